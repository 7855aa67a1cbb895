/*
 * zkvc.h - Groth16 prover for the matrix-multiplication statement Y = X W on
 * BN254, for AMD MI355X (gfx950).
 *
 * The statement follows the paper's use case (Section I and Figure 1): a
 * client holds X, a server holds the weights W, returns Y = X W and proves
 * that Y is correct without revealing W.  X and Y are public inputs; W is
 * private.  Gen, Prove and Verify are the three algorithms of a zk-SNARK
 * (Section II); the backend is Groth16 (Section IV, zkVC-G).  Two circuits
 * are provided: the per-product R1CS and the paper's constraint-reduced
 * polynomial circuit with prefix-sum queries (Section III-A, III-B), plus the
 * remaining rows of the ablation in Table II.
 *
 * Conventions for every entry point:
 *   - All integers are little-endian.  Field elements at this interface are
 *     canonical integers (value < modulus) unless a flag selects the
 *     library's internal layout (ZKVC_LAYOUT_MONT: 8 words holding
 *     x * 2^261 mod modulus).
 *   - A G1 point is (x, y); a G2 point is (x0, x1, y0, y1) with x = x0 + x1 i
 *     over Fq2 = Fq[i]/(i^2 + 1).  The all-zero encoding is the point at
 *     infinity.
 *   - Ownership: the caller owns every buffer it passes (host or device) and
 *     keeps it alive for the duration of the call.  The library owns proving
 *     keys until zkvc_pk_free and its own scratch memory.
 *   - Streams: hip_stream is a hipStream_t (NULL = the default stream).  Every
 *     call is synchronous with respect to its outputs: when it returns, host
 *     outputs are written and device outputs are complete.  Calls on
 *     different streams may run concurrently, except that two calls using
 *     the same proving key must not overlap.
 *   - Errors: negative return codes; no exception crosses this interface and
 *     nothing aborts.  zkvc_strerror gives the last error message of the
 *     calling thread.
 */
#ifndef ZKVC_H
#define ZKVC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ZKVC_OK 0
#define ZKVC_EINVAL (-1)  /* null pointer, empty or oversized shape, bad flag, value out of range */
#define ZKVC_ENOMEM (-2)  /* device allocation failed or exceeded ZKVC_MEMORY_BUDGET_MB */
#define ZKVC_EDEVICE (-3) /* a HIP runtime error */
#define ZKVC_EFORMAT (-4) /* malformed verification-key blob */

typedef struct { uint32_t l[8]; } zkvc_fr;
typedef struct { uint32_t x[8], y[8]; } zkvc_g1;
typedef struct { uint32_t x0[8], x1[8], y0[8], y1[8]; } zkvc_g2;
typedef struct { zkvc_g1 A; zkvc_g2 B; zkvc_g1 C; } zkvc_proof; /* 256 bytes */

/* Constraint systems (Section III and Table II). */
enum {
  ZKVC_PLAIN = 0,     /* one constraint per product x_ik w_kj; the output sum is folded
                         into the last product's constraint: a*b*n constraints */
  ZKVC_CRPC_PSQ = 1,  /* CRPC with prefix sums: n constraints X_k(z) W_k(z) = s_k - s_(k-1) */
  ZKVC_PLAIN_ADD = 2, /* per-product plus one long-addition constraint per output */
  ZKVC_PLAIN_PSQ = 3, /* per-product with prefix sums in place of products */
  ZKVC_CRPC = 4       /* CRPC with products and one final addition: n + 1 constraints */
};

typedef struct {
  uint32_t a, n, b; /* X is a x n, W is n x b, Y is a x b */
  uint32_t kind;    /* one of the ZKVC_* circuit kinds above */
} zkvc_shape;

typedef struct zkvc_pk zkvc_pk; /* opaque proving key, resident in device memory */

/* Flags for zkvc_ntt_fr, zkvc_msm_g1, zkvc_msm_g2, zkvc_fixed_base_*. */
#define ZKVC_NTT_INVERSE 1u  /* inverse transform, including the 1/N factor */
#define ZKVC_NTT_COSET 2u    /* forward: input j scaled by g^j first; inverse: output j scaled by g^-j; g = 5 */
#define ZKVC_LAYOUT_MONT 4u  /* operands in the library's internal Montgomery layout */

/*
 * Gen (Section II; Groth16 key generation for the circuit of `shape`).
 * Shapes: a, n, b >= 1, a <= 65535, a n b <= 2^28, QAP domain <= 2^28.
 * toxic = {tau, alpha, beta, gamma, delta}: nonzero elements of Fr, canonical;
 * tau must lie outside the evaluation domain (tau^N != 1).  z is the public
 * CRPC evaluation point (Section III-A's variable Z), required nonzero for the
 * CRPC kinds and ignored otherwise.  On success *pk_out receives a proving
 * key in device memory.  The verification key is serialized into vk; if vk
 * is NULL only the required size is written to *vk_len.  On input *vk_len
 * is the capacity of vk.  Errors: ZKVC_EINVAL (bad shape/kind/toxic/z, or vk
 * too small), ZKVC_ENOMEM, ZKVC_EDEVICE.
 */
int zkvc_setup(const zkvc_shape* shape, const zkvc_fr toxic[5], const zkvc_fr* z, zkvc_pk** pk_out,
               uint8_t* vk, size_t* vk_len, void* hip_stream);

/* Releases a proving key and its device memory.  NULL is accepted. */
int zkvc_pk_free(zkvc_pk* pk);

/*
 * Prove (Section II; Groth16 proof that Y = X W).
 * X: host int8 a x n row-major; W: host int8 n x b row-major (private);
 * r, s: the prover's blinding scalars, canonical Fr (the caller draws them).
 * Writes Y = X W (host int32 a x b row-major) and the 256-byte proof.
 * Errors: ZKVC_EINVAL (null pointer, r or s >= r), ZKVC_ENOMEM, ZKVC_EDEVICE.
 */
int zkvc_prove(const zkvc_pk* pk, const int8_t* X, const int8_t* W, const zkvc_fr* r, const zkvc_fr* s,
               int32_t* Y_out, zkvc_proof* proof_out, void* hip_stream);

/*
 * Prove with device-resident operands (Section II; the same proof as
 * zkvc_prove): d_X (int8 a x n row-major), d_W (int8 n x b row-major) and
 * d_Y (int32 a x b row-major, written) are device buffers on the proving
 * key's device, owned by the caller; nothing crosses PCIe but the 256-byte
 * proof (host).  The call is synchronous: d_Y and *proof_out are complete
 * when it returns.  Errors: ZKVC_EINVAL (null pointer, a buffer that is not
 * device memory of the key's device, r or s >= r), ZKVC_ENOMEM, ZKVC_EDEVICE.
 */
int zkvc_prove_device(const zkvc_pk* pk, const int8_t* d_X, const int8_t* d_W, const zkvc_fr* r, const zkvc_fr* s,
                      int32_t* d_Y, zkvc_proof* proof_out, void* hip_stream);

/* One proof of a batch (zkvc_prove_batch): the arguments of zkvc_prove. */
typedef struct {
  const zkvc_pk* pk;      /* proving key of this proof's shape and circuit kind */
  const int8_t* X;        /* host int8 a x n row-major (public) */
  const int8_t* W;        /* host int8 n x b row-major (private) */
  zkvc_fr r, s;           /* blinding scalars, canonical Fr */
  int32_t* Y_out;         /* host int32 a x b row-major, written */
  zkvc_proof* proof_out;  /* host, written */
} zkvc_prove_job;

/*
 * Batched proving (the same statement as zkvc_prove, many at once).  The
 * proofs may use keys of different shapes and kinds, and a key may repeat.
 * All stages run once for the whole batch: the witnesses, the quotient
 * transforms of all proofs of one domain size in shared launches, and every
 * multi-scalar multiplication of the batch in three shared pipelines (G1
 * queries, the G2 query, the H query).  Every proof and Y equal, bit for bit,
 * what zkvc_prove returns for the same job.  Synchronous; the library keeps
 * one batch context per (device, stream), so calls on one stream serialize
 * and calls on different streams run concurrently.  Keys are only read.
 * Errors: ZKVC_EINVAL (no jobs, null pointer, r or s >= r, a key on another
 * device), ZKVC_ENOMEM, ZKVC_EDEVICE.
 */
int zkvc_prove_batch(const zkvc_prove_job* jobs, size_t njobs, void* hip_stream);

/*
 * Graph replay of repeated proofs (off by default).  When on, zkvc_prove and
 * zkvc_prove_batch capture the device work of a composition (the sequence of
 * keys of a call, on one stream) into a HIP graph the second time it runs in
 * a row on a context, and replay that graph for later calls of the same
 * composition: one launch instead of one per kernel, with only X and W
 * restaged.  Results are bit-identical either way.  Off by default because
 * the eager launches on the context's three streams measured faster (the
 * graph's nodes are dispatched in capture order, which delays the lanes
 * captured last).  The proving server always launches eagerly.  enable: 1
 * on, 0 off (process-wide, affects later calls).  Returns the previous
 * setting.  Host only; never fails.
 */
int zkvc_set_graphs(int enable);

/*
 * Proving server (continuous batching).  One worker thread proves submitted
 * jobs in batches: each batch takes the queued jobs in order while they fit
 * max_batch and memory_budget, and is enqueued while the previous batch is
 * still on the device, so jobs that arrive during a batch overlap it.
 * memory_budget (bytes; 0 = no limit) bounds the estimated device workspace
 * of the jobs in flight, the batch being admitted plus the one still on the
 * device; a job's estimate is zkvc_pk_info().prove_bytes, and a job whose
 * estimate alone exceeds the budget is rejected at submission.  Workspace
 * buffers replaced by growth are freed when nothing is in flight.  Every
 * result equals zkvc_prove's for the same job, bit for bit.  The server is
 * created on the current device and owns its own streams.
 */
typedef struct zkvc_server zkvc_server;
typedef struct {
  uint32_t max_batch;      /* most proofs per batch, >= 1 */
  uint64_t memory_budget;  /* bytes of estimated workspace in flight, 0 = unlimited */
} zkvc_server_config;
typedef struct {
  int32_t status;          /* ZKVC_OK, or the error code of the job's batch */
  uint32_t batch_size;     /* proofs in the batch that carried the job */
  double queue_ms;         /* submission to the start of its batch */
  double latency_ms;       /* submission to Y and the proof written */
} zkvc_server_result;
/* Errors: ZKVC_EINVAL (null pointer, max_batch 0). */
int zkvc_server_create(const zkvc_server_config* config, zkvc_server** server_out);
/* Queues one job and returns its ticket.  X and W are copied before return;
 * Y_out and proof_out must stay valid until zkvc_server_wait returns for the
 * ticket.  Errors: ZKVC_EINVAL (null pointer, r or s >= r, key on another
 * device, server stopping), ZKVC_ENOMEM (the job's estimate exceeds the
 * memory budget). */
int zkvc_server_submit(zkvc_server* server, const zkvc_prove_job* job, uint64_t* ticket);
/* Blocks until the job is done (results written), then reports it; each
 * ticket is reported once.  Errors: ZKVC_EINVAL (unknown ticket),
 * ZKVC_EDEVICE (the worker could not start). */
int zkvc_server_wait(zkvc_server* server, uint64_t ticket, zkvc_server_result* result);
/* Proves every job still queued, stops the worker and frees the server.
 * NULL is accepted. */
int zkvc_server_destroy(zkvc_server* server);

/*
 * Verify (Section II; the Groth16 pairing-product equation), on the host.
 * vk: blob written by zkvc_setup; X: int8 a x n; Y: int32 a x b (the shape is
 * read from vk).  Returns 1 if the proof is valid for (X, Y), 0 if not
 * (including points off the curve, at infinity, or B outside the order-r
 * subgroup), ZKVC_EFORMAT for a malformed blob, ZKVC_EINVAL for null pointers.
 */
int zkvc_verify(const uint8_t* vk, size_t vk_len, const int8_t* X, const int32_t* Y,
                const zkvc_proof* proof);

/*
 * In-place number-theoretic transform over Fr of N = 2^log_n elements on the
 * device (d_data: N elements of 8 words), natural order in and out:
 *   forward: X_k = sum_j x_j omega^(jk), omega = 5^((r-1)/N)
 *   inverse: x_j = N^-1 sum_k X_k omega^(-jk)
 * plus the coset scalings of ZKVC_NTT_COSET.  This is the transform the QAP
 * quotient uses (Section II: the QAP comes from the R1CS by interpolation).
 * 0 <= log_n <= 28.  Elements must be < r.  Errors: ZKVC_EINVAL, ZKVC_ENOMEM,
 * ZKVC_EDEVICE.
 */
int zkvc_ntt_fr(void* d_data, uint32_t log_n, uint32_t flags, void* hip_stream);

/*
 * Multi-scalar multiplication sum_i s_i P_i over G1: the operation that
 * Groth16's Prove (Section II; the backend of Section IV) spends its time on,
 * computing the A, B1, L and H query sums of the proof from the witness and
 * the quotient coefficients.  d_points: n affine points (16 words each); d_scalars: n Fr
 * elements (8 words each); both in device memory.  Points must lie on the
 * curve (the all-zero encoding, infinity, is allowed); scalars must be < r.
 * The result is written to *out (host).  n = 0 gives infinity.
 * Errors: ZKVC_EINVAL, ZKVC_ENOMEM, ZKVC_EDEVICE.
 */
int zkvc_msm_g1(const void* d_points, const void* d_scalars, size_t n, uint32_t flags, zkvc_g1* out,
                void* hip_stream);

/* As zkvc_msm_g1 over G2: the B query sum of Groth16's Prove (Section II),
 * the proof's G2 element.  d_points: n affine points of 32 words each
 * (x0, x1, y0, y1), which must lie in the order-r subgroup of the twist;
 * d_scalars as for zkvc_msm_g1.  The result is written to *out (host).
 * n = 0 gives infinity.  Errors: ZKVC_EINVAL, ZKVC_ENOMEM, ZKVC_EDEVICE. */
int zkvc_msm_g2(const void* d_points, const void* d_scalars, size_t n, uint32_t flags, zkvc_g2* out,
                void* hip_stream);

/*
 * zkvc_msm_g1 without allocating, for callers that cannot allocate memory:
 * code under HIP graph capture, tight serving loops, and hosts that forbid
 * device allocation.  Same arguments, layout, flags and result as
 * zkvc_msm_g1 (the same kernels; the window width and task size always
 * follow the built-in rules, never the autotuner's).  Its workspace is a
 * fixed 56 MiB device array that each GPU holds from the library's load
 * until the process ends, plus a fixed host array; no hipMalloc, hipFree or
 * pinned allocation happens in the call.  n <= 65536; a larger n is rejected
 * with ZKVC_EINVAL before anything is launched.  Calls in one process are
 * serialized by a lock, since every call on a GPU shares that GPU's array
 * (overlapping calls would race on it); the array keeps the last call's
 * contents, and nothing in the pipeline reads a location it has not written
 * in the same call.  Synchronous like zkvc_msm_g1.  Errors: ZKVC_EINVAL,
 * ZKVC_EDEVICE.
 */
int zkvc_msm_g1_noalloc(const void* d_points, const void* d_scalars, size_t n, uint32_t flags, zkvc_g1* out,
                        void* hip_stream);

/* Message for the last error on the calling thread (or for the code if none). */
const char* zkvc_strerror(int err);

/* ---------------------------------------------------------------- support calls */

/*
 * Fixed-base batch multiplication (Groth16 key generation): out_i = [k_i] G
 * for the standard generator G of G1 (resp. G2), written as affine points.
 * d_scalars: n Fr elements (device); d_points_out: n points (device, 16 or
 * 32 words each).  ZKVC_LAYOUT_MONT selects the internal layout for both.
 */
int zkvc_fixed_base_g1(const void* d_scalars, size_t n, void* d_points_out, uint32_t flags, void* hip_stream);
int zkvc_fixed_base_g2(const void* d_scalars, size_t n, void* d_points_out, uint32_t flags, void* hip_stream);

/* Sizes of a proving key's queries (number of points). */
typedef struct {
  uint32_t a, n, b, kind;
  uint32_t log_n;       /* QAP domain size N = 2^log_n */
  uint64_t num_vars;    /* full assignment length */
  uint64_t num_public;  /* l: public inputs excluding the constant */
  uint64_t a_query, b_query, l_query, h_query;
  uint64_t device_bytes; /* proving key plus its proving workspace */
  uint64_t prove_bytes;  /* estimated device workspace of one proof in a batch (server admission) */
} zkvc_pk_info_t;
int zkvc_pk_info(const zkvc_pk* pk, zkvc_pk_info_t* info);

/* Query identifiers for zkvc_pk_export. */
enum { ZKVC_Q_A = 0, ZKVC_Q_B1 = 1, ZKVC_Q_B2 = 2, ZKVC_Q_L = 3, ZKVC_Q_H = 4, ZKVC_Q_CONST = 5 };
/*
 * Copies entries [start, start + count) of a proving-key query to host memory
 * as canonical affine points (zkvc_g1, or zkvc_g2 for ZKVC_Q_B2).  For
 * ZKVC_Q_CONST the entries are alpha1, beta1, delta1 (zkvc_g1) followed by
 * beta2, delta2 (zkvc_g2), and start/count are ignored.  Query order, with
 * variables numbered 0 = constant, then x (a*n), y (a*b), w (n*b), auxiliary:
 *   A:      [u_i(tau)]1 for i = 0 .. l, then (PLAIN_ADD, CRPC) the auxiliary variables
 *   B1, B2: [v_i(tau)]1,2 for the w variables, then (PLAIN_ADD, CRPC) the constant
 *   L:      [(beta u_i + alpha v_i + w_i)(tau)/delta]1 for the w, then auxiliary variables
 *   H:      [(tau^N - 1)/delta * L'_a(tau)]1 for a = 0 .. N-1, where L'_a is the
 *           Lagrange basis polynomial of the coset g H = {5 omega_N^a} at the
 *           point 5 omega_N^a (omega_N = w^(2^(28-log_n)), w = 5^((r-1)/2^28)):
 *           L'_a(X) = (X^N - 5^N) x_a / (N 5^N (X - x_a)).  The prover takes h
 *           = (A B - C) / Z as its values on that coset, so sum_a h(x_a) H_a
 *           equals the textbook sum_j h_j [tau^j (tau^N - 1)/delta]1
 *           (Section II, Groth16 Prove): the proof is the same.
 * Used to spot-check keys.  Errors: ZKVC_EINVAL (unknown query or range).
 */
int zkvc_pk_export(const zkvc_pk* pk, uint32_t query, uint64_t start, uint64_t count, void* host_out);

/* Per-stage device times (milliseconds, from HIP events on the calling
 * stream) of the last zkvc_prove with this key: witness and evaluation
 * vectors, the QAP quotient, then from the end of the quotient to the end of
 * the last multi-scalar multiplication (the G1 and G2 queries other than H
 * start right after the witness, on the key's own streams, overlapping the
 * quotient), then the host-side plane combination and assembly left after
 * the device work, and the wall time of the whole call. */
typedef struct {
  float witness_ms, ntt_ms, msm_ms, host_ms, total_ms;
} zkvc_prove_stats;
int zkvc_pk_last_stats(const zkvc_pk* pk, zkvc_prove_stats* out);

/*
 * Autotuner.  Times candidate settings on synthetic inputs on the device
 * (hip_stream) and keeps the fastest for the rest of the process: the MSM
 * window width for wide scalars and the thread-task size per power-of-two
 * size 2^min_log..2^max_log (G2 up to 2^18), and the largest sub-transform per
 * NTT pass per domain size.  Proving keys built later use the tuned values
 * too; results never depend on them (bit-exact either way), only speed.
 * Returns the number of settings chosen (>= 0) or an error: ZKVC_EINVAL
 * (unknown target, sizes outside 4 <= min_log <= max_log <= 22),
 * ZKVC_ENOMEM, ZKVC_EDEVICE.
 */
#define ZKVC_TUNE_MSM_G1 1u
#define ZKVC_TUNE_MSM_G2 2u
#define ZKVC_TUNE_NTT 4u
int zkvc_autotune(uint32_t what, uint32_t min_log, uint32_t max_log, void* hip_stream);
/* The tuned settings as text, one "<key> <log2 size> <value>" line each
 * (keys msm_g1, msm_g2, msm_kdiv, ntt); with buf NULL only the size
 * (including the terminating zero) is written to *len.  Host only. */
int zkvc_tune_export(char* buf, size_t* len);
/* Loads settings in the export format (value 0 restores the built-in rule).
 * All lines are checked before any is applied.  ZKVC_EINVAL on a malformed
 * line or a value out of range.  Host only. */
int zkvc_tune_import(const char* text);

/*
 * Elementwise field operations on device arrays, for arithmetic parity
 * tests.  field: 0 = Fq, 1 = Fr.  op: 0 add, 1 sub, 2 mul, 3 sqr, 4 inv
 * (of nonzero), 5 to-internal (canonical -> Montgomery), 6 from-internal.
 * Inputs and output are n elements of 8 words in device memory; a, b and
 * out are canonical integers except for ops 5 and 6.
 */
int zkvc_field_op(uint32_t field, uint32_t op, const void* d_a, const void* d_b, void* d_out, size_t n,
                  void* hip_stream);

/*
 * Kernel profiling with HIP events on the launching stream.  zkvc_profile_begin
 * clears earlier records and turns recording on; every instrumented launch
 * then records a start and stop event and its algorithmic work units (bucket
 * additions for MSM accumulation, butterflies for NTT passes, elements for
 * the others).  zkvc_profile_read turns recording off, waits for the events
 * and writes one aggregate per kernel name (up to `capacity`; *count receives
 * the number of kernels seen).  Recording adds two event records per launch;
 * for the single-kernel scopes (the MSM bucket accumulation, the quotient's
 * last NTT kernel) the two events are bound to the kernel's own dispatch on
 * eager streams (hipExtLaunchKernel), so they time the kernel itself and add
 * no marker packet between it and the next launch.
 */
typedef struct {
  char name[48];
  uint64_t launches;
  double total_ms;
  double work;
} zkvc_kernel_stat;
int zkvc_profile_begin(void);
int zkvc_profile_read(zkvc_kernel_stat* out, int capacity, int* count);
/* Restricts recording to the instrumented launches whose names (as reported
 * by zkvc_profile_read) are listed in `kernels`, comma separated; NULL or ""
 * records every launch again.  Timing a few kernels then costs two event
 * records per launch of those kernels only.  Takes effect for launches
 * enqueued afterwards.  Host only; ZKVC_EINVAL if the list is 4096 bytes or
 * longer. */
int zkvc_profile_select(const char* kernels);

/* ---------------------------------------------------------------- Spartan (zkVC-S) */

/*
 * The paper's second backend, Spartan (Section II names it among the
 * transparent SNARKs; Section IV uses it for zkVC-S; Table II times it beside
 * Groth16), for the CRPC kinds (ZKVC_CRPC_PSQ, ZKVC_CRPC).  The paper fixes
 * neither its commitment nor its curve; this implementation takes Spartan's
 * NIZK with a verifier that evaluates the constraint matrices itself, over
 * the BN254 scalar field, with the witness committed row by row by Pedersen
 * commitments in G1 (square-root layout), without zero-knowledge blinding,
 * and Fiat-Shamir by SHA-256.  The witness half of z (W entries, then the
 * auxiliary values, zero-padded to 2^(sy-1)) is a rows x cols matrix; a proof
 * is, all little-endian and canonical:
 *   rows commitments (64 bytes each, affine x then y, all-zero = infinity),
 *   sx rounds x 4 values of sum-check 1 (32 bytes each),
 *   vA, vB, vC, sy rounds x 3 values of sum-check 2, and cols opening values.
 * The caller supplies the commitment generators (cols points of G1, none at
 * infinity); their discrete logarithms must be unknown to provers (e.g. a
 * hash-to-curve), which the library cannot check.
 */
typedef struct zkvc_spartan_key zkvc_spartan_key; /* opaque, device-resident */
typedef struct {
  uint64_t constraints;   /* m: rows of the R1CS */
  uint32_t sx, sy;        /* variables of the two sum-checks: 2^sx >= m rows, 2^sy entries of z */
  uint32_t rows, cols;    /* the witness matrix; cols generators are needed */
  uint64_t proof_bytes;
} zkvc_spartan_info_t;
/* Sizes of the Spartan instance of a shape (host only).  Errors: ZKVC_EINVAL
 * (bad shape, or a kind other than the CRPC ones). */
int zkvc_spartan_info(const zkvc_shape* shape, zkvc_spartan_info_t* out);
/* Key for a shape: z (the public CRPC point, nonzero) and the cols
 * generators (host, canonical affine).  Errors: ZKVC_EINVAL, ZKVC_ENOMEM,
 * ZKVC_EDEVICE. */
int zkvc_spartan_setup(const zkvc_shape* shape, const zkvc_fr* z, const zkvc_g1* gens, size_t ngens,
                       zkvc_spartan_key** key_out, void* hip_stream);
int zkvc_spartan_key_free(zkvc_spartan_key* key);
/* Proves Y = X W (X, W host int8 row-major); writes Y (host int32) and the
 * proof (proof_len must equal the info's proof_bytes).  Synchronous.  Calls
 * with one key serialize.  Errors: ZKVC_EINVAL, ZKVC_ENOMEM, ZKVC_EDEVICE. */
int zkvc_spartan_prove(zkvc_spartan_key* key, const int8_t* X, const int8_t* W, int32_t* Y_out, uint8_t* proof,
                       size_t proof_len, void* hip_stream);
/* Host verifier: 1 valid, 0 invalid (including a proof of the wrong length,
 * values out of range or points off the curve), <0 for bad arguments. */
int zkvc_spartan_verify(const zkvc_shape* shape, const zkvc_fr* z, const zkvc_g1* gens, size_t ngens,
                        const int8_t* X, const int32_t* Y, const uint8_t* proof, size_t proof_len);

/*
 * Integer-VALU peak microbenchmark.  Every field product of the prover is a
 * column of 32x32 -> 64-bit multiply-adds (v_mad_u64_u32), so the rate at
 * which the device issues that instruction is the roofline of the bucket
 * accumulation and NTT kernels.  Runs 8 blocks of 256 threads per compute
 * unit, each thread 16 independent multiply-add chains of 4 * iters steps,
 * on hip_stream (one warm-up launch, one timed with HIP events), and reports:
 * the multiply-adds executed and their rate over the timed launch; the shader
 * clock during the loop (clock counter against the constant-rate counter);
 * and lane operations per compute unit per clock (64 would be one wave64
 * instruction per cycle per compute unit).  1 <= iters <= 2^20.
 * Errors: ZKVC_EINVAL, ZKVC_ENOMEM, ZKVC_EDEVICE.
 */
typedef struct {
  double mads;                /* multiply-adds executed by the timed launch */
  double ms;                  /* its duration (HIP events) */
  double mad_per_s;           /* mads / duration */
  double clock_ghz;           /* average shader clock over the blocks' loops */
  double lane_ops_per_cu_clk; /* mad_per_s / (compute units * clock) */
  uint32_t compute_units;
} zkvc_valu_peak_t;
int zkvc_valu_peak(uint32_t iters, zkvc_valu_peak_t* out, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ZKVC_H */
