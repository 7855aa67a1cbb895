// C-ABI entry points for the standalone kernels: NTT, MSM, fixed-base
// multiplication and elementwise field operations.
#include <cstring>

#include "api_common.hpp"
#include "field.hpp"
#include "msm.hpp"
#include "ntt.hpp"

using namespace zkvc;

namespace {

__global__ void k_field_op(int field, int op, const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (field == 0) {
    Fq x = Fq::load(a + 8ull * i), y = b ? Fq::load(b + 8ull * i) : Fq::zero(), z;
    if (op <= 4) {
      x = Fq::to_mont(x);
      y = Fq::to_mont(y);
    }
    switch (op) {
      case 0: z = Fq::add(x, y); break;
      case 1: z = Fq::sub(x, y); break;
      case 2: z = Fq::mul(x, y); break;
      case 3: z = Fq::sqr(x); break;
      case 4: z = Fq::inv(x); break;
      case 5: z = Fq::to_mont(x); break;
      default: z = Fq::from_mont(x); break;
    }
    if (op <= 4) z = Fq::from_mont(z);
    z.store(out + 8ull * i);
  } else {
    Fr x = Fr::load(a + 8ull * i), y = b ? Fr::load(b + 8ull * i) : Fr::zero(), z;
    if (op <= 4) {
      x = Fr::to_mont(x);
      y = Fr::to_mont(y);
    }
    switch (op) {
      case 0: z = Fr::add(x, y); break;
      case 1: z = Fr::sub(x, y); break;
      case 2: z = Fr::mul(x, y); break;
      case 3: z = Fr::sqr(x); break;
      case 4: z = Fr::inv(x); break;
      case 5: z = Fr::to_mont(x); break;
      default: z = Fr::from_mont(x); break;
    }
    if (op <= 4) z = Fr::from_mont(z);
    z.store(out + 8ull * i);
  }
}

}  // namespace

namespace zkvc {

void g1_to_abi(const host::G1J& p, zkvc_g1* out) {
  std::memset(out, 0, sizeof(*out));
  if (p.is_inf()) return;
  host::HFq x, y;
  p.to_affine(x, y);
  x.to_u32(out->x);
  y.to_u32(out->y);
}

void g2_to_abi(const host::G2J& p, zkvc_g2* out) {
  std::memset(out, 0, sizeof(*out));
  if (p.is_inf()) return;
  host::HFq2 x, y;
  p.to_affine(x, y);
  x.c0.to_u32(out->x0);
  x.c1.to_u32(out->x1);
  y.c0.to_u32(out->y0);
  y.c1.to_u32(out->y1);
}

}  // namespace zkvc

extern "C" {

int zkvc_ntt_fr(void* d_data, uint32_t log_n, uint32_t flags, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(log_n <= 28, "log_n must be <= 28");
    ZK_REQUIRE((flags & ~(ZKVC_NTT_INVERSE | ZKVC_NTT_COSET | ZKVC_LAYOUT_MONT)) == 0, "unknown NTT flag");
    const size_t n = (size_t)1 << log_n;
    require_device_range(d_data, n * 32, "d_data");
    hipStream_t st = (hipStream_t)hip_stream;
    const NttTables& T = ntt_tables(current_device());
    const bool canon = !(flags & ZKVC_LAYOUT_MONT);
    const bool inverse = flags & ZKVC_NTT_INVERSE;
    const bool coset = flags & ZKVC_NTT_COSET;
    NttFuse f;
    f.in_canonical = canon;
    f.out_canonical = canon;
    if (!inverse) {
      if (coset) f.pre_coset = 1;
    } else {
      f.post_const = T.ninv + 8 * log_n;
      if (coset) {
        f.post_coset = -1;
        f.post_bitrev = true;
      }
    }
    uint32_t* data = static_cast<uint32_t*>(d_data);
    ntt_launch(data, (int)log_n, false, inverse, f, st);
    bitrev_launch(data, (int)log_n, st);
    ZK_HIP(hipStreamSynchronize(st));
  });
}

int zkvc_msm_g1(const void* d_points, const void* d_scalars, size_t n, uint32_t flags, zkvc_g1* out,
                void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(out != nullptr, "out is null");
    ZK_REQUIRE((flags & ~ZKVC_LAYOUT_MONT) == 0, "unknown MSM flag");
    if (n == 0) {
      std::memset(out, 0, sizeof(*out));
      return;
    }
    require_device_range(d_points, n * 64, "d_points");
    require_device_range(d_scalars, n * 32, "d_scalars");
    hipStream_t st = (hipStream_t)hip_stream;
    StreamWorkspace& sw = stream_workspace(st);
    std::lock_guard<std::mutex> lock(sw.mu);
    const uint32_t* pts = static_cast<const uint32_t*>(d_points);
    if (!(flags & ZKVC_LAYOUT_MONT)) {
      uint32_t* conv = sw.ws.get(1, n * 64);
      points_to_mont_g1(pts, conv, n, st);
      pts = conv;
    }
    MsmInput in;
    in.points = pts;
    in.npoints = n;
    in.scalars = static_cast<const uint32_t*>(d_scalars);
    in.nscalars = n;
    in.scalars_mont = flags & ZKVC_LAYOUT_MONT;
    in.max_bits = 253;
    g1_to_abi(msm_g1(in, sw.ws, st), out);
  });
}

int zkvc_msm_g2(const void* d_points, const void* d_scalars, size_t n, uint32_t flags, zkvc_g2* out,
                void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(out != nullptr, "out is null");
    ZK_REQUIRE((flags & ~ZKVC_LAYOUT_MONT) == 0, "unknown MSM flag");
    if (n == 0) {
      std::memset(out, 0, sizeof(*out));
      return;
    }
    require_device_range(d_points, n * 128, "d_points");
    require_device_range(d_scalars, n * 32, "d_scalars");
    hipStream_t st = (hipStream_t)hip_stream;
    StreamWorkspace& sw = stream_workspace(st);
    std::lock_guard<std::mutex> lock(sw.mu);
    const uint32_t* pts = static_cast<const uint32_t*>(d_points);
    if (!(flags & ZKVC_LAYOUT_MONT)) {
      uint32_t* conv = sw.ws.get(1, n * 128);
      points_to_mont_g2(pts, conv, n, st);
      pts = conv;
    }
    MsmInput in;
    in.points = pts;
    in.npoints = n;
    in.scalars = static_cast<const uint32_t*>(d_scalars);
    in.nscalars = n;
    in.scalars_mont = flags & ZKVC_LAYOUT_MONT;
    in.max_bits = 253;
    g2_to_abi(msm_g2(in, sw.ws, st), out);
  });
}

int zkvc_fixed_base_g1(const void* d_scalars, size_t n, void* d_points_out, uint32_t flags, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE((flags & ~ZKVC_LAYOUT_MONT) == 0, "unknown flag");
    if (n == 0) return;
    require_device_range(d_scalars, n * 32, "d_scalars");
    require_device_range(d_points_out, n * 64, "d_points_out");
    hipStream_t st = (hipStream_t)hip_stream;
    StreamWorkspace& sw = stream_workspace(st);
    std::lock_guard<std::mutex> lock(sw.mu);
    const bool mont = flags & ZKVC_LAYOUT_MONT;
    fixed_base_g1(static_cast<const uint32_t*>(d_scalars), mont, n, static_cast<uint32_t*>(d_points_out), !mont,
                  sw.ws, st);
    ZK_HIP(hipStreamSynchronize(st));
  });
}

int zkvc_fixed_base_g2(const void* d_scalars, size_t n, void* d_points_out, uint32_t flags, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE((flags & ~ZKVC_LAYOUT_MONT) == 0, "unknown flag");
    if (n == 0) return;
    require_device_range(d_scalars, n * 32, "d_scalars");
    require_device_range(d_points_out, n * 128, "d_points_out");
    hipStream_t st = (hipStream_t)hip_stream;
    StreamWorkspace& sw = stream_workspace(st);
    std::lock_guard<std::mutex> lock(sw.mu);
    const bool mont = flags & ZKVC_LAYOUT_MONT;
    fixed_base_g2(static_cast<const uint32_t*>(d_scalars), mont, n, static_cast<uint32_t*>(d_points_out), !mont,
                  sw.ws, st);
    ZK_HIP(hipStreamSynchronize(st));
  });
}

int zkvc_field_op(uint32_t field, uint32_t op, const void* d_a, const void* d_b, void* d_out, size_t n,
                  void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(field <= 1 && op <= 6, "bad field or op");
    if (n == 0) return;
    ZK_REQUIRE(n < (1ull << 31), "n too large");
    require_device_range(d_a, n * 32, "d_a");
    const bool binary = op <= 2;
    if (binary) require_device_range(d_b, n * 32, "d_b");
    require_device_range(d_out, n * 32, "d_out");
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_field_op, dim3(cdiv(n, 128)), dim3(128), 0, st, (int)field, (int)op,
                       static_cast<const uint32_t*>(d_a), binary ? static_cast<const uint32_t*>(d_b) : nullptr,
                       static_cast<uint32_t*>(d_out), (uint32_t)n);
    ZK_HIP(hipGetLastError());
    ZK_HIP(hipStreamSynchronize(st));
  });
}

const char* zkvc_strerror(int err) {
  const std::string& m = last_error();
  if (!m.empty()) return m.c_str();
  switch (err) {
    case ZKVC_OK: return "ok";
    case ZKVC_EINVAL: return "invalid argument";
    case ZKVC_ENOMEM: return "out of device memory";
    case ZKVC_EDEVICE: return "HIP runtime error";
    case ZKVC_EFORMAT: return "malformed verification key";
    default: return "unknown error";
  }
}

}  // extern "C"
