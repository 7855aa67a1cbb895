// C-ABI entry points for Groth16: setup, prove, verify and proving-key access.
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "api_common.hpp"
#include "prover.hpp"

using namespace zkvc;

namespace {

size_t vk_size(const Layout& L) { return 8 + 24 + 32 + 64 + 3 * 128 + 8 + 64 * (L.ell + 1); }

}  // namespace

extern "C" {

int zkvc_setup(const zkvc_shape* shape, const zkvc_fr toxic[5], const zkvc_fr* z, zkvc_pk** pk_out, uint8_t* vk,
               size_t* vk_len, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(shape && toxic && vk_len, "null argument");
    const Layout L = r1cs_layout(shape->a, shape->n, shape->b, shape->kind);
    const size_t need = vk_size(L);
    if (vk == nullptr) {
      *vk_len = need;
      return;
    }
    ZK_REQUIRE(pk_out != nullptr, "pk_out is null");
    ZK_REQUIRE(*vk_len >= need, "vk buffer too small");
    host::HFr tox[5];
    for (int k = 0; k < 5; k++) tox[k] = fr_in(toxic[k], "toxic waste");
    host::HFr zz;
    const bool use_z = kind_uses_z(L.kind);
    if (use_z) {
      ZK_REQUIRE(z != nullptr, "this circuit kind needs z");
      zz = fr_in(*z, "z");
    }
    std::vector<uint8_t> blob;
    zkvc_pk* pk = groth16_setup(L, tox, use_z ? &zz : nullptr, blob, (hipStream_t)hip_stream);
    std::memcpy(vk, blob.data(), blob.size());
    *vk_len = blob.size();
    *pk_out = pk;
  });
}

int zkvc_pk_free(zkvc_pk* pk) {
  return guarded([&] { delete pk; });
}

int zkvc_prove(const zkvc_pk* pk, const int8_t* X, const int8_t* W, const zkvc_fr* r, const zkvc_fr* s,
               int32_t* Y_out, zkvc_proof* proof_out, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(pk && X && W && r && s && Y_out && proof_out, "null argument");
    zkvc_pk* k = const_cast<zkvc_pk*>(pk);
    std::lock_guard<std::mutex> lock(k->mu);
    const host::HFr rr = fr_in(*r, "r"), ss = fr_in(*s, "s");
    int dev = current_device();
    ZK_REQUIRE(dev == k->device, "the proving key lives on another device");
    groth16_prove(k, X, W, rr, ss, Y_out, proof_out, (hipStream_t)hip_stream);
  });
}

namespace {
// A caller's device buffer: memory of the given device (device or managed).
void require_device_buffer(const void* p, int dev, const char* what) {
  hipPointerAttribute_t at{};
  const hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(ZKVC_EINVAL, std::string(what) + " is not a device buffer");
  }
  ZK_REQUIRE(at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged,
             std::string(what) + " is not a device buffer");
  ZK_REQUIRE(at.device == dev, std::string(what) + " lives on another device");
}
}  // namespace

int zkvc_prove_device(const zkvc_pk* pk, const int8_t* d_X, const int8_t* d_W, const zkvc_fr* r, const zkvc_fr* s,
                      int32_t* d_Y, zkvc_proof* proof_out, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(pk && d_X && d_W && r && s && d_Y && proof_out, "null argument");
    zkvc_pk* k = const_cast<zkvc_pk*>(pk);
    std::lock_guard<std::mutex> lock(k->mu);
    const host::HFr rr = fr_in(*r, "r"), ss = fr_in(*s, "s");
    int dev = current_device();
    ZK_REQUIRE(dev == k->device, "the proving key lives on another device");
    require_device_buffer(d_X, dev, "X");
    require_device_buffer(d_W, dev, "W");
    require_device_buffer(d_Y, dev, "Y");
    groth16_prove(k, d_X, d_W, rr, ss, d_Y, proof_out, (hipStream_t)hip_stream, true);
  });
}

namespace {
// One batch context per (device, stream), created on first use and kept until
// the process ends.  The table is never destroyed: a context's destructor
// synchronizes and destroys streams and events, and a static destructor
// would run those HIP calls during exit(), after the runtime (and a profiler
// attached to it) has begun tearing down, which aborts the process.  The
// operating system reclaims the memory.
struct BatchCtxEntry {
  std::mutex mu;
  std::unique_ptr<ProveCtx> ctx;
};
BatchCtxEntry& batch_ctx(int dev, hipStream_t st) {
  static std::mutex* mu = new std::mutex();
  static auto* table = new std::map<std::pair<int, hipStream_t>, BatchCtxEntry*>();
  std::lock_guard<std::mutex> lock(*mu);
  BatchCtxEntry*& e = (*table)[{dev, st}];
  if (!e) e = new BatchCtxEntry();
  return *e;
}
}  // namespace

int zkvc_prove_batch(const zkvc_prove_job* jobs, size_t njobs, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(jobs && njobs > 0, "no proof jobs");
    const int dev = current_device();
    std::vector<ProveJob> pj(njobs);
    for (size_t j = 0; j < njobs; j++) {
      const zkvc_prove_job& in = jobs[j];
      ZK_REQUIRE(in.pk && in.X && in.W && in.Y_out && in.proof_out, "null argument in a proof job");
      ZK_REQUIRE(in.pk->device == dev, "a proving key lives on another device");
      pj[j].pk = in.pk;
      pj[j].X = in.X;
      pj[j].W = in.W;
      pj[j].r = fr_in(in.r, "r");
      pj[j].s = fr_in(in.s, "s");
      pj[j].Y = in.Y_out;
      pj[j].out = in.proof_out;
    }
    BatchCtxEntry& e = batch_ctx(dev, (hipStream_t)hip_stream);
    std::lock_guard<std::mutex> lock(e.mu);
    if (!e.ctx) e.ctx.reset(new ProveCtx());
    groth16_prove_batch(*e.ctx, pj.data(), njobs, (hipStream_t)hip_stream);
  });
}

int zkvc_set_graphs(int enable) { return set_graphs(enable); }

int zkvc_verify(const uint8_t* vk, size_t vk_len, const int8_t* X, const int32_t* Y, const zkvc_proof* proof) {
  int result = 0;
  const int rc = guarded([&] {
    ZK_REQUIRE(vk && X && Y && proof, "null argument");
    result = groth16_verify(vk, vk_len, X, Y, proof);
  });
  return rc < 0 ? rc : result;
}

int zkvc_pk_info(const zkvc_pk* pk, zkvc_pk_info_t* info) {
  return guarded([&] {
    ZK_REQUIRE(pk && info, "null argument");
    const Layout& L = pk->L;
    auto total = [](const std::vector<Seg>& v) { return v.empty() ? 0ull : (unsigned long long)(v.back().index + v.back().count); };
    info->a = L.a;
    info->n = L.n;
    info->b = L.b;
    info->kind = L.kind;
    info->log_n = (uint32_t)L.log_n;
    info->num_vars = L.nv;
    info->num_public = L.ell;
    info->a_query = total(L.segA);
    info->b_query = total(L.segB);
    info->l_query = total(L.segL);
    info->h_query = L.N;
    const size_t ctx_bytes = pk->ctx ? pk->ctx->device_bytes() : 0;
    info->device_bytes = pk->key_bytes + pk->ws.bytes() + ctx_bytes;
    info->prove_bytes = prove_footprint(L);
  });
}

int zkvc_pk_export(const zkvc_pk* pk, uint32_t query, uint64_t start, uint64_t count, void* host_out) {
  return guarded([&] {
    ZK_REQUIRE(pk && host_out, "null argument");
    if (query == ZKVC_Q_CONST) {
      zkvc_g1* g1 = static_cast<zkvc_g1*>(host_out);
      g1_to_abi(pk->alpha1, &g1[0]);
      g1_to_abi(pk->beta1, &g1[1]);
      g1_to_abi(pk->delta1, &g1[2]);
      zkvc_g2* g2 = reinterpret_cast<zkvc_g2*>(g1 + 3);
      g2_to_abi(pk->beta2, &g2[0]);
      g2_to_abi(pk->delta2, &g2[1]);
      return;
    }
    const Layout& L = pk->L;
    const DevBuf* buf = nullptr;
    std::vector<Seg> segs;
    switch (query) {
      case ZKVC_Q_A: buf = &pk->qA; segs = L.segA; break;
      case ZKVC_Q_B1: buf = &pk->qB1; segs = L.segB; break;
      case ZKVC_Q_B2: buf = &pk->qB2; segs = L.segB; break;
      case ZKVC_Q_L: buf = &pk->qL; segs = L.segL; break;
      case ZKVC_Q_H: buf = &pk->qH; if (L.segH.count) segs.push_back(L.segH); break;
      default: throw Error(ZKVC_EINVAL, "unknown query");
    }
    const uint64_t size = segs.empty() ? 0 : segs.back().index + segs.back().count;
    ZK_REQUIRE(start <= size && count <= size - start, "range outside the query");
    const int words = query == ZKVC_Q_B2 ? 32 : 16;
    std::vector<uint32_t> raw(count * words);
    // query index -> stored point: the first copy of the range holding it
    for (const Seg& sg : segs) {
      const uint64_t lo = std::max<uint64_t>(start, sg.index), hi = std::min<uint64_t>(start + count, sg.index + sg.count);
      if (lo >= hi) continue;
      ZK_HIP(hipMemcpy(raw.data() + (lo - start) * words, buf->get() + (sg.point_offset + (lo - sg.index)) * words,
                       (hi - lo) * words * 4, hipMemcpyDeviceToHost));
    }
    for (uint64_t k = 0; k < count; k++) {
      const uint32_t* p = raw.data() + k * words;
      bool zero = true;
      for (int q = 0; q < words; q++) zero = zero && p[q] == 0;
      if (words == 16) {
        zkvc_g1* o = static_cast<zkvc_g1*>(host_out) + k;
        std::memset(o, 0, sizeof(*o));
        if (!zero) {
          host::HFq::from_dev(p).to_u32(o->x);
          host::HFq::from_dev(p + 8).to_u32(o->y);
        }
      } else {
        zkvc_g2* o = static_cast<zkvc_g2*>(host_out) + k;
        std::memset(o, 0, sizeof(*o));
        if (!zero) {
          host::HFq::from_dev(p).to_u32(o->x0);
          host::HFq::from_dev(p + 8).to_u32(o->x1);
          host::HFq::from_dev(p + 16).to_u32(o->y0);
          host::HFq::from_dev(p + 24).to_u32(o->y1);
        }
      }
    }
  });
}

int zkvc_pk_last_stats(const zkvc_pk* pk, zkvc_prove_stats* out) {
  return guarded([&] {
    ZK_REQUIRE(pk && out, "null argument");
    *out = pk->last;
  });
}

}  // extern "C"
