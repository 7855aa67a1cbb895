// Groth16 entry points (setup, prove, verify, proving-key management).
#include "api_common.hpp"

using namespace zkvc;

extern "C" {
int zkvc_setup(const zkvc_shape*, const zkvc_fr*, const zkvc_fr*, zkvc_pk**, uint8_t*, size_t*, void*) {
  return guarded([&] { throw Error(ZKVC_EINVAL, "setup not available yet"); });
}
int zkvc_pk_free(zkvc_pk*) { return 0; }
int zkvc_prove(const zkvc_pk*, const int8_t*, const int8_t*, const zkvc_fr*, const zkvc_fr*, int32_t*, zkvc_proof*,
               void*) {
  return guarded([&] { throw Error(ZKVC_EINVAL, "prove not available yet"); });
}
int zkvc_verify(const uint8_t*, size_t, const int8_t*, const int32_t*, const zkvc_proof*) {
  return guarded([&] { throw Error(ZKVC_EINVAL, "verify not available yet"); });
}
int zkvc_pk_info(const zkvc_pk*, zkvc_pk_info_t*) { return ZKVC_EINVAL; }
int zkvc_pk_export(const zkvc_pk*, uint32_t, uint64_t, uint64_t, void*) { return ZKVC_EINVAL; }
int zkvc_pk_last_stats(const zkvc_pk*, zkvc_prove_stats*) { return ZKVC_EINVAL; }
}
