// Shared helpers for the C-ABI translation units: exception guard, argument checks.
#pragma once
#include <exception>
#include <new>
#include <string>

#include "host_field.hpp"
#include "util.hpp"
#include "zkvc.h"

namespace zkvc {

const std::string& last_error();

// Runs fn, mapping exceptions to the ABI's negative codes; never throws.
template <class Fn>
int guarded(Fn&& fn) {
  try {
    set_last_error("");
    fn();
    return ZKVC_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return ZKVC_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return ZKVC_EDEVICE;
  } catch (...) {
    set_last_error("unknown failure");
    return ZKVC_EDEVICE;
  }
}

// Checks that p is non-null, 16-byte aligned device memory and that [p, p + bytes)
// lies inside the allocation that holds p.  (A sub-allocator such as a caching
// allocator can hide a too-small buffer inside a larger block: callers remain
// responsible for passing buffers of the documented size.)
void require_device_range(const void* p, size_t bytes, const char* name);

// A canonical Fr argument of the ABI (rejects values >= r with ZKVC_EINVAL).
inline host::HFr fr_in(const zkvc_fr& v, const char* name) {
  ZK_REQUIRE(host::HFr::canonical_ok(v.l), std::string(name) + " must be below the group order r");
  return host::HFr::from_u32(v.l);
}

void g1_to_abi(const host::G1J& p, zkvc_g1* out);
void g2_to_abi(const host::G2J& p, zkvc_g2* out);

}  // namespace zkvc
