// Exclusive prefix sums over u32 arrays on the device.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "util.hpp"

namespace zkvc {

// out[i] = sum_{j<i} f(in[j]) with f(x) = x if div == 0, else ceil(x / div).
// Optionally writes the grand total and the maximum of f(in[i]) to device words.
// n may be any size up to 2^31; uses workspace slots [slot, slot + 1].
void scan_exclusive(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t div, uint32_t* d_total,
                    uint32_t* d_max, Workspace& ws, int slot, hipStream_t st);

// Two scans of n words each (f = identity), in one launch when n is small.
void scan_exclusive2(const uint32_t* in0, uint32_t* out0, uint32_t* d_total0, const uint32_t* in1, uint32_t* out1,
                     uint32_t* d_total1, uint32_t n, Workspace& ws, int slot, hipStream_t st);

}  // namespace zkvc
