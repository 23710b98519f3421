// Self-test of the vertex programs' rounded arithmetic: the library's
// reciprocal and square root against the compiler's IEEE sequences.
#pragma once

#include "vr_device.h"

namespace vr {

// One operand per thread: the float32 with bit pattern first + i.  Counts
// (one atomic per wavefront) the operands whose result differs in any bit;
// out[i] receives the result when out is not NULL.
__global__ __launch_bounds__(256) void k_math_selftest(uint32_t fn, uint64_t first, uint64_t n, float *out,
                                                       unsigned long long *mismatches) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const float x = __uint_as_float((uint32_t)(first + i));
        float got, want;
        if (fn == 0) {
            got = recip_rn(x);
            want = 1.0f / x;
        } else if (fn == 1) {
            got = sqrt_rn(x);
            want = __builtin_sqrtf(x);
        } else {
            got = inv_sqrt_rn(x);
            want = 1.0f / __builtin_sqrtf(x);
        }
        bad = __float_as_uint(got) != __float_as_uint(want);
        if (out) out[i] = got;
    }
    const uint64_t m = ballot(bad);
    if (m && lane_id() == 0) atomicAdd(mismatches, (unsigned long long)__popcll(m));
}

}  // namespace vr
