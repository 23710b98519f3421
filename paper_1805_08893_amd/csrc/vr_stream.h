// Triangle setup: the stage that consumes the geometry stage's output queue
// in a streaming pipeline (Section 4.2).  One lane per triangle reads the
// clip-space row of its three corners, divides by w, maps to the viewport
// and writes {xmin, ymin, xmax, ymax} and {area, flags, 0, 0} as two float4.
#pragma once

#include "vr_device.h"

namespace vr {

__global__ __launch_bounds__(256) void k_setup(const f4 *corners, uint32_t T, uint32_t width, uint32_t height,
                                               f4 *records, const unsigned long long *chunk_counters,
                                               unsigned long long *totals) {
    __shared__ uint32_t s_part[4];
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    uint32_t vis = 0;
    if (t < T) {
        const float hw = 0.5f * (float)width, hh = 0.5f * (float)height;
        float sx[3], sy[3];
        bool front = true;
#pragma unroll
        for (uint32_t k = 0; k < 3; ++k) {
            const f4 c = corners[9ull * t + 3 * k];   // row 0 of corner k: clip x, y, z, w
            front = front && c.w > 0.0f;
            sx[k] = (c.x / c.w + 1.0f) * hw;
            sy[k] = (c.y / c.w + 1.0f) * hh;
        }
        f4 box = {0.0f, 0.0f, 0.0f, 0.0f}, rest = {0.0f, 0.0f, 0.0f, 0.0f};
        if (front) {
            const float area = (sx[1] - sx[0]) * (sy[2] - sy[0]) - (sx[2] - sx[0]) * (sy[1] - sy[0]);
            const float x0 = fmaxf(fminf(fminf(sx[0], sx[1]), sx[2]), 0.0f);
            const float x1 = fminf(fmaxf(fmaxf(sx[0], sx[1]), sx[2]), (float)width);
            const float y0 = fmaxf(fminf(fminf(sy[0], sy[1]), sy[2]), 0.0f);
            const float y1 = fminf(fmaxf(fmaxf(sy[0], sy[1]), sy[2]), (float)height);
            vis = (area > 0.0f && x0 < x1 && y0 < y1) ? 1u : 0u;
            box = f4{x0, y0, x1, y1};
            rest = f4{area, __uint_as_float(vis), 0.0f, 0.0f};
        }
        records[2ull * t] = box;
        records[2ull * t + 1] = rest;
    }
    // visible count: a wave reduction, then one atomic per workgroup
    uint32_t w = (uint32_t)__popcll(ballot(vis != 0));
    if (lane_id() == 0) s_part[threadIdx.x / kWave] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&totals[0], (unsigned long long)(s_part[0] + s_part[1] + s_part[2] + s_part[3]));
        if (blockIdx.x == 0 && chunk_counters) {
            atomicAdd(&totals[1], chunk_counters[0]);
            atomicAdd(&totals[2], chunk_counters[1]);
        }
    }
}

}  // namespace vr
