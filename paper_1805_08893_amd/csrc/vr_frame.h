// Many draws in one persistent launch per variant (a frame).
//
// The streaming pipeline of the paper processes the index buffer batch by
// batch (Sections 3 and 4.2); a frame applies that to a list of draws of
// uneven size at once.  Every draw keeps exactly the units the single-draw
// path computes: static batches, dynamic batches from its plan, ballot
// batches (one wavefront each) or naive chunks of 256 corners.  The draws are
// grouped by variant (dedup mode and vertex program) through an order array;
// a prepare kernel counts each draw's units and prefix-sums them in that
// order, so every variant owns one contiguous range of units.  One persistent
// kernel per variant, compiled for that variant alone (so its registers and
// LDS are those of the variant, not of the widest one), deals its range out
// to its workgroups in chunks of frame_chunk(mode) units, round robin, finds each
// unit's draw by binary search in an LDS copy of the range's draw bases, and
// runs the single-draw device function.  Per-unit aggregates are reduced per
// draw afterwards, so no same-address atomics are on the hot path.
#pragma once

#include "vr_kernels.h"

namespace vr {

enum FrameMode : uint32_t { kFrameSort = 0, kFrameHash = 1, kFramePHash = 2, kFrameBallot = 3, kFrameNaive = 4 };
constexpr uint32_t kFrameNT = 256;
// Consecutive units a workgroup takes at a time.  A workgroup runs its
// units one after another, each a chain of index load, vertex gather,
// shading and stores, so larger chunks leave a longer tail: 16 naive units
// per chunk made the scene's naive variants 2-3 times slower than 4, and a
// deduplicated unit is several times longer than a naive one.
__host__ __device__ constexpr uint32_t frame_chunk(uint32_t mode) { return mode == kFrameNaive ? 2u : 1u; }
constexpr uint32_t kFrameMaxDraws = 4096;
static_assert(VR_MAX_FRAME_DRAWS <= kFrameMaxDraws, "k_frame_prepare holds every draw of a frame");

// One persistent launch of a frame: the draws of one variant (order
// positions [lo, hi)), its kernel's LDS and its grid.
struct FrameVariant {
    uint32_t mode, kind, lo, hi, grid, unit_lds, ballot_stride, lds_total;
    uint32_t occ;   // hashing variant held to eight wavefronts per SIMD (its LDS allows them)
};

struct DrawDesc {
    const uint32_t *idx;
    const f4 *vtx;
    f4 *corners;
    unsigned long long *counters;
    const uint32_t *plan;
    uint32_t V, T, batch_tris, num_batches;
    uint32_t shader, mode, kind;
    uint32_t max_idx, max_uniq, hash_bits, probes;
    uint32_t slot_cap;   // aggregate slots the host reserved for the draw's batches
};

// Batches of a plan that start before triangle T.  A plan built for a
// longer stream with the same start, cut at T, is the plan of the first T
// triangles: greedy batching closes a batch without looking past it.
__device__ __forceinline__ uint32_t plan_prefix_batches(const uint32_t *plan, uint32_t T) {
    const uint32_t B = plan[0];
    if (plan[1 + B] <= T) return B;
    uint32_t lo = 0, hi = B;   // plan[1 + lo] < T <= plan[1 + hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (plan[1 + mid] < T) lo = mid;
        else hi = mid;
    }
    return hi;
}

// Units (workgroup tasks) and aggregate slots of a draw.  A plan with more
// batches than the host reserved slots for (one built with a smaller N_u or
// N_pmax than the draw states) raises VR_ERR_CAPACITY and is cut to the
// reserved slots, so no aggregate lands outside the draw's range.
__device__ __forceinline__ void frame_draw_units(const DrawDesc &D, uint32_t &units, uint32_t &slots,
                                                 uint32_t *err) {
    if (D.mode == kFrameNaive) {
        units = slots = (uint32_t)((3ull * D.T + 255) / 256);
        return;
    }
    uint32_t nb = D.T == 0 ? 0u : (D.plan ? plan_prefix_batches(D.plan, D.T) : D.num_batches);
    if (nb > D.slot_cap) {
        raise_error(err, VR_ERR_CAPACITY);
        nb = D.slot_cap;
    }
    slots = nb;
    units = D.mode == kFrameBallot ? (nb + 3) / 4 : nb;   // four wavefronts, four ballot batches
}

// One workgroup: unit and slot bases of the draws in variant order
// (position k is draw order[k]), totals last.  Thread t owns positions
// t*E .. t*E+E-1 (E <= kFrameMaxDraws / 1024); their counts are kept in
// registers between the scan and the writes.
__global__ __launch_bounds__(1024) void k_frame_prepare(const DrawDesc *draws, const uint32_t *order, uint32_t n,
                                                        uint32_t *unit_base, uint32_t *slot_base, uint32_t *err) {
    constexpr uint32_t kE = kFrameMaxDraws / 1024;
    __shared__ uint32_t tmp[16];
    const uint32_t E = (n + 1023) / 1024;
    const uint32_t lo = min(n, threadIdx.x * E), hi = min(n, lo + E);
    uint32_t cu[kE], cs[kE];
    uint32_t su = 0, ss = 0;
#pragma unroll
    for (uint32_t j = 0; j < kE; ++j) {
        cu[j] = cs[j] = 0;
        if (lo + j < hi) frame_draw_units(draws[order[lo + j]], cu[j], cs[j], err);
        su += cu[j];
        ss += cs[j];
    }
    uint32_t tu, ts;
    uint32_t ru = block_excl_scan<1024>(su, tmp, tu);
    uint32_t rs = block_excl_scan<1024>(ss, tmp, ts);
#pragma unroll
    for (uint32_t j = 0; j < kE; ++j) {
        if (lo + j < hi) {
            unit_base[lo + j] = ru;
            slot_base[lo + j] = rs;
        }
        ru += cu[j];
        rs += cs[j];
    }
    if (threadIdx.x == 0) {
        unit_base[n] = tu;
        slot_base[n] = ts;
    }
}

__device__ __forceinline__ DrawArgs frame_args(const DrawDesc &D, unsigned long long *agg, uint32_t *err,
                                               unsigned long long *total_inv) {
    DrawArgs A{};
    A.idx = D.idx;
    A.vtx = D.vtx;
    A.V = D.V;
    A.T = D.T;
    A.batch_tris = D.batch_tris;
    A.num_batches = D.num_batches;
    A.plan = D.plan;
    A.corners = D.corners;
    A.agg = agg;
    A.err = err;
    A.total_inv = total_inv;
    A.hash_bits = D.hash_bits;
    A.probes = D.probes;
    A.max_idx = D.max_idx;
    A.max_uniq = D.max_uniq;
    A.need_prefix = 0;
    A.status_cap = 0xFFFFFFFFu;
    return A;
}

template <int MODE, int KIND>
__device__ __forceinline__ void frame_unit(const DrawArgs &A, const vr_shader_params &sh, uint32_t local,
                                           uint32_t nb, unsigned char *smem, uint32_t ballot_stride) {
    if (MODE == kFrameSort) {
        dedup_unit<kFrameNT, kSort, KIND>(A, sh, local, nb, smem);
    } else if (MODE == kFrameHash) {
        dedup_unit<kFrameNT, kHash, KIND>(A, sh, local, nb, smem);
    } else if (MODE == kFramePHash) {
        dedup_unit<kFrameNT, kPHash, KIND>(A, sh, local, nb, smem);
    } else if (MODE == kFrameBallot) {
        const uint32_t w = threadIdx.x / kWave;
        const uint32_t b = 4 * local + w;
        unsigned char *mine = smem + w * ballot_stride;
        if (b < nb) ballot_batch<KIND>(A, sh, b, nb, mine);
        __syncthreads();
    } else {
        const unsigned long long agg = naive_chunk<KIND>(A, sh, local, (f4 *)smem);
        if (threadIdx.x == 0) A.agg[local] = agg;
    }
}

// The persistent kernel of one variant: the draws at order positions
// [lo, hi), whose units are unit_base[lo] .. unit_base[hi] - 1.  Dynamic LDS:
// the variant's largest unit layout, then its draw bases (hi - lo + 1 words).
// With OCC (hashing variants whose LDS lets eight workgroups reside) the
// kernel is held to eight wavefronts per SIMD, as in a single draw.  The
// read-only inputs are restrict: k_frame_prepare writes them before the
// launch and nothing writes them during it, which lets the compiler read the
// descriptors and shader parameters with scalar loads.
template <int MODE, int KIND, bool OCC>
__global__ __launch_bounds__(kFrameNT) __attribute__((amdgpu_waves_per_eu(OCC ? 8 : 1))) void k_frame(const DrawDesc *__restrict__ draws,
                                                    const uint32_t *__restrict__ order, uint32_t lo, uint32_t hi,
                                                    const vr_shader_params *__restrict__ shaders,
                                                    const uint32_t *__restrict__ unit_base,
                                                    const uint32_t *__restrict__ slot_base,
                                                    unsigned long long *agg, uint32_t unit_lds,
                                                    uint32_t ballot_stride, uint32_t *err,
                                                    unsigned long long *total_inv) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const uint32_t m = hi - lo;
    uint32_t *s_base = (uint32_t *)(smem + unit_lds);
    for (uint32_t k = threadIdx.x; k <= m; k += kFrameNT) s_base[k] = unit_base[lo + k];
    __syncthreads();
    const uint32_t U = s_base[m];
    const uint32_t G = gridDim.x;
    constexpr uint32_t kChunk = frame_chunk(MODE);
    uint32_t kd = 0xFFFFFFFFu;   // the draw whose descriptor is loaded
    DrawArgs A{};
    const vr_shader_params *sh = shaders;
    uint32_t nb = 0;
    // The draw index and everything loaded through it are the same in every
    // lane; reading the LDS bases through readfirstlane lets the compiler see
    // that, so the descriptor and the shader parameters stay in scalar
    // registers (as kernel arguments do in a single draw) instead of taking
    // vector registers and vector loads.
    auto base_at = [&](uint32_t k) { return (uint32_t)__builtin_amdgcn_readfirstlane(s_base[k]); };
    for (uint32_t c0 = base_at(0) + blockIdx.x * kChunk; c0 < U; c0 += G * kChunk) {
        // the draw of unit c0: largest k with s_base[k] <= c0
        uint32_t a = 0, b = m;   // invariant: s_base[a] <= c0 < s_base[b]
        while (b - a > 1) {
            const uint32_t mid = (a + b) / 2;
            if (base_at(mid) <= c0) a = mid;
            else b = mid;
        }
        uint32_t k = a;
        for (uint32_t u = c0; u < min(U, c0 + kChunk); ++u) {
            while (u >= base_at(k + 1)) ++k;   // units of empty draws are skipped
            if (k != kd) {   // descriptors are loaded once per draw, not per unit
                kd = k;
                const DrawDesc D = draws[order[lo + k]];
                A = frame_args(D, agg + slot_base[lo + k], err, total_inv);
                sh = shaders + D.shader;
                nb = slot_base[lo + k + 1] - slot_base[lo + k];
            }
            frame_unit<MODE, KIND>(A, *sh, u - base_at(k), nb, smem, ballot_stride);
        }
    }
}

// Per draw (order position d): counters = the sum of its aggregates;
// dtot[d] = its invocations.  One wavefront per draw, 16 per workgroup.
__global__ __launch_bounds__(1024) void k_frame_finish(const DrawDesc *draws, const uint32_t *order, uint32_t n,
                                                       const uint32_t *slot_base, const unsigned long long *agg,
                                                       unsigned long long *dtot) {
    const uint32_t d = blockIdx.x * 16 + threadIdx.x / kWave;
    if (d >= n) return;
    unsigned long long sum = 0;
    const uint32_t i1 = slot_base[d + 1];
    for (uint32_t i = slot_base[d] + lane_id(); i < i1; i += 4 * kWave) {   // four loads in flight
        unsigned long long v[4];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) v[j] = i + j * kWave < i1 ? agg[i + j * kWave] : 0ull;
        sum += v[0] + v[1] + v[2] + v[3];
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) sum += __shfl_xor(sum, s, kWave);
    if (lane_id() == 0) {
        const unsigned long long inv = sum & 0xFFFFFFFFull, units = sum >> 32;
        unsigned long long *c = draws[order[d]].counters;
        if (c) {
            c[0] = inv;
            c[1] = units;
            c[2] = 0;
            c[3] = 0;
        }
        dtot[d] = inv;
    }
}

__global__ __launch_bounds__(1024) void k_frame_total(const unsigned long long *dtot, uint32_t n,
                                                      unsigned long long *total_inv) {
    __shared__ unsigned long long part[16];
    unsigned long long sum = 0;
    for (uint32_t d = threadIdx.x; d < n; d += 1024) sum += dtot[d];
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) sum += __shfl_xor(sum, s, kWave);
    if (lane_id() == 0) part[threadIdx.x / kWave] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 16; ++w) t += part[w];
        *total_inv += t;
    }
}

}  // namespace vr
