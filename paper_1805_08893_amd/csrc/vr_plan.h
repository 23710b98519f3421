// Dynamic batching on the device (Section 3.4, "Dynamic batching").
//
// The cut rule is a sequential greedy chain: starting at a batch start,
// whole triangles are added while the batch has at most N_u distinct indices
// and at most N_pmax triangles; the first triangle that would break a limit
// starts the next batch.  The chain is made parallel by speculation:
//   spec   one wavefront per segment of SEG triangles runs the chain from
//          the segment's first triangle, marking cuts in a bitmap and
//          recording the batch still open at the segment end;
//   fix    one wavefront per segment s >= 1 continues the chain of segment
//          s-1 from that open batch into s until it produces a cut that s
//          already holds: from there on both chains coincide (the greedy
//          rule is deterministic from any cut), so only the bits before the
//          meeting point change;
//   walk   a single wavefront visits the segments whose fix started from a
//          batch start that changed meanwhile and redoes them in order;
//   pack   the bitmap is compacted into the plan [B, start_0.., T].
// The result equals the sequential chain exactly for any segment length.
#pragma once

#include "vr_device.h"

namespace vr {

constexpr uint32_t kPlanSeg = 512;        // triangles per segment (multiple of 64)

struct PlanArgs {
    const uint32_t *idx;
    uint32_t V, T;
    uint32_t cap, tmax;                   // N_u, N_pmax
    uint32_t nseg;
    uint32_t hs_bits;                     // per-wave set size: 2^hs_bits slots
    unsigned long long *bits;             // cut bitmap, ceil(T/64) words
    uint32_t *spec_last;                  // [nseg] batch open at the segment end (speculative)
    uint32_t *fix_from;                   // [nseg] batch start the fix of s started from
    uint32_t *fix_last;                   // [nseg] batch open at the end of s after its fix
    uint32_t *err;
};

// Per-wavefront set of the open batch's distinct indices: slot = (stamp << 32
// | key) with the batch's stamp, plus the first corner position at which the
// key entered the batch.  A new stamp empties the set in O(1).
struct WaveSet {
    unsigned long long *tab;
    uint32_t *pos;
    uint32_t bits;
    uint32_t mask;
    uint32_t stamp;
};

__device__ __forceinline__ void waveset_init(WaveSet &S) {
    for (uint32_t i = lane_id(); i <= S.mask; i += kWave) {
        S.tab[i] = 0ull;
        S.pos[i] = kEmpty;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    S.stamp = 1;
}

// Finds or claims the slot of `key` under the current stamp.  A claimant
// resets the slot's first position.
__device__ __forceinline__ uint32_t waveset_slot(WaveSet &S, uint32_t key) {
    const unsigned long long want = ((unsigned long long)S.stamp << 32) | key;
    uint32_t p = hash_slot(key, S.bits);
    for (;;) {
        unsigned long long cur = __hip_atomic_load(&S.tab[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == want) return p;
        if ((uint32_t)(cur >> 32) != S.stamp) {
            unsigned long long seen = atomicCAS(&S.tab[p], cur, want);
            if (seen == cur) {
                S.pos[p] = kEmpty;
                return p;
            }
            if (seen == want) return p;
            continue;   // another key took it: look again at the same slot
        }
        p = (p + 1) & S.mask;
    }
}

__device__ __forceinline__ unsigned long long word_mask(uint32_t lo, uint32_t hi) {
    // bits [lo, hi) of one 64-bit word, 0 <= lo <= hi <= 64
    const unsigned long long a = lo >= 64 ? 0ull : (~0ull << lo);
    const unsigned long long b = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    return a & b;
}

// Clears cut bits [lo, hi) (lanes work on consecutive words).
__device__ __forceinline__ void bits_clear(unsigned long long *bits, uint32_t lo, uint32_t hi) {
    if (lo >= hi) return;
    const uint32_t w0 = lo / 64, w1 = (hi - 1) / 64;
    for (uint32_t w = w0 + lane_id(); w <= w1; w += kWave) {
        const uint32_t a = w == w0 ? lo % 64 : 0, b = w == w1 ? (hi - 1) % 64 + 1 : 64;
        atomicAnd(&bits[w], ~word_mask(a, b));
    }
}

__device__ __forceinline__ bool bit_test(unsigned long long *bits, uint32_t t) {
    return (atomicOr(&bits[t / 64], 0ull) >> (t % 64)) & 1ull;
}

__device__ __forceinline__ void bit_set(unsigned long long *bits, uint32_t t) {
    atomicOr(&bits[t / 64], 1ull << (t % 64));
}

// Runs the greedy chain with a batch opened at `start`, over triangles
// [start, limit).  Every cut c (start of a new batch, c < limit) is passed
// to on_cut(c), which returns true to stop the scan there.  Returns the
// start of the batch open at `limit`, or the stopping cut.  Wave-uniform.
template <typename OnCut>
__device__ uint32_t greedy_chain(const PlanArgs &P, WaveSet &S, uint32_t start, uint32_t limit, OnCut on_cut) {
    const uint32_t lane = lane_id();
    uint32_t bstart = start, cur = start, distinct = 0;
    ++S.stamp;
    while (cur < limit) {
        const uint32_t t = cur + lane;
        const bool act = t < limit;
        uint32_t k[3] = {0, 0, 0}, sl[3] = {0, 0, 0};
        if (act) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                uint32_t v = P.idx[3ull * t + c];
                if (v >= P.V) {
                    raise_error(P.err, VR_ERR_INDEX_RANGE);
                    v = 0;
                }
                k[c] = v;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) sl[c] = waveset_slot(S, k[c]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (act) {
#pragma unroll
            for (int c = 0; c < 3; ++c) atomicMin(&S.pos[sl[c]], 3 * t + c);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        uint32_t fresh = 0;
        if (act) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                fresh += __hip_atomic_load(&S.pos[sl[c]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) ==
                         3 * t + c;
        }
        const uint32_t incl = wave_incl_scan(fresh);
        const bool ok = act && distinct + incl <= P.cap && t - bstart + 1 <= P.tmax;
        const uint64_t okm = ballot(ok);
        const uint32_t acc = (uint32_t)__popcll(okm);
        const uint32_t nact = min((uint32_t)kWave, limit - cur);
        if (acc == nact) {
            distinct += __builtin_amdgcn_readlane(incl, nact - 1);
            cur += acc;
        } else {
            const uint32_t c = cur + acc;
            if (on_cut(c)) return c;
            ++S.stamp;          // the triangle at c opens a new batch
            bstart = c;
            cur = c;
            distinct = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    return bstart;
}

__device__ __forceinline__ uint32_t seg_begin(uint32_t s) { return s * kPlanSeg; }
__device__ __forceinline__ uint32_t seg_end(const PlanArgs &P, uint32_t s) {
    return min(P.T, (s + 1) * kPlanSeg);
}

// LDS per wavefront for the chain: 12 bytes per set slot.
__global__ __launch_bounds__(64) void k_plan_spec(PlanArgs P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    WaveSet S{(unsigned long long *)smem, (uint32_t *)(smem + (8u << P.hs_bits)), P.hs_bits,
              (1u << P.hs_bits) - 1, 0};
    const uint32_t s = blockIdx.x;
    if (s >= P.nseg) return;
    waveset_init(S);
    const uint32_t b = seg_begin(s), e = seg_end(P, s);
    // the segment owns bit words [b/64, ceil(e/64)); start from clean words
    bits_clear(P.bits, b, (e + 63) & ~63u);
    __threadfence();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane_id() == 0) bit_set(P.bits, b);
    const uint32_t last = greedy_chain(P, S, b, e, [&](uint32_t c) {
        if (lane_id() == 0) bit_set(P.bits, c);
        return false;
    });
    if (lane_id() == 0) {
        P.spec_last[s] = last;
        P.fix_from[s] = b;       // segment 0 is exact from the start
        P.fix_last[s] = last;
    }
}

// Continues the chain from batch start q (which lies before segment s and
// whose batch is still open at the segment's first triangle) through s.
// Rewrites s's cut bits up to the first cut s already holds.
__device__ __forceinline__ void fix_segment(const PlanArgs &P, WaveSet &S, uint32_t s, uint32_t q) {
    const uint32_t b = seg_begin(s), e = seg_end(P, s);
    uint32_t clr = b;
    bool synced = false;
    const uint32_t last = greedy_chain(P, S, q, e, [&](uint32_t c) {
        // c >= b: the batch from q covers every triangle before segment s
        uint32_t had = 0;
        if (lane_id() == 0) had = bit_test(P.bits, c);
        had = __builtin_amdgcn_readfirstlane(had);
        bits_clear(P.bits, clr, c);
        __threadfence();
        if (had) {
            synced = true;
            return true;
        }
        if (lane_id() == 0) bit_set(P.bits, c);
        clr = c + 1;
        return false;
    });
    if (!synced) bits_clear(P.bits, clr, e);
    __threadfence();
    if (lane_id() == 0) {
        P.fix_from[s] = q;
        P.fix_last[s] = synced ? P.fix_last[s] : last;
    }
}

__global__ __launch_bounds__(64) void k_plan_fix(PlanArgs P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    WaveSet S{(unsigned long long *)smem, (uint32_t *)(smem + (8u << P.hs_bits)), P.hs_bits,
              (1u << P.hs_bits) - 1, 0};
    const uint32_t s = blockIdx.x + 1;
    if (s >= P.nseg) return;
    waveset_init(S);
    fix_segment(P, S, s, P.spec_last[s - 1]);
}

// Single wavefront: walks the segments in order and redoes every segment
// whose fix started from a batch start other than its predecessor's final
// open batch.  Segment 0 is always exact.
__global__ __launch_bounds__(64) void k_plan_walk(PlanArgs P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    WaveSet S{(unsigned long long *)smem, (uint32_t *)(smem + (8u << P.hs_bits)), P.hs_bits,
              (1u << P.hs_bits) - 1, 0};
    waveset_init(S);
    const uint32_t lane = lane_id();
    uint32_t s = 1;
    uint32_t prev_last = P.fix_last[0];
    while (s < P.nseg) {
        // 64 segments at a time: the first one whose fix used a stale start
        const uint32_t j = s + lane;
        bool bad = false;
        if (j < P.nseg) {
            const uint32_t pl = (lane == 0) ? prev_last : P.fix_last[j - 1];
            bad = P.fix_from[j] != pl;
        }
        const uint64_t badm = ballot(bad);
        if (!badm) {
            const uint32_t adv = min((uint32_t)kWave, P.nseg - s);
            prev_last = __builtin_amdgcn_readfirstlane(P.fix_last[s + adv - 1]);
            s += adv;
            continue;
        }
        const uint32_t f = (uint32_t)__ffsll((long long)badm) - 1;
        s += f;
        if (f > 0) prev_last = __builtin_amdgcn_readfirstlane(P.fix_last[s - 1]);
        fix_segment(P, S, s, prev_last);
        __threadfence();
        prev_last = __builtin_amdgcn_readfirstlane(P.fix_last[s]);
        ++s;
    }
}

// Compaction of the cut bitmap into the plan.
__global__ __launch_bounds__(256) void k_plan_count(const unsigned long long *bits, uint32_t nwords,
                                                    uint32_t *block_sums) {
    __shared__ uint32_t tmp[4];
    const uint32_t w = blockIdx.x * 256 + threadIdx.x;
    const uint32_t c = w < nwords ? (uint32_t)__popcll(bits[w]) : 0u;
    uint32_t total;
    block_excl_scan<256>(c, tmp, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// One workgroup turns the block sums into exclusive offsets, writes B and
// the final entry T.
__global__ __launch_bounds__(1024) void k_plan_scan(uint32_t *block_sums, uint32_t nblocks, uint32_t *plan,
                                                    uint32_t T) {
    __shared__ uint32_t tmp[16];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nblocks; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nblocks ? block_sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan<1024>(v, tmp, total);
        if (i < nblocks) block_sums[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        plan[0] = carry;
        plan[1 + carry] = T;
    }
}

__global__ __launch_bounds__(256) void k_plan_write(const unsigned long long *bits, uint32_t nwords,
                                                    const uint32_t *block_offsets, uint32_t *plan) {
    __shared__ uint32_t tmp[4];
    const uint32_t w = blockIdx.x * 256 + threadIdx.x;
    unsigned long long m = w < nwords ? bits[w] : 0ull;
    uint32_t total;
    uint32_t r = block_offsets[blockIdx.x] + block_excl_scan<256>((uint32_t)__popcll(m), tmp, total);
    while (m) {
        const uint32_t b = (uint32_t)__ffsll((long long)m) - 1;
        plan[1 + r++] = w * 64 + b;
        m &= m - 1;
    }
}

}  // namespace vr
