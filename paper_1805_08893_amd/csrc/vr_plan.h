// Dynamic batching on the device (Section 3.4, "Dynamic batching").
//
// The cut rule is a sequential greedy chain: starting at a batch start,
// whole triangles are added while the batch has at most N_u distinct indices
// and at most N_pmax triangles; the first triangle that would break a limit
// starts the next batch.  The chain is made parallel by speculation:
//   spec   one wavefront per segment of kPlanSeg triangles runs the chain
//          from the segment's first triangle, marking cuts in the segment's
//          bitmap words and recording the batch still open at its end;
//   fix    one wavefront per segment s >= 1 continues the chain of segment
//          s-1 from that open batch into s until it produces a cut that s
//          already holds: from there on both chains coincide (the greedy
//          rule is deterministic from any cut), so only the bits before the
//          meeting point change;
//   walk   one wavefront visits the segments whose fix started from a batch
//          start that changed meanwhile and redoes them in order; then the
//          whole workgroup compacts the bitmap into [B, start_0.., T].
// The result equals the sequential chain exactly for any segment length.
// Indices and cut bits live in LDS while a chain runs: global memory sees one
// coalesced index load and one bitmap write-back per segment.
#pragma once

#include "vr_device.h"

namespace vr {

constexpr uint32_t kPlanSeg = 512;            // triangles per segment (multiple of 64)
constexpr uint32_t kSegWords = kPlanSeg / 64; // bitmap words per segment
static_assert(kPlanSeg >= VR_MAX_BATCH_DYNAMIC, "a batch must not outgrow one segment");

struct PlanArgs {
    const uint32_t *idx;
    uint32_t V, T;
    uint32_t cap, tmax;                   // N_u, N_pmax
    uint32_t nseg, nwords;
    uint32_t hs_bits;                     // per-wave set size: 2^hs_bits slots
    unsigned long long *bits;             // cut bitmap, nwords words (kSegWords per segment)
    uint32_t *spec_last;                  // [nseg] batch open at the segment end (speculative)
    uint32_t *fix_from;                   // [nseg] batch start the fix of s started from
    uint32_t *fix_last;                   // [nseg] batch open at the end of s after its fix
    uint32_t *plan;                       // output [B, starts.., T]
    uint32_t *err;
};

// LDS of one chain-running wavefront.
struct ChainLds {
    uint32_t *tab;             // set of the open batch's indices (kEmpty = free)
    uint32_t *pos;             // first corner position of each key in the open batch
    uint32_t *cache;           // indices of triangles [c0, c0 + cn)
    unsigned long long *sbits; // the segment's kSegWords bitmap words
    uint32_t hs_bits, mask;
    uint32_t c0, cn;
};

__host__ __device__ inline uint32_t plan_chain_lds(uint32_t hs_bits) {
    return (8u << hs_bits) + 3u * 4u * 2u * kPlanSeg + 8u * kSegWords;
}

__device__ __forceinline__ ChainLds chain_lds(unsigned char *smem, uint32_t hs_bits) {
    ChainLds S;
    S.tab = (uint32_t *)smem;
    S.pos = (uint32_t *)(smem + (4u << hs_bits));
    S.cache = (uint32_t *)(smem + (8u << hs_bits));
    S.sbits = (unsigned long long *)(smem + (8u << hs_bits) + 3u * 4u * 2u * kPlanSeg);
    S.hs_bits = hs_bits;
    S.mask = (1u << hs_bits) - 1;
    S.c0 = S.cn = 0;
    return S;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Empties the set (a new batch opens).
__device__ __forceinline__ void chain_clear_set(ChainLds &S) {
    for (uint32_t i = lane_id(); i <= S.mask; i += kWave) {
        S.tab[i] = kEmpty;
        S.pos[i] = kEmpty;
    }
    wave_sync_lds();
}

// Stages the indices of triangles [t0, t1) (at most 2 * kPlanSeg) in LDS,
// with the range check applied once here.
__device__ __forceinline__ void chain_load(const PlanArgs &P, ChainLds &S, uint32_t t0, uint32_t t1) {
    if (t1 - t0 > 2 * kPlanSeg) {   // cannot happen while N_pmax <= kPlanSeg
        raise_error(P.err, VR_ERR_DEVICE);
        t1 = t0 + 2 * kPlanSeg;
    }
    const uint32_t n = 3 * (t1 - t0);
    const uint32_t *src = P.idx + 3ull * t0;
    for (uint32_t i = lane_id(); i < n; i += kWave) {
        uint32_t v = src[i];
        if (v >= P.V) {
            raise_error(P.err, VR_ERR_INDEX_RANGE);
            v = 0;
        }
        S.cache[i] = v;
    }
    S.c0 = t0;
    S.cn = t1 - t0;
}

// Finds or inserts `key` (linear probing; the set never fills: it holds at
// most N_u + 192 keys in 2 * (N_u + 192) or more slots).
__device__ __forceinline__ uint32_t chain_slot(ChainLds &S, uint32_t key) {
    uint32_t p = hash_slot(key, S.hs_bits);
    for (;;) {
        const uint32_t prev = atomicCAS(&S.tab[p], kEmpty, key);
        if (prev == kEmpty || prev == key) return p;
        p = (p + 1) & S.mask;
    }
}

__device__ __forceinline__ unsigned long long word_mask(uint32_t lo, uint32_t hi) {
    // bits [lo, hi) of one 64-bit word, 0 <= lo <= hi <= 64
    const unsigned long long a = lo >= 64 ? 0ull : (~0ull << lo);
    const unsigned long long b = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    return a & b;
}

// Segment-local bit operations on the LDS copy (positions relative to the
// segment's first triangle).
__device__ __forceinline__ void sbits_clear(ChainLds &S, uint32_t lo, uint32_t hi) {
    const uint32_t w = lane_id();
    if (lo < hi && w < kSegWords) {
        const uint32_t a = max(lo, w * 64), b = min(hi, w * 64 + 64);
        if (a < b) S.sbits[w] &= ~word_mask(a - w * 64, b - w * 64);
    }
}
__device__ __forceinline__ bool sbits_test(const ChainLds &S, uint32_t t) { return (S.sbits[t / 64] >> (t % 64)) & 1ull; }
__device__ __forceinline__ void sbits_set(ChainLds &S, uint32_t t) {
    if (lane_id() == 0) S.sbits[t / 64] |= 1ull << (t % 64);
}

// Runs the greedy chain with a batch opened at `start`, over triangles
// [start, limit) (all staged in the LDS cache).  Every cut c (the start of
// a new batch, c < limit) is passed to on_cut(c), which returns true to stop
// the scan there.  Returns the start of the batch open at `limit`, or the
// stopping cut.  Wave-uniform.
template <typename OnCut>
__device__ uint32_t greedy_chain(const PlanArgs &P, ChainLds &S, uint32_t start, uint32_t limit, OnCut on_cut) {
    const uint32_t lane = lane_id();
    uint32_t bstart = start, cur = start, distinct = 0;
    chain_clear_set(S);
    while (cur < limit) {
        const uint32_t t = cur + lane;
        const bool act = t < limit;
        uint32_t sl0 = 0, sl1 = 0, sl2 = 0;
        if (act) {
            const uint32_t *k = S.cache + 3 * (t - S.c0);
            sl0 = chain_slot(S, k[0]);
            sl1 = chain_slot(S, k[1]);
            sl2 = chain_slot(S, k[2]);
        }
        wave_sync_lds();
        if (act) {
            atomicMin(&S.pos[sl0], 3 * t);
            atomicMin(&S.pos[sl1], 3 * t + 1);
            atomicMin(&S.pos[sl2], 3 * t + 2);
        }
        wave_sync_lds();
        uint32_t fresh = 0;
        if (act) fresh = (S.pos[sl0] == 3 * t) + (S.pos[sl1] == 3 * t + 1) + (S.pos[sl2] == 3 * t + 2);
        const uint32_t incl = wave_incl_scan(fresh);
        const bool ok = act && distinct + incl <= P.cap && t - bstart + 1 <= P.tmax;
        const uint32_t acc = (uint32_t)__popcll(ballot(ok));
        const uint32_t nact = min((uint32_t)kWave, limit - cur);
        if (acc == nact) {
            distinct += __builtin_amdgcn_readlane(incl, nact - 1);
            cur += acc;
        } else {
            const uint32_t c = cur + acc;
            if (on_cut(c)) return c;
            chain_clear_set(S);   // the triangle at c opens a new batch
            bstart = c;
            cur = c;
            distinct = 0;
        }
        wave_sync_lds();
    }
    return bstart;
}

__device__ __forceinline__ uint32_t seg_begin(uint32_t s) { return s * kPlanSeg; }
__device__ __forceinline__ uint32_t seg_end(const PlanArgs &P, uint32_t s) { return min(P.T, (s + 1) * kPlanSeg); }

__device__ __forceinline__ void sbits_store(const PlanArgs &P, const ChainLds &S, uint32_t s) {
    const uint32_t w = lane_id();
    const uint32_t gw = s * kSegWords + w;
    if (w < kSegWords && gw < P.nwords) P.bits[gw] = S.sbits[w];
}

__device__ __forceinline__ void sbits_load(const PlanArgs &P, ChainLds &S, uint32_t s) {
    const uint32_t w = lane_id();
    const uint32_t gw = s * kSegWords + w;
    if (w < kSegWords) S.sbits[w] = gw < P.nwords ? P.bits[gw] : 0ull;
}

__global__ __launch_bounds__(64) void k_plan_spec(PlanArgs P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    ChainLds S = chain_lds(smem, P.hs_bits);
    const uint32_t s = blockIdx.x;
    if (s >= P.nseg) return;
    const uint32_t b = seg_begin(s), e = seg_end(P, s);
    chain_load(P, S, b, e);
    if (lane_id() < kSegWords) S.sbits[lane_id()] = 0ull;
    wave_sync_lds();
    sbits_set(S, 0);
    const uint32_t last = greedy_chain(P, S, b, e, [&](uint32_t c) {
        sbits_set(S, c - b);
        return false;
    });
    wave_sync_lds();
    sbits_store(P, S, s);
    if (lane_id() == 0) {
        P.spec_last[s] = last;
        P.fix_from[s] = b;       // segment 0 is exact from the start
        P.fix_last[s] = last;
    }
}

// Continues the chain from batch start q (in segment s-1, its batch still
// open at segment s's first triangle) through s, rewriting s's cut bits up to
// the first cut s already holds.  The caller has loaded s's bits into LDS.
__device__ __forceinline__ uint32_t fix_segment(const PlanArgs &P, ChainLds &S, uint32_t s, uint32_t q,
                                                uint32_t old_last) {
    const uint32_t b = seg_begin(s), e = seg_end(P, s);
    chain_load(P, S, q, e);
    wave_sync_lds();
    uint32_t clr = 0;
    bool synced = false;
    const uint32_t last = greedy_chain(P, S, q, e, [&](uint32_t c) {
        // c >= b: the batch from q covers every triangle before segment s
        const uint32_t lc = c - b;
        const bool had = sbits_test(S, lc);
        sbits_clear(S, clr, lc);
        wave_sync_lds();
        if (had) {
            synced = true;
            return true;
        }
        sbits_set(S, lc);
        clr = lc + 1;
        wave_sync_lds();
        return false;
    });
    if (!synced) sbits_clear(S, clr, e - b);
    wave_sync_lds();
    return synced ? old_last : last;
}

__global__ __launch_bounds__(64) void k_plan_fix(PlanArgs P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    ChainLds S = chain_lds(smem, P.hs_bits);
    const uint32_t s = blockIdx.x + 1;
    if (s >= P.nseg) return;
    sbits_load(P, S, s);
    const uint32_t q = P.spec_last[s - 1];
    const uint32_t last = fix_segment(P, S, s, q, P.spec_last[s]);
    sbits_store(P, S, s);
    if (lane_id() == 0) {
        P.fix_from[s] = q;
        P.fix_last[s] = last;
    }
}

// Walk and pack, one workgroup.  A segment s >= 1 is consistent when its fix
// started from its predecessor's final open batch.  All threads flag the
// inconsistent segments of a page in LDS; wavefront 0 then visits them in
// order, redoing each from the true open batch, and re-checks the successor
// of every redone segment whose open batch changed.  Finally the workgroup
// compacts the bitmap into the plan, whole segments per thread.
constexpr uint32_t kWalkPage = 65536;      // segments flagged per pass (8 KB of LDS)

__global__ __launch_bounds__(1024) void k_plan_walk_pack(PlanArgs P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ uint32_t tmp[16];
    __shared__ unsigned long long sbad[kWalkPage / 64];
    __shared__ uint32_t s_prev_last;
    if (threadIdx.x == 0) s_prev_last = P.fix_last[0];
    for (uint32_t page = 0; page * kWalkPage < P.nseg; ++page) {
        const uint32_t s0 = page * kWalkPage, s1 = min(P.nseg, s0 + kWalkPage);
        for (uint32_t w = threadIdx.x; w < kWalkPage / 64; w += 1024) sbad[w] = 0ull;
        __syncthreads();
        for (uint32_t s = max(s0, 1u) + threadIdx.x; s < s1; s += 1024)
            if (P.fix_from[s] != P.fix_last[s - 1]) atomicOr(&sbad[(s - s0) / 64], 1ull << ((s - s0) % 64));
        __syncthreads();
        if (threadIdx.x < kWave) {
            ChainLds S = chain_lds(smem, P.hs_bits);
            uint32_t prev_last = s_prev_last;   // true open batch at the end of segment s0 - 1
            uint32_t s = max(s0, 1u);
            bool recheck = page > 0 && s_prev_last != P.fix_last[s0 - 1];
            if (s0 == 0) prev_last = P.fix_last[0];
            while (s < s1) {
                const uint32_t ls = s - s0;
                const bool flagged = (sbad[ls / 64] >> (ls % 64)) & 1ull;
                if (!flagged && !recheck) {
                    // jump to the next flagged segment; everything before it is final
                    uint32_t nxt = s1;
                    for (uint32_t w = ls / 64; w < (s1 - s0 + 63) / 64; ++w) {
                        unsigned long long m = sbad[w];
                        if (w == ls / 64) m &= ~0ull << (ls % 64);
                        if (m) {
                            nxt = s0 + w * 64 + (uint32_t)__ffsll((long long)m) - 1;
                            break;
                        }
                    }
                    if (nxt >= s1) {
                        prev_last = P.fix_last[s1 - 1];
                        s = s1;
                        break;
                    }
                    s = nxt;
                    prev_last = P.fix_last[s - 1];
                    continue;
                }
                recheck = false;
                if (P.fix_from[s] != prev_last) {
                    const uint32_t old_last = P.fix_last[s];
                    sbits_load(P, S, s);
                    const uint32_t last = fix_segment(P, S, s, prev_last, old_last);
                    sbits_store(P, S, s);
                    if (lane_id() == 0) {
                        P.fix_from[s] = prev_last;
                        P.fix_last[s] = last;
                    }
                    recheck = last != old_last;   // the successor's start moved
                    prev_last = last;
                } else {
                    prev_last = P.fix_last[s];
                }
                ++s;
            }
            if (lane_id() == 0) s_prev_last = prev_last;
        }
        __threadfence();
        __syncthreads();
        __threadfence();
    }
    // compaction: thread t owns whole segments [t*E, t*E + E)
    const uint32_t E = (P.nseg + 1023) / 1024;
    const uint32_t lo = min(P.nseg, threadIdx.x * E), hi = min(P.nseg, lo + E);
    const uint32_t w0 = lo * kSegWords, w1 = min(P.nwords, hi * kSegWords);
    uint32_t cnt = 0;
    for (uint32_t w = w0; w < w1; ++w) cnt += (uint32_t)__popcll(P.bits[w]);
    uint32_t total;
    uint32_t r = block_excl_scan<1024>(cnt, tmp, total);
    for (uint32_t w = w0; w < w1; ++w) {
        unsigned long long m = P.bits[w];
        while (m) {
            const uint32_t bit = (uint32_t)__ffsll((long long)m) - 1;
            P.plan[1 + r++] = w * 64 + bit;
            m &= m - 1;
        }
    }
    if (threadIdx.x == 0) {
        P.plan[0] = total;
        P.plan[1 + total] = P.T;
    }
}

}  // namespace vr
