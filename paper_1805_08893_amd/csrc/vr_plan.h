// Dynamic batching on the device (Section 3.4, "Dynamic batching").
//
// The cut rule is a sequential greedy chain: a batch that starts at triangle
// c takes whole triangles while it has at most N_u distinct indices and at
// most N_pmax triangles; the first triangle that would break a limit starts
// the next batch.  Write next(c) for the end of the batch that starts at c;
// the plan is the chain 0, next(0), next(next(0)), ...  It is computed
// exactly, in parallel, in three steps:
//
//  1. next(c) for every c (k_plan_next).  A workgroup stages the indices of
//     a block of starts plus N_pmax triangles in LDS and finds every corner's
//     previous occurrence in that window (hash slots, bucketed by a counting
//     sort).  The distinct count of the full N_pmax window of every start
//     follows from a difference array; where it is within N_u, next(c) is
//     the window's end.  Otherwise the start's lane finds the cut: a corner
//     is new to the batch [c, e) exactly when its previous occurrence lies
//     before c, so the count of a shorter batch is the window's count minus
//     the new corners of the triangles dropped from its end; the lane drops
//     triangles from the end while the count is over N_u (or, when the
//     window is more than twice over, adds them from c until it would be).
//  2. Transfer tables (k_plan_table, k_plan_compose).  The triangles are cut
//     into segments of L >= N_pmax triangles.  The chain's state at a
//     segment boundary is its first position at or after the boundary, which
//     lies within N_pmax triangles of it.  For every possible entry offset a
//     table gives the exit offset at the segment's end (one lane per entry
//     follows next() in LDS); tables of consecutive ranges are composed into
//     one, level by level, until few remain, and each composition records
//     every member table's entry for every entry of its group.
//  3. Resolution (k_plan_top, k_plan_resolve, k_plan_emit).  The top tables
//     are applied in order from entry 0 and entries are pushed down the
//     levels through those records; at level 0 every segment takes its
//     entry, walks next() from it to list its batch starts, and copies them
//     into [B, start_0, .., start_{B-1}, T] at an offset found by a
//     decoupled look-back.
// Every step does bounded parallel work whatever the batch structure; the
// result equals the sequential chain exactly.
#pragma once

#include "vr_device.h"

namespace vr {

constexpr uint16_t kEnd = 0xFFFF;                            // table value: the chain has ended
constexpr uint32_t kNone = 0xFFFF;                           // no previous / next occurrence

constexpr uint32_t ceil_log2(uint32_t x) { return x <= 1 ? 0 : 1 + ceil_log2((x + 1) / 2); }

// Primitive-cap classes: the planner's kernels are instantiated for caps up
// to 256, 512, 1024, 2048 and 4096 triangles.
__host__ __device__ inline uint32_t plan_class(uint32_t tmax) {
    uint32_t c = 256;
    while (c < tmax) c <<= 1;
    return c;
}

// Tables composed per group: as many as fit in 64 KB of LDS, at most 32.
__host__ __device__ inline uint32_t plan_fan_in(uint32_t tmax) {
    const uint32_t f = 32768u / tmax;
    return f < 2 ? 2 : (f > 32 ? 32 : f);
}

// k_plan_next for caps up to TMC triangles: one start per thread, the
// window of the block's starts plus TMC triangles, corners per thread, a
// power-of-two hash table at most 8/9 full.
template <uint32_t TMC>
struct NextClass {
    static constexpr uint32_t threads = TMC == 512 ? 1024 : (TMC == 1024 ? 256 : 512);
    static constexpr uint32_t starts = threads;
    static constexpr uint32_t tris = starts + TMC;
    static constexpr uint32_t corners = 3 * tris;
    static constexpr uint32_t per = (corners + threads - 1) / threads;
    static constexpr uint32_t bits = ceil_log2(corners + corners / 8);
    static constexpr uint32_t slots = 1u << bits;
    // LDS: keys -> corner positions grouped by slot (+ the difference array),
    // the hash table -> bucket starts | ends, slot counts -> previous
    // occurrences packed per triangle (three 16-bit positions in 64 bits)
    static constexpr uint32_t prev_words = (slots / 4 > tris + 4) ? slots / 4 : tris + 4;
    static constexpr uint32_t lds = 4 * corners + 4 * slots + 8 * prev_words + 64;
    static_assert(slots % threads == 0, "table slots split evenly over the threads");
    static_assert(slots >= corners + corners / 8 && corners < kNone, "window fits the table and 16-bit positions");
    static_assert(2 * corners + 4 * (starts + 1) <= 4 * corners, "difference array fits behind the positions");
    static_assert(lds <= 160 * 1024, "window fits the LDS");
};

// k_plan_check for caps up to TMC triangles: one window per workgroup.  The
// table is sized for the class whatever N_pmax: a sparser table keeps the
// longest probe chain of a lockstep round short on windows of distinct
// indices.
template <uint32_t TMC>
struct CheckClass {
    static constexpr uint32_t threads = TMC <= 1024 ? 256 : 1024;
    static constexpr uint32_t per = 3 * TMC / threads;
    static constexpr uint32_t bits = ceil_log2(3 * TMC) + 1 < 14 ? ceil_log2(3 * TMC) + 1 : 14;
    static_assert((1u << bits) >= 3 * TMC + 3 * TMC / 4, "check table must hold every corner");
};

struct PlanArgs {
    const uint32_t *idx;
    uint32_t V, T;
    uint32_t cap, tmax;        // N_u, N_pmax
    uint32_t seg_len, nseg;    // L and the number of segments
    uint32_t *next;            // [T]
    uint32_t *err;
    uint32_t *fail;            // holds `epoch` once an aligned window is over budget
    uint32_t epoch;            // this planning call's number (never 0)
};

// True when the aligned chain of this call was verified (the general
// kernels then have nothing to do).
__device__ __forceinline__ bool plan_is_aligned(const uint32_t *fail, uint32_t epoch) { return *fail != epoch; }

__device__ __forceinline__ uint32_t seg_lo(const PlanArgs &P, uint32_t s) { return s * P.seg_len; }
__device__ __forceinline__ uint32_t seg_hi(const PlanArgs &P, uint32_t s) { return min(P.T, (s + 1) * P.seg_len); }

// ---------------------------------------------------------------------------
// 0. Aligned fast path.  If every aligned window [k N_pmax, (k+1) N_pmax)
// holds at most N_u distinct indices, the greedy chain is 0, N_pmax,
// 2 N_pmax, ...: from a start k N_pmax every prefix of the window stays
// within the budget, so the batch takes all N_pmax triangles (or the rest of
// the stream).  One workgroup per window counts its distinct indices in an
// LDS hash set; a window over the budget stores the call's epoch in *fail
// (every writer stores the same value).  Indices >= V raise
// VR_ERR_INDEX_RANGE here, since the general pass may not run.
// ---------------------------------------------------------------------------
template <uint32_t TMC>
__global__ __launch_bounds__(CheckClass<TMC>::threads) void k_plan_check(PlanArgs P, uint32_t *plan) {
    using C = CheckClass<TMC>;
    constexpr uint32_t NT = C::threads, kPer = C::per, kBits = C::bits;
    __shared__ __attribute__((aligned(16))) uint32_t s_tab[1u << kBits];
    __shared__ uint32_t s_tmp[NT / kWave];
    const uint32_t tid = threadIdx.x;
    const uint32_t t0 = blockIdx.x * P.tmax, t1 = min(P.T, t0 + P.tmax);
    const uint32_t n = 3 * (t1 - t0);
    // the aligned chain [K, 0, N_pmax, .., (K-1) N_pmax, T], written before
    // it is verified: when a window fails, the general planner's kernels
    // overwrite the count, the starts and the end
    if (tid == 0) {
        plan[1 + blockIdx.x] = t0;
        if (blockIdx.x == 0) {
            plan[0] = gridDim.x;
            plan[1 + gridDim.x] = P.T;
        }
    }
    // every load is issued before the first is checked, so their latencies overlap
    uint32_t key[kPer];
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t i = tid + NT * k;
        key[k] = i < n ? P.idx[3ull * t0 + i] : 0u;
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        if (tid + NT * k < n && key[k] >= P.V) {
            raise_error(P.err, VR_ERR_INDEX_RANGE);
            key[k] = 0;
        }
    }
    constexpr uint32_t mask = (1u << kBits) - 1;
    for (uint32_t q = 4 * tid; q <= mask; q += 4 * NT) *(uint4 *)&s_tab[q] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
    __syncthreads();
    uint32_t slot[kPer], pending = 0, fresh = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        slot[k] = hash_slot(key[k], kBits);
        if (tid + NT * k < n) pending |= 1u << k;
    }
    while (pending) {   // lockstep linear probing; the table never fills
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) {
            if (pending & (1u << k)) {
                const uint32_t prev = atomicCAS(&s_tab[slot[k]], kEmpty, key[k]);
                if (prev == kEmpty || prev == key[k]) {
                    fresh += prev == kEmpty;
                    pending &= ~(1u << k);
                } else {
                    slot[k] = (slot[k] + 1) & mask;
                }
            }
        }
    }
    uint32_t distinct;
    block_excl_scan<NT>(fresh, s_tmp, distinct);
    if (tid == 0 && distinct > P.cap) *P.fail = P.epoch;
}

// ---------------------------------------------------------------------------
// 1. next(c) for every start c
// ---------------------------------------------------------------------------
template <uint32_t TMC>
__global__ __launch_bounds__(NextClass<TMC>::threads) void k_plan_next(PlanArgs P) {
    using Win = NextClass<TMC>;
    constexpr uint32_t NT = Win::threads, kNextBlock = Win::starts, kNextTris = Win::tris, kNextSlots = Win::slots;
    if (plan_is_aligned(P.fail, P.epoch)) return;
    // LDS regions are reused once their first contents are dead:
    //   s_a: indices (insert) -> corner positions grouped by slot + start counts
    //   s_tab: keys (insert) -> bucket start | bucket end << 16 per slot
    //   s_cnt: slot counts -> 3 x 16-bit previous occurrence per triangle
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    uint32_t *s_a = (uint32_t *)smem;
    uint32_t *s_tab = s_a + 3 * kNextTris;
    unsigned long long *s_cntprev = (unsigned long long *)(s_tab + kNextSlots);
    uint32_t *s_tmp = (uint32_t *)(s_cntprev + Win::prev_words);
    uint16_t *s_cnt = (uint16_t *)s_cntprev;
    unsigned long long *s_prev = s_cntprev;
    uint32_t *s_key = s_a;
    uint16_t *s_arr = (uint16_t *)s_a;                       // 3 * kNextTris entries
    int *s_diff = (int *)(s_a + (3 * kNextTris + 1) / 2);    // kNextBlock + 1 entries
    uint32_t *s_se = s_tab;
    constexpr uint32_t E = kNextSlots / NT;   // slots per thread in the clears and the scan
    static_assert(E % 8 == 0, "slots are handled in 16-byte LDS accesses");
    const uint32_t tid = threadIdx.x;
    const uint32_t c0 = blockIdx.x * kNextBlock;
    const uint32_t r1 = min(P.T, c0 + kNextBlock + P.tmax);
    const uint32_t n = 3 * (r1 - c0);

    // three loads per thread issued before the first is checked (latencies overlap)
    for (uint32_t i0 = 0; i0 < n; i0 += 3 * NT) {
        uint32_t v[3];
#pragma unroll
        for (uint32_t r = 0; r < 3; ++r) {
            const uint32_t i = i0 + r * NT + tid;
            v[r] = i < n ? P.idx[3ull * c0 + i] : 0u;
        }
#pragma unroll
        for (uint32_t r = 0; r < 3; ++r) {
            const uint32_t i = i0 + r * NT + tid;
            if (i < n) {
                if (v[r] >= P.V) {
                    raise_error(P.err, VR_ERR_INDEX_RANGE);
                    v[r] = 0;
                }
                s_key[i] = v[r];
            }
        }
    }
#pragma unroll
    for (uint32_t j = 0; j < E / 4; ++j)
        ((uint4 *)(s_tab + tid * E))[j] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
#pragma unroll
    for (uint32_t j = 0; j < E / 8; ++j) ((uint4 *)(s_cnt + tid * E))[j] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    // insertion: every thread owns corners tid + NT*k (k < kPer) and probes
    // them in lockstep rounds so their LDS round trips overlap
    constexpr uint32_t kBits = Win::bits;
    constexpr uint32_t kPer = Win::per;
    uint32_t key[kPer], slot[kPer];
    uint64_t pending = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t i = tid + NT * k;
        key[k] = i < n ? s_key[i] : 0u;
        slot[k] = hash_slot(key[k], kBits);
        if (i < n) pending |= 1ull << k;
    }
    while (pending) {
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) {
            if (pending & (1ull << k)) {
                const uint32_t prev = atomicCAS(&s_tab[slot[k]], kEmpty, key[k]);
                if (prev == kEmpty || prev == key[k]) pending &= ~(1ull << k);
                else slot[k] = (slot[k] + 1) & (kNextSlots - 1);
            }
        }
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t i = tid + NT * k;
        if (i < n) {
            // counts per slot (16-bit LDS words are updated through their 32-bit word)
            atomicAdd((uint32_t *)&s_cnt[slot[k] & ~1u], (slot[k] & 1u) ? 0x10000u : 1u);
        }
    }
    __syncthreads();
    {   // bucket starts: exclusive scan of the counts, E slots per thread;
        // each slot's word becomes start | end << 16 with the end (the fill
        // cursor) starting at the start
        const uint4 *c4 = (const uint4 *)(s_cnt + tid * E);
        auto half_sum = [](uint32_t w) { return (w & 0xFFFFu) + (w >> 16); };
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t j = 0; j < E / 8; ++j) {
            const uint4 w = c4[j];
            sum += half_sum(w.x) + half_sum(w.y) + half_sum(w.z) + half_sum(w.w);
        }
        uint32_t total;
        uint32_t run = block_excl_scan<NT>(sum, s_tmp, total);
        uint4 *o4 = (uint4 *)(s_se + tid * E);
#pragma unroll
        for (uint32_t j = 0; j < E / 8; ++j) {
            const uint4 w = c4[j];
            const uint32_t cw[4] = {w.x, w.y, w.z, w.w};
            uint32_t o[8];
#pragma unroll
            for (uint32_t h = 0; h < 4; ++h) {
                o[2 * h] = run * 0x10001u;
                run += cw[h] & 0xFFFFu;
                o[2 * h + 1] = run * 0x10001u;
                run += cw[h] >> 16;
            }
            o4[2 * j] = make_uint4(o[0], o[1], o[2], o[3]);
            o4[2 * j + 1] = make_uint4(o[4], o[5], o[6], o[7]);
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t i = tid + NT * k;
        if (i < n) {
            const uint32_t sl = slot[k];
            const uint32_t old = atomicAdd(&s_se[sl], 0x10000u);
            s_arr[old >> 16] = (uint16_t)i;
        }
    }
    for (uint32_t c = tid; c <= kNextBlock; c += NT) s_diff[c] = 0;
    __syncthreads();
    // previous occurrence of every corner inside the window (bucket order is
    // arbitrary, so take the largest position below the corner's own), and
    // the difference array of the full-window distinct counts: corner p is
    // new to the N_pmax-triangle window starting at c exactly for
    // prev(p) < 3c <= p < 3c + 3*N_pmax
    // every thread walks the buckets of its kPer corners in lockstep
    const uint32_t span = 3 * P.tmax;
    uint32_t q[kPer], qe[kPer], best[kPer];
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t i = tid + NT * k;
        const uint32_t se = i < n ? s_se[slot[k]] : 0u;
        q[k] = se & 0xFFFFu;
        qe[k] = se >> 16;
        best[k] = kNone;
    }
    for (bool more = true; more;) {
        more = false;
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) {
            if (q[k] < qe[k]) {
                const uint32_t i = tid + NT * k;
                const uint32_t a = s_arr[q[k]++];
                if (a < i && (best[k] == kNone || a > best[k])) best[k] = a;
                more |= q[k] < qe[k];
            }
        }
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t i = tid + NT * k;
        uint32_t lo = 1, hi = 0;
        if (i < n) {
            ((uint16_t *)s_prev)[4 * (i / 3) + i % 3] = (uint16_t)best[k];
            const uint32_t lo_prev = best[k] == kNone ? 0u : best[k] / 3 + 1;
            const uint32_t lo_win = i + 1 > span ? (i + 1 - span + 2) / 3 : 0u;
            lo = max(lo_prev, lo_win);
            hi = min(i / 3, kNextBlock - 1);
        }
        // many corners start at 0 (no earlier occurrence in the first window):
        // one atomic per wavefront for them; ends past the last start are
        // never read and are dropped
        const uint64_t at0 = ballot(lo == 0 && lo <= hi);
        if (at0 && lane_id() == (uint32_t)__builtin_ctzll(at0)) atomicAdd(&s_diff[0], (int)__popcll(at0));
        if (lo <= hi) {
            if (lo != 0) atomicAdd(&s_diff[lo], 1);
            if (hi + 1 < kNextBlock) atomicAdd(&s_diff[hi + 1], -1);
        }
    }
    __syncthreads();
    // full-window distinct count of this lane's start (inclusive scan of the
    // difference array; each thread owns one start)
    uint32_t dfull;
    {
        uint32_t total;
        const int d = s_diff[tid];
        dfull = block_excl_scan<NT>((uint32_t)d, s_tmp, total) + (uint32_t)d;
    }
    const uint32_t c = c0 + tid;
    if (c < P.T) {
        const uint32_t lim = min(P.T, c + P.tmax);
        uint32_t t = lim;
        if (dfull > P.cap) {
            // the budget breaks inside the window (kNone + 1 wraps to 0, so a
            // missing previous occurrence always counts as new).  Each corner
            // counts on its own (new iff its previous occurrence lies before the
            // start), so the count of a shorter batch is the window's count
            // minus the new corners of the triangles dropped from its end.
            // Where the window is at most twice over the budget the cut is
            // found from the end, else from the start.
            const uint32_t first = 3 * tid;
            auto fresh = [&](unsigned long long x) {
                return ((uint32_t)((x + 1) & 0xFFFF) <= first) + ((uint32_t)(((x >> 16) + 1) & 0xFFFF) <= first) +
                       ((uint32_t)(((x >> 32) + 1) & 0xFFFF) <= first);
            };
            if (dfull - P.cap <= P.cap) {
                uint32_t distinct = dfull;
                t = lim;
                while (distinct > P.cap) {   // ends by t = c + 1: one triangle never exceeds N_u >= 3
                    unsigned long long pr[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) pr[u] = t > c + u ? s_prev[t - 1 - u - c0] : 0ull;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (distinct > P.cap) {
                            distinct -= fresh(pr[u]);
                            --t;
                        }
                    }
                }
            } else {
                uint32_t distinct = 0;
                t = c;
                bool stop = false;
                while (!stop && t < lim) {
                    unsigned long long pr[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) pr[u] = s_prev[t - c0 + u];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (!stop && t < lim) {
                            const uint32_t f = fresh(pr[u]);
                            if (distinct + f > P.cap) stop = true;
                            else {
                                distinct += f;
                                ++t;
                            }
                        }
                    }
                }
            }
        }
        P.next[c] = t;
    }
}

// ---------------------------------------------------------------------------
// 2. Transfer tables.  Table layout: tmax entries of uint16 per range; entry
// j = the chain's first position at or after the range's start boundary is
// boundary + j; value = its first position at or after the range's end
// boundary minus that boundary, or kEnd once the chain has reached T.  One
// lane per entry follows next() through the segment (staged in LDS).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_plan_table(PlanArgs P, uint16_t *tab) {
    extern __shared__ __attribute__((aligned(16))) uint32_t s_nx[];   // seg_len entries
    if (plan_is_aligned(P.fail, P.epoch)) return;
    const uint32_t s = blockIdx.x;
    const uint32_t b = seg_lo(P, s), e = seg_hi(P, s), len = e - b;
    {   // 16-byte loads: a segment starts at a multiple of 2048 entries
        const uint4 *src = (const uint4 *)(P.next + b);
        for (uint32_t i = threadIdx.x; i < len / 4; i += 256) ((uint4 *)s_nx)[i] = src[i];
        for (uint32_t i = len / 4 * 4 + threadIdx.x; i < len; i += 256) s_nx[i] = P.next[b + i];
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < P.tmax; j += 256) {
        uint16_t out = kEnd;
        if (j < len) {
            uint32_t x = b + j;
            while (x < e) x = s_nx[x - b];
            out = x >= P.T ? kEnd : (uint16_t)(x - e);
        }
        tab[(size_t)s * P.tmax + j] = out;
    }
}

// Composes tables [g*fan, min(count, g*fan + fan)) of `in` into table g of
// `out` (fan = plan_fan_in(tmax)).  On the way it records, for every entry j
// of the group, the entry of each member table (`pre`, laid out as `in`):
// once the group's entry is known, a member's entry is one lookup.
__global__ __launch_bounds__(512) void k_plan_compose(uint32_t tmax, uint32_t count, const uint16_t *in,
                                                      uint16_t *out, uint16_t *pre, const uint32_t *fail,
                                                      uint32_t epoch) {
    extern __shared__ uint16_t s_t[];   // fan * tmax
    if (plan_is_aligned(fail, epoch)) return;
    const uint32_t fan = plan_fan_in(tmax);
    const uint32_t g = blockIdx.x;
    const uint32_t k0 = g * fan, k1 = min(count, k0 + fan);
    const uint32_t m = (k1 - k0) * tmax;
    for (uint32_t i = threadIdx.x; i < m; i += 512) s_t[i] = in[(size_t)k0 * tmax + i];
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < tmax; j += 512) {
        uint32_t x = j;
        for (uint32_t k = 0; k < k1 - k0; ++k) {
            pre[(size_t)(k0 + k) * tmax + j] = (uint16_t)x;
            if (x != kEnd) x = s_t[k * tmax + x];
        }
        out[(size_t)g * tmax + j] = (uint16_t)x;
    }
}

// One workgroup: applies the (at most fan) top tables in order starting
// from entry 0 and records each table's entry.
__global__ __launch_bounds__(256) void k_plan_top(uint32_t tmax, uint32_t count, const uint16_t *tab,
                                                  uint16_t *entry, const uint32_t *fail, uint32_t epoch) {
    extern __shared__ uint16_t s_t[];
    if (plan_is_aligned(fail, epoch)) return;
    const uint32_t m = count * tmax;
    for (uint32_t i = threadIdx.x; i < m; i += 256) s_t[i] = tab[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0;
        for (uint32_t k = 0; k < count; ++k) {
            entry[k] = (uint16_t)x;
            if (x != kEnd) x = s_t[k * tmax + x];
        }
    }
}

// Pushes entries one level down: table i of a level (of `count`) gets its
// entry from its group's entry up_entry[i / fan] through the member entries
// `pre` recorded by k_plan_compose.  One thread per table.
__global__ __launch_bounds__(256) void k_plan_resolve(uint32_t tmax, uint32_t count, const uint16_t *pre,
                                                      const uint16_t *up_entry, uint16_t *entry,
                                                      const uint32_t *fail, uint32_t epoch) {
    if (plan_is_aligned(fail, epoch)) return;
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const uint32_t x = up_entry[i / plan_fan_in(tmax)];
    entry[i] = x == kEnd ? kEnd : pre[(size_t)i * tmax + x];
}

// Level 0, merged with listing and packing.  Segment s receives its entry
// (`mode`): 0, directly from `up` (the tables have one level); 1, from its
// group's entry at level 1 (`up`, pushed down by k_plan_top and
// k_plan_resolve) through the member entries k_plan_compose recorded
// (`pre0`); 2, with exactly two levels, from its group's entry found by the
// block itself, walking the level-1 tables before its group (`up`, staged in
// LDS) from entry 0, then through `pre0` (no k_plan_top launch).  One thread
// follows next() from the entry (next() of the
// segment staged in LDS) and lists the segment's batch starts; the segment
// publishes its count and resolves its offset in the plan with a decoupled
// look-back over the segments, then the block copies its starts there.  The
// status words hold [63:32] the call's epoch, [31:30] a flag (1 count, 2
// prefix including the segment), [29:0] the count, so words left by earlier
// calls read as not ready and nothing needs clearing.  The last segment
// writes B and T.
__device__ __forceinline__ uint32_t plan_lookback(unsigned long long *status, uint32_t s, uint32_t cnt,
                                                  uint32_t epoch, uint32_t *err) {
    const uint32_t lane = lane_id();
    const unsigned long long tag = (unsigned long long)epoch << 32;
    uint32_t excl = 0;
    int64_t hi = (int64_t)s;   // the window is segments hi - 64 .. hi - 1, lane i reading hi - 1 - i
    uint32_t spins = 0;
    while (hi > 0) {
        const int64_t j = hi - 1 - (int64_t)lane;
        const unsigned long long w =
            j >= 0 ? __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : (tag | (2u << 30));
        const uint32_t flag = (w >> 32) == epoch ? (uint32_t)(w >> 30) & 3u : 0u;
        const uint64_t inc = ballot(flag == 2);
        const uint64_t need = inc ? ((inc & (~inc + 1)) << 1) - 1 : ~0ull;
        if (ballot(flag == 0) & need) {
            if (++spins > (1u << 26)) {
                if (lane == 0) raise_error(err, VR_ERR_DEVICE);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const uint32_t v = ((need >> lane) & 1ull) ? (uint32_t)w & 0x3FFFFFFFu : 0u;
        excl += (uint32_t)__builtin_amdgcn_readlane(wave_incl_scan(v), kWave - 1);
        if (inc) break;
        hi -= kWave;
    }
    if (lane == 0)
        __hip_atomic_store(&status[s], tag | (2ull << 30) | (excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

__global__ __launch_bounds__(256) void k_plan_emit(PlanArgs P, const uint16_t *pre0, const uint16_t *up,
                                                   uint32_t mode, unsigned long long *status, uint32_t *plan) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ uint32_t s_cnt, s_off;
    if (plan_is_aligned(P.fail, P.epoch)) return;
    const uint32_t tid = threadIdx.x, s = blockIdx.x;
    const uint32_t b = seg_lo(P, s), e = seg_hi(P, s), len = e - b;
    uint32_t *s_nx = (uint32_t *)smem;                    // seg_len entries
    uint32_t *s_cut = s_nx + P.seg_len;                   // seg_len entries
    uint16_t *s_t = (uint16_t *)(s_cut + P.seg_len);      // mode 2: level-1 tables before the group
    const uint32_t g = s / plan_fan_in(P.tmax);
    // 16-byte loads: next() of a segment starts at a multiple of 2048 entries
    // and the level-1 tables at a 256-byte boundary of the planner's scratch
    {
        const uint4 *src = (const uint4 *)(P.next + b);
        for (uint32_t i = tid; i < len / 4; i += 256) ((uint4 *)s_nx)[i] = src[i];
        for (uint32_t i = len / 4 * 4 + tid; i < len; i += 256) s_nx[i] = P.next[b + i];
    }
    const uint32_t m = mode == 2 ? g * P.tmax : 0u;
    for (uint32_t i = tid; i < m / 8; i += 256) ((uint4 *)s_t)[i] = ((const uint4 *)up)[i];
    for (uint32_t i = m / 8 * 8 + tid; i < m; i += 256) s_t[i] = up[i];
    __syncthreads();
    if (tid == 0) {
        uint32_t x;
        if (mode == 0) {
            x = up[s];
        } else if (mode == 1) {
            x = up[g];
        } else {
            x = 0;
            for (uint32_t k = 0; k < g && x != kEnd; ++k) x = s_t[k * P.tmax + x];
        }
        if (mode != 0 && x != kEnd) x = pre0[(size_t)s * P.tmax + x];
        uint32_t n = 0;
        if (x != kEnd)
            for (uint32_t t = b + x; t < e; t = s_nx[t - b]) s_cut[n++] = t;
        s_cnt = n;
        if (s == 0) __hip_atomic_store(&status[0], ((unsigned long long)P.epoch << 32) | (2ull << 30) | n,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else __hip_atomic_store(&status[s], ((unsigned long long)P.epoch << 32) | (1ull << 30) | n,
                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t cnt = s_cnt;
    if (tid < kWave) {
        const uint32_t off = s == 0 ? 0u : plan_lookback(status, s, cnt, P.epoch, P.err);
        if (tid == 0) s_off = off;
    }
    __syncthreads();
    const uint32_t off = s_off;
    for (uint32_t i = tid; i < cnt; i += 256) plan[1 + off + i] = s_cut[i];
    if (s + 1 == P.nseg && tid == 0) {
        plan[0] = off + cnt;
        plan[1 + off + cnt] = P.T;
    }
}

}  // namespace vr
