// Geometry-stage kernels for gfx950: naive, LDS sort / hash / parallel-hash
// deduplication over static or dynamic batches, and wave64 ballot rounds.
#pragma once

#include "vr_device.h"

namespace vr {

typedef float f4 __attribute__((ext_vector_type(4)));

enum DedupMode { kSort = 0, kHash = 1, kPHash = 2 };

// Everything a draw kernel reads besides the shader parameters.
struct DrawArgs {
    const uint32_t *idx;        // uint32[3T]
    const f4 *vtx;              // [V][2] float4
    uint32_t V, T;
    uint32_t batch_tris;        // static batches: N_p
    uint32_t num_batches;       // static batches: ceil(T / N_p)
    const uint32_t *plan;       // dynamic batches: [B, start_0 .. start_{B-1}, T]
    f4 *corners;                // [3T][3]
    uint32_t *tris;             // [3T]
    f4 *verts;                  // [..][3]
    uint16_t *local_idx;        // [3T]
    uint32_t *unit_offsets;     // [units + 1]
    uint32_t *unit_inv;         // [units]
    unsigned long long *counters;   // [4]
    unsigned long long *agg;    // per batch: (units << 32) | invocations
    unsigned long long *status; // look-back words, zero at launch (cleared by k_finish)
    uint32_t *err;              // first device-side error
    unsigned long long *total_inv;  // invocations since the last vr_sync
    uint32_t hash_bits;         // log2 of the LDS hash-table size
    uint32_t probes;            // parallel hashing: per-lane probes
    uint32_t max_idx;           // LDS capacity in corners (3 * max triangles per unit)
    uint32_t max_uniq;          // LDS capacity in shaded vertices
    uint32_t need_prefix;       // tris / verts / unit arrays requested
    uint32_t status_cap;        // look-back words available
    uint32_t stream_verts;      // no corners: shaded vertices stream out through an NT-row stage
};

// Units a launch may take: the plan's count, bounded by the look-back
// capacity (a plan built for other limits raises an error instead of
// overrunning scratch).
__device__ __forceinline__ uint32_t launch_units(const DrawArgs &A, uint32_t nb) {
    if (A.need_prefix && nb > A.status_cap) {
        raise_error(A.err, VR_ERR_CAPACITY);
        return A.status_cap;
    }
    return nb;
}

__device__ __forceinline__ uint32_t batch_count(const DrawArgs &A) {
    return A.plan ? A.plan[0] : A.num_batches;
}

__device__ __forceinline__ void batch_range(const DrawArgs &A, uint32_t b, uint32_t &t0, uint32_t &t1) {
    if (A.plan) {   // the plan may be that of a longer stream with the same start
        t0 = A.plan[1 + b];
        t1 = min(A.plan[2 + b], A.T);
    } else {
        t0 = b * A.batch_tris;
        t1 = min(A.T, t0 + A.batch_tris);
    }
}

// Index fetch with the range check fused in: an index >= V raises
// VR_ERR_INDEX_RANGE and is replaced by 0 so no access leaves the buffers.
__device__ __forceinline__ uint32_t checked_index(const DrawArgs &A, uint32_t k) {
    if (k >= A.V) {
        raise_error(A.err, VR_ERR_INDEX_RANGE);
        k = 0;
    }
    return k;
}

__device__ __forceinline__ uint32_t fetch_index(const DrawArgs &A, uint64_t pos) {
    return checked_index(A, A.idx[pos]);
}

// The indices idx[base .. base + n) into dst[0 .. n), checked as
// fetch_index does, by NT threads; each thread issues three loads before it
// uses the first, so that their latencies overlap.
template <uint32_t NT>
__device__ __forceinline__ void load_indices(const DrawArgs &A, uint64_t base, uint32_t n, uint32_t *dst,
                                             uint32_t tid) {
    for (uint32_t i0 = 0; i0 < n; i0 += 3 * NT) {
        uint32_t v[3];
#pragma unroll
        for (uint32_t r = 0; r < 3; ++r) {
            const uint32_t i = i0 + r * NT + tid;
            v[r] = i < n ? A.idx[base + i] : 0u;
        }
#pragma unroll
        for (uint32_t r = 0; r < 3; ++r) {
            const uint32_t i = i0 + r * NT + tid;
            if (i < n) dst[i] = checked_index(A, v[r]);
        }
    }
}

// Shades the vertex whose 32 input bytes are (a, b) into dst[0..2].
template <int KIND>
__device__ __forceinline__ void shade_raw_to_lds(const vr_shader_params &sh, f4 a, f4 b, f4 *dst) {
    float4 o0, o1, o2;
    shade_vertex<KIND>(sh, make_float4(a.x, a.y, a.z, a.w), make_float4(b.x, b.y, b.z, b.w), o0, o1, o2);
    dst[0] = f4{o0.x, o0.y, o0.z, o0.w};
    dst[1] = f4{o1.x, o1.y, o1.z, o1.w};
    dst[2] = f4{o2.x, o2.y, o2.z, o2.w};
}

template <int KIND>
__device__ __forceinline__ void shade_to_lds(const DrawArgs &A, const vr_shader_params &sh, uint32_t v,
                                             f4 *dst) {
    const f4 a = A.vtx[2ull * v], b = A.vtx[2ull * v + 1];
    float4 o0, o1, o2;
    shade_vertex<KIND>(sh, make_float4(a.x, a.y, a.z, a.w), make_float4(b.x, b.y, b.z, b.w), o0, o1, o2);
    dst[0] = f4{o0.x, o0.y, o0.z, o0.w};
    dst[1] = f4{o1.x, o1.y, o1.z, o1.w};
    dst[2] = f4{o2.x, o2.y, o2.z, o2.w};
}

// Assembly (Section 4.2): every corner of the unit's triangles receives its
// shaded vertex.  The unit's corner rows are one contiguous span, so lane q
// stores float4 q of the span: fully coalesced 16-byte stores.
template <int NT, typename LocalT>
__device__ __forceinline__ void write_unit(const DrawArgs &A, uint32_t t0, uint32_t ntri, const LocalT *s_local,
                                           const f4 *s_sv, uint32_t inv, uint32_t vbase, uint32_t unit,
                                           uint32_t tid, bool verts_written = false) {
    const uint32_t ncorner = 3 * ntri;
    if (A.corners) {
        // float4 q of the span is part q % 3 of corner q / 3.  Lane tid takes
        // q = tid + NT i; NT is a power of two, so NT = r (mod 3) with r = 1
        // or 2, and for i = 3 m + j the corner is NT m + kj[j] and the part
        // pj[j], both fixed per lane: no division in the loop.  Three rows per
        // lane at a time, so that their LDS reads overlap.
        constexpr uint32_t r = NT % 3;
        static_assert(r != 0, "the workgroup size is a power of two");
        uint32_t kj[3], pj[3];
#pragma unroll
        for (uint32_t j = 0; j < 3; ++j) {
            const uint32_t m = tid + r * j;
            kj[j] = (NT - r) / 3 * j + m / 3;
            pj[j] = m % 3;
        }
        f4 *dst = A.corners + 9ull * t0;
        const uint32_t cnt = 9 * ntri, klast = ncorner - 1;
        for (uint32_t q = tid, kb = 0; q < cnt; q += 3 * NT, kb += NT) {
            uint32_t at[3];
            f4 row[3];
            // rows past the span read the last corner (kept in bounds) and are not stored
#pragma unroll
            for (uint32_t j = 0; j < 3; ++j) at[j] = 3 * (uint32_t)s_local[min(kb + kj[j], klast)] + pj[j];
#pragma unroll
            for (uint32_t j = 0; j < 3; ++j) row[j] = s_sv[at[j]];
#pragma unroll
            for (uint32_t j = 0; j < 3; ++j)
                if (q + j * NT < cnt) __builtin_nontemporal_store(row[j], dst + q + j * NT);
        }
    }
    if (A.tris || A.local_idx) {
        for (uint32_t k = tid; k < ncorner; k += NT) {
            const uint32_t l = s_local[k];
            if (A.tris) A.tris[3ull * t0 + k] = vbase + l;
            if (A.local_idx) A.local_idx[3ull * t0 + k] = (uint16_t)l;
        }
    }
    if (A.verts && !verts_written) {
        f4 *dst = A.verts + 3ull * vbase;
        for (uint32_t q = tid; q < 3 * inv; q += NT) __builtin_nontemporal_store(s_sv[q], dst + q);
    }
    if (tid == 0) {
        if (A.unit_offsets) A.unit_offsets[unit] = t0;
        if (A.unit_inv) A.unit_inv[unit] = inv;
    }
}

// ---------------------------------------------------------------------------
// End of a batched draw: each workgroup sums a slice of the per-batch
// aggregates and adds it to the counters (zeroed by the draw's first
// kernel) and to the context total, one atomic per counter and workgroup,
// and clears its slice of the look-back words for the next launch.
__global__ __launch_bounds__(256) void k_finish(const uint32_t *plan, uint32_t num_batches, uint32_t status_cap,
                                                const unsigned long long *agg, unsigned long long *status,
                                                unsigned long long *counters, unsigned long long *total_inv) {
    __shared__ unsigned long long part[4];
    uint32_t nb = plan ? plan[0] : num_batches;
    if (nb > status_cap) nb = status_cap;
    unsigned long long sum = 0;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nb; i += gridDim.x * 256) {
        sum += agg[i];
        if (status) status[i] = 0;
    }
    for (int d = 32; d > 0; d >>= 1) sum += __shfl_down(sum, d, kWave);
    if (lane_id() == 0) part[threadIdx.x / kWave] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        const unsigned long long inv = t & 0xFFFFFFFFull, units = t >> 32;
        if (counters) {
            atomicAdd(&counters[0], inv);
            atomicAdd(&counters[1], units);
        }
        atomicAdd(total_inv, inv);
    }
}

// The draw's first kernel clears its counters before k_finish adds to them.
__device__ __forceinline__ void clear_counters(const DrawArgs &A) {
    if (blockIdx.x == 0 && threadIdx.x < 4 && A.counters) A.counters[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// Naive (Section 3.3): no reuse, every corner is shaded.  One lane per
// corner (three invocations per triangle as in the paper's one thread per
// triangle); the block's corner rows are staged in LDS and stored
// contiguously.
// ---------------------------------------------------------------------------
// One chunk of 256 corners (256 threads); s_sv holds 768 float4.  Returns
// the chunk's aggregate ((triangles started) << 32 | invocations).
template <int KIND>
__device__ __forceinline__ unsigned long long naive_chunk(const DrawArgs &A, const vr_shader_params &sh,
                                                          uint32_t chunk, f4 *s_sv) {
    const uint32_t tid = threadIdx.x;
    const uint64_t n = 3ull * A.T;
    const uint64_t c0 = (uint64_t)chunk * 256;
    const uint32_t cnt = (uint32_t)min<uint64_t>(256, n - c0);
    if (tid < cnt) {
        const uint64_t c = c0 + tid;
        const uint32_t v = fetch_index(A, c);
        shade_to_lds<KIND>(A, sh, v, s_sv + 3 * tid);
        const uint32_t corner = (uint32_t)(c % 3);
        if (A.tris) A.tris[c] = (uint32_t)c;
        if (A.local_idx) A.local_idx[c] = (uint16_t)corner;
        if (corner == 0) {
            const uint32_t t = (uint32_t)(c / 3);
            if (A.unit_offsets) A.unit_offsets[t] = t;
            if (A.unit_inv) A.unit_inv[t] = 3;
        }
    }
    __syncthreads();
    for (uint32_t q = tid; q < 3 * cnt; q += 256) {
        if (A.corners) __builtin_nontemporal_store(s_sv[q], A.corners + 3 * c0 + q);
        if (A.verts) __builtin_nontemporal_store(s_sv[q], A.verts + 3 * c0 + q);
    }
    __syncthreads();
    const uint64_t tris_started = (c0 + cnt + 2) / 3 - (c0 + 2) / 3;
    return (tris_started << 32) | cnt;
}

template <int KIND>
__global__ __launch_bounds__(256) void k_naive(DrawArgs A, vr_shader_params sh) {
    __shared__ f4 s_sv[256 * 3];
    naive_chunk<KIND>(A, sh, blockIdx.x, s_sv);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long n = 3ull * A.T;
        if (A.unit_offsets) A.unit_offsets[A.T] = A.T;
        if (A.counters) {
            A.counters[0] = n;
            A.counters[1] = A.T;
            A.counters[2] = 0;
            A.counters[3] = 0;
        }
        atomicAdd(A.total_inv, n);
    }
}

// ---------------------------------------------------------------------------
// Two-pass reference (Section 4.2, Table 2), not streaming: every vertex of
// the buffer is shaded once by a first kernel, referenced or not; a second
// kernel assembles the corners from the shaded buffer in global memory.
// ---------------------------------------------------------------------------
// 256 vertices per workgroup: shaded into LDS, then stored as one contiguous
// span of rows (plain stores, so the rows stay in the caches for the gather).
template <int KIND>
__global__ __launch_bounds__(256) void k_multi_shade(DrawArgs A, vr_shader_params sh, f4 *shaded) {
    __shared__ f4 s_sv[256 * 3];
    const uint32_t v0 = blockIdx.x * 256, tid = threadIdx.x;
    const uint32_t cnt = min(256u, A.V - v0);
    if (tid < cnt) shade_to_lds<KIND>(A, sh, v0 + tid, s_sv + 3 * tid);
    __syncthreads();
    f4 *dst = shaded + 3ull * v0;
    for (uint32_t q = tid; q < 3 * cnt; q += 256) dst[q] = s_sv[q];
}

// 256 corners per workgroup: each lane gathers its corner's three rows from
// the shaded buffer into LDS, then the block's rows are stored as one
// contiguous span (fully coalesced 16-byte stores).  The single unit's
// counters and offsets come from block 0.
__global__ __launch_bounds__(256) void k_multi_assemble(DrawArgs A, const f4 *shaded) {
    __shared__ f4 s_rows[256 * 3];
    const uint64_t n = 3ull * A.T, c0 = (uint64_t)blockIdx.x * 256;
    const uint32_t tid = threadIdx.x;
    const uint32_t cnt = (uint32_t)min<uint64_t>(256, n - c0);
    if (tid < cnt) {
        const uint32_t v = fetch_index(A, c0 + tid);
        const f4 *src = shaded + 3ull * v;
        s_rows[3 * tid] = src[0];
        s_rows[3 * tid + 1] = src[1];
        s_rows[3 * tid + 2] = src[2];
        if (A.tris) A.tris[c0 + tid] = v;
    }
    __syncthreads();
    if (A.corners)
        for (uint32_t q = tid; q < 3 * cnt; q += 256) __builtin_nontemporal_store(s_rows[q], A.corners + 3 * c0 + q);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (A.counters) {
            A.counters[0] = A.V;
            A.counters[1] = 1;
            A.counters[2] = 0;
            A.counters[3] = 0;
        }
        if (A.unit_offsets) {
            A.unit_offsets[0] = 0;
            A.unit_offsets[1] = A.T;
        }
        if (A.unit_inv) A.unit_inv[0] = A.V;
        atomicAdd(A.total_inv, (unsigned long long)A.V);
    }
}

// ---------------------------------------------------------------------------
// LDS layout of the dedup kernel (bytes), shared with the host launcher.
// ---------------------------------------------------------------------------
struct DedupLds {
    uint32_t keys, local, pairs, stab, table, first, uniq, sv, tmp, total;
};

__host__ __device__ inline uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

__host__ __device__ inline uint32_t pow2_ceil(uint32_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Count groups per digit of the sort's radix passes: rounds x wavefronts,
// padded to whole words.
__host__ __device__ inline uint32_t sort_groups(uint32_t max_idx, uint32_t nt) {
    const uint32_t g = (max_idx + nt - 1) / nt * (nt / 64);
    return (g + 3u) & ~3u;
}

// The local ids and the unique list live from deduplication to the end of
// the unit; the shaded vertices (written after deduplication) share their
// region with what deduplication alone uses: the indices, then the sort's
// two position buffers and its per-digit counts (uint8) and offsets
// (uint16), or the hash table and the first-position words.  sv_rows shaded vertices are
// kept: every unique vertex of a unit when corners are assembled, else one
// stage of nt rows through which the shaded vertices stream out.
__host__ __device__ inline DedupLds dedup_lds_layout(int mode, uint32_t max_idx, uint32_t max_uniq,
                                                     uint32_t hash_bits, uint32_t nt, uint32_t sv_rows) {
    DedupLds L{};
    uint32_t off = 0;
    if (mode == kSort) {
        // The sort writes the local ids and the unique list only after its
        // last pass, so they sit in the space of its count tables, past the
        // buffers the run-end scan still reads and past the shaded vertices
        // (written from the start once the sort's buffers are dead).
        uint32_t d = 0;
        L.keys = d;  d += align16(4 * max_idx);
        L.pairs = d; d += align16(4 * max_idx);   // two uint16 position buffers
        L.stab = d;  d += 3u * 256u * sort_groups(max_idx, nt);
        L.sv = 0;
        uint32_t lu = max(align16(48 * sv_rows), L.stab);
        L.local = lu; lu += align16(2 * max_idx);   // uint16 ids < max_idx
        L.uniq = lu;  lu += align16(4 * max_uniq);
        L.table = L.first = 0;
        off = max(lu, d);
    } else {
        L.local = off; off += align16(2 * max_idx);   // uint16: hash slots < 8192, then ids < max_idx
        L.uniq = off;  off += align16(4 * max_uniq);
        L.sv = off;
        uint32_t d = off;
        L.keys = d;    d += align16(4 * max_idx);
        L.pairs = L.stab = 0;
        L.table = d; d += align16(4u << hash_bits);
        L.first = d; d += align16(4u << hash_bits);
        off = max(align16(off + 48 * sv_rows), align16(d));
    }
    L.tmp = off;  off += 64;
    L.total = off;
    return L;
}

// Ranks flagged entries of a unit in index order with a blocked scan:
// thread t owns entries [t*E, t*E+E).  flag(i) is evaluated once and kept
// in a register mask (E <= 32).  Returns the number of flagged entries.
template <int NT, typename FlagF, typename EmitF>
__device__ __forceinline__ uint32_t rank_flagged(uint32_t n, uint32_t *s_tmp, FlagF flag, EmitF emit) {
    const uint32_t E = (n + NT - 1) / NT;
    const uint32_t lo = min(n, threadIdx.x * E), hi = min(n, lo + E);
    uint32_t mask = 0, cnt = 0;
    for (uint32_t i = lo; i < hi; ++i)
        if (flag(i)) {
            mask |= 1u << (i - lo);
            ++cnt;
        }
    uint32_t total;
    uint32_t r = block_excl_scan<NT>(cnt, s_tmp, total);   // has barriers
    for (uint32_t i = lo; i < hi; ++i)
        if (mask & (1u << (i - lo))) emit(i, r++);
    return total;
}

// LSD radix sort of a unit's positions by index (Algorithm 2's sort): 8-bit
// digits of (index - unit minimum), `passes` of them.  Within a pass, element
// x of the current order is handled in round x / NT by thread x % NT; its
// stable destination is the offset of (digit, round, wavefront) plus its
// rank among the wavefront's lanes with the same digit, found with 8
// ballots.  Counts (uint8) and offsets (uint16) are stored per digit
// contiguously in `tab`, so the thread owning a digit scans them with word
// accesses and clears the counts for the next pass.  RR is the round count
// when known at compile time (R == RR), else 8 (R <= 8).  Returns the sorted
// order (one of the two position buffers).
template <int NT, uint32_t RR>
__device__ __forceinline__ const uint16_t *radix_passes(const uint32_t *s_keys, uint16_t *src, uint16_t *dst,
                                                        uint32_t n, uint32_t R, uint32_t kmin, uint32_t passes,
                                                        uint32_t Gp, unsigned char *tab, uint32_t *s_tmp) {
    constexpr uint32_t NW = NT / kWave;
    constexpr uint32_t DP = NT >= 256 ? 1u : 256u / NT;   // digits per thread in the scan
    const uint32_t tid = threadIdx.x, w = tid / kWave;
    uint32_t *s_c32 = (uint32_t *)tab;              // [256][Gp] uint8 counts
    uint2 *s_o64 = (uint2 *)(tab + 256 * Gp);       // [256][Gp] uint16 offsets
    const uint16_t *s_o16 = (const uint16_t *)s_o64;
    uint8_t *s_c8 = (uint8_t *)s_c32;
    for (uint32_t pass = 0; pass < passes; ++pass) {
        uint32_t dig[RR], rank[RR], pos[RR];
#pragma unroll
        for (uint32_t r = 0; r < RR; ++r) {
            if (RR == 8 && r >= R) break;
            const uint32_t x = r * NT + tid;
            const bool act = x < n;
            const uint32_t p = act ? src[x] : 0u;
            const uint32_t d = act ? ((s_keys[p] - kmin) >> (8 * pass)) & 0xFFu : 0u;
            // lanes with the same digit: for each bit, the lanes that agree
            // on it are m where the bit is set and ~m where it is clear
            const uint64_t act_m = ballot(act);
            uint32_t plo = (uint32_t)act_m, phi = (uint32_t)(act_m >> 32);
            const uint32_t nd = ~d;
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                // nx = ~0 where the bit is clear, 0 where it is set (one signed
                // bit-field extract, kept opaque so that it is not rebuilt from
                // compares and selects)
                uint32_t nx;
                asm volatile("v_bfe_i32 %0, %1, %2, 1" : "=v"(nx) : "v"(nd), "n"(bit));
                const uint64_t m = ballot(nx == 0u);
                plo &= (uint32_t)m ^ nx;
                phi &= (uint32_t)(m >> 32) ^ nx;
            }
            const uint64_t peers = ((uint64_t)phi << 32) | plo;
            const uint32_t rk = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
            // digit x group index in 24-bit products (full-rate multiplies)
            if (act && rk == 0) s_c8[__umul24(d, Gp) + r * NW + w] = (uint8_t)__popcll(peers);
            dig[r] = d;
            rank[r] = rk;
            pos[r] = p;
        }
        __syncthreads();
        {   // exclusive offsets in (digit, round, wavefront) order
            const uint32_t d0 = tid * DP, words = Gp / 4;
            uint32_t sum = 0;
            if (d0 < 256)
                for (uint32_t j = 0; j < DP * words; ++j) {
                    const uint32_t c = s_c32[d0 * words + j];
                    sum += (c & 0xFFu) + ((c >> 8) & 0xFFu) + ((c >> 16) & 0xFFu) + (c >> 24);
                }
            uint32_t total;
            uint32_t run = block_excl_scan<NT>(sum, s_tmp, total);
            if (d0 < 256)
                for (uint32_t j = 0; j < DP * words; ++j) {
                    const uint32_t c = s_c32[d0 * words + j];
                    s_c32[d0 * words + j] = 0;   // counts start at zero next pass
                    const uint32_t o0 = run, o1 = o0 + (c & 0xFFu), o2 = o1 + ((c >> 8) & 0xFFu),
                                   o3 = o2 + ((c >> 16) & 0xFFu);
                    run = o3 + (c >> 24);
                    s_o64[d0 * words + j] = make_uint2(o0 | (o1 << 16), o2 | (o3 << 16));
                }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < RR; ++r) {
            if (RR == 8 && r >= R) break;
            const uint32_t x = r * NT + tid;
            if (x < n) dst[s_o16[__umul24(dig[r], Gp) + r * NW + w] + rank[r]] = (uint16_t)pos[r];
        }
        __syncthreads();
        uint16_t *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// ---------------------------------------------------------------------------
// Batched deduplication + shading + assembly (Algorithms 2 and 3, and the
// parallel-hashing variant).  Workgroup u owns unit u (no atomics to pick
// work); a unit of n corners is deduplicated in LDS into inv unique
// vertices with canonical local ids:
//   sort  - ascending rank among distinct indices (Algorithm 2),
//   hash  - first-occurrence order (Algorithm 3, ids made independent of
//           the insertion races by ranking each slot's first position),
//   phash - as hash, but a lane that fails `probes` linear probes hands its
//           key to a wavefront-cooperative probe of 64 slots at a time.
// ---------------------------------------------------------------------------
template <int NT, int MODE, int KIND>
__device__ __forceinline__ void dedup_unit(const DrawArgs &A, const vr_shader_params &sh, uint32_t u, uint32_t nb,
                                           unsigned char *smem) {
    // without corners, units whose unique vertices would not leave room for
    // several workgroups per CU stream them out through an NT-row stage
    const bool stream = A.stream_verts != 0;
    const DedupLds L = dedup_lds_layout(MODE, A.max_idx, A.max_uniq, A.hash_bits, NT, stream ? NT : A.max_uniq);
    uint32_t *s_keys = (uint32_t *)(smem + L.keys);
    uint16_t *s_local = (uint16_t *)(smem + L.local);
    uint32_t *s_uniq = (uint32_t *)(smem + L.uniq);
    f4 *s_sv = (f4 *)(smem + L.sv);
    uint32_t *s_tmp = (uint32_t *)(smem + L.tmp);
    __shared__ uint32_t s_vbase;

    const uint32_t tid = threadIdx.x, lane = lane_id();
    {
        uint32_t t0, t1;
        batch_range(A, u, t0, t1);
        uint32_t n = 3 * (t1 - t0);
        const bool fits = t1 >= t0 && n <= A.max_idx;   // false only for a plan built with other limits
        if (!fits) {
            if (tid == 0) raise_error(A.err, VR_ERR_CAPACITY);
            n = 0;
        }

        load_indices<NT>(A, 3ull * t0, n, s_keys, tid);

        uint32_t inv;
        if (MODE == kSort) {
            // LSD radix sort of the positions by index (radix_passes), only
            // as many passes as the unit's index range needs
            uint16_t *s_pos0 = (uint16_t *)(smem + L.pairs);
            uint16_t *s_pos1 = s_pos0 + A.max_idx;
            const uint32_t R = (n + NT - 1) / NT;   // <= 8: the launcher sizes NT >= max_idx / 8
            const uint32_t Gp = sort_groups(A.max_idx, NT);
            uint32_t *s_c32 = (uint32_t *)(smem + L.stab);                     // [256][Gp] uint8 counts
            __syncthreads();
            uint32_t kmin = kEmpty, kmax = 0;
            for (uint32_t i = tid; i < n; i += NT) {
                const uint32_t k = s_keys[i];
                kmin = min(kmin, k);
                kmax = max(kmax, k);
                s_pos0[i] = (uint16_t)i;
            }
            for (uint32_t i = tid; i < 64 * Gp; i += NT) s_c32[i] = 0;
            block_reduce_minmax<NT>(kmin, kmax, s_tmp);
            const uint32_t span = n ? kmax - kmin : 0u;
            const uint32_t passes = span ? (32u - __builtin_clz(span) + 7u) / 8u : 0u;
            // the round count fixed at compile time where it is small
            const uint16_t *src;
            if (R <= 1) src = radix_passes<NT, 1>(s_keys, s_pos0, s_pos1, n, R, kmin, passes, Gp, smem + L.stab, s_tmp);
            else if (R == 2) src = radix_passes<NT, 2>(s_keys, s_pos0, s_pos1, n, R, kmin, passes, Gp, smem + L.stab, s_tmp);
            else if (R == 3) src = radix_passes<NT, 3>(s_keys, s_pos0, s_pos1, n, R, kmin, passes, Gp, smem + L.stab, s_tmp);
            else src = radix_passes<NT, 8>(s_keys, s_pos0, s_pos1, n, R, kmin, passes, Gp, smem + L.stab, s_tmp);
            // run ends of the sorted indices; the exclusive prefix over run
            // ends is the rank of every entry's run (Algorithm 2's marks and
            // prefix sum)
            __syncthreads();
            const uint32_t E = (n + NT - 1) / NT;
            const uint32_t lo = min(n, tid * E), hi = min(n, lo + E);
            uint32_t cnt = 0;
            for (uint32_t i = lo; i < hi; ++i) cnt += (i + 1 == n || s_keys[src[i]] != s_keys[src[i + 1]]);
            uint32_t r = block_excl_scan<NT>(cnt, s_tmp, inv);
            for (uint32_t i = lo; i < hi; ++i) {
                const uint32_t p = src[i], k = s_keys[p];
                s_local[p] = (uint16_t)r;
                if (i + 1 == n || k != s_keys[src[i + 1]]) s_uniq[r++] = k;
            }
        } else {
            uint32_t *s_table = (uint32_t *)(smem + L.table);
            uint32_t *s_first = (uint32_t *)(smem + L.first);
            const uint32_t S = 1u << A.hash_bits, mask = S - 1;
            // Ids are visible only in the indexed outputs and local ids; then
            // they are made canonical (first-occurrence order).  Otherwise a
            // key's id comes from a counter taken by the lane that inserted
            // it (Algorithm 3), and the corners are the same either way.
            const bool canon = A.need_prefix || A.local_idx;
            __shared__ uint32_t s_count;
            for (uint32_t s = tid; s < S; s += NT) {
                s_table[s] = kEmpty;
                s_first[s] = kEmpty;
            }
            if (tid == 0) s_count = 0;
            __syncthreads();
            // the inserting lane of a new key takes the next id
            auto take_id = [&](uint32_t slot, uint32_t key) {
                const uint32_t id = atomicAdd(&s_count, 1u);
                s_first[slot] = id;
                if (id < A.max_uniq) s_uniq[id] = key;
            };
            if (MODE == kHash) {
                for (uint32_t i = tid; i < n; i += NT) {
                    const uint32_t k = s_keys[i];
                    uint32_t p = hash_slot(k, A.hash_bits);
                    for (uint32_t probe = 0;; ++probe) {   // linear probing; S >= distinct keys
                        const uint32_t prev = atomicCAS(&s_table[p], kEmpty, k);
                        if (prev == kEmpty && !canon) take_id(p, k);
                        if (prev == kEmpty || prev == k) break;
                        if (probe >= mask) {              // table full: only with foreign plans
                            raise_error(A.err, VR_ERR_CAPACITY);
                            break;
                        }
                        p = (p + 1) & mask;
                    }
                    s_local[i] = (uint16_t)p;
                    if (canon) atomicMin(&s_first[p], i);
                }
            } else {
                // wave-uniform sweep so the cooperative path sees every lane
                for (uint32_t base = (tid / kWave) * kWave; base < n; base += NT) {
                    const uint32_t i = base + lane;
                    const bool act = i < n;
                    const uint32_t k = act ? s_keys[i] : 0u;
                    uint32_t p = hash_slot(k, A.hash_bits);
                    uint32_t slot = 0;
                    bool placed = !act;
                    for (uint32_t r = 0; r < A.probes && !placed; ++r) {
                        const uint32_t prev = atomicCAS(&s_table[p], kEmpty, k);
                        if (prev == kEmpty && !canon) take_id(p, k);
                        if (prev == kEmpty || prev == k) {
                            slot = p;
                            placed = true;
                        } else {
                            p = (p + 1) & mask;
                        }
                    }
                    uint64_t pend = ballot(!placed);
                    while (pend) {
                        const uint32_t Lr = (uint32_t)__ffsll((long long)pend) - 1;
                        const uint32_t key = __builtin_amdgcn_readlane(k, Lr);
                        uint32_t start = __builtin_amdgcn_readlane(p, Lr);
                        for (uint32_t sweep = 0;; ++sweep) {
                            if (sweep > 2 * (mask + 1)) {     // table full: only with foreign plans
                                if (lane == 0) raise_error(A.err, VR_ERR_CAPACITY);
                                break;
                            }
                            const uint32_t s = (start + lane) & mask;
                            const uint32_t val = __hip_atomic_load(&s_table[s], __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                            const uint64_t hit = ballot(val == kEmpty || val == key);
                            if (!hit) {
                                start = (start + kWave) & mask;
                                continue;
                            }
                            const uint32_t w = (uint32_t)__ffsll((long long)hit) - 1;
                            const uint32_t ws = (start + w) & mask;
                            uint32_t got = 0;
                            if (lane == w) {
                                got = atomicCAS(&s_table[ws], kEmpty, key);
                                if (got == kEmpty && !canon) take_id(ws, key);
                            }
                            got = __builtin_amdgcn_readlane(got, w);
                            if (got == kEmpty || got == key) {
                                if (lane == Lr) {
                                    slot = ws;
                                    placed = true;
                                }
                                break;
                            }
                            start = ws;   // lost the slot to another key: continue past it
                        }
                        pend &= pend - 1;
                    }
                    if (act) {
                        s_local[i] = (uint16_t)slot;
                        if (canon) atomicMin(&s_first[slot], i);
                    }
                }
            }
            __syncthreads();
            if (canon) {
                // canonical ids: a slot's id is the rank of its first position;
                // every flag is read before the scan's barriers, so the first
                // position can overwrite its slot's word with the rank
                inv = rank_flagged<NT>(
                    n, s_tmp, [&](uint32_t i) { return s_first[s_local[i]] == i; },
                    [&](uint32_t i, uint32_t r) {
                        s_uniq[r] = s_keys[i];
                        s_first[s_local[i]] = r;
                    });
                __syncthreads();
            } else {
                inv = s_count;
            }
            for (uint32_t i = tid; i < n; i += NT) s_local[i] = (uint16_t)s_first[s_local[i]];
        }

        if (inv > A.max_uniq) {   // only with a plan built for a larger N_u
            if (tid == 0) raise_error(A.err, VR_ERR_CAPACITY);
            inv = 0;
        }
        // publish this unit's invocation count early; resolve after shading
        // (before it when the shaded vertices stream out)
        if (A.need_prefix && tid == 0) lookback_publish(A.status, u, (1ull << 32) | inv);
        __syncthreads();
        if (!stream)
            for (uint32_t j = tid; j < inv; j += NT) shade_to_lds<KIND>(A, sh, s_uniq[j], s_sv + 3 * j);
        if (tid < kWave) {   // the first wavefront, whole (NT >= 64)
            uint32_t vb = 0;
            if (A.need_prefix) vb = (uint32_t)lookback_resolve(A.status, u, (1ull << 32) | inv, A.err);
            if (tid == 0) {
                s_vbase = vb;
                if (A.unit_offsets && u + 1 == nb) A.unit_offsets[nb] = A.T;
            }
        }
        __syncthreads();
        if (stream) {
            // NT unique vertices at a time: shaded into the stage, then stored
            // as one contiguous span of rows
            f4 *dst = A.verts ? A.verts + 3ull * s_vbase : nullptr;
            for (uint32_t j0 = 0; j0 < inv; j0 += NT) {
                const uint32_t rows = min((uint32_t)NT, inv - j0);
                if (tid < rows) shade_to_lds<KIND>(A, sh, s_uniq[j0 + tid], s_sv + 3 * tid);
                __syncthreads();
                if (dst)
                    for (uint32_t q = tid; q < 3 * rows; q += NT)
                        __builtin_nontemporal_store(s_sv[q], dst + 3ull * j0 + q);
                __syncthreads();
            }
        }
        if (fits && (inv > 0 || n == 0))
            write_unit<NT>(A, t0, t1 - t0, s_local, s_sv, inv, s_vbase, u, tid, stream);
        if (tid == 0 && A.agg) A.agg[u] = (1ull << 32) | inv;
        __syncthreads();   // the caller may reuse the LDS for the next unit
    }
}

// Units from base on: unit base + workgroup index (stride 0), or
// grid-stride over every unit from base on (stride = the grid).  Grid-stride
// serves the units of a dynamic draw beyond the fewest it can have within
// the same launch; it is used without prefix outputs only, since the
// look-back needs each unit's predecessor running or done.  With OCC the
// kernel is held to eight wavefronts per SIMD (seven for the sort, whose
// registers would otherwise spill): the host picks it only when the unit's
// LDS lets that many workgroups reside, and then the extra wavefronts hide
// more of a unit's serial latency; otherwise the bound would only add
// spills.
template <int NT, int MODE, int KIND, bool OCC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC ? (MODE == kSort ? 7 : 8) : 1))) void k_dedup(DrawArgs A, vr_shader_params sh, uint32_t base, uint32_t stride) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    if (base == 0) clear_counters(A);
    const uint32_t nb = launch_units(A, batch_count(A));
    for (uint64_t u = (uint64_t)base + blockIdx.x; u < nb; u += stride ? stride : nb)
        dedup_unit<NT, MODE, KIND>(A, sh, (uint32_t)u, nb, smem);
}

// ---------------------------------------------------------------------------
// Wave64 ballot rounds (Algorithm 1 on a 64-lane wavefront).  One wavefront
// owns a batch and cuts it into rounds: it fetches 21 whole triangles (63
// indices, one per lane) at a time and resolves them one distinct value at
// a time: the lowest unresolved lane's index is broadcast (readlane), every
// lane holding the same index is resolved together (ballot), and if no lane
// holds it yet the lowest free lane takes it.  The first triangle that would
// need a 65th lane ends the round; lanes taken by rejected triangles are
// released, so a round shades exactly its distinct indices.
// ---------------------------------------------------------------------------
struct RoundState {
    uint32_t my_id;   // the vertex this lane shades in the round
    uint32_t fill;    // lanes in use (= invocations of the round)
    f4 va, vb;        // its input, loaded when the lane took it (output sweep only)
};

// Indices of a batch a wavefront keeps in LDS (the rest, for batches of more
// than 256 triangles, is fetched per group of 21 triangles).
constexpr uint32_t kBallotPrefetch = 768;

// LDS of one ballot wavefront: 64 shaded vertices, the prefetched indices, a
// hand-over area for new values (2 x 64 words) and a lane number per corner.
__host__ __device__ inline uint32_t ballot_lds_bytes(uint32_t batch_tris) {
    const uint32_t pre = 3 * batch_tris < kBallotPrefetch ? 3 * batch_tris : kBallotPrefetch;
    return 64 * 48 + 4 * pre + 2 * 64 * 4 + ((3 * batch_tris + 15u) & ~15u);
}

// Processes one round starting at triangle `cur` of the batch starting at
// t0; returns the round's end.  The batch's first `pre` indices are in
// s_keys; s_new is the wavefront's hand-over area.  When s_map is not NULL
// it receives each corner's lane (local id).
//
// A group of 21 triangles is resolved by votes, one per distinct value: the
// lowest unresolved lane broadcasts its index, and ballots give the lanes
// holding it (whose first occurrence is that lane) and the lane that already
// owns it.  Values no lane owns then get the next free lanes in the order of
// their first lanes (a popcount of the first-occurrence mask below), and the
// first lane hands the value to the lane of its slot through LDS.  This is
// the sequential assignment of Algorithm 1, with the slot bookkeeping taken
// out of the per-value loop (the scalar unit, shared by a CU's wavefronts,
// bounds this loop).
__device__ __forceinline__ uint32_t ballot_round(const DrawArgs &A, uint32_t t0, uint32_t cur, uint32_t t1,
                                                 const uint32_t *s_keys, uint32_t pre, uint32_t *s_new,
                                                 uint8_t *s_map, RoundState &st) {
    const uint32_t lane = lane_id();
    uint32_t my_id = kEmpty, my_intro = kEmpty, fill = 0, done = 0;
    f4 va = {}, vb = {};
    for (;;) {
        const uint32_t gt = min(21u, t1 - cur);
        const uint32_t nc = 3 * gt;
        const bool act = lane < nc;
        const uint32_t pos = __umul24(3u, cur - t0) + lane;   // cur - t0 < 2^24 (a batch)
        const uint32_t k = act ? (pos < pre ? s_keys[pos] : fetch_index(A, 3ull * cur + lane)) : kEmpty;
        // one vote per distinct value, lowest unresolved lane first: that
        // lane is the value's first occurrence in the group
        uint64_t pend = ballot(act);
        uint32_t first = lane, owner = kEmpty;
        if (fill == 0) {   // nothing owned yet in this round
            while (pend) {
                const uint32_t pick = (uint32_t)__builtin_ctzll(pend);
                const uint32_t cv = __builtin_amdgcn_readlane(k, pick);
                const uint64_t same = ballot(k == cv);
                first = __builtin_amdgcn_inverse_ballot_w64(same) ? pick : first;
                pend &= ~same;
            }
        } else {
            while (pend) {
                const uint32_t pick = (uint32_t)__builtin_ctzll(pend);
                const uint32_t cv = __builtin_amdgcn_readlane(k, pick);
                const uint64_t same = ballot(k == cv);
                // the owning lane, or lane 63 when none owns it (checked below)
                const uint32_t ol = (uint32_t)__builtin_ctzll(ballot(my_id == cv) | (1ull << 63));
                const bool in = __builtin_amdgcn_inverse_ballot_w64(same);
                first = in ? pick : first;
                owner = in ? ol : owner;
                pend &= ~same;
            }
            // a candidate owner counts only if it holds the lane's index
            const uint32_t held = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(owner << 2), (int)my_id);
            if (!act || held != k) owner = kEmpty;
        }
        // first occurrences of values no lane owns yet
        const uint64_t fresh = ballot(act && owner == kEmpty && first == lane);
        const uint32_t slot = owner != kEmpty ? owner
                                              : fill + (uint32_t)__popcll(fresh & ((1ull << first) - 1ull));
        if (act && owner == kEmpty && first == lane && slot < (uint32_t)kWave) {
            s_new[slot] = k;
            s_new[kWave + slot] = done + lane;
        }
        wave_sync_lds();
        const uint32_t f = fill + (uint32_t)__popcll(fresh);
        if (lane >= fill && lane < f) {
            my_id = s_new[lane];
            my_intro = s_new[kWave + lane];
            if (s_map) {   // the output sweep: the load overlaps the rest of the round
                va = A.vtx[2ull * my_id];
                vb = A.vtx[2ull * my_id + 1];
            }
        }
        const uint64_t bad = ballot(act && slot >= (uint32_t)kWave);
        const uint32_t acc = bad ? ((uint32_t)__ffsll((long long)bad) - 1) / 3 : gt;
        if (s_map && lane < 3 * acc) s_map[done + lane] = (uint8_t)slot;
        done += 3 * acc;
        cur += acc;
        if (bad) {
            const uint64_t keep = ballot(my_intro < done);
            fill = (uint32_t)__popcll(keep);
            if (!((keep >> lane) & 1ull)) my_id = kEmpty;
            break;
        }
        fill = f;
        if (cur >= t1) break;
    }
    st.my_id = my_id;
    st.fill = fill;
    st.va = va;
    st.vb = vb;
    return cur;
}

// One batch processed by one wavefront in its private LDS area of
// ballot_lds_bytes(batch_tris) bytes.  The batch's indices are loaded once,
// up front; only wavefront-level synchronisation is used, so several
// wavefronts of a workgroup can work on different batches.
template <int KIND>
__device__ __forceinline__ void ballot_batch(const DrawArgs &A, const vr_shader_params &sh, uint32_t b, uint32_t nb,
                                             unsigned char *lds) {
    const uint32_t lane = lane_id();
    uint32_t t0, t1;
    batch_range(A, b, t0, t1);
    if (t1 < t0 || 3 * (t1 - t0) > A.max_idx) {   // only with a plan built for other limits
        if (lane == 0) raise_error(A.err, VR_ERR_CAPACITY);
        t1 = t0;
    }
    const uint32_t cap = A.max_idx < kBallotPrefetch ? A.max_idx : kBallotPrefetch;
    f4 *s_sv = (f4 *)lds;
    uint32_t *s_keys = (uint32_t *)(lds + 64 * 48);
    uint32_t *s_new = s_keys + cap;
    uint8_t *s_map = (uint8_t *)(s_new + 2 * kWave);
    const uint32_t pre = min(3 * (t1 - t0), cap);
    load_indices<kWave>(A, 3ull * t0, pre, s_keys, lane);
    wave_sync_lds();
    uint32_t vbase = 0, ubase = b;
    RoundState st;
    if (A.need_prefix) {
        // counting sweep: the batch's rounds and invocations, published
        // before any output so later batches can resolve their prefix
        uint32_t rounds = 0, inv = 0;
        for (uint32_t cur = t0; cur < t1; ++rounds) {
            cur = ballot_round(A, t0, cur, t1, s_keys, pre, s_new, nullptr, st);
            inv += st.fill;
        }
        const uint64_t agg = ((uint64_t)rounds << 32) | inv;
        if (lane == 0) lookback_publish(A.status, b, agg);
        const uint64_t ex = lookback_resolve(A.status, b, agg, A.err);
        vbase = __builtin_amdgcn_readfirstlane((uint32_t)ex);
        ubase = __builtin_amdgcn_readfirstlane((uint32_t)((ex >> 32) & 0x3FFFFFFFu));
    }
    uint32_t r = 0, inv = 0;
    for (uint32_t cur = t0; cur < t1; ++r) {
        const uint32_t end = ballot_round(A, t0, cur, t1, s_keys, pre, s_new, s_map, st);
        if (lane < st.fill) shade_raw_to_lds<KIND>(sh, st.va, st.vb, s_sv + 3 * lane);
        wave_sync_lds();
        write_unit<64>(A, cur, end - cur, s_map, s_sv, st.fill, vbase, ubase + r, lane);
        wave_sync_lds();
        vbase += st.fill;
        inv += st.fill;
        cur = end;
    }
    if (A.unit_offsets && b + 1 == nb && lane == 0) A.unit_offsets[ubase + r] = A.T;
    if (lane == 0 && A.agg) A.agg[b] = ((unsigned long long)r << 32) | inv;
}

// Two wavefronts per workgroup, one batch each (batch 2 * workgroup +
// wavefront); `stride` is the per-wavefront LDS area.  Two measured faster
// than four and eight, and about as fast as one.
constexpr uint32_t kBallotWaves = 2;

template <int KIND>
__global__ __launch_bounds__(kBallotWaves * 64) void k_ballot(DrawArgs A, vr_shader_params sh, uint32_t stride) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    clear_counters(A);
    const uint32_t nb = launch_units(A, batch_count(A));
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t b = blockIdx.x * kBallotWaves + w;
    if (b >= nb) return;   // only wavefront-level synchronisation follows
    ballot_batch<KIND>(A, sh, b, nb, smem + w * stride);
}

}  // namespace vr
