// Parallel random walk (Section 5) on the reuse machinery: an agent's
// "index" is its packed cell key x | y << 16, and the expensive per-index
// program is the search of the cell's most likely moves, which agents on the
// same cell share.  One workgroup deduplicates the cells of a batch of
// agents in an LDS hash table, evaluates each distinct cell once and then
// moves every agent of the batch.
#pragma once

#include "vr_device.h"

namespace vr {

constexpr uint32_t kWalkKeep = 8;          // options kept per cell
constexpr uint32_t kWalkMaxBatch = 512;    // agents per workgroup
constexpr uint32_t kWalkThreads = 512;     // threads per batch workgroup (4 per cell searched)

struct WalkArgs {
    const uint32_t *keys_in;
    uint32_t *keys_out;
    const float *activity;   // grid * grid, cell (x, y) at y * grid + x
    const int8_t *moves;     // (dx, dy) per move
    const float *weights;    // per move
    const float *uniforms;   // per agent, [0, 1)
    uint32_t n, grid, num_moves, batch;
    unsigned long long *agg;        // per batch: (1 << 32) | evaluations
    unsigned long long *counters;   // {evaluations, units, 0, 0} or NULL
    unsigned long long *total_inv;
    uint32_t *err;
};

// Inserts candidate (l, m) into the kept list (descending, ties keep the
// earlier entry first) by a fixed compare-and-shift network, so no index is
// dynamic and the list stays in registers.
__device__ __forceinline__ void walk_insert(float (&L)[kWalkKeep], uint32_t (&mi)[kWalkKeep], float l, uint32_t m) {
    if (!(l > L[kWalkKeep - 1])) return;
#pragma unroll
    for (uint32_t j = kWalkKeep - 1; j >= 1; --j) {
        const bool above_prev = l > L[j - 1];   // l goes above position j - 1
        const bool above_cur = l > L[j];
        L[j] = above_prev ? L[j - 1] : (above_cur ? l : L[j]);
        mi[j] = above_prev ? mi[j - 1] : (above_cur ? m : mi[j]);
    }
    const bool top = l > L[0];
    mi[0] = top ? m : mi[0];
    L[0] = top ? l : L[0];
}

__device__ __forceinline__ void walk_clear(float (&L)[kWalkKeep], uint32_t (&mi)[kWalkKeep]) {
#pragma unroll
    for (uint32_t j = 0; j < kWalkKeep; ++j) {
        L[j] = -1.0f;   // below every likelihood (activities and weights are >= 0)
        mi[j] = 0;
    }
}

// The kWalkKeep most likely moves among moves [m0, m1) from cell (x, y):
// likelihood = activity of the target times the move's weight (one FP32
// product), moves leaving the grid skipped, descending with ties to the
// lower move index.  The activity is read from `act`, a window of the field
// with row pitch `pitch` whose first cell is (ox, oy) and which holds every
// in-grid target (the whole field, or a tile staged in LDS).  Returns the
// number of moves that stay in the grid.
__device__ __forceinline__ uint32_t walk_search(const WalkArgs &W, uint32_t x, uint32_t y, uint32_t m0, uint32_t m1,
                                                float (&L)[kWalkKeep], uint32_t (&mi)[kWalkKeep], const float *act,
                                                uint32_t pitch, int32_t ox, int32_t oy) {
    uint32_t valid = 0;
    for (uint32_t m = m0; m < m1; ++m) {
        const int32_t tx = (int32_t)x + W.moves[2 * m], ty = (int32_t)y + W.moves[2 * m + 1];
        if (tx < 0 || ty < 0 || tx >= (int32_t)W.grid || ty >= (int32_t)W.grid) continue;
        ++valid;
        walk_insert(L, mi, act[(uint32_t)(ty - oy) * pitch + (uint32_t)(tx - ox)] * W.weights[m], m);
    }
    return valid;
}

// The cell's options searched by one thread; returns the count kept.
__device__ __forceinline__ uint32_t walk_options(const WalkArgs &W, uint32_t x, uint32_t y, float (&L)[kWalkKeep],
                                                 uint32_t (&mi)[kWalkKeep]) {
    walk_clear(L, mi);
    const uint32_t valid = walk_search(W, x, y, 0, W.num_moves, L, mi, W.activity, W.grid, 0, 0);
    return valid < kWalkKeep ? valid : kWalkKeep;
}

// Merges the kept list of lane (lane ^ mask) into this lane's.  For the
// lower lane of the pair, whose moves all precede the partner's, inserting
// the partner's entries in their order keeps ties to the lower move index.
__device__ __forceinline__ void walk_merge_xor(float (&L)[kWalkKeep], uint32_t (&mi)[kWalkKeep], int mask) {
    float PL[kWalkKeep];
    uint32_t PM[kWalkKeep];
#pragma unroll
    for (uint32_t j = 0; j < kWalkKeep; ++j) {
        PL[j] = __shfl_xor(L[j], mask, kWave);
        PM[j] = (uint32_t)__shfl_xor((int)mi[j], mask, kWave);
    }
#pragma unroll
    for (uint32_t j = 0; j < kWalkKeep; ++j) walk_insert(L, mi, PL[j], PM[j]);
}

// One agent's move: the first option whose running FP32 sum exceeds u times
// the options' sum (the last one when rounding leaves none); an agent whose
// options sum to zero stays.  The loops run over all kWalkKeep positions
// with the count as a predicate, so the arrays stay in registers.
__device__ __forceinline__ uint32_t walk_choose(const WalkArgs &W, uint32_t key, float u, const float (&L)[kWalkKeep],
                                                const uint32_t (&mi)[kWalkKeep], uint32_t k) {
    float S = 0.0f;
#pragma unroll
    for (uint32_t j = 0; j < kWalkKeep; ++j)
        if (j < k) S += L[j];
    if (k == 0 || !(S > 0.0f)) return key;
    const float t = u * S;
    float run = 0.0f;
    bool found = false;
    uint32_t m = 0;
#pragma unroll
    for (uint32_t j = 0; j < kWalkKeep; ++j) {
        if (j < k) {
            run += L[j];
            if (!found) m = mi[j];   // ends on the first option past the target, else the last one
            found = found || run > t;
        }
    }
    const uint32_t x = (key & 0xFFFFu) + (uint32_t)(int32_t)W.moves[2 * m];
    const uint32_t y = (key >> 16) + (uint32_t)(int32_t)W.moves[2 * m + 1];
    return (x & 0xFFFFu) | (y << 16);
}

// A key outside the grid raises VR_ERR_INDEX_RANGE; the agent stays.
__device__ __forceinline__ bool walk_key_ok(const WalkArgs &W, uint32_t key) {
    if ((key & 0xFFFFu) < W.grid && (key >> 16) < W.grid) return true;
    raise_error(W.err, VR_ERR_INDEX_RANGE);
    return false;
}

// No reuse: every agent evaluates its own cell.
__global__ __launch_bounds__(256) void k_walk_naive(WalkArgs W) {
    const uint32_t a = blockIdx.x * 256 + threadIdx.x;
    if (a < W.n) {
        const uint32_t key = W.keys_in[a];
        uint32_t out = key;
        if (walk_key_ok(W, key)) {
            float L[kWalkKeep];
            uint32_t mi[kWalkKeep];
            const uint32_t k = walk_options(W, key & 0xFFFFu, key >> 16, L, mi);
            out = walk_choose(W, key, W.uniforms[a], L, mi, k);
        }
        W.keys_out[a] = out;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (W.counters) {
            W.counters[0] = W.n;
            W.counters[1] = W.n;
            W.counters[2] = 0;
            W.counters[3] = 0;
        }
        atomicAdd(W.total_inv, (unsigned long long)W.n);
    }
}

// One batch of up to kWalkMaxBatch agents per workgroup of NT threads: the
// batch's cells go into an LDS hash table (linear probing, 2 x kWalkMaxBatch
// slots); the lane that inserts a cell takes the next id; each distinct cell
// is evaluated once into LDS; every agent then takes its move from its
// cell's options.
// Activity cells a batch can stage in LDS: the bounding box of its distinct
// cells grown by the longest move, when it holds at most this many cells.
constexpr uint32_t kWalkTile = 4096;

template <int NT>
__global__ __launch_bounds__(NT) void k_walk_hash(WalkArgs W) {
    constexpr uint32_t S = 2 * kWalkMaxBatch, mask = S - 1;
    // s_raw holds the hash table and the slot ids while the batch's cells are
    // inserted, then the staged activity tile
    __shared__ uint32_t s_raw[kWalkTile];
    uint32_t *s_table = s_raw, *s_id = s_raw + S;
    float *s_tile = (float *)s_raw;
    __shared__ uint32_t s_key[kWalkMaxBatch], s_uniq[kWalkMaxBatch];
    __shared__ uint16_t s_slot[kWalkMaxBatch];
    __shared__ float s_L[kWalkMaxBatch][kWalkKeep];
    __shared__ uint16_t s_mi[kWalkMaxBatch][kWalkKeep];
    __shared__ uint8_t s_k[kWalkMaxBatch];
    __shared__ uint32_t s_count, s_box[5];   // min x, min y, max x, max y, longest move
    const uint32_t tid = threadIdx.x, b = blockIdx.x;
    if (b == 0 && tid < 4 && W.counters) W.counters[tid] = 0;   // k_finish adds to them afterwards
    const uint32_t a0 = b * W.batch, cnt = min(W.batch, W.n - a0);
    for (uint32_t s = tid; s < S; s += NT) s_table[s] = kEmpty;
    if (tid == 0) {
        s_count = 0;
        s_box[0] = s_box[1] = 0xFFFFFFFFu;
        s_box[2] = s_box[3] = s_box[4] = 0;
    }
    __syncthreads();
    for (uint32_t i = tid; i < cnt; i += NT) {
        const uint32_t key = W.keys_in[a0 + i];
        s_key[i] = key;
        uint32_t p = hash_slot(key, 10);   // S = 1024 slots
        for (;;) {                          // at most cnt <= S / 2 distinct keys: a free slot exists
            const uint32_t prev = atomicCAS(&s_table[p], kEmpty, key);
            if (prev == kEmpty) {
                const uint32_t id = atomicAdd(&s_count, 1u);
                s_id[p] = id;
                s_uniq[id] = key;
                break;
            }
            if (prev == key) break;
            p = (p + 1) & mask;
        }
        s_slot[i] = (uint16_t)p;
    }
    for (uint32_t m = tid; m < W.num_moves; m += NT) {
        const int32_t dx = W.moves[2 * m], dy = W.moves[2 * m + 1];
        atomicMax(&s_box[4], (uint32_t)max(max(dx, -dx), max(dy, -dy)));
    }
    __syncthreads();
    const uint32_t inv = s_count;
    for (uint32_t i = tid; i < cnt; i += NT) s_slot[i] = (uint16_t)s_id[s_slot[i]];   // slot -> id
    for (uint32_t j = tid; j < inv; j += NT) {
        const uint32_t key = s_uniq[j], x = key & 0xFFFFu, y = key >> 16;
        if (x < W.grid && y < W.grid) {
            atomicMin(&s_box[0], x);
            atomicMin(&s_box[1], y);
            atomicMax(&s_box[2], x);
            atomicMax(&s_box[3], y);
        }
    }
    __syncthreads();   // the table and ids are dead from here on
    // the tile: the cells' bounding box grown by the longest move, clipped
    const int32_t R = (int32_t)s_box[4];
    const bool any = s_box[0] <= s_box[2];
    const int32_t tx0 = any ? max(0, (int32_t)s_box[0] - R) : 0, ty0 = any ? max(0, (int32_t)s_box[1] - R) : 0;
    const int32_t tx1 = any ? min((int32_t)W.grid - 1, (int32_t)s_box[2] + R) : 0;
    const int32_t ty1 = any ? min((int32_t)W.grid - 1, (int32_t)s_box[3] + R) : 0;
    const uint32_t tw = (uint32_t)(tx1 - tx0 + 1), th = (uint32_t)(ty1 - ty0 + 1);
    const bool tiled = any && tw * th <= kWalkTile;
    if (tiled) {
        for (uint32_t c = tid; c < tw * th; c += NT) {
            const uint32_t r = c / tw;
            s_tile[c] = W.activity[(uint32_t)(ty0 + (int32_t)r) * W.grid + (uint32_t)tx0 + (c - r * tw)];
        }
        __syncthreads();
    }
    const float *act = tiled ? (const float *)s_tile : W.activity;
    const uint32_t pitch = tiled ? tw : W.grid;
    const int32_t ox = tiled ? tx0 : 0, oy = tiled ? ty0 : 0;
    // four lanes per distinct cell, each searching a quarter of the moves;
    // the quad's lists are merged lane 1 into 0 and 3 into 2, then 2 into 0
    const uint32_t quarter = (W.num_moves + 3) / 4;
    for (uint32_t base = 0; base < inv; base += NT / 4) {   // uniform trip count: every lane shuffles
        const uint32_t j = base + tid / 4, q = tid % 4;
        const bool has = j < inv;
        const uint32_t key = has ? s_uniq[j] : 0u;
        const bool ok = has && (key & 0xFFFFu) < W.grid && (key >> 16) < W.grid;
        if (has && !ok && q == 0) raise_error(W.err, VR_ERR_INDEX_RANGE);
        float L[kWalkKeep];
        uint32_t mi[kWalkKeep];
        walk_clear(L, mi);
        uint32_t valid = 0;
        if (ok)
            valid = walk_search(W, key & 0xFFFFu, key >> 16, min(W.num_moves, q * quarter),
                                min(W.num_moves, (q + 1) * quarter), L, mi, act, pitch, ox, oy);
        walk_merge_xor(L, mi, 1);
        walk_merge_xor(L, mi, 2);
        valid += (uint32_t)__shfl_xor((int)valid, 1, kWave);
        valid += (uint32_t)__shfl_xor((int)valid, 2, kWave);
        if (has && q == 0) {
#pragma unroll
            for (uint32_t r = 0; r < kWalkKeep; ++r) {
                s_L[j][r] = L[r];
                s_mi[j][r] = (uint16_t)mi[r];
            }
            s_k[j] = (uint8_t)(ok ? min(valid, kWalkKeep) : 0u);
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < cnt; i += NT) {
        const uint32_t key = s_key[i];
        const uint32_t id = s_slot[i];
        float L[kWalkKeep];
        uint32_t mi[kWalkKeep];
#pragma unroll
        for (uint32_t q = 0; q < kWalkKeep; ++q) {
            L[q] = s_L[id][q];
            mi[q] = s_mi[id][q];
        }
        W.keys_out[a0 + i] = walk_choose(W, key, W.uniforms[a0 + i], L, mi, s_k[id]);
    }
    if (tid == 0) W.agg[b] = (1ull << 32) | inv;
}

}  // namespace vr
