/*
 * vro.c -- CPU oracle for on-the-fly vertex reuse.  TEST INFRASTRUCTURE
 * ONLY: loaded by the test suite, the smoke check and the benchmark's
 * CPU-baseline leg, never by the product path.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).  Every
 * floating-point step of the vertex programs is spelled out with fmaf and
 * correctly rounded '/' and sqrtf so the FP32 results are reproducible
 * bit for bit by any IEEE-754 implementation of the same sequence.
 *
 * What each part follows in the paper:
 *   - Input model: indexed triangle lists, consecutive triples (Section 3).
 *   - Static batching: fixed triangle ranges per batch (Section 3.3).
 *   - Dynamic batching: front-to-back scan counting unique indices, a batch
 *     closes when the unique budget N or the primitive cap would be
 *     exceeded (Section 3.4, "Dynamic batching").
 *   - Warp voting: a batch is processed in rounds, each round holds at most
 *     one wave worth of distinct indices; a new round may shade a vertex
 *     again (Section 3.3, Algorithm 1).
 *   - Sorting: unit-local ids are the prefix sum over run ends of the sorted
 *     indices, i.e. the ascending rank among distinct values (Algorithm 2).
 *   - Hashing / parallel hashing: one entry per distinct index; ids are
 *     fixed to first-occurrence order (Algorithm 3 and the parallel-hashing
 *     paragraph; the paper's slot numbers depend on atomic races).
 *   - Naive: every corner shaded separately (Section 3.3).
 *   - Reuse metric: ideal reuse = duplicates / index count (Section 4.1,
 *     Table 1).
 *   - FIFO post-transform cache: the classic k-entry FIFO (Section 2).
 */
#include "vro.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define EMPTY_STAMP 0u

/* ------------------------------------------------------------------------
 * Argument rules
 * ---------------------------------------------------------------------- */
static int is_dynamic(int s) { return s >= VRO_DYN_SORT && s <= VRO_DYN_BALLOT; }
static int is_ballot(int s) { return s == VRO_STATIC_BALLOT || s == VRO_DYN_BALLOT; }

static uint32_t max_batch_tris(int s)
{
    switch (s) {
    case VRO_NAIVE:
    case VRO_MULTI: return 0xFFFFFFFFu;
    case VRO_STATIC_BALLOT: return 1024;
    case VRO_STATIC_SORT:
    case VRO_STATIC_HASH: return 256;
    default: return 4096;
    }
}

uint64_t vro_units_bound(int strategy, uint64_t num_tris, uint32_t batch_tris)
{
    if (strategy == VRO_MULTI) return 1;
    if (strategy == VRO_STATIC_SORT || strategy == VRO_STATIC_HASH)
        return batch_tris ? (num_tris + batch_tris - 1) / batch_tris : 0;
    return num_tris;
}

int vro_check_args(uint64_t num_indices, uint32_t num_vertices, const vro_shader *sh,
                   int strategy, uint32_t batch_tris, const vro_opts *opts,
                   const vro_outputs *out, uint32_t *resolved_max_unique)
{
    if (!sh || !out) return VRO_ERR_ARG;
    if (num_indices % 3 != 0 || num_indices > 3ull * ((1ull << 30) - 1)) return VRO_ERR_ARG;
    if (strategy < VRO_NAIVE || strategy > VRO_MULTI) return VRO_ERR_ARG;
    /* MULTI's unit is the whole vertex buffer: no 16-bit local ids */
    if (strategy == VRO_MULTI && out && out->local_idx) return VRO_ERR_ARG;
    if (batch_tris == 0 || batch_tris > max_batch_tris(strategy)) return VRO_ERR_ARG;
    if (sh->kind > 2 || sh->num_lights > VRO_MAX_LIGHTS || sh->spec_squarings > 8 ||
        sh->iterations > 4096)
        return VRO_ERR_ARG;

    uint32_t nu = 0, wg = 0, slots = 0, probes = 0;
    if (opts) { nu = opts->max_unique; wg = opts->wg_size; slots = opts->hash_slots; probes = opts->hash_probes; }
    if (wg != 0 && (wg % 64 != 0 || wg > 1024)) return VRO_ERR_ARG;
    if (probes > 64) return VRO_ERR_ARG;
    if (is_dynamic(strategy)) {
        if (nu == 0) {
            nu = 64u * ((batch_tris + 63u) / 64u);
            if (nu > 4096) nu = 4096;
        }
        if (nu < 3 || nu > 4096) return VRO_ERR_ARG;
    } else {
        nu = 0;
    }
    if (slots != 0) {
        uint32_t need = is_dynamic(strategy) ? nu : 3u * batch_tris;
        if ((slots & (slots - 1)) != 0 || slots < need || slots > 8192) return VRO_ERR_ARG;
    }
    uint64_t T = num_indices / 3;
    if (out->verts && out->verts_cap < (strategy == VRO_MULTI ? (uint64_t)num_vertices : 3 * T))
        return VRO_ERR_CAPACITY;
    if ((out->unit_offsets || out->unit_invocations) &&
        out->units_cap < vro_units_bound(strategy, T, batch_tris))
        return VRO_ERR_CAPACITY;
    if (resolved_max_unique) *resolved_max_unique = nu;
    return VRO_OK;
}

/* ------------------------------------------------------------------------
 * Small helpers
 * ---------------------------------------------------------------------- */
int64_t vro_count_unique(const uint32_t *idx, uint64_t n, uint32_t V)
{
    unsigned char *seen = (unsigned char *)calloc(V ? V : 1, 1);
    if (!seen) return -1;
    int64_t u = 0;
    for (uint64_t k = 0; k < n; ++k) {
        if (idx[k] >= V) { free(seen); return -1; }
        if (!seen[idx[k]]) { seen[idx[k]] = 1; ++u; }
    }
    free(seen);
    return u;
}

int64_t vro_fifo_misses(const uint32_t *idx, uint64_t n, uint32_t V, uint32_t k)
{
    for (uint64_t i = 0; i < n; ++i)
        if (idx[i] >= V) return -1;
    if (k == 0) return (int64_t)n;
    unsigned char *in = (unsigned char *)calloc(V ? V : 1, 1);
    uint32_t *ring = (uint32_t *)malloc(sizeof(uint32_t) * k);
    if (!in || !ring) { free(in); free(ring); return -1; }
    uint64_t head = 0, size = 0;
    int64_t misses = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t v = idx[i];
        if (in[v]) continue;                 /* hit: FIFO order unchanged */
        ++misses;
        if (size == k) {                     /* evict the oldest entry    */
            in[ring[head]] = 0;
            ring[head] = v;
            head = (head + 1) % k;
        } else {
            ring[(head + size) % k] = v;
            ++size;
        }
        in[v] = 1;
    }
    free(in);
    free(ring);
    return misses;
}

/* Parallel per-processor LRU post-transform caches (Section 4.1, Table 1).
 * The index stream is cut into chunks of `per_cycle` indices.  With
 * contiguous != 0 the chunks are split into `procs` consecutive runs of
 * ceil(chunks / procs), run p on processor p, one chunk per shading cycle;
 * otherwise chunk c runs on processor c mod procs in its cycle c / procs.
 * A processor looks
 * every index of its chunk up in its own LRU cache of `entries` shaded
 * vertices as the cache stood after its previous cycle: a hit reuses the
 * result, a miss is shaded in this cycle (duplicates inside one chunk are
 * processed concurrently and all miss).  Then the chunk's indices enter the
 * cache in stream order, each moving to the most-recent end, the least
 * recently used entry leaving when the cache is full.  Processors share
 * nothing, so they are simulated one after another.  Returns the hits, or
 * -1 for an index >= V or an allocation failure. */
typedef struct {
    uint32_t cap, mask, head, tail, size;   /* doubly linked list, most recent at head */
    uint32_t *key, *prev, *next;            /* per entry                               */
    uint32_t *slot;                         /* open addressing: entry + 1, 0 = empty   */
} lru_cache;

static uint32_t lru_hash(uint32_t v, uint32_t mask) { return (v * 2654435761u) & mask; }

static uint32_t lru_find(const lru_cache *c, uint32_t v)   /* entry index or UINT32_MAX */
{
    for (uint32_t h = lru_hash(v, c->mask);; h = (h + 1) & c->mask) {
        if (c->slot[h] == 0) return UINT32_MAX;
        if (c->key[c->slot[h] - 1] == v) return c->slot[h] - 1;
    }
}

static void lru_unlink(lru_cache *c, uint32_t e)
{
    if (c->prev[e] != UINT32_MAX) c->next[c->prev[e]] = c->next[e]; else c->head = c->next[e];
    if (c->next[e] != UINT32_MAX) c->prev[c->next[e]] = c->prev[e]; else c->tail = c->prev[e];
}

static void lru_push_front(lru_cache *c, uint32_t e)
{
    c->prev[e] = UINT32_MAX;
    c->next[e] = c->head;
    if (c->head != UINT32_MAX) c->prev[c->head] = e; else c->tail = e;
    c->head = e;
}

static void lru_erase_key(lru_cache *c, uint32_t v)   /* backward-shift deletion */
{
    uint32_t h = lru_hash(v, c->mask);
    while (c->key[c->slot[h] - 1] != v) h = (h + 1) & c->mask;
    for (uint32_t j = (h + 1) & c->mask;; j = (j + 1) & c->mask) {
        if (c->slot[j] == 0) break;
        const uint32_t home = lru_hash(c->key[c->slot[j] - 1], c->mask);
        /* the entry at j may move to h if h lies cyclically in [home, j) */
        if (((j - home) & c->mask) >= ((j - h) & c->mask)) {
            c->slot[h] = c->slot[j];
            h = j;
        }
    }
    c->slot[h] = 0;
}

static void lru_touch(lru_cache *c, uint32_t v)
{
    uint32_t e = lru_find(c, v);
    if (e != UINT32_MAX) { lru_unlink(c, e); lru_push_front(c, e); return; }
    if (c->size == c->cap) {                       /* reuse the least recent entry */
        e = c->tail;
        lru_unlink(c, e);
        lru_erase_key(c, c->key[e]);
    } else {
        e = c->size++;
    }
    c->key[e] = v;
    uint32_t h = lru_hash(v, c->mask);
    while (c->slot[h] != 0) h = (h + 1) & c->mask;
    c->slot[h] = e + 1;
    lru_push_front(c, e);
}

int64_t vro_parallel_cache_hits(const uint32_t *idx, uint64_t n, uint32_t V, uint32_t procs, uint32_t per_cycle,
                                uint32_t entries, int contiguous)
{
    for (uint64_t i = 0; i < n; ++i)
        if (idx[i] >= V) return -1;
    if (procs == 0 || per_cycle == 0) return -1;
    if (entries == 0) return 0;
    uint32_t slots = 2;
    while (slots < 2 * entries) slots <<= 1;
    lru_cache c;
    c.cap = entries;
    c.mask = slots - 1;
    c.key = (uint32_t *)malloc(sizeof(uint32_t) * entries);
    c.prev = (uint32_t *)malloc(sizeof(uint32_t) * entries);
    c.next = (uint32_t *)malloc(sizeof(uint32_t) * entries);
    c.slot = (uint32_t *)malloc(sizeof(uint32_t) * slots);
    if (!c.key || !c.prev || !c.next || !c.slot) {
        free(c.key); free(c.prev); free(c.next); free(c.slot);
        return -1;
    }
    int64_t hits = 0;
    const uint64_t chunks = (n + per_cycle - 1) / per_cycle;
    const uint64_t run = (chunks + procs - 1) / procs;
    for (uint32_t p = 0; p < procs && p < chunks; ++p) {
        c.head = c.tail = UINT32_MAX;
        c.size = 0;
        memset(c.slot, 0, sizeof(uint32_t) * slots);
        const uint64_t first = contiguous ? p * run : p, step = contiguous ? 1 : procs;
        const uint64_t last = contiguous ? (first + run < chunks ? first + run : chunks) : chunks;
        for (uint64_t ch = first; ch < last; ch += step) {
            const uint64_t a = ch * per_cycle, b = a + per_cycle < n ? a + per_cycle : n;
            for (uint64_t i = a; i < b; ++i) hits += lru_find(&c, idx[i]) != UINT32_MAX;
            for (uint64_t i = a; i < b; ++i) lru_touch(&c, idx[i]);
        }
    }
    free(c.key); free(c.prev); free(c.next); free(c.slot);
    return hits;
}

/* ------------------------------------------------------------------------
 * Parallel random walk (Section 5).  An agent's reuse "index" is its packed
 * cell key x | y << 16; agents on the same cell see the same move
 * likelihoods, so a batch evaluates each distinct cell once.
 * ---------------------------------------------------------------------- */
#define VRO_WALK_KEEP 8

/* The VRO_WALK_KEEP most likely moves from cell (x, y): likelihood =
 * activity(target) * weight(move) in FP32, moves leaving the grid skipped,
 * kept in decreasing likelihood with ties to the lower move index.  Returns
 * how many were kept. */
static uint32_t walk_top(uint32_t x, uint32_t y, const float *act, uint32_t G, const int8_t *mv, const float *w,
                         uint32_t M, float *L, uint32_t *mi)
{
    uint32_t k = 0;
    for (uint32_t m = 0; m < M; ++m) {
        const int64_t tx = (int64_t)x + mv[2 * m], ty = (int64_t)y + mv[2 * m + 1];
        if (tx < 0 || ty < 0 || tx >= (int64_t)G || ty >= (int64_t)G) continue;
        const float l = act[(uint64_t)ty * G + (uint64_t)tx] * w[m];
        uint32_t j = k;                      /* insertion point: after every entry >= l */
        while (j > 0 && l > L[j - 1]) --j;
        if (j >= VRO_WALK_KEEP) continue;
        for (uint32_t t = (k < VRO_WALK_KEEP ? k : VRO_WALK_KEEP - 1); t > j; --t) { L[t] = L[t - 1]; mi[t] = mi[t - 1]; }
        L[j] = l;
        mi[j] = m;
        if (k < VRO_WALK_KEEP) ++k;
    }
    return k;
}

/* One agent's move: target u * S with S the FP32 sum of the kept
 * likelihoods in order; the first option whose running sum exceeds the
 * target is taken (the last one if rounding leaves none); an agent whose
 * options sum to zero stays. */
static uint32_t walk_choose(uint32_t key, float u, const float *L, const uint32_t *mi, uint32_t k, const int8_t *mv)
{
    float S = 0.0f;
    for (uint32_t j = 0; j < k; ++j) S += L[j];
    if (k == 0 || !(S > 0.0f)) return key;
    const float t = u * S;
    uint32_t pick = k - 1;
    float run = 0.0f;
    for (uint32_t j = 0; j < k; ++j) {
        run += L[j];
        if (run > t) { pick = j; break; }
    }
    const uint32_t x = (key & 0xFFFFu) + (uint32_t)(int32_t)mv[2 * mi[pick]];
    const uint32_t y = (key >> 16) + (uint32_t)(int32_t)mv[2 * mi[pick] + 1];
    return (x & 0xFFFFu) | (y << 16);
}

uint32_t vro_walk_options(uint32_t x, uint32_t y, const float *activity, uint32_t grid, const int8_t *moves,
                          const float *weights, uint32_t num_moves, float *L, uint32_t *move_index)
{
    return walk_top(x, y, activity, grid, moves, weights, num_moves, L, move_index);
}

uint32_t vro_walk_choose(uint32_t key, float u, const float *L, const uint32_t *move_index, uint32_t k,
                         const int8_t *moves)
{
    return walk_choose(key, u, L, move_index, k, moves);
}

int vro_walk_step(const uint32_t *keys_in, uint32_t n, const float *activity, uint32_t grid, const int8_t *moves,
                  const float *weights, uint32_t num_moves, const float *uniforms, int strategy, uint32_t batch,
                  uint32_t *keys_out, uint64_t *counters)
{
    if (counters) memset(counters, 0, 4 * sizeof(uint64_t));
    if (grid == 0 || grid > 32768 || num_moves == 0 || num_moves > 65535) return VRO_ERR_ARG;
    if (strategy != VRO_NAIVE && strategy != VRO_STATIC_SORT && strategy != VRO_STATIC_HASH) return VRO_ERR_ARG;
    if (strategy != VRO_NAIVE && (batch == 0 || batch > 512)) return VRO_ERR_ARG;
    if (n && (!keys_in || !keys_out || !uniforms || !activity || !moves || !weights)) return VRO_ERR_ARG;
    for (uint32_t a = 0; a < n; ++a)
        if ((keys_in[a] & 0xFFFFu) >= grid || (keys_in[a] >> 16) >= grid) {
            if (counters) counters[3] = VRO_ERR_INDEX_RANGE;
            return VRO_ERR_INDEX_RANGE;
        }
    float L[VRO_WALK_KEEP];
    uint32_t mi[VRO_WALK_KEEP];
    uint64_t inv = 0, units = 0;
    if (strategy == VRO_NAIVE) {
        for (uint32_t a = 0; a < n; ++a) {
            const uint32_t k = walk_top(keys_in[a] & 0xFFFFu, keys_in[a] >> 16, activity, grid, moves, weights,
                                        num_moves, L, mi);
            keys_out[a] = walk_choose(keys_in[a], uniforms[a], L, mi, k, moves);
        }
        inv = units = n;
    } else {
        /* per batch: each distinct cell once (first occurrence order) */
        uint32_t *slot = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)grid * grid);
        float *bL = (float *)malloc(sizeof(float) * VRO_WALK_KEEP * batch);
        uint32_t *bm = (uint32_t *)malloc(sizeof(uint32_t) * VRO_WALK_KEEP * batch);
        uint32_t *bk = (uint32_t *)malloc(sizeof(uint32_t) * batch);
        uint32_t *cell = (uint32_t *)malloc(sizeof(uint32_t) * batch);
        if (!slot || !bL || !bm || !bk || !cell) {
            free(slot); free(bL); free(bm); free(bk); free(cell);
            return VRO_ERR_ARG;
        }
        for (size_t c = 0; c < (size_t)grid * grid; ++c) slot[c] = UINT32_MAX;
        for (uint32_t a0 = 0; a0 < n; a0 += batch) {
            const uint32_t a1 = n - a0 < batch ? n : a0 + batch;
            uint32_t d = 0;
            for (uint32_t a = a0; a < a1; ++a) {
                const uint32_t c = (keys_in[a] >> 16) * grid + (keys_in[a] & 0xFFFFu);
                if (slot[c] == UINT32_MAX) {
                    slot[c] = d;
                    cell[d] = c;
                    bk[d] = walk_top(keys_in[a] & 0xFFFFu, keys_in[a] >> 16, activity, grid, moves, weights,
                                     num_moves, bL + VRO_WALK_KEEP * d, bm + VRO_WALK_KEEP * d);
                    ++d;
                }
                const uint32_t s = slot[c];
                keys_out[a] = walk_choose(keys_in[a], uniforms[a], bL + VRO_WALK_KEEP * s, bm + VRO_WALK_KEEP * s,
                                          bk[s], moves);
            }
            for (uint32_t j = 0; j < d; ++j) slot[cell[j]] = UINT32_MAX;
            inv += d;
            ++units;
        }
        free(slot); free(bL); free(bm); free(bk); free(cell);
    }
    if (counters) { counters[0] = inv; counters[1] = units; }
    return VRO_OK;
}

/* ------------------------------------------------------------------------
 * Triangle setup, the stage that consumes the geometry stage's output queue
 * (Section 4.2): each assembled triangle's clip-space corners are divided by
 * w, mapped to a width x height viewport, and the triangle gets its screen
 * bounding box (clamped to the viewport) and signed area.  It is visible when
 * every w > 0, the area is positive (counter-clockwise, front facing) and the
 * clamped box is not empty.  A triangle with a corner at w <= 0 gets an all
 * zero record.  FP32, in the order written.
 * ---------------------------------------------------------------------- */
uint64_t vro_setup(const float *corners, uint64_t T, uint32_t width, uint32_t height, float *records)
{
    const float hw = 0.5f * (float)width, hh = 0.5f * (float)height;
    uint64_t visible = 0;
    for (uint64_t t = 0; t < T; ++t) {
        float *r = records + 8 * t;
        memset(r, 0, 8 * sizeof(float));
        float sx[3], sy[3];
        int front = 1;
        for (int k = 0; k < 3; ++k) {
            const float *c = corners + 12 * (3 * t + (uint64_t)k);
            if (!(c[3] > 0.0f)) front = 0;
            sx[k] = (c[0] / c[3] + 1.0f) * hw;
            sy[k] = (c[1] / c[3] + 1.0f) * hh;
        }
        if (!front) continue;
        const float area = (sx[1] - sx[0]) * (sy[2] - sy[0]) - (sx[2] - sx[0]) * (sy[1] - sy[0]);
        float x0 = fminf(fminf(sx[0], sx[1]), sx[2]), x1 = fmaxf(fmaxf(sx[0], sx[1]), sx[2]);
        float y0 = fminf(fminf(sy[0], sy[1]), sy[2]), y1 = fmaxf(fmaxf(sy[0], sy[1]), sy[2]);
        x0 = fmaxf(x0, 0.0f);
        y0 = fmaxf(y0, 0.0f);
        x1 = fminf(x1, (float)width);
        y1 = fminf(y1, (float)height);
        const int vis = area > 0.0f && x0 < x1 && y0 < y1;
        r[0] = x0;
        r[1] = y0;
        r[2] = x1;
        r[3] = y1;
        r[4] = area;
        const uint32_t flag = vis ? 1u : 0u;
        memcpy(r + 5, &flag, 4);
        visible += (uint64_t)vis;
    }
    return visible;
}

/* Stamp set over vertex ids: membership test in O(1) without clearing. */
typedef struct {
    uint32_t *stamp;
    uint32_t *slot;
    uint32_t cur;
} stamp_set;

static int sset_init(stamp_set *s, uint32_t V)
{
    s->stamp = (uint32_t *)calloc(V ? V : 1, sizeof(uint32_t));
    s->slot = (uint32_t *)calloc(V ? V : 1, sizeof(uint32_t));
    s->cur = EMPTY_STAMP;
    return s->stamp && s->slot;
}
static void sset_free(stamp_set *s) { free(s->stamp); free(s->slot); }
static void sset_clear(stamp_set *s) { ++s->cur; }   /* 2^32 units never reached */

/*
 * Greedy cut rule of dynamic batching (Section 3.4): starting at triangle
 * `a`, keep adding whole triangles while the unit's distinct-index count
 * stays <= cap and its triangle count stays <= tmax.  The first triangle that
 * would break a limit opens the next unit.  Writes unit start offsets into
 * `starts` (which receives at most b-a entries) and returns how many.
 */
static uint64_t greedy_units(const uint32_t *idx, uint64_t a, uint64_t b, uint32_t cap,
                             uint64_t tmax, stamp_set *set, uint32_t *starts)
{
    uint64_t n = 0, cur = a;
    while (cur < b) {
        uint64_t start = cur;
        uint32_t distinct = 0;
        sset_clear(set);
        starts[n++] = (uint32_t)start;
        while (cur < b && cur - start < tmax) {
            const uint32_t *t = idx + 3 * cur;
            uint32_t fresh = 0;
            for (int c = 0; c < 3; ++c) {
                int dup_in_tri = 0;
                for (int e = 0; e < c; ++e) dup_in_tri |= (t[e] == t[c]);
                if (!dup_in_tri && set->stamp[t[c]] != set->cur) ++fresh;
            }
            if (distinct + fresh > cap) break;
            for (int c = 0; c < 3; ++c) set->stamp[t[c]] = set->cur;
            distinct += fresh;
            ++cur;
        }
    }
    return n;
}

int64_t vro_plan_dynamic(const uint32_t *idx, uint64_t T, uint32_t V, uint32_t max_unique,
                         uint32_t max_tris, uint32_t *offsets, uint64_t cap)
{
    if (max_unique < 3 || max_tris == 0) return -1;
    for (uint64_t k = 0; k < 3 * T; ++k)
        if (idx[k] >= V) return -1;
    stamp_set set;
    uint32_t *starts = (uint32_t *)malloc(sizeof(uint32_t) * (T ? T : 1));
    if (!starts || !sset_init(&set, V)) { free(starts); return -1; }
    uint64_t B = greedy_units(idx, 0, T, max_unique, max_tris, &set, starts);
    if (offsets && cap >= B + 1) {
        memcpy(offsets, starts, sizeof(uint32_t) * B);
        offsets[B] = (uint32_t)T;
    }
    sset_free(&set);
    free(starts);
    return (int64_t)B;
}

/* ------------------------------------------------------------------------
 * Normative vertex programs, FP32 (every operation written out)
 * ---------------------------------------------------------------------- */
static float dot3f(const float *a, const float *b)
{
    return fmaf(a[2], b[2], fmaf(a[1], b[1], a[0] * b[0]));
}
/* row r of a row-major matrix with 4 columns applied to (p, 1) */
static float xform_row_f(const float *M, int r, const float *p)
{
    return fmaf(M[4 * r + 2], p[2], fmaf(M[4 * r + 1], p[1], fmaf(M[4 * r + 0], p[0], M[4 * r + 3])));
}
static void normalize3f(float *x)
{
    float s = dot3f(x, x);
    float q = 1.0f / sqrtf(s);
    x[0] = x[0] * q;
    x[1] = x[1] * q;
    x[2] = x[2] * q;
}

void vro_shade(const vro_shader *sh, const float *vin, float *vout)
{
    float p[3] = {vin[0], vin[1], vin[2]};
    const float *nin = vin + 3;
    if (sh->kind == 2) {                       /* OFFSET: refine along the normal */
        const float *c = sh->coef;
        float ph = dot3f(c + 4, p);
        float h = 0.0f;
        for (uint32_t it = 0; it < sh->iterations; ++it) {
            float g = fmaf(fmaf(fmaf(c[3], h, c[2]), h, c[1]), h, ph);
            h = fmaf(c[0], g - h, h);
        }
        for (int i = 0; i < 3; ++i) p[i] = fmaf(h, nin[i], p[i]);
    }
    for (int r = 0; r < 4; ++r) vout[r] = xform_row_f(sh->mvp, r, p);
    float n[3] = {dot3f(sh->normal + 0, nin), dot3f(sh->normal + 3, nin), dot3f(sh->normal + 6, nin)};
    normalize3f(n);
    vout[4] = n[0];
    vout[5] = n[1];
    vout[6] = n[2];
    vout[7] = vin[6];
    vout[8] = vin[7];
    float col[3] = {sh->ambient[0], sh->ambient[1], sh->ambient[2]};
    if (sh->kind == 1) {                       /* PHONG with point lights */
        float w[3] = {xform_row_f(sh->model, 0, p), xform_row_f(sh->model, 1, p),
                      xform_row_f(sh->model, 2, p)};
        float vd[3] = {sh->eye[0] - w[0], sh->eye[1] - w[1], sh->eye[2] - w[2]};
        normalize3f(vd);
        for (uint32_t l = 0; l < sh->num_lights; ++l) {
            const float *L = sh->lights[l];
            float d[3] = {L[0] - w[0], L[1] - w[1], L[2] - w[2]};
            float d2 = dot3f(d, d);
            float inv = 1.0f / sqrtf(d2);
            float ld[3] = {d[0] * inv, d[1] * inv, d[2] * inv};
            float ndl = dot3f(n, ld);
            float df = ndl > 0.0f ? ndl : 0.0f;
            float two_ndl = 2.0f * ndl;
            float rr[3] = {fmaf(two_ndl, n[0], -ld[0]), fmaf(two_ndl, n[1], -ld[1]),
                           fmaf(two_ndl, n[2], -ld[2])};
            float rv = dot3f(rr, vd);
            float sp = rv > 0.0f ? rv : 0.0f;
            for (uint32_t s = 0; s < sh->spec_squarings; ++s) sp = sp * sp;
            float att = 1.0f / fmaf(sh->katt, d2, 1.0f);
            float k = att * fmaf(sh->ks, sp, sh->kd * df);
            col[0] = fmaf(k, L[3], col[0]);
            col[1] = fmaf(k, L[4], col[1]);
            col[2] = fmaf(k, L[5], col[2]);
        }
    }
    vout[9] = col[0];
    vout[10] = col[1];
    vout[11] = col[2];
}

/* Same program in float64 (inputs widened exactly). */
static double dot3d(const double *a, const double *b) { return fma(a[2], b[2], fma(a[1], b[1], a[0] * b[0])); }
static double xform_row_d(const float *M, int r, const double *p)
{
    return fma((double)M[4 * r + 2], p[2],
               fma((double)M[4 * r + 1], p[1], fma((double)M[4 * r + 0], p[0], (double)M[4 * r + 3])));
}
static void normalize3d(double *x)
{
    double q = 1.0 / sqrt(dot3d(x, x));
    x[0] *= q;
    x[1] *= q;
    x[2] *= q;
}

void vro_shade_f64(const vro_shader *sh, const float *vin, double *vout)
{
    double p[3] = {vin[0], vin[1], vin[2]};
    double nin[3] = {vin[3], vin[4], vin[5]};
    if (sh->kind == 2) {
        double c[7];
        for (int i = 0; i < 7; ++i) c[i] = sh->coef[i];
        double ph = dot3d(c + 4, p), h = 0.0;
        for (uint32_t it = 0; it < sh->iterations; ++it) {
            double g = fma(fma(fma(c[3], h, c[2]), h, c[1]), h, ph);
            h = fma(c[0], g - h, h);
        }
        for (int i = 0; i < 3; ++i) p[i] = fma(h, nin[i], p[i]);
    }
    for (int r = 0; r < 4; ++r) vout[r] = xform_row_d(sh->mvp, r, p);
    double N[9];
    for (int i = 0; i < 9; ++i) N[i] = sh->normal[i];
    double n[3] = {dot3d(N + 0, nin), dot3d(N + 3, nin), dot3d(N + 6, nin)};
    normalize3d(n);
    vout[4] = n[0];
    vout[5] = n[1];
    vout[6] = n[2];
    vout[7] = vin[6];
    vout[8] = vin[7];
    double col[3] = {sh->ambient[0], sh->ambient[1], sh->ambient[2]};
    if (sh->kind == 1) {
        double w[3] = {xform_row_d(sh->model, 0, p), xform_row_d(sh->model, 1, p),
                       xform_row_d(sh->model, 2, p)};
        double vd[3] = {sh->eye[0] - w[0], sh->eye[1] - w[1], sh->eye[2] - w[2]};
        normalize3d(vd);
        for (uint32_t l = 0; l < sh->num_lights; ++l) {
            const float *L = sh->lights[l];
            double d[3] = {L[0] - w[0], L[1] - w[1], L[2] - w[2]};
            double d2 = dot3d(d, d);
            double inv = 1.0 / sqrt(d2);
            double ld[3] = {d[0] * inv, d[1] * inv, d[2] * inv};
            double ndl = dot3d(n, ld);
            double df = ndl > 0.0 ? ndl : 0.0;
            double rr[3] = {fma(2.0 * ndl, n[0], -ld[0]), fma(2.0 * ndl, n[1], -ld[1]),
                            fma(2.0 * ndl, n[2], -ld[2])};
            double rv = dot3d(rr, vd);
            double sp = rv > 0.0 ? rv : 0.0;
            for (uint32_t s = 0; s < sh->spec_squarings; ++s) sp = sp * sp;
            double att = 1.0 / fma((double)sh->katt, d2, 1.0);
            double k = att * fma((double)sh->ks, sp, (double)sh->kd * df);
            for (int i = 0; i < 3; ++i) col[i] = fma(k, (double)L[3 + i], col[i]);
        }
    }
    vout[9] = col[0];
    vout[10] = col[1];
    vout[11] = col[2];
}

/* ------------------------------------------------------------------------
 * One draw through the geometry stage
 * ---------------------------------------------------------------------- */
static void set_counters(vro_outputs *out, uint64_t inv, uint64_t units, uint64_t uniq, uint64_t st)
{
    if (out && out->counters) {
        out->counters[0] = inv;
        out->counters[1] = units;
        out->counters[2] = uniq;
        out->counters[3] = st;
    }
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* The non-streaming reference of Section 4.2 (Table 2): a first pass
 * shades every vertex of the vertex buffer once, referenced or not, and a
 * second pass assembles each corner from the shaded buffer.  The draw is a
 * single unit whose local ids are the vertex indices themselves. */
static int multi_draw(const uint32_t *idx, uint64_t T, const float *vertices, uint32_t V,
                      const vro_shader *sh, uint64_t U, vro_outputs *out)
{
    float *shaded = (float *)malloc(sizeof(float) * VRO_OUT_FLOATS * (V ? V : 1));
    if (!shaded) { set_counters(out, 0, 0, 0, VRO_ERR_ARG); return VRO_ERR_ARG; }
    for (uint32_t v = 0; v < V; ++v)
        vro_shade(sh, vertices + (uint64_t)VRO_IN_FLOATS * v, shaded + (uint64_t)VRO_OUT_FLOATS * v);
    if (out->verts) memcpy(out->verts, shaded, sizeof(float) * VRO_OUT_FLOATS * V);
    for (uint64_t k = 0; k < 3 * T; ++k) {
        if (out->tris) out->tris[k] = idx[k];
        if (out->corners)
            memcpy(out->corners + VRO_OUT_FLOATS * k, shaded + (uint64_t)VRO_OUT_FLOATS * idx[k],
                   sizeof(float) * VRO_OUT_FLOATS);
    }
    if (out->unit_offsets) { out->unit_offsets[0] = 0; out->unit_offsets[1] = (uint32_t)T; }
    if (out->unit_invocations) out->unit_invocations[0] = V;
    free(shaded);
    set_counters(out, V, 1, U, VRO_OK);
    return VRO_OK;
}

int vro_process_draw(const uint32_t *idx, uint64_t num_indices, const float *vertices,
                     uint32_t V, const vro_shader *sh, int strategy, uint32_t batch_tris,
                     const vro_opts *opts, vro_outputs *out)
{
    uint32_t nu = 0;
    int rc = vro_check_args(num_indices, V, sh, strategy, batch_tris, opts, out, &nu);
    if (rc != VRO_OK) { set_counters(out, 0, 0, 0, (uint64_t)rc); return rc; }
    if (num_indices && (!idx || !vertices)) { set_counters(out, 0, 0, 0, VRO_ERR_ARG); return VRO_ERR_ARG; }
    const uint64_t T = num_indices / 3;
    int64_t U = vro_count_unique(idx, num_indices, V);
    if (U < 0) { set_counters(out, 0, 0, 0, VRO_ERR_INDEX_RANGE); return VRO_ERR_INDEX_RANGE; }
    if (T == 0) {
        if (out->unit_offsets) out->unit_offsets[0] = 0;
        set_counters(out, 0, 0, 0, VRO_OK);
        return VRO_OK;
    }

    if (strategy == VRO_MULTI) return multi_draw(idx, T, vertices, V, sh, (uint64_t)U, out);

    /* 1. Partition the triangles into units (whole triangles only). */
    stamp_set set;
    uint32_t *batch = (uint32_t *)malloc(sizeof(uint32_t) * (T + 1));
    uint32_t *unit = (uint32_t *)malloc(sizeof(uint32_t) * (T + 1));
    if (!batch || !unit || !sset_init(&set, V)) { free(batch); free(unit); return VRO_ERR_ARG; }
    uint64_t nb = 0;
    if (strategy == VRO_NAIVE) {
        for (uint64_t t = 0; t < T; ++t) batch[nb++] = (uint32_t)t;
    } else if (!is_dynamic(strategy)) {
        for (uint64_t t = 0; t < T; t += batch_tris) batch[nb++] = (uint32_t)t;
    } else {
        nb = greedy_units(idx, 0, T, nu, batch_tris, &set, batch);
    }
    batch[nb] = (uint32_t)T;
    uint64_t nunits = 0;
    if (is_ballot(strategy)) {                 /* rounds of <= 64 distinct */
        for (uint64_t b = 0; b < nb; ++b)
            nunits += greedy_units(idx, batch[b], batch[b + 1], VRO_WAVE, (uint64_t)-1, &set,
                                   unit + nunits);
    } else {
        memcpy(unit, batch, sizeof(uint32_t) * nb);
        nunits = nb;
    }
    unit[nunits] = (uint32_t)T;

    /* 2-5. Per unit: distinct list, local ids, shade, assemble. */
    uint64_t maxlen = 0;
    for (uint64_t u = 0; u < nunits; ++u)
        if (unit[u + 1] - unit[u] > maxlen) maxlen = unit[u + 1] - unit[u];
    uint32_t *uniq = (uint32_t *)malloc(sizeof(uint32_t) * 3 * maxlen);
    uint32_t *local = (uint32_t *)malloc(sizeof(uint32_t) * 3 * maxlen);
    float *sv = (float *)malloc(sizeof(float) * VRO_OUT_FLOATS * 3 * maxlen);
    if (!uniq || !local || !sv) { rc = VRO_ERR_ARG; goto done; }

    uint64_t vbase = 0;
    for (uint64_t u = 0; u < nunits; ++u) {
        const uint64_t t0 = unit[u], t1 = unit[u + 1];
        const uint32_t *ui = idx + 3 * t0;
        const uint64_t ncorner = 3 * (t1 - t0);
        uint32_t inv = 0;
        if (strategy == VRO_NAIVE) {
            for (uint64_t k = 0; k < ncorner; ++k) { uniq[k] = ui[k]; local[k] = (uint32_t)k; }
            inv = (uint32_t)ncorner;
        } else {
            sset_clear(&set);
            for (uint64_t k = 0; k < ncorner; ++k) {   /* first-occurrence order */
                uint32_t v = ui[k];
                if (set.stamp[v] != set.cur) {
                    set.stamp[v] = set.cur;
                    set.slot[v] = inv;
                    uniq[inv++] = v;
                }
            }
            if (strategy == VRO_STATIC_SORT || strategy == VRO_DYN_SORT) {
                qsort(uniq, inv, sizeof(uint32_t), cmp_u32);  /* ascending rank */
                for (uint32_t j = 0; j < inv; ++j) set.slot[uniq[j]] = j;
            }
            for (uint64_t k = 0; k < ncorner; ++k) local[k] = set.slot[ui[k]];
        }
        if (out->verts || out->corners)
            for (uint32_t j = 0; j < inv; ++j)
                vro_shade(sh, vertices + (uint64_t)VRO_IN_FLOATS * uniq[j], sv + (uint64_t)VRO_OUT_FLOATS * j);
        if (out->verts)
            memcpy(out->verts + VRO_OUT_FLOATS * vbase, sv, sizeof(float) * VRO_OUT_FLOATS * inv);
        for (uint64_t k = 0; k < ncorner; ++k) {
            const uint64_t g = 3 * t0 + k;
            if (out->tris) out->tris[g] = (uint32_t)(vbase + local[k]);
            if (out->local_idx) out->local_idx[g] = (uint16_t)local[k];
            if (out->corners)
                memcpy(out->corners + VRO_OUT_FLOATS * g, sv + (uint64_t)VRO_OUT_FLOATS * local[k],
                       sizeof(float) * VRO_OUT_FLOATS);
        }
        if (out->unit_offsets) out->unit_offsets[u] = (uint32_t)t0;
        if (out->unit_invocations) out->unit_invocations[u] = inv;
        vbase += inv;
    }
    if (out->unit_offsets) out->unit_offsets[nunits] = (uint32_t)T;
    set_counters(out, vbase, nunits, (uint64_t)U, VRO_OK);
    rc = VRO_OK;
done:
    free(uniq);
    free(local);
    free(sv);
    free(batch);
    free(unit);
    sset_free(&set);
    return rc;
}
