/*
 * vro.h -- CPU oracle for on-the-fly vertex reuse (Kenzel et al., "On-the-fly
 * Vertex Reuse for Massively-Parallel Software Geometry Processing").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the GPU library; the two agree only through the
 * written specification of the geometry stage.
 *
 * Everything here is plain, sequential and host-side: batches are formed by
 * walking the triangle list front to back, each unit's distinct indices are
 * found with a stamp array, and every unique vertex is shaded with the
 * normative FP32 vertex programs.  Function-level comments cite the paper
 * section, algorithm or table each step follows.
 *
 * Parity pins: every function has at least one test that checks it against
 * something other than itself (closed forms, special cases, brute force or
 * a float64 evaluation).  None is "parity unpinned".
 */
#ifndef VRO_H
#define VRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VRO_OK = 0,
    VRO_ERR_ARG = 1,          /* bad argument, nothing written            */
    VRO_ERR_INDEX_RANGE = 2,  /* an index >= num_vertices                 */
    VRO_ERR_CAPACITY = 3      /* an output capacity is too small          */
};

enum {
    VRO_NAIVE = 0,            /* no reuse: 3 invocations per triangle      */
    VRO_STATIC_BALLOT = 1,    /* static batches, rounds of <= 64 distinct  */
    VRO_STATIC_SORT = 2,      /* static batches, ascending-rank local ids  */
    VRO_STATIC_HASH = 3,      /* static batches, first-occurrence ids      */
    VRO_DYN_SORT = 4,         /* dynamic batches, ascending-rank ids       */
    VRO_DYN_HASH = 5,         /* dynamic batches, first-occurrence ids     */
    VRO_DYN_PHASH = 6,        /* dynamic batches, first-occurrence ids     */
    VRO_DYN_BALLOT = 7,       /* dynamic batches split into ballot rounds  */
    VRO_MULTI = 8             /* two passes: shade all V, then assemble    */
};

#define VRO_WAVE 64           /* distinct-index capacity of a ballot round */
#define VRO_MAX_LIGHTS 16
#define VRO_OUT_FLOATS 12     /* clip xyzw, normal xyz, uv, rgb            */
#define VRO_IN_FLOATS 8       /* pos xyz, normal xyz, uv                   */

typedef struct {
    uint32_t max_unique;      /* N_u for dynamic batching; 0 = default     */
    uint32_t wg_size;         /* GPU launch shape only: ignored here       */
    uint32_t hash_slots;      /* GPU launch shape only: ignored here       */
    uint32_t hash_probes;     /* GPU launch shape only: ignored here       */
} vro_opts;

typedef struct {
    uint32_t kind;            /* 0 MVP, 1 PHONG, 2 OFFSET                  */
    uint32_t num_lights;      /* PHONG: 0..16                              */
    uint32_t iterations;      /* OFFSET: refinement steps                  */
    uint32_t spec_squarings;  /* PHONG: specular exponent 2^s              */
    float mvp[16];            /* row-major 4x4                             */
    float model[12];          /* row-major 3x4                             */
    float normal[9];          /* row-major 3x3                             */
    float eye[3];
    float ambient[3];
    float kd, ks, katt;
    float coef[8];            /* OFFSET: c0 c1 c2 c3 cvec.xyz (unused)     */
    float lights[VRO_MAX_LIGHTS][6]; /* position xyz, colour rgb           */
} vro_shader;

typedef struct {
    float *corners;           /* [3T][12] or NULL                          */
    uint32_t *tris;           /* [3T] indices into verts, or NULL          */
    float *verts;             /* [verts_cap][12] or NULL                   */
    uint64_t verts_cap;       /* >= 3T (MULTI: >= V) when verts != NULL    */
    uint16_t *local_idx;      /* [3T] unit-local ids, or NULL              */
    uint32_t *unit_offsets;   /* [units_cap + 1] triangle offsets, or NULL */
    uint32_t *unit_invocations; /* [units_cap] or NULL                     */
    uint64_t units_cap;       /* >= vro_units_bound(...) when unit arrays  */
    uint64_t *counters;       /* [4]: invocations, units, unique, status   */
} vro_outputs;

/* Upper bound on the number of units a strategy can produce. */
uint64_t vro_units_bound(int strategy, uint64_t num_tris, uint32_t batch_tris);

/* Argument check shared by every entry point; returns VRO_OK or
 * VRO_ERR_ARG / VRO_ERR_CAPACITY and writes nothing. */
int vro_check_args(uint64_t num_indices, uint32_t num_vertices, const vro_shader *sh,
                   int strategy, uint32_t batch_tris, const vro_opts *opts,
                   const vro_outputs *out, uint32_t *resolved_max_unique);

/* Dynamic batching (Section 3.4): greedy front-to-back cuts.  Writes B+1
 * triangle offsets (offsets[0] = 0, offsets[B] = T) when offsets != NULL and
 * cap >= B+1; returns B, or -1 on an out-of-range index or bad argument. */
int64_t vro_plan_dynamic(const uint32_t *indices, uint64_t num_tris, uint32_t num_vertices,
                         uint32_t max_unique, uint32_t max_tris, uint32_t *offsets,
                         uint64_t cap);

/* The full geometry stage for one draw, synchronous, host pointers. */
int vro_process_draw(const uint32_t *indices, uint64_t num_indices, const float *vertices,
                     uint32_t num_vertices, const vro_shader *shader, int strategy,
                     uint32_t batch_tris, const vro_opts *opts, vro_outputs *out);

/* One vertex through the normative FP32 vertex program. */
void vro_shade(const vro_shader *sh, const float *vin, float *vout);
/* The same program evaluated in float64 (used to bound FP32 rounding). */
void vro_shade_f64(const vro_shader *sh, const float *vin, double *vout);

/* Distinct indices referenced by the buffer (-1 on an out-of-range index). */
int64_t vro_count_unique(const uint32_t *indices, uint64_t n, uint32_t num_vertices);

/* Misses of a k-entry FIFO post-transform cache over the index stream
 * (Section 2): a hit does not reorder, a miss inserts and evicts the oldest. */
int64_t vro_fifo_misses(const uint32_t *indices, uint64_t n, uint32_t num_vertices, uint32_t k);

/* Section 4.1, Table 1: hits of `procs` parallel per-processor LRU caches of
 * `entries` shaded vertices each; chunks of `per_cycle` indices go to the
 * processors in consecutive runs (contiguous != 0) or round robin; lookups
 * see the cache as it stood after the processor's previous cycle (no hit
 * among concurrently shaded duplicates).  -1 on a bad index. */
/* Section 5, parallel random walk: one step of n agents on a grid x grid
 * domain.  keys are packed cells x | y << 16; activity is float32[grid *
 * grid] (cell (x, y) at y * grid + x); moves are int8 (dx, dy) pairs with
 * float32 weights; uniforms are the agents' random numbers in [0, 1).  A
 * cell's options are its 8 most likely moves (activity of the target times
 * the move's weight, moves leaving the grid skipped, ties to the lower move
 * index); an agent takes the first option whose running FP32 sum exceeds
 * u * (sum of the options), and stays when they sum to zero.  NAIVE
 * evaluates every agent's cell; STATIC_SORT / STATIC_HASH evaluate each
 * distinct cell of a batch of `batch` agents (<= 512) once.  counters =
 * {cell evaluations, units, 0, status}. */
/* The pieces of a step, for the tests: a cell's options (count returned,
 * likelihoods and move indices in order) and one agent's choice. */
uint32_t vro_walk_options(uint32_t x, uint32_t y, const float *activity, uint32_t grid, const int8_t *moves,
                          const float *weights, uint32_t num_moves, float *L, uint32_t *move_index);
uint32_t vro_walk_choose(uint32_t key, float u, const float *L, const uint32_t *move_index, uint32_t k,
                         const int8_t *moves);
int vro_walk_step(const uint32_t *keys_in, uint32_t n, const float *activity, uint32_t grid, const int8_t *moves,
                  const float *weights, uint32_t num_moves, const float *uniforms, int strategy, uint32_t batch,
                  uint32_t *keys_out, uint64_t *counters);

/* Triangle setup of T assembled triangles (corners as written by a draw):
 * records float[T][8] = {xmin, ymin, xmax, ymax, area, flags (uint32: 1 =
 * visible), 0, 0}; returns the number of visible triangles. */
uint64_t vro_setup(const float *corners, uint64_t T, uint32_t width, uint32_t height, float *records);

int64_t vro_parallel_cache_hits(const uint32_t *indices, uint64_t n, uint32_t num_vertices, uint32_t procs,
                                uint32_t per_cycle, uint32_t entries, int contiguous);

#ifdef __cplusplus
}
#endif
#endif
