/*
 * vr.h -- C ABI of the MI355X geometry stage with on-the-fly vertex reuse
 * (Kenzel, Kerbl, Tatzgern, Ivanchenko, Schmalstieg, Steinberger, "On-the-fly
 * Vertex Reuse for Massively-Parallel Software Geometry Processing").
 *
 * Problem statement (Section 4.2, "Rasterization"): the geometry stage gets
 * a stream of indices and a vertex buffer, groups the triangles into batches,
 * shades each vertex a batch references once, and writes every triangle with
 * its shaded vertices to an output queue.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are device pointers (HBM), caller-owned, and must
 *    stay valid until the work enqueued on the context's stream completes.
 *    Host structs (shader parameters, options, output descriptors) are copied
 *    during the call.
 *  - Work is enqueued on the context's HIP stream and the call returns
 *    without waiting.  vr_sync() waits and reports device-side errors.
 *  - Errors are returned as vr_status; nothing aborts or throws across the
 *    ABI.  Argument errors are detected on the host before anything is
 *    enqueued and leave every output untouched.  vr_last_error() returns a
 *    text for the last failing call on a context.
 *  - A context is used by one host thread at a time.
 *
 * Data layout (all little-endian, tightly packed):
 *  - indices:  uint32[3T], a triangle list; triangle t uses entries 3t..3t+2
 *              (Section 3).  Every index must be < num_vertices.
 *  - vertices: float32[V][8] = {px, py, pz, nx, ny, nz, u, v}; 32-byte rows,
 *              the buffer 16-byte aligned.
 *  - a shaded vertex: float32[12] = {clip x, y, z, w, n'x, n'y, n'z, u, v,
 *              r, g, b}, 48 bytes.
 */
#ifndef VR_H
#define VR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vr_ctx vr_ctx;

typedef enum {
    VR_OK = 0,
    VR_ERR_ARG = 1,          /* invalid argument; nothing was enqueued          */
    VR_ERR_INDEX_RANGE = 2,  /* (from vr_sync) an index >= num_vertices; the
                                outputs of the affected draws are undefined    */
    VR_ERR_CAPACITY = 3,     /* an output capacity is below the documented bound */
    VR_ERR_OOM = 4,          /* device memory for the context's scratch failed  */
    VR_ERR_DEVICE = 5,       /* a HIP call failed, or a device-side wait ran out */
    VR_ERR_BUSY = 6,         /* the object is in a state that forbids the call   */
    VR_CANCELLED = 7         /* (server) the request was cancelled before launch */
} vr_status;

/*
 * Reuse strategies (Section 3).  A "unit" is the set of triangles that share
 * one deduplication: a static batch, a dynamic batch, or a ballot round.
 *  NAIVE          one unit per triangle; every corner is shaded (Section 3.3,
 *                 "Statically batched naive").
 *  STATIC_BALLOT  batches of batch_tris triangles (Section 3.3); each batch
 *                 is cut into rounds, the longest runs of whole triangles with
 *                 at most 64 distinct indices (Algorithm 1 on a 64-lane
 *                 wavefront); ids in first-occurrence order.
 *  STATIC_SORT    static batches; local id = ascending rank among the batch's
 *                 distinct indices (Algorithm 2 applied to a static batch).
 *  STATIC_HASH    static batches; ids in first-occurrence order (Algorithm 3
 *                 applied to a static batch).
 *  DYN_SORT       dynamic batches (Section 3.4): the longest runs of whole
 *                 triangles with at most max_unique distinct indices and at
 *                 most batch_tris triangles; ascending-rank ids (Algorithm 2).
 *  DYN_HASH       dynamic batches, LDS hash table (Algorithm 3), ids in
 *                 first-occurrence order.
 *  DYN_PHASH      dynamic batches, bounded per-lane probing then
 *                 wavefront-cooperative probing (Section 3.4, "parallel
 *                 hashing"); ids in first-occurrence order.
 *  DYN_BALLOT     dynamic batches cut into ballot rounds as STATIC_BALLOT.
 *  MULTI          the non-streaming two-pass reference of Section 4.2
 *                 (Table 2): one kernel shades every vertex of the buffer
 *                 once, referenced or not (invocations = num_vertices), a
 *                 second gathers the corners from the shaded buffer.  One
 *                 unit spans the draw; its local ids are the vertex indices,
 *                 so tris = indices and verts holds all num_vertices shaded
 *                 vertices in buffer order.  batch_tris is ignored (>= 1);
 *                 local_idx is not available (VR_ERR_ARG); not accepted in
 *                 frames or by the server.
 * Hash-table slot numbers depend on atomic races; exported ids never do.
 */
typedef enum {
    VR_NAIVE = 0,
    VR_STATIC_BALLOT = 1,
    VR_STATIC_SORT = 2,
    VR_STATIC_HASH = 3,
    VR_DYN_SORT = 4,
    VR_DYN_HASH = 5,
    VR_DYN_PHASH = 6,
    VR_DYN_BALLOT = 7,
    VR_MULTI = 8
} vr_strategy;

/* Limits on batch_tris per strategy (argument error beyond them).  A DYN_*
 * sort, hash or parallel-hash draw must also fit one workgroup: at most
 * 1024 threads (a unit of at most 8 indices per thread for the sort, 32 for
 * the hashes) and the device's LDS per workgroup (160 KB on gfx950), which
 * holds 48 bytes per unique vertex when corners are requested and an
 * NT-row stage otherwise; vr_process_draw returns VR_ERR_ARG before any
 * launch for a configuration that does not fit. */
#define VR_MAX_BATCH_STATIC 256        /* STATIC_SORT, STATIC_HASH            */
#define VR_MAX_BATCH_BALLOT 1024       /* STATIC_BALLOT                       */
#define VR_MAX_BATCH_DYNAMIC 4096      /* DYN_* (the triangle cap N_pmax)     */
#define VR_MAX_UNIQUE 4096             /* DYN_* unique budget N_u             */
#define VR_MAX_HASH_SLOTS 8192         /* opts.hash_slots                     */
#define VR_MAX_INDICES 3221225469ull   /* num_indices < 3 * 2^30              */
#define VR_MAX_LIGHTS 16

typedef struct {
    uint32_t max_unique;   /* N_u for DYN_*: 0 = 64*ceil(batch_tris/64) capped
                              at 4096, else 3..4096.  Ignored by static modes. */
    uint32_t wg_size;      /* 0 = automatic, else a multiple of 64 <= 1024;
                              changes launch shape only, never results.        */
    uint32_t hash_slots;   /* 0 = automatic, else a power of two >= the unit's
                              distinct bound (N_u, or 3*batch_tris) and <= 8192;
                              never changes results.                            */
    uint32_t hash_probes;  /* DYN_PHASH per-lane probes before the cooperative
                              path: 0 = 4, else <= 64; never changes results.   */
    const uint32_t *d_plan; /* DYN_*: a plan written by vr_plan_dynamic() with
                              the same indices, max_unique and batch_tris, or
                              NULL to build one on the context's stream.       */
} vr_opts;

typedef struct {
    uint32_t kind;            /* 0 MVP, 1 PHONG, 2 OFFSET                       */
    uint32_t num_lights;      /* PHONG: 0..16                                   */
    uint32_t iterations;      /* OFFSET: refinement steps, <= 4096              */
    uint32_t spec_squarings;  /* PHONG: specular exponent 2^s, s <= 8           */
    float mvp[16];            /* row-major 4x4 applied to (p, 1)                */
    float model[12];          /* row-major 3x4: world position for lighting     */
    float normal[9];          /* row-major 3x3 normal matrix                    */
    float eye[3];
    float ambient[3];
    float kd, ks, katt;       /* diffuse, specular, distance attenuation        */
    float coef[8];            /* OFFSET: c0 c1 c2 c3 cvec.xyz, [7] unused       */
    float lights[VR_MAX_LIGHTS][6]; /* position xyz, colour rgb                 */
} vr_shader_params;

/*
 * Outputs of one draw (device pointers; any may be NULL).
 *  corners           float[3T][12]: corner k of triangle t at row 3t+k, the
 *                    shaded vertex of indices[3t+k] (the assembled triangle).
 *  tris              uint32[3T]: tris[3t+k] = vbase(unit) + local id, an index
 *                    into verts.
 *  verts             float[verts_cap][12]: unit u's shaded vertices at rows
 *                    vbase(u) .. vbase(u)+inv(u)-1, vbase = sum of earlier
 *                    units' invocations.  verts_cap >= 3T (MULTI: >= num_vertices)
 *                    when verts != NULL.
 *  local_idx         uint16[3T]: the unit-local id of every corner.
 *  unit_offsets      uint32[units_cap+1]: first triangle of every unit, then T.
 *  unit_invocations  uint32[units_cap]: vertex-shader invocations per unit.
 *                    units_cap >= T, or >= ceil(T/batch_tris) for
 *                    STATIC_SORT / STATIC_HASH, or >= 1 for MULTI, when
 *                    either unit array is set.
 *  counters          uint64[4]: {invocations, units, 0, 0}, overwritten.
 */
typedef struct {
    float *corners;
    uint32_t *tris;
    float *verts;
    uint64_t verts_cap;
    uint16_t *local_idx;
    uint32_t *unit_offsets;
    uint32_t *unit_invocations;
    uint64_t units_cap;
    uint64_t *counters;
} vr_outputs;

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Scratch memory is allocated on
 * first use, grows as needed and is released by vr_destroy(). */
vr_status vr_create(vr_ctx **ctx, int device, void *hip_stream);
void vr_destroy(vr_ctx *ctx);
/* Re-target the context to another stream of the same device. */
vr_status vr_set_stream(vr_ctx *ctx, void *hip_stream);

/* Host-only argument check used by every draw entry point: returns VR_OK,
 * VR_ERR_ARG or VR_ERR_CAPACITY and touches no device. */
vr_status vr_check_args(uint64_t num_indices, uint32_t num_vertices,
                        const vr_shader_params *shader, vr_strategy strategy,
                        uint32_t batch_tris, const vr_opts *opts, const vr_outputs *out);

/*
 * Dynamic batching (Section 3.4): scan the triangles front to back and close
 * a batch when adding the next triangle would exceed max_unique distinct
 * indices or max_tris triangles.  Runs on the device.  Writes into d_plan
 * (uint32[T+2], caller-owned): d_plan[0] = B, d_plan[1..B+1] = the batch
 * start triangles followed by T.  plan_cap is the length of d_plan in
 * elements and must be >= T+2.  max_unique in 3..4096, max_tris in 1..4096.
 */
vr_status vr_plan_dynamic(vr_ctx *ctx, const uint32_t *d_indices, uint64_t num_indices,
                          uint32_t num_vertices, uint32_t max_unique, uint32_t max_tris,
                          uint32_t *d_plan, uint64_t plan_cap);

/*
 * One draw: batch, deduplicate, shade each unit-unique vertex once with the
 * vertex program in `shader`, and assemble the outputs described above
 * (Algorithms 1-3, Section 4.2).  batch_tris is N_p for static strategies
 * and the triangle cap for dynamic ones; NAIVE accepts any value >= 1.
 * num_indices == 0 is valid and writes zero counters.  An out-of-range index
 * is reported by the next vr_sync() as VR_ERR_INDEX_RANGE.
 */
vr_status vr_process_draw(vr_ctx *ctx, const uint32_t *d_indices, uint64_t num_indices,
                          const float *d_vertices, uint32_t num_vertices,
                          const vr_shader_params *shader, vr_strategy strategy,
                          uint32_t batch_tris, const vr_opts *opts, const vr_outputs *out);

/*
 * Allocation-free draw, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, and harnesses that
 * forbid hipMalloc.  Same arguments, outputs, semantics and errors as
 * vr_process_draw, except:
 *  - the per-batch aggregates and look-back words live in one static
 *    device array of the library, 16 bytes per batch for at most
 *    VR_NOALLOC_MAX_BATCHES batches (8 MiB), which every GPU the library
 *    runs on holds until the process ends (its address is looked up once
 *    per device by vr_create);
 *  - a draw whose batch bound exceeds VR_NOALLOC_MAX_BATCHES is rejected
 *    with VR_ERR_CAPACITY before anything is enqueued (the bound is
 *    ceil(T / batch_tris) for static strategies and
 *    T / min(batch_tris, ceil((N_u - 2) / 3)) + 1 for dynamic ones; NAIVE
 *    uses no batch scratch);
 *  - DYN_* need opts->d_plan (built beforehand by vr_plan_dynamic) and
 *    MULTI needs out->verts (its shaded buffer): VR_ERR_ARG otherwise;
 *  - kernel timing (vr_set_kernel_timing) records nothing for it.
 * The call performs no hipMalloc, hipFree or other allocation.  Every call
 * on a GPU shares that GPU's array and the array keeps the last call's
 * contents (the look-back words are zero again after every draw): calls
 * that overlap on one GPU, from any contexts or streams, race and must be
 * ordered by the caller.  VR_ERR_DEVICE if the array could not be set up.
 */
#define VR_NOALLOC_MAX_BATCHES 524288u
vr_status vr_process_draw_noalloc(vr_ctx *ctx, const uint32_t *d_indices, uint64_t num_indices,
                                  const float *d_vertices, uint32_t num_vertices,
                                  const vr_shader_params *shader, vr_strategy strategy,
                                  uint32_t batch_tris, const vr_opts *opts, const vr_outputs *out);

/*
 * Streaming (Sections 4.2 and 5): index chunks are drawn as they arrive with
 * strategies that need no analysis of the index buffer (NAIVE, STATIC_*),
 * each into one of `slots` corner buffers of chunk_tris triangles (owned by
 * the stream), and a consumer on a second HIP stream runs triangle setup on
 * every finished buffer: the clip-space corners are divided by w and mapped
 * to a width x height viewport; each triangle gets its bounding box clamped
 * to the viewport and its signed area, and is visible when every w > 0, the
 * area is positive (counter-clockwise) and the box is not empty (a corner at
 * w <= 0 gives an all-zero record).  Records land in d_records (caller-owned,
 * float[records_cap][8] = {xmin, ymin, xmax, ymax, area, flags, 0, 0}, flags
 * a uint32 with bit 0 = visible) at the triangle's position in the stream.
 * A buffer is drawn into again only after the consumer has finished it
 * (events), so memory stays bounded for any stream length.  Static batches
 * restart at every chunk.  A stream belongs to its context and must be
 * destroyed before it; push is not thread safe.  Errors: VR_ERR_ARG (slots outside 1..8,
 * chunk_tris outside 1..2^24, a dynamic strategy, a chunk above chunk_tris),
 * VR_ERR_CAPACITY (records_cap exceeded), draw errors as vr_process_draw.
 */
typedef struct vr_stream vr_stream;
vr_status vr_stream_create(vr_ctx *ctx, uint32_t slots, uint32_t chunk_tris, uint32_t width, uint32_t height,
                           float *d_records, uint64_t records_cap, vr_stream **stream);
vr_status vr_stream_push(vr_stream *stream, const uint32_t *d_indices, uint64_t num_indices, const float *d_vertices,
                         uint32_t num_vertices, const vr_shader_params *shader, vr_strategy strategy,
                         uint32_t batch_tris);
/* Waits for both stages; totals since creation: triangles pushed, visible
 * triangles, vertex-shader invocations. */
vr_status vr_stream_finish(vr_stream *stream, uint64_t *h_triangles, uint64_t *h_visible, uint64_t *h_invocations);
void vr_stream_destroy(vr_stream *stream);

/*
 * Parallel random walk (Section 5): one step of num_agents agents on a
 * grid x grid domain, reusing the per-cell move search among agents on the
 * same cell.  d_keys_in / d_keys_out: uint32[num_agents] packed cells
 * x | y << 16 (may be the same buffer); d_activity: float32[grid * grid],
 * cell (x, y) at y * grid + x; d_moves: int8[2 * num_moves] (dx, dy);
 * d_weights: float32[num_moves]; d_uniforms: float32[num_agents] in [0, 1).
 * A cell's options are its 8 most likely moves (likelihood = activity of the
 * target times the move's weight in FP32, moves leaving the grid skipped,
 * ties to the lower move index); an agent takes the first option whose
 * running FP32 sum exceeds u * (sum of the options) and stays when they sum
 * to zero.  NAIVE searches every agent's cell; STATIC_HASH searches each
 * distinct cell of every batch of batch_agents (1..512) agents once.
 * d_counters: uint64[4] {cell searches, units, 0, 0} or NULL.  A key outside
 * the grid leaves its agent in place and is reported by the next vr_sync()
 * as VR_ERR_INDEX_RANGE.  grid <= 32768, num_moves <= 65535.
 */
vr_status vr_walk_step(vr_ctx *ctx, const uint32_t *d_keys_in, uint32_t num_agents, const float *d_activity,
                       uint32_t grid, const int8_t *d_moves, const float *d_weights, uint32_t num_moves,
                       const float *d_uniforms, vr_strategy strategy, uint32_t batch_agents, uint32_t *d_keys_out,
                       uint64_t *d_counters);

/* Wait for the context's stream.  Returns the first device-side error raised
 * since the previous vr_sync (then clears it) and, when h_invocations is not
 * NULL, the vertex-shader invocations of all draws since then. */
vr_status vr_sync(vr_ctx *ctx, uint64_t *h_invocations);

/*
 * Frames: many draws in one persistent launch (the streaming geometry stage
 * of Section 4.2 applied to a list of draws of uneven size).  Each draw is
 * processed exactly as vr_process_draw would process it with only `corners`
 * and `counters` requested, so every draw keeps its own batches, ids and
 * invocation counts.  Dynamic draws need their plan (vr_plan_dynamic with the
 * same indices, max_unique and batch_tris) in d_plan, or the plan of any
 * longer index buffer that starts with this draw's indices: greedy batching
 * never looks past the end of the batch it closes, so the plan of a prefix
 * of the stream is the longer plan cut at the prefix's end (the last batch
 * shortened to end there).
 */
typedef struct vr_frame vr_frame;

typedef struct {
    const uint32_t *d_indices;   /* uint32[num_indices]                            */
    uint64_t num_indices;
    const float *d_vertices;     /* float32[num_vertices][8], 16-byte aligned      */
    uint32_t num_vertices;
    uint32_t shader;             /* index into the frame's shader table            */
    vr_strategy strategy;
    uint32_t batch_tris;         /* as for vr_process_draw                         */
    uint32_t max_unique;         /* DYN_*: N_u, 0 = default                        */
    const uint32_t *d_plan;      /* DYN_*: required; ignored otherwise             */
    float *d_corners;            /* float32[3T][12], required, 16-byte aligned     */
    uint64_t *d_counters;        /* uint64[4] {invocations, units, 0, 0} or NULL   */
} vr_draw;

#define VR_MAX_FRAME_DRAWS 4096

/* Validate and upload a frame (draw and shader tables are copied to device
 * memory owned by the frame; the device buffers named in the draws must stay
 * valid while the frame exists).  With capture_graph != 0 the frame's
 * launches are captured once into a hipGraph that vr_frame_run replays.
 * Returns VR_ERR_ARG for more than VR_MAX_FRAME_DRAWS draws, a shader index
 * out of range, a dynamic draw without a plan, a sort draw of more than 682
 * or a hash draw of more than 2730 triangles per batch (the frame kernel runs
 * 256 threads per unit), or any per-draw argument error (vr_last_error names
 * the draw). */
vr_status vr_frame_create(vr_ctx *ctx, const vr_draw *draws, uint32_t num_draws, const vr_shader_params *shaders,
                          uint32_t num_shaders, int capture_graph, vr_frame **frame);
/* Enqueue the frame on its context's stream (a graph launch when captured). */
vr_status vr_frame_run(vr_frame *frame);
/* Wait for the context's stream and release the frame. */
void vr_frame_destroy(vr_frame *frame);
/* One-shot frame: create, run, wait and destroy (synchronous). */
vr_status vr_process_draws(vr_ctx *ctx, const vr_draw *draws, uint32_t num_draws, const vr_shader_params *shaders,
                           uint32_t num_shaders);

/*
 * Autotuning support: time candidate configurations on a sample draw (the
 * paper picks its batch sizes by such a search, Sections 4.2 and 5).  For
 * every candidate the draw is processed with per-corner output into context
 * scratch: the plan is built (timed as plan_ms) for dynamic strategies, one
 * untimed warm-up, then `reps` timed draws (kernel_ms = the fastest of them,
 * main kernel only: the repetition least disturbed by other device work).  Invalid candidates get kernel_ms = -1.  *best receives the index
 * of the fastest valid candidate by kernel_ms.  Synchronous; allocates
 * scratch as needed.
 */
typedef struct {
    vr_strategy strategy;
    uint32_t batch_tris;
    uint32_t max_unique;      /* DYN_*: 0 = default                            */
    uint32_t wg_size;         /* 0 = automatic                                 */
    float kernel_ms;          /* out                                           */
    float plan_ms;            /* out: dynamic strategies, else 0               */
    uint64_t invocations;     /* out                                           */
} vr_tune_candidate;

vr_status vr_autotune(vr_ctx *ctx, const uint32_t *d_indices, uint64_t num_indices, const float *d_vertices,
                      uint32_t num_vertices, const vr_shader_params *shader, vr_tune_candidate *cands,
                      uint32_t num_cands, uint32_t reps, uint32_t *best);

/*
 * Kernel timing (a measurement aid, off by default).  While enabled, every
 * vr_process_draw records a pair of HIP events on the context's stream
 * around its main kernel, every vr_plan_dynamic around its kernels and every
 * vr_frame_run around the whole frame.
 * vr_kernel_times waits for the stream and returns the elapsed milliseconds
 * of the launches recorded since its previous call, in submission order
 * (at most `cap`; *count receives how many were recorded, which may exceed
 * cap), then forgets them.
 */
vr_status vr_set_kernel_timing(vr_ctx *ctx, int enable);
vr_status vr_kernel_times(vr_ctx *ctx, float *ms, uint32_t cap, uint32_t *count);

/*
 * Self-test of the vertex programs' rounded arithmetic.  The programs need
 * correctly rounded division and square root (IEEE-754 round to nearest
 * even); the library computes them with short sequences on the operands
 * whose intermediates stay normal and with the compiler's full IEEE
 * sequences on the rest.  This call evaluates the library's version of
 * `fn` (0 = 1/x, 1 = sqrt(x), 2 = 1/sqrt(x) with both operations rounded)
 * on the float32 operands whose bit patterns are first .. first + count - 1
 * and compares each result bit for bit with the compiler's IEEE sequence.
 * *h_mismatches (host) receives the number of operands that differ; d_out
 * (device, `count` floats, or NULL) receives the results.  The full range
 * (first 0, count 2^32) takes a few milliseconds.  Runs on the context's
 * stream and waits for it.
 * Errors: VR_ERR_ARG (NULL ctx or h_mismatches, fn > 2, first + count >
 * 2^32), VR_ERR_OOM, VR_ERR_DEVICE.
 */
vr_status vr_math_selftest(vr_ctx *ctx, uint32_t fn, uint64_t first, uint64_t count, float *d_out,
                           uint64_t *h_mismatches);

/*
 * Request server: continuous batching of draw requests against meshes that
 * stay resident in device memory (the geometry stage of Section 4.2 fed by
 * a stream of requests instead of one draw call).
 *
 * A server owns its own HIP stream, a device arena of `budget_bytes` for
 * request outputs, and a scheduler thread.  vr_server_submit queues a
 * request and returns at once.  The scheduler admits requests in submission
 * order while their outputs (3T shaded corners, 144 bytes per triangle) fit
 * in the arena, and launches "ticks": one frame launch over the admitted
 * requests, at most max_tick_draws requests and max_tick_tris triangles,
 * with at most max_inflight ticks queued on the device.  Requests that
 * arrive while ticks run join the next tick.  Each request is processed
 * exactly as vr_process_draw would process its draw (bit-identical corners
 * and counts, alone or in any mix).  A finished request keeps its memory
 * until vr_server_release.  With max_tick_draws = 1 every request gets its
 * own launch (the per-draw baseline).
 *
 * Threading: submit, poll, release, cancel and stats may be called from any
 * host thread; destroy from one thread after all others have stopped using
 * the server.
 */
typedef struct vr_server vr_server;

typedef struct {
    uint64_t budget_bytes;    /* arena for request outputs, allocated at create */
    uint32_t max_inflight;    /* ticks queued on the device at once, 1..8; 0 -> 2 */
    uint32_t max_tick_draws;  /* requests per tick, 1..VR_MAX_FRAME_DRAWS; 0 -> 1024 */
    uint64_t max_tick_tris;   /* triangles per tick; 0 = no limit (a tick always
                                 takes at least one request)                    */
} vr_server_config;

typedef struct {
    uint32_t mesh;            /* from vr_server_add_mesh                        */
    uint32_t num_tris;        /* the first num_tris triangles of the mesh       */
    vr_strategy strategy;
    uint32_t batch_tris;      /* as for vr_process_draw                         */
    uint32_t max_unique;      /* DYN_*: N_u, 0 = default                        */
    uint32_t pad;
    uint64_t user;            /* opaque, returned in the completion             */
    vr_shader_params shader;  /* copied at submit                               */
} vr_request;

typedef struct {
    uint64_t ticket, user;
    int32_t status;           /* VR_OK, VR_CANCELLED, or the device error of its tick */
    uint32_t tick;            /* tick that processed it                         */
    uint64_t num_tris, invocations, units;
    const float *d_corners;   /* float32[3 num_tris][12] in the arena; valid until
                                 vr_server_release                              */
    double t_submit, t_admit, t_launch, t_done;   /* seconds since create; t_done
                                 is when the scheduler saw the tick finish     */
} vr_completion;

typedef struct {
    uint64_t submitted, completed, cancelled, rejected, ticks;
    uint64_t budget_bytes, reserved_bytes, peak_reserved_bytes;
    uint64_t pending, admitted, inflight_ticks;
    uint64_t max_pending, max_tick_draws, admission_blocked;
    uint64_t plan_bytes;      /* cached dynamic plans (outside the budget)      */
} vr_server_stats;

/* Allocates the arena and starts the scheduler on `device`.  VR_ERR_ARG for
 * out-of-range settings, VR_ERR_OOM if the arena cannot be allocated. */
vr_status vr_server_create(int device, const vr_server_config *cfg, vr_server **server);
/* Registers a resident mesh (caller-owned buffers that must outlive the
 * server).  Synchronous: checks on the device that every index is below
 * num_vertices (VR_ERR_INDEX_RANGE otherwise), so requests cannot fault.
 * Dynamic plans of the whole mesh are built on first use for each
 * (max_unique, batch_tris) and cached; a request on a prefix uses the cached
 * plan cut at its end. */
vr_status vr_server_add_mesh(vr_server *server, const uint32_t *d_indices, uint64_t num_indices,
                             const float *d_vertices, uint32_t num_vertices, uint32_t *mesh);
/* Queues a request.  VR_ERR_ARG for an unknown mesh, num_tris beyond the
 * mesh, or any argument vr_process_draw would reject; VR_ERR_CAPACITY when
 * its output can never fit in the budget; VR_ERR_BUSY after destroy began. */
vr_status vr_server_submit(vr_server *server, const vr_request *request, uint64_t *ticket);
/* Queues requests[0..n) in order under one acquisition of the server's lock,
 * so the scheduler sees them together (a burst is not split into ticks by
 * the caller's submission rate).  Each request is checked as by
 * vr_server_submit; at the first rejected one the call stops and returns its
 * status.  *accepted = the number queued (their tickets in tickets[0..*accepted));
 * the rejected request and the ones after it are not queued.  VR_ERR_ARG for
 * NULL pointers. */
vr_status vr_server_submit_many(vr_server *server, const vr_request *requests, uint32_t n, uint64_t *tickets,
                                uint32_t *accepted);
/* Returns up to `cap` finished requests, oldest first, waiting up to
 * timeout_ms for the first one (0 = do not wait). */
vr_status vr_server_poll(vr_server *server, vr_completion *out, uint32_t cap, uint32_t *count, uint32_t timeout_ms);
/* Frees a finished request's memory.  VR_ERR_BUSY if it has not finished,
 * VR_ERR_ARG for an unknown ticket. */
vr_status vr_server_release(vr_server *server, uint64_t ticket);
/* Copies a finished request's corners (144 bytes per triangle) to host
 * memory `dst` of `bytes` bytes (synchronous).  VR_ERR_BUSY if it has not
 * finished, VR_ERR_CAPACITY if bytes is too small. */
vr_status vr_server_fetch(vr_server *server, uint64_t ticket, void *dst, uint64_t bytes);
/* Cancels a request that has not been launched (it completes with
 * VR_CANCELLED); VR_ERR_BUSY once launched. */
vr_status vr_server_cancel(vr_server *server, uint64_t ticket);
vr_status vr_server_stats_get(vr_server *server, vr_server_stats *stats);
/* Cancels what is not launched, waits for the device, frees everything. */
void vr_server_destroy(vr_server *server);
const char *vr_server_last_error(const vr_server *server);

/*
 * The server's admission and tick policy on a simulated clock (host only, no
 * device): requests (sorted by arrival) reserve `bytes`, ticks run one after
 * another on a simulated device taking tick_fixed_s + tick_s_per_tri x (their
 * triangles), a finished request is released `hold` seconds after it
 * finishes, and a request with cancel_at >= 0 is cancelled at that time if
 * it has not been launched.
 */
typedef struct {
    double arrival, cancel_at, hold;
    uint64_t num_tris, bytes;
} vr_sim_request;

typedef struct {
    int32_t status;
    uint32_t tick;
    double t_admit, t_launch, t_done, t_release;   /* -1 when it did not happen */
    uint64_t offset;          /* arena offset while admitted                    */
} vr_sim_result;

vr_status vr_server_simulate(const vr_server_config *cfg, const vr_sim_request *requests, uint32_t num_requests,
                             double tick_fixed_s, double tick_s_per_tri, vr_sim_result *results,
                             vr_server_stats *stats);

/* Text of the last error on ctx (or of the last vr_create failure when ctx
 * is NULL).  Valid until the next call on the same context. */
const char *vr_last_error(const vr_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
