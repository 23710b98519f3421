// Host runtime of the geometry stage: the C ABI declared in include/vr.h.
// Validates arguments, owns per-context device scratch (grow-only), builds
// dynamic batch plans on the device and dispatches the draw kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "vr.h"
#include "vr_kernels.h"
#include "vr_plan.h"
#include "vr_frame.h"

using namespace vr;

namespace {

thread_local std::string g_create_error;

// Device words owned by a context: error code and the invocation total
// since the last vr_sync.
struct CtxWords {
    uint32_t err;
    uint32_t pad;
    unsigned long long total_inv;
};

struct Scratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct vr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cus = 256;
    size_t lds_limit = 65536;
    std::string error;
    CtxWords *d_words = nullptr;
    Scratch status, agg, plan, plan_work, tune;
    uint32_t host_err = 0;   // data error found on the host, reported by vr_sync
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;   // reused event pairs
    size_t ev_used = 0;
};

namespace {

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev_ >= 0) (void)hipSetDevice(prev_);
    }

  private:
    int prev_ = -1;
};

vr_status fail(vr_ctx *c, vr_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->error = buf;
    else g_create_error = buf;
    return s;
}

#define VR_HIP(ctx, call)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail((ctx), VR_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Grow-only scratch.  The stream is drained before a buffer is replaced
// because enqueued kernels may still use the old one.
vr_status ensure(vr_ctx *c, Scratch &s, size_t bytes, bool zero = false) {
    if (bytes <= s.bytes) return VR_OK;
    bytes = std::max<size_t>(bytes, 2 * s.bytes);
    if (s.ptr) {
        VR_HIP(c, hipStreamSynchronize(c->stream));
        VR_HIP(c, hipFree(s.ptr));
        s.ptr = nullptr;
        s.bytes = 0;
    }
    if (hipMalloc(&s.ptr, bytes) != hipSuccess) {
        s.ptr = nullptr;
        return fail(c, VR_ERR_OOM, "scratch allocation of %zu bytes failed", bytes);
    }
    s.bytes = bytes;
    if (zero) VR_HIP(c, hipMemsetAsync(s.ptr, 0, bytes, c->stream));
    return VR_OK;
}

// Event pair around the next launches when kernel timing is on.
struct TimedRegion {
    vr_ctx *c;
    hipEvent_t stop = nullptr;
    explicit TimedRegion(vr_ctx *ctx) : c(ctx) {
        if (!c->timing) return;
        if (c->ev_used == c->ev_pool.size()) {
            hipEvent_t a = nullptr, b = nullptr;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
            c->ev_pool.push_back({a, b});
        }
        auto &pr = c->ev_pool[c->ev_used++];
        (void)hipEventRecord(pr.first, c->stream);
        stop = pr.second;
    }
    void done() {
        if (stop) (void)hipEventRecord(stop, c->stream);
        stop = nullptr;
    }
    ~TimedRegion() { done(); }
};

bool is_dynamic(vr_strategy s) { return s >= VR_DYN_SORT && s <= VR_DYN_BALLOT; }
bool is_ballot(vr_strategy s) { return s == VR_STATIC_BALLOT || s == VR_DYN_BALLOT; }

uint32_t batch_limit(vr_strategy s) {
    switch (s) {
    case VR_NAIVE: return 0xFFFFFFFFu;
    case VR_STATIC_BALLOT: return VR_MAX_BATCH_BALLOT;
    case VR_STATIC_SORT:
    case VR_STATIC_HASH: return VR_MAX_BATCH_STATIC;
    default: return VR_MAX_BATCH_DYNAMIC;
    }
}

uint32_t default_max_unique(uint32_t batch_tris) {
    return std::min<uint32_t>(VR_MAX_UNIQUE, 64u * ((batch_tris + 63u) / 64u));
}

uint64_t units_bound(vr_strategy s, uint64_t T, uint32_t batch_tris) {
    if (s == VR_STATIC_SORT || s == VR_STATIC_HASH) return (T + batch_tris - 1) / batch_tris;
    return T;
}

// Upper bound on dynamic batches: a closed batch holds at least
// min(N_pmax, ceil((N_u - 2) / 3)) triangles.
uint64_t dyn_batch_bound(uint64_t T, uint32_t nu, uint32_t tmax) {
    const uint64_t m = std::max<uint64_t>(1, std::min<uint64_t>(tmax, (nu - 2 + 2) / 3));
    return T / m + 1;
}

uint32_t log2u(uint32_t x) {
    uint32_t b = 0;
    while ((1u << b) < x) ++b;
    return b;
}

struct Resolved {
    uint32_t nu = 0, nt = 0, max_idx = 0, max_uniq = 0, hash_bits = 0, probes = 4;
};

vr_status check_args(vr_ctx *c, uint64_t num_indices, const vr_shader_params *sh, vr_strategy strategy,
                     uint32_t batch_tris, const vr_opts *opts, const vr_outputs *out, Resolved *res) {
    if (!sh || !out) return fail(c, VR_ERR_ARG, "shader and outputs must not be NULL");
    if (num_indices % 3 != 0) return fail(c, VR_ERR_ARG, "num_indices %llu is not a multiple of 3",
                                          (unsigned long long)num_indices);
    if (num_indices > VR_MAX_INDICES) return fail(c, VR_ERR_ARG, "more than 2^30-1 triangles");
    if ((int)strategy < 0 || strategy > VR_DYN_BALLOT) return fail(c, VR_ERR_ARG, "unknown strategy %d", (int)strategy);
    if (batch_tris == 0 || batch_tris > batch_limit(strategy))
        return fail(c, VR_ERR_ARG, "batch_tris %u outside 1..%u for this strategy", batch_tris, batch_limit(strategy));
    if (sh->kind > 2) return fail(c, VR_ERR_ARG, "unknown shader kind %u", sh->kind);
    if (sh->num_lights > VR_MAX_LIGHTS) return fail(c, VR_ERR_ARG, "num_lights %u > 16", sh->num_lights);
    if (sh->spec_squarings > 8) return fail(c, VR_ERR_ARG, "spec_squarings %u > 8", sh->spec_squarings);
    if (sh->iterations > 4096) return fail(c, VR_ERR_ARG, "iterations %u > 4096", sh->iterations);
    vr_opts o{};
    if (opts) o = *opts;
    if (o.wg_size != 0 && (o.wg_size % 64 != 0 || o.wg_size > 1024))
        return fail(c, VR_ERR_ARG, "wg_size %u is not a multiple of 64 up to 1024", o.wg_size);
    if (o.hash_probes > 64) return fail(c, VR_ERR_ARG, "hash_probes %u > 64", o.hash_probes);
    Resolved r;
    if (is_dynamic(strategy)) {
        r.nu = o.max_unique ? o.max_unique : default_max_unique(batch_tris);
        if (r.nu < 3 || r.nu > VR_MAX_UNIQUE) return fail(c, VR_ERR_ARG, "max_unique %u outside 3..512", r.nu);
        r.max_idx = 3 * batch_tris;
        r.max_uniq = std::min(r.nu, r.max_idx);
    } else {
        r.max_idx = 3 * batch_tris;
        r.max_uniq = 3 * batch_tris;
    }
    if (strategy == VR_NAIVE) r.max_idx = r.max_uniq = 3;
    if (o.hash_slots != 0) {
        const uint32_t need = is_dynamic(strategy) ? r.nu : 3u * batch_tris;
        if ((o.hash_slots & (o.hash_slots - 1)) != 0 || o.hash_slots < need || o.hash_slots > 4096)
            return fail(c, VR_ERR_ARG, "hash_slots %u: need a power of two in %u..4096", o.hash_slots, need);
    }
    const uint64_t T = num_indices / 3;
    if (out->verts && out->verts_cap < 3 * T)
        return fail(c, VR_ERR_CAPACITY, "verts_cap %llu < 3T", (unsigned long long)out->verts_cap);
    if ((out->unit_offsets || out->unit_invocations) && out->units_cap < units_bound(strategy, T, batch_tris))
        return fail(c, VR_ERR_CAPACITY, "units_cap %llu below the bound %llu", (unsigned long long)out->units_cap,
                    (unsigned long long)units_bound(strategy, T, batch_tris));
    // launch shape (never changes results)
    if (strategy != VR_NAIVE && !is_ballot(strategy)) {
        uint32_t want = o.wg_size ? o.wg_size : std::max<uint32_t>(64, std::min<uint32_t>(256, r.max_uniq));
        uint32_t nt = 64;
        while (nt * 2 <= want && nt < 512) nt *= 2;
        // the sort keeps at most 8 rounds of elements per thread in registers
        if (strategy == VR_STATIC_SORT || strategy == VR_DYN_SORT)
            while (nt * 8 < r.max_idx) nt *= 2;
        r.nt = nt;
        const uint32_t slots = o.hash_slots ? o.hash_slots : std::max<uint32_t>(8, 1u << log2u(2 * r.max_uniq));
        r.hash_bits = log2u(slots);
        r.probes = o.hash_probes ? o.hash_probes : 4;
    } else {
        r.nt = is_ballot(strategy) ? 64 : 256;
    }
    if (res) *res = r;
    return VR_OK;
}

template <int NT, int MODE, int KIND>
void launch_dedup(vr_ctx *c, const DrawArgs &A, const vr_shader_params &sh, uint32_t lds, uint64_t units) {
    hipLaunchKernelGGL((k_dedup<NT, MODE, KIND>), dim3((uint32_t)units), dim3(NT), lds, c->stream, A, sh);
}

template <int MODE, int KIND>
void dispatch_nt(vr_ctx *c, uint32_t nt, const DrawArgs &A, const vr_shader_params &sh, uint32_t lds, uint64_t units) {
    switch (nt) {
    case 64: launch_dedup<64, MODE, KIND>(c, A, sh, lds, units); break;
    case 128: launch_dedup<128, MODE, KIND>(c, A, sh, lds, units); break;
    case 256: launch_dedup<256, MODE, KIND>(c, A, sh, lds, units); break;
    default: launch_dedup<512, MODE, KIND>(c, A, sh, lds, units); break;
    }
}

template <int MODE>
void dispatch_kind(vr_ctx *c, uint32_t kind, uint32_t nt, const DrawArgs &A, const vr_shader_params &sh, uint32_t lds,
                   uint64_t units) {
    if (kind == 0) dispatch_nt<MODE, 0>(c, nt, A, sh, lds, units);
    else if (kind == 1) dispatch_nt<MODE, 1>(c, nt, A, sh, lds, units);
    else dispatch_nt<MODE, 2>(c, nt, A, sh, lds, units);
}

template <int KIND>
void launch_ballot(vr_ctx *c, const DrawArgs &A, const vr_shader_params &sh, uint32_t lds, uint64_t batches) {
    hipLaunchKernelGGL(k_ballot<KIND>, dim3((uint32_t)batches), dim3(64), lds, c->stream, A, sh);
}

template <int KIND>
void launch_naive(vr_ctx *c, const DrawArgs &A, const vr_shader_params &sh) {
    const uint64_t blocks = (3ull * A.T + 255) / 256;
    hipLaunchKernelGGL(k_naive<KIND>, dim3((uint32_t)blocks), dim3(256), 0, c->stream, A, sh);
}

__global__ void k_empty_draw(unsigned long long *counters, uint32_t *unit_offsets) {
    if (threadIdx.x < 4 && counters) counters[threadIdx.x] = 0;
    if (threadIdx.x == 0 && unit_offsets) unit_offsets[0] = 0;
}

__global__ void k_plan_empty(uint32_t *plan) {
    if (threadIdx.x == 0) {
        plan[0] = 0;
        plan[1] = 0;
    }
}

// Builds the plan of a dynamic draw on the context's stream (see vr_plan.h).
vr_status build_plan(vr_ctx *c, const uint32_t *d_idx, uint32_t T, uint32_t V, uint32_t nu, uint32_t tmax,
                     uint32_t *d_plan) {
    if (T == 0) {
        hipLaunchKernelGGL(k_plan_empty, dim3(1), dim3(64), 0, c->stream, d_plan);
        return VR_OK;
    }
    // segment length: a power of two >= N_pmax, 2048 up to 4M triangles, then
    // growing to 8192 so that large draws keep a modest number of segments
    uint32_t L = 2048;
    while (L < 8192 && (uint64_t)L * 2048 < T) L <<= 1;
    const uint32_t nseg = (T + L - 1) / L;
    std::vector<uint32_t> counts{nseg};
    while (counts.back() > kFanIn) counts.push_back((counts.back() + kFanIn - 1) / kFanIn);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t bytes = al(4ull * T) * 2 + al(4ull * nseg);
    std::vector<size_t> tab_off, ent_off;
    for (uint32_t cnt : counts) {
        tab_off.push_back(bytes);
        bytes += al(2ull * cnt * tmax);
        ent_off.push_back(bytes);
        bytes += al(2ull * cnt);
    }
    vr_status st = ensure(c, c->plan_work, bytes);
    if (st != VR_OK) return st;
    unsigned char *base = (unsigned char *)c->plan_work.ptr;
    uint32_t *next = (uint32_t *)base;
    uint32_t *cuts = (uint32_t *)(base + al(4ull * T));
    uint32_t *ncuts = (uint32_t *)(base + 2 * al(4ull * T));
    auto tab = [&](size_t l) { return (uint16_t *)(base + tab_off[l]); };
    auto ent = [&](size_t l) { return (uint16_t *)(base + ent_off[l]); };
    PlanArgs P{};
    P.idx = d_idx;
    P.V = V;
    P.T = T;
    P.cap = nu;
    P.tmax = tmax;
    P.seg_len = L;
    P.nseg = nseg;
    P.next = next;
    P.err = &c->d_words->err;
    TimedRegion timed(c);
    hipLaunchKernelGGL(k_plan_next, dim3((T + kNextBlock - 1) / kNextBlock), dim3(256), 0, c->stream, P);
    hipLaunchKernelGGL(k_plan_table, dim3(nseg), dim3(256), 4 * L, c->stream, P, tab(0));
    const uint32_t grp_lds = 2 * kFanIn * tmax;
    for (size_t l = 0; l + 1 < counts.size(); ++l)
        hipLaunchKernelGGL(k_plan_compose, dim3(counts[l + 1]), dim3(512), grp_lds, c->stream, tmax, counts[l],
                           (const uint16_t *)tab(l), tab(l + 1));
    const size_t top = counts.size() - 1;
    hipLaunchKernelGGL(k_plan_top, dim3(1), dim3(256), 2 * counts[top] * tmax, c->stream, tmax, counts[top],
                       (const uint16_t *)tab(top), ent(top));
    for (size_t l = top; l-- > 0;)
        hipLaunchKernelGGL(k_plan_resolve, dim3(counts[l + 1]), dim3(256), grp_lds, c->stream, tmax, counts[l],
                           (const uint16_t *)tab(l), (const uint16_t *)ent(l + 1), ent(l));
    hipLaunchKernelGGL(k_plan_emit, dim3(nseg), dim3(64), 4 * L, c->stream, P, (const uint16_t *)ent(0), cuts, ncuts);
    if (nseg <= kPackSegs)
        hipLaunchKernelGGL(k_plan_pack_seg, dim3(nseg), dim3(64), 0, c->stream, P, (const uint32_t *)cuts,
                           (const uint32_t *)ncuts, d_plan);
    else
        hipLaunchKernelGGL(k_plan_pack, dim3(1), dim3(1024), 0, c->stream, P, (const uint32_t *)cuts, ncuts, d_plan);
    VR_HIP(c, hipGetLastError());
    return VR_OK;
}

}  // namespace

struct vr_frame {
    vr_ctx *c = nullptr;
    uint32_t n = 0;
    void *mem = nullptr;
    DrawDesc *d_draws = nullptr;
    vr_shader_params *d_shaders = nullptr;
    uint32_t *d_unit_base = nullptr, *d_slot_base = nullptr;
    unsigned long long *d_agg = nullptr, *d_dtot = nullptr;
    uint32_t unit_lds = 0, ballot_stride = 0, lds_total = 0, grid = 1;
    bool index_error = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void frame_enqueue(vr_frame *f, hipStream_t s) {
    if (f->n == 0) return;
    vr_ctx *c = f->c;
    hipLaunchKernelGGL(k_frame_prepare, dim3(1), dim3(1024), 0, s, (const DrawDesc *)f->d_draws, f->n, f->d_unit_base,
                       f->d_slot_base);
    hipLaunchKernelGGL(k_frame, dim3(f->grid), dim3(kFrameNT), f->lds_total, s, (const DrawDesc *)f->d_draws, f->n,
                       (const vr_shader_params *)f->d_shaders, (const uint32_t *)f->d_unit_base,
                       (const uint32_t *)f->d_slot_base, f->d_agg, f->unit_lds, f->ballot_stride, &c->d_words->err,
                       &c->d_words->total_inv);
    hipLaunchKernelGGL(k_frame_finish, dim3(f->n), dim3(64), 0, s, (const DrawDesc *)f->d_draws,
                       (const uint32_t *)f->d_slot_base, (const unsigned long long *)f->d_agg, f->d_dtot);
    hipLaunchKernelGGL(k_frame_total, dim3(1), dim3(1024), 0, s, (const unsigned long long *)f->d_dtot, f->n,
                       &c->d_words->total_inv);
}

uint32_t frame_mode(vr_strategy s) {
    switch (s) {
    case VR_NAIVE: return kFrameNaive;
    case VR_STATIC_BALLOT:
    case VR_DYN_BALLOT: return kFrameBallot;
    case VR_STATIC_SORT:
    case VR_DYN_SORT: return kFrameSort;
    case VR_DYN_PHASH: return kFramePHash;
    default: return kFrameHash;
    }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

vr_status vr_create(vr_ctx **out, int device, void *hip_stream) {
    if (!out) return fail(nullptr, VR_ERR_ARG, "ctx pointer is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return fail(nullptr, VR_ERR_DEVICE, "HIP device %d not available", device);
    vr_ctx *c = new vr_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->num_cus = prop.multiProcessorCount;
        c->lds_limit = prop.sharedMemPerBlock;
    }
    if (hipMalloc((void **)&c->d_words, sizeof(CtxWords)) != hipSuccess ||
        hipMemset(c->d_words, 0, sizeof(CtxWords)) != hipSuccess) {
        if (c->d_words) (void)hipFree(c->d_words);
        delete c;
        return fail(nullptr, VR_ERR_OOM, "context allocation failed");
    }
    *out = c;
    return VR_OK;
}

void vr_destroy(vr_ctx *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (Scratch *s : {&c->status, &c->agg, &c->plan, &c->plan_work, &c->tune})
        if (s->ptr) (void)hipFree(s->ptr);
    for (auto &pr : c->ev_pool) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    if (c->d_words) (void)hipFree(c->d_words);
    delete c;
}

vr_status vr_set_stream(vr_ctx *c, void *hip_stream) {
    if (!c) return VR_ERR_ARG;
    c->stream = (hipStream_t)hip_stream;
    return VR_OK;
}

vr_status vr_check_args(uint64_t num_indices, uint32_t num_vertices, const vr_shader_params *shader,
                        vr_strategy strategy, uint32_t batch_tris, const vr_opts *opts, const vr_outputs *out) {
    (void)num_vertices;
    return check_args(nullptr, num_indices, shader, strategy, batch_tris, opts, out, nullptr);
}

vr_status vr_plan_dynamic(vr_ctx *c, const uint32_t *d_indices, uint64_t num_indices, uint32_t num_vertices,
                          uint32_t max_unique, uint32_t max_tris, uint32_t *d_plan, uint64_t plan_cap) {
    if (!c) return VR_ERR_ARG;
    if (num_indices % 3 != 0 || num_indices > VR_MAX_INDICES)
        return fail(c, VR_ERR_ARG, "num_indices must be a multiple of 3 below 3*2^30");
    if (max_unique < 3 || max_unique > VR_MAX_UNIQUE) return fail(c, VR_ERR_ARG, "max_unique outside 3..512");
    if (max_tris == 0 || max_tris > VR_MAX_BATCH_DYNAMIC) return fail(c, VR_ERR_ARG, "max_tris outside 1..512");
    const uint64_t T = num_indices / 3;
    if (!d_plan || plan_cap < T + 2) return fail(c, VR_ERR_CAPACITY, "plan buffer must hold T+2 entries");
    if (T && !d_indices) return fail(c, VR_ERR_ARG, "indices are NULL");
    DeviceGuard g(c->device);
    if (T && num_vertices == 0) {
        if (!c->host_err) c->host_err = VR_ERR_INDEX_RANGE;
        return VR_OK;
    }
    return build_plan(c, d_indices, (uint32_t)T, num_vertices, max_unique, max_tris, d_plan);
}

vr_status vr_process_draw(vr_ctx *c, const uint32_t *d_indices, uint64_t num_indices, const float *d_vertices,
                          uint32_t num_vertices, const vr_shader_params *shader, vr_strategy strategy,
                          uint32_t batch_tris, const vr_opts *opts, const vr_outputs *out) {
    if (!c) return VR_ERR_ARG;
    Resolved r;
    vr_status st = check_args(c, num_indices, shader, strategy, batch_tris, opts, out, &r);
    if (st != VR_OK) return st;
    const uint64_t T = num_indices / 3;
    if (T && (!d_indices || !d_vertices)) return fail(c, VR_ERR_ARG, "indices or vertices are NULL");
    if (d_vertices && ((uintptr_t)d_vertices & 15)) return fail(c, VR_ERR_ARG, "vertices must be 16-byte aligned");
    if (out->corners && ((uintptr_t)out->corners & 15)) return fail(c, VR_ERR_ARG, "corners must be 16-byte aligned");
    if (out->verts && ((uintptr_t)out->verts & 15)) return fail(c, VR_ERR_ARG, "verts must be 16-byte aligned");
    DeviceGuard g(c->device);
    if (T == 0) {
        hipLaunchKernelGGL(k_empty_draw, dim3(1), dim3(64), 0, c->stream, (unsigned long long *)out->counters,
                           out->unit_offsets);
        VR_HIP(c, hipGetLastError());
        return VR_OK;
    }
    if (num_vertices == 0) {   // every index is out of range
        if (!c->host_err) c->host_err = VR_ERR_INDEX_RANGE;
        return VR_OK;
    }

    DrawArgs A{};
    A.idx = d_indices;
    A.vtx = (const f4 *)d_vertices;
    A.V = num_vertices;
    A.T = (uint32_t)T;
    A.batch_tris = batch_tris;
    A.corners = (f4 *)out->corners;
    A.tris = out->tris;
    A.verts = (f4 *)out->verts;
    A.local_idx = out->local_idx;
    A.unit_offsets = out->unit_offsets;
    A.unit_inv = out->unit_invocations;
    A.counters = (unsigned long long *)out->counters;
    A.err = &c->d_words->err;
    A.total_inv = &c->d_words->total_inv;
    A.hash_bits = r.hash_bits;
    A.probes = r.probes;
    A.max_idx = r.max_idx;
    A.max_uniq = r.max_uniq;
    A.need_prefix = (out->tris || out->verts || out->unit_offsets || out->unit_invocations) ? 1u : 0u;

    const vr_shader_params &sh = *shader;
    if (strategy == VR_NAIVE) {
        TimedRegion timed(c);
        if (sh.kind == 0) launch_naive<0>(c, A, sh);
        else if (sh.kind == 1) launch_naive<1>(c, A, sh);
        else launch_naive<2>(c, A, sh);
        VR_HIP(c, hipGetLastError());
        return VR_OK;
    }

    uint64_t nb_bound;
    if (is_dynamic(strategy)) {
        const uint32_t *plan = opts ? opts->d_plan : nullptr;
        if (!plan) {
            st = ensure(c, c->plan, 4ull * (T + 2));
            if (st != VR_OK) return st;
            st = build_plan(c, d_indices, (uint32_t)T, num_vertices, r.nu, batch_tris, (uint32_t *)c->plan.ptr);
            if (st != VR_OK) return st;
            plan = (const uint32_t *)c->plan.ptr;
        }
        A.plan = plan;
        A.num_batches = 0;
        nb_bound = dyn_batch_bound(T, r.nu, batch_tris);
    } else {
        A.plan = nullptr;
        A.num_batches = (uint32_t)((T + batch_tris - 1) / batch_tris);
        nb_bound = A.num_batches;
    }
    // one workgroup per batch; a dynamic launch covers the batch bound and
    // workgroups past the plan's count return at once
    st = ensure(c, c->agg, 8ull * nb_bound);
    if (st != VR_OK) return st;
    A.agg = (unsigned long long *)c->agg.ptr;
    if (A.need_prefix) {
        st = ensure(c, c->status, 8ull * nb_bound, /*zero=*/true);
        if (st != VR_OK) return st;
        A.status = (unsigned long long *)c->status.ptr;
        A.status_cap = (uint32_t)nb_bound;
    } else {
        A.status = nullptr;
        A.status_cap = (uint32_t)nb_bound;
    }
    TimedRegion timed(c);
    if (is_ballot(strategy)) {
        const uint32_t lds = 64 * 48 + ((3 * batch_tris + 15) & ~15u);
        if (sh.kind == 0) launch_ballot<0>(c, A, sh, lds, nb_bound);
        else if (sh.kind == 1) launch_ballot<1>(c, A, sh, lds, nb_bound);
        else launch_ballot<2>(c, A, sh, lds, nb_bound);
    } else {
        const int mode = (strategy == VR_STATIC_SORT || strategy == VR_DYN_SORT) ? kSort
                         : (strategy == VR_DYN_PHASH)                             ? kPHash
                                                                                  : kHash;
        const uint32_t lds = dedup_lds_layout(mode, r.max_idx, r.max_uniq, r.hash_bits).total;
        if (lds > c->lds_limit)
            return fail(c, VR_ERR_ARG, "LDS need %u B exceeds the %zu B limit (lower hash_slots or batch_tris)", lds,
                        c->lds_limit);
        if (mode == kSort) dispatch_kind<kSort>(c, sh.kind, r.nt, A, sh, lds, nb_bound);
        else if (mode == kHash) dispatch_kind<kHash>(c, sh.kind, r.nt, A, sh, lds, nb_bound);
        else dispatch_kind<kPHash>(c, sh.kind, r.nt, A, sh, lds, nb_bound);
    }
    timed.done();
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, c->stream, A.plan, A.num_batches, A.status_cap,
                       (const unsigned long long *)A.agg, A.status, A.counters, A.total_inv);
    VR_HIP(c, hipGetLastError());
    return VR_OK;
}

vr_status vr_sync(vr_ctx *c, uint64_t *h_invocations) {
    if (!c) return VR_ERR_ARG;
    DeviceGuard g(c->device);
    VR_HIP(c, hipStreamSynchronize(c->stream));
    CtxWords w{};
    VR_HIP(c, hipMemcpy(&w, c->d_words, sizeof w, hipMemcpyDeviceToHost));
    VR_HIP(c, hipMemset(c->d_words, 0, sizeof w));
    if (h_invocations) *h_invocations = w.total_inv;
    uint32_t e = c->host_err ? c->host_err : w.err;
    c->host_err = 0;
    if (e == VR_ERR_INDEX_RANGE) return fail(c, VR_ERR_INDEX_RANGE, "an index is >= num_vertices");
    if (e != 0) return fail(c, (vr_status)e, "device-side error %u", e);
    return VR_OK;
}

vr_status vr_frame_create(vr_ctx *c, const vr_draw *draws, uint32_t n, const vr_shader_params *shaders,
                          uint32_t ns, int capture_graph, vr_frame **out) {
    if (!c || !out) return VR_ERR_ARG;
    *out = nullptr;
    if (n > VR_MAX_FRAME_DRAWS) return fail(c, VR_ERR_ARG, "a frame holds at most %d draws", VR_MAX_FRAME_DRAWS);
    if (n && (!draws || !shaders || ns == 0)) return fail(c, VR_ERR_ARG, "draws and shaders must not be NULL");
    std::vector<DrawDesc> desc(n);
    uint64_t slots = 0;
    uint32_t unit_lds = 256 * 48, ballot_stride = 0;
    bool index_error = false;
    for (uint32_t d = 0; d < n; ++d) {
        const vr_draw &D = draws[d];
        if (D.shader >= ns) return fail(c, VR_ERR_ARG, "draw %u: shader %u out of range", d, D.shader);
        vr_opts o{};
        o.max_unique = D.max_unique;
        o.d_plan = D.d_plan;
        vr_outputs ov{};
        ov.corners = D.d_corners;
        ov.counters = D.d_counters;
        Resolved r;
        vr_status st = check_args(c, D.num_indices, &shaders[D.shader], D.strategy, D.batch_tris, &o, &ov, &r);
        if (st != VR_OK) return fail(c, st, "draw %u: %s", d, c->error.c_str());
        const uint64_t T = D.num_indices / 3;
        if (T && (!D.d_indices || !D.d_vertices || !D.d_corners))
            return fail(c, VR_ERR_ARG, "draw %u: indices, vertices and corners are required", d);
        if (((uintptr_t)D.d_vertices & 15) || ((uintptr_t)D.d_corners & 15))
            return fail(c, VR_ERR_ARG, "draw %u: vertices and corners must be 16-byte aligned", d);
        if (is_dynamic(D.strategy) && T && !D.d_plan)
            return fail(c, VR_ERR_ARG, "draw %u: a dynamic draw in a frame needs its plan", d);
        if (T && D.num_vertices == 0) index_error = true;
        DrawDesc &X = desc[d];
        X.idx = D.d_indices;
        X.vtx = (const f4 *)D.d_vertices;
        X.corners = (f4 *)D.d_corners;
        X.counters = (unsigned long long *)D.d_counters;
        X.plan = is_dynamic(D.strategy) ? D.d_plan : nullptr;
        X.V = D.num_vertices;
        X.T = (T && D.num_vertices == 0) ? 0u : (uint32_t)T;
        X.batch_tris = D.batch_tris;
        X.num_batches = is_dynamic(D.strategy) ? 0u : (uint32_t)((T + D.batch_tris - 1) / D.batch_tris);
        X.shader = D.shader;
        X.mode = frame_mode(D.strategy);
        X.kind = shaders[D.shader].kind;
        X.max_idx = r.max_idx;
        X.max_uniq = r.max_uniq;
        X.hash_bits = r.hash_bits;
        X.probes = r.probes;
        if (X.mode == kFrameNaive) {
            slots += (3 * T + 255) / 256;
        } else {
            slots += is_dynamic(D.strategy) ? dyn_batch_bound(T, r.nu, D.batch_tris) : X.num_batches;
            if (X.mode == kFrameBallot) {
                ballot_stride = std::max(ballot_stride, align16(64 * 48 + 3 * D.batch_tris));
            } else {
                unit_lds = std::max(unit_lds, dedup_lds_layout((int)X.mode, r.max_idx, r.max_uniq, r.hash_bits).total);
            }
        }
    }
    unit_lds = align16(std::max(unit_lds, 4 * ballot_stride));
    const uint32_t lds_total = unit_lds + 4 * (n + 1);
    if (lds_total > c->lds_limit)
        return fail(c, VR_ERR_ARG, "frame needs %u B of LDS per workgroup (limit %zu)", lds_total, c->lds_limit);

    DeviceGuard g(c->device);
    vr_frame *f = new vr_frame();
    f->c = c;
    f->n = n;
    f->unit_lds = unit_lds;
    f->ballot_stride = ballot_stride;
    f->lds_total = lds_total;
    f->index_error = index_error;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_draws = 0, o_sh = al(sizeof(DrawDesc) * n), o_ub = o_sh + al(sizeof(vr_shader_params) * ns),
                 o_sb = o_ub + al(4ull * (n + 1)), o_agg = o_sb + al(4ull * (n + 1)), o_dt = o_agg + al(8 * (slots + 1)),
                 total = o_dt + al(8ull * (n + 1));
    if (hipMalloc(&f->mem, total) != hipSuccess) {
        delete f;
        return fail(c, VR_ERR_OOM, "frame allocation of %zu bytes failed", total);
    }
    unsigned char *m = (unsigned char *)f->mem;
    f->d_draws = (DrawDesc *)(m + o_draws);
    f->d_shaders = (vr_shader_params *)(m + o_sh);
    f->d_unit_base = (uint32_t *)(m + o_ub);
    f->d_slot_base = (uint32_t *)(m + o_sb);
    f->d_agg = (unsigned long long *)(m + o_agg);
    f->d_dtot = (unsigned long long *)(m + o_dt);
    hipError_t e = hipSuccess;
    if (n) e = hipMemcpy(f->d_draws, desc.data(), sizeof(DrawDesc) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess && n) e = hipMemcpy(f->d_shaders, shaders, sizeof(vr_shader_params) * ns, hipMemcpyHostToDevice);
    int per_cu = 0;
    if (e == hipSuccess &&
        (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_frame, kFrameNT, lds_total) != hipSuccess || per_cu < 1))
        per_cu = 1;
    f->grid = (uint32_t)std::max(1, c->num_cus * per_cu);
    if (e == hipSuccess && capture_graph && n) {
        hipStream_t cs = nullptr;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            frame_enqueue(f, cs);
            e = hipStreamEndCapture(cs, &f->graph);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&f->exec, f->graph, nullptr, nullptr, 0);
        if (cs) (void)hipStreamDestroy(cs);
    }
    if (e != hipSuccess) {
        vr_frame_destroy(f);
        return fail(c, VR_ERR_DEVICE, "frame setup: %s", hipGetErrorString(e));
    }
    *out = f;
    return VR_OK;
}

vr_status vr_frame_run(vr_frame *f) {
    if (!f) return VR_ERR_ARG;
    vr_ctx *c = f->c;
    DeviceGuard g(c->device);
    if (f->index_error && !c->host_err) c->host_err = VR_ERR_INDEX_RANGE;
    TimedRegion timed(c);
    if (f->exec) VR_HIP(c, hipGraphLaunch(f->exec, c->stream));
    else frame_enqueue(f, c->stream);
    timed.done();
    VR_HIP(c, hipGetLastError());
    return VR_OK;
}

void vr_frame_destroy(vr_frame *f) {
    if (!f) return;
    DeviceGuard g(f->c->device);
    (void)hipStreamSynchronize(f->c->stream);
    if (f->exec) (void)hipGraphExecDestroy(f->exec);
    if (f->graph) (void)hipGraphDestroy(f->graph);
    if (f->mem) (void)hipFree(f->mem);
    delete f;
}

vr_status vr_process_draws(vr_ctx *c, const vr_draw *draws, uint32_t n, const vr_shader_params *shaders, uint32_t ns) {
    vr_frame *f = nullptr;
    vr_status st = vr_frame_create(c, draws, n, shaders, ns, 0, &f);
    if (st != VR_OK) return st;
    st = vr_frame_run(f);
    vr_frame_destroy(f);
    return st;
}

vr_status vr_autotune(vr_ctx *c, const uint32_t *d_idx, uint64_t num_indices, const float *d_vtx, uint32_t V,
                      const vr_shader_params *sh, vr_tune_candidate *cands, uint32_t ncand, uint32_t reps,
                      uint32_t *best) {
    if (!c || !sh || (ncand && !cands)) return VR_ERR_ARG;
    if (num_indices % 3 != 0 || num_indices > VR_MAX_INDICES) return fail(c, VR_ERR_ARG, "bad num_indices");
    const uint64_t T = num_indices / 3;
    if (reps == 0) reps = 1;
    DeviceGuard g(c->device);
    // scratch: corners, plan, counters
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_plan = al(48ull * 3 * T), o_cnt = o_plan + al(4ull * (T + 2)), total = o_cnt + 256;
    vr_status st = ensure(c, c->tune, total);
    if (st != VR_OK) return st;
    unsigned char *m = (unsigned char *)c->tune.ptr;
    float *corners = (float *)m;
    uint32_t *plan = (uint32_t *)(m + o_plan);
    uint64_t *counters = (uint64_t *)(m + o_cnt);
    // the search's invocations and errors are its own: keep the caller's
    VR_HIP(c, hipStreamSynchronize(c->stream));
    CtxWords saved{};
    VR_HIP(c, hipMemcpy(&saved, c->d_words, sizeof saved, hipMemcpyDeviceToHost));
    VR_HIP(c, hipMemset(c->d_words, 0, sizeof saved));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    VR_HIP(c, hipEventCreate(&e0));
    VR_HIP(c, hipEventCreate(&e1));
    const bool was_timing = c->timing;
    c->timing = false;
    float best_ms = -1.0f;
    uint32_t best_i = 0;
    for (uint32_t i = 0; i < ncand; ++i) {
        vr_tune_candidate &k = cands[i];
        k.kernel_ms = -1.0f;
        k.plan_ms = 0.0f;
        k.invocations = 0;
        vr_opts o{};
        o.max_unique = k.max_unique;
        o.wg_size = k.wg_size;
        vr_outputs out{};
        out.corners = corners;
        out.counters = counters;
        Resolved r;
        if (check_args(c, num_indices, sh, k.strategy, k.batch_tris, &o, &out, &r) != VR_OK) continue;
        if (is_dynamic(k.strategy)) {
            (void)hipEventRecord(e0, c->stream);
            if (vr_plan_dynamic(c, d_idx, num_indices, V, r.nu, k.batch_tris, plan, T + 2) != VR_OK) continue;
            (void)hipEventRecord(e1, c->stream);
            VR_HIP(c, hipEventSynchronize(e1));
            VR_HIP(c, hipEventElapsedTime(&k.plan_ms, e0, e1));
            o.d_plan = plan;
        }
        if (vr_process_draw(c, d_idx, num_indices, d_vtx, V, sh, k.strategy, k.batch_tris, &o, &out) != VR_OK) continue;
        c->timing = true;
        const size_t first = c->ev_used;
        bool ok = true;
        for (uint32_t rep = 0; rep < reps && ok; ++rep)
            ok = vr_process_draw(c, d_idx, num_indices, d_vtx, V, sh, k.strategy, k.batch_tris, &o, &out) == VR_OK;
        c->timing = false;
        VR_HIP(c, hipStreamSynchronize(c->stream));
        float sum = 0.0f;
        for (size_t j = first; j < c->ev_used; ++j) {
            float ms = 0.0f;
            VR_HIP(c, hipEventElapsedTime(&ms, c->ev_pool[j].first, c->ev_pool[j].second));
            sum += ms;
        }
        const size_t timed = c->ev_used - first;
        c->ev_used = first;
        if (!ok || timed == 0) continue;
        VR_HIP(c, hipMemcpy(&k.invocations, counters, sizeof(uint64_t), hipMemcpyDeviceToHost));
        k.kernel_ms = sum / (float)timed;
        if (best_ms < 0.0f || k.kernel_ms < best_ms) {
            best_ms = k.kernel_ms;
            best_i = i;
        }
    }
    c->timing = was_timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    VR_HIP(c, hipStreamSynchronize(c->stream));
    CtxWords mine{};
    VR_HIP(c, hipMemcpy(&mine, c->d_words, sizeof mine, hipMemcpyDeviceToHost));
    VR_HIP(c, hipMemcpy(c->d_words, &saved, sizeof saved, hipMemcpyHostToDevice));
    if (best) *best = best_i;
    if (mine.err) return fail(c, (vr_status)mine.err, "device-side error %u during the search", mine.err);
    return best_ms < 0.0f ? fail(c, VR_ERR_ARG, "no valid candidate") : VR_OK;
}

vr_status vr_set_kernel_timing(vr_ctx *c, int enable) {
    if (!c) return VR_ERR_ARG;
    c->timing = enable != 0;
    return VR_OK;
}

vr_status vr_kernel_times(vr_ctx *c, float *ms, uint32_t cap, uint32_t *count) {
    if (!c) return VR_ERR_ARG;
    DeviceGuard g(c->device);
    VR_HIP(c, hipStreamSynchronize(c->stream));
    const size_t n = c->ev_used;
    for (size_t i = 0; i < n && i < cap && ms; ++i)
        VR_HIP(c, hipEventElapsedTime(&ms[i], c->ev_pool[i].first, c->ev_pool[i].second));
    if (count) *count = (uint32_t)n;
    c->ev_used = 0;
    return VR_OK;
}

const char *vr_last_error(const vr_ctx *c) { return c ? c->error.c_str() : g_create_error.c_str(); }

}  // extern "C"
