// Host runtime of the geometry stage: the C ABI declared in include/vr.h.
// Validates arguments, owns per-context device scratch (grow-only), builds
// dynamic batch plans on the device and dispatches the draw kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vr.h"
#include "vr_kernels.h"
#include "vr_plan.h"
#include "vr_frame.h"
#include "vr_sched.h"
#include "vr_walk.h"
#include "vr_stream.h"
#include "vr_selftest.h"

using namespace vr;

namespace {

thread_local std::string g_create_error;

// Device words owned by a context: error code and the invocation total
// since the last vr_sync.
struct CtxWords {
    uint32_t err;
    uint32_t plan_fail;   // epoch of the last planning call whose aligned chain failed
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
    Scratch status, agg, plan, plan_work, tune, shaded;   // shaded: MULTI's vertex pass
    Scratch plan_status;                                   // the planner's epoch-tagged look-back words
    Scratch selftest;                                      // vr_math_selftest's counter
    uint32_t host_err = 0;   // data error found on the host, reported by vr_sync
    uint32_t plan_epoch = 0;  // numbers planning calls (0 is never used)
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
    explicit TimedRegion(vr_ctx *ctx, bool enabled = true) : c(ctx) {
        if (!c->timing || !enabled) return;
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
    case VR_NAIVE:
    case VR_MULTI: return 0xFFFFFFFFu;
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
    if (s == VR_MULTI) return 1;
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

vr_status check_args(vr_ctx *c, uint64_t num_indices, uint32_t num_vertices, const vr_shader_params *sh,
                     vr_strategy strategy, uint32_t batch_tris, const vr_opts *opts, const vr_outputs *out,
                     Resolved *res) {
    if (!sh || !out) return fail(c, VR_ERR_ARG, "shader and outputs must not be NULL");
    if (num_indices % 3 != 0) return fail(c, VR_ERR_ARG, "num_indices %llu is not a multiple of 3",
                                          (unsigned long long)num_indices);
    if (num_indices > VR_MAX_INDICES) return fail(c, VR_ERR_ARG, "more than 2^30-1 triangles");
    if ((int)strategy < 0 || strategy > VR_MULTI) return fail(c, VR_ERR_ARG, "unknown strategy %d", (int)strategy);
    if (strategy == VR_MULTI && out->local_idx)
        return fail(c, VR_ERR_ARG, "MULTI has no unit-local ids (its unit is the whole vertex buffer)");
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
        if (r.nu < 3 || r.nu > VR_MAX_UNIQUE)
            return fail(c, VR_ERR_ARG, "max_unique %u outside 3..%u", r.nu, (unsigned)VR_MAX_UNIQUE);
        r.max_idx = 3 * batch_tris;
        r.max_uniq = std::min(r.nu, r.max_idx);
    } else {
        r.max_idx = 3 * batch_tris;
        r.max_uniq = 3 * batch_tris;
    }
    if (strategy == VR_NAIVE || strategy == VR_MULTI) r.max_idx = r.max_uniq = 3;
    if (o.hash_slots != 0) {
        const uint32_t need = is_dynamic(strategy) ? r.nu : 3u * batch_tris;
        if ((o.hash_slots & (o.hash_slots - 1)) != 0 || o.hash_slots < need || o.hash_slots > VR_MAX_HASH_SLOTS)
            return fail(c, VR_ERR_ARG, "hash_slots %u: need a power of two in %u..%u", o.hash_slots, need,
                        (unsigned)VR_MAX_HASH_SLOTS);
    }
    const uint64_t T = num_indices / 3;
    const uint64_t vneed = strategy == VR_MULTI ? (uint64_t)num_vertices : 3 * T;
    if (out->verts && out->verts_cap < vneed)
        return fail(c, VR_ERR_CAPACITY, "verts_cap %llu < %llu", (unsigned long long)out->verts_cap,
                    (unsigned long long)vneed);
    if ((out->unit_offsets || out->unit_invocations) && out->units_cap < units_bound(strategy, T, batch_tris))
        return fail(c, VR_ERR_CAPACITY, "units_cap %llu below the bound %llu", (unsigned long long)out->units_cap,
                    (unsigned long long)units_bound(strategy, T, batch_tris));
    // launch shape (never changes results)
    if (strategy != VR_NAIVE && strategy != VR_MULTI && !is_ballot(strategy)) {
        uint32_t want = o.wg_size ? o.wg_size : std::max<uint32_t>(64, std::min<uint32_t>(256, r.max_uniq));
        uint32_t nt = 64;
        while (nt * 2 <= want && nt < 1024) nt *= 2;
        // the sort keeps at most 8 rounds of elements per thread in registers;
        // the canonical ranking keeps at most 32 flags per thread in a mask
        const uint32_t per = (strategy == VR_STATIC_SORT || strategy == VR_DYN_SORT) ? 8u : 32u;
        while (nt * per < r.max_idx && nt < 1024) nt *= 2;
        if (nt * per < r.max_idx)
            return fail(c, VR_ERR_ARG, "batch_tris %u: a unit of %u indices needs more than 1024 threads", batch_tris,
                        r.max_idx);
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

// A static draw's units are exactly known.  A dynamic draw has at least
// ceil(T / N_pmax) units (exactly that many when every batch is full) and at
// most the host-side bound.  The launch has one workgroup per unit of the
// fewest; without prefix outputs (units in any order) the same workgroups
// take the rest grid-stride, else a second launch has one workgroup per
// possible further unit.
template <int NT, int MODE, int KIND, bool OCC>
void launch_dedup(vr_ctx *c, const DrawArgs &A, const vr_shader_params &sh, uint32_t lds, uint64_t units) {
    uint64_t first = units;
    if (A.plan) first = std::min<uint64_t>(units, (A.T + A.batch_tris - 1) / A.batch_tris);
    const bool stride = A.plan && !A.need_prefix && first > 0 && units > first;
    if (first)
        hipLaunchKernelGGL((k_dedup<NT, MODE, KIND, OCC>), dim3((uint32_t)first), dim3(NT), lds, c->stream, A, sh,
                           0u, stride ? (uint32_t)first : 0u);
    if (units > first && !stride)
        hipLaunchKernelGGL((k_dedup<NT, MODE, KIND, OCC>), dim3((uint32_t)(units - first)), dim3(NT), lds,
                           c->stream, A, sh, (uint32_t)first, 0u);
}

// Whether a dedup launch of nt threads and lds bytes per workgroup takes the
// occupancy-bound kernel: only for 128 and 256 threads, and only when the
// LDS lets eight wavefronts per SIMD reside (seven for the sort).
bool dedup_occupancy_bound(const vr_ctx *c, int mode, uint32_t nt, uint32_t lds) {
    if (nt != 128 && nt != 256) return false;
    const uint32_t target = mode == kSort ? 7u : 8u;          // wavefronts per SIMD
    const uint32_t groups = target * 4u / (nt / kWave);        // workgroups per CU for them
    return (uint64_t)groups * (lds + 64u) <= c->lds_limit;     // + the kernel's static LDS
}

template <int MODE, int KIND>
void dispatch_nt(vr_ctx *c, uint32_t nt, const DrawArgs &A, const vr_shader_params &sh, uint32_t lds, uint64_t units) {
    const bool occ = dedup_occupancy_bound(c, MODE, nt, lds);
    switch (nt) {
    case 64: launch_dedup<64, MODE, KIND, false>(c, A, sh, lds, units); break;
    case 128:
        if (occ) launch_dedup<128, MODE, KIND, true>(c, A, sh, lds, units);
        else launch_dedup<128, MODE, KIND, false>(c, A, sh, lds, units);
        break;
    case 256:
        if (occ) launch_dedup<256, MODE, KIND, true>(c, A, sh, lds, units);
        else launch_dedup<256, MODE, KIND, false>(c, A, sh, lds, units);
        break;
    case 512: launch_dedup<512, MODE, KIND, false>(c, A, sh, lds, units); break;
    default: launch_dedup<1024, MODE, KIND, false>(c, A, sh, lds, units); break;
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
void launch_ballot(vr_ctx *c, const DrawArgs &A, const vr_shader_params &sh, uint32_t stride, uint64_t batches) {
    hipLaunchKernelGGL(k_ballot<KIND>, dim3((uint32_t)((batches + kBallotWaves - 1) / kBallotWaves)),
                       dim3(kBallotWaves * 64), kBallotWaves * stride, c->stream, A, sh, stride);
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

__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) p[i] = v;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free draw (vr_process_draw_noalloc): the
// per-batch aggregates, then the look-back words, of at most
// VR_NOALLOC_MAX_BATCHES batches.  Every GPU holds its own copy for the life
// of the process.  In host code `scratch` names a host-side stand-in, never
// the device memory: the device address comes from hipGetSymbolAddress, once
// per device (scratch_setup, called by vr_create), and only that address is
// handed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[16ull * VR_NOALLOC_MAX_BATCHES];

struct ScratchSlot {
    bool tried = false;
    unsigned char *ptr = nullptr;   // device address of `scratch` on this device
    std::string error;
};
std::mutex g_scratch_mu;
std::map<int, ScratchSlot> g_scratch;

// With `device` current: looks up the array's address on it and zeroes its
// look-back words (a fill kernel, waited for), once per device.  Every draw
// that uses look-back words clears the ones it used in its k_finish, so they
// are zero again at the start of the next call.
void scratch_setup(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchSlot &S = g_scratch[device];
    if (S.tried) return;
    S.tried = true;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        S.error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return;
    }
    unsigned long long *words = (unsigned long long *)((unsigned char *)p + 8ull * VR_NOALLOC_MAX_BATCHES);
    hipLaunchKernelGGL(k_fill_u64, dim3(256), dim3(256), 0, nullptr, words, (uint64_t)VR_NOALLOC_MAX_BATCHES, 0ull);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        S.error = std::string("clearing the look-back words: ") + hipGetErrorString(e);
        return;
    }
    S.ptr = (unsigned char *)p;
}

// The device address of `scratch` on `device`, or NULL (then *why is set).
unsigned char *scratch_ptr(int device, std::string *why) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(device);
    if (it == g_scratch.end() || !it->second.ptr) {
        *why = it == g_scratch.end() ? std::string("not set up") : it->second.error;
        return nullptr;
    }
    return it->second.ptr;
}

// The aligned check and next() for the primitive-cap class TMC.
template <uint32_t TMC>
void launch_plan_first(vr_ctx *c, const PlanArgs &P, uint32_t K, uint32_t *d_plan) {
    using W = NextClass<TMC>;
    hipLaunchKernelGGL(k_plan_check<TMC>, dim3(K), dim3(CheckClass<TMC>::threads), 0, c->stream, P, d_plan);
    hipLaunchKernelGGL(k_plan_next<TMC>, dim3((P.T + W::starts - 1) / W::starts), dim3(W::threads), W::lds,
                       c->stream, P);
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
    while (L < tmax) L <<= 1;
    const uint32_t nseg = (T + L - 1) / L;
    const uint32_t fan = plan_fan_in(tmax);
    std::vector<uint32_t> counts{nseg};
    while (counts.back() > fan) counts.push_back((counts.back() + fan - 1) / fan);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t bytes = al(4ull * T);
    std::vector<size_t> tab_off, ent_off, pre_off;
    for (size_t l = 0; l < counts.size(); ++l) {
        const uint32_t cnt = counts[l];
        tab_off.push_back(bytes);
        bytes += al(2ull * cnt * tmax);
        ent_off.push_back(bytes);
        bytes += al(2ull * cnt);
        pre_off.push_back(bytes);   // member entries, for the levels that are composed
        if (l + 1 < counts.size()) bytes += al(2ull * cnt * tmax);
    }
    vr_status st = ensure(c, c->plan_work, bytes);
    if (st != VR_OK) return st;
    // words tagged with a planning call's epoch: only ever written by the
    // planner, zeroed when allocated, so no stale word carries a later epoch
    st = ensure(c, c->plan_status, 8ull * nseg, /*zero=*/true);
    if (st != VR_OK) return st;
    unsigned char *base = (unsigned char *)c->plan_work.ptr;
    uint32_t *next = (uint32_t *)base;
    auto tab = [&](size_t l) { return (uint16_t *)(base + tab_off[l]); };
    auto ent = [&](size_t l) { return (uint16_t *)(base + ent_off[l]); };
    auto pre = [&](size_t l) { return (uint16_t *)(base + pre_off[l]); };
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
    P.fail = &c->d_words->plan_fail;
    if (++c->plan_epoch == 0) c->plan_epoch = 1;
    P.epoch = c->plan_epoch;
    TimedRegion timed(c);
    const uint32_t K = (T + tmax - 1) / tmax;
    switch (plan_class(tmax)) {
    case 256: launch_plan_first<256>(c, P, K, d_plan); break;
    case 512: launch_plan_first<512>(c, P, K, d_plan); break;
    case 1024: launch_plan_first<1024>(c, P, K, d_plan); break;
    case 2048: launch_plan_first<2048>(c, P, K, d_plan); break;
    default: launch_plan_first<4096>(c, P, K, d_plan); break;
    }
    hipLaunchKernelGGL(k_plan_table, dim3(nseg), dim3(256), 4 * L, c->stream, P, tab(0));
    const uint32_t grp_lds = 2 * fan * tmax;
    for (size_t l = 0; l + 1 < counts.size(); ++l)
        hipLaunchKernelGGL(k_plan_compose, dim3(counts[l + 1]), dim3(512), grp_lds, c->stream, tmax, counts[l],
                           (const uint16_t *)tab(l), tab(l + 1), pre(l), (const uint32_t *)P.fail, P.epoch);
    const size_t top = counts.size() - 1;
    // with two levels every emit block walks the (at most fan) level-1
    // tables before its group itself, so the top kernel is not launched
    const uint32_t emit_mode = top == 0 ? 0u : (top == 1 ? 2u : 1u);
    if (emit_mode != 2)
        hipLaunchKernelGGL(k_plan_top, dim3(1), dim3(256), 2 * counts[top] * tmax, c->stream, tmax, counts[top],
                           (const uint16_t *)tab(top), ent(top), (const uint32_t *)P.fail, P.epoch);
    for (size_t l = top; l-- > 1;)
        hipLaunchKernelGGL(k_plan_resolve, dim3((counts[l] + 255) / 256), dim3(256), 0, c->stream, tmax, counts[l],
                           (const uint16_t *)pre(l), (const uint16_t *)ent(l + 1), ent(l), (const uint32_t *)P.fail,
                           P.epoch);
    // level 0: entries, batch starts and packing in one launch
    const uint16_t *up = emit_mode == 0 ? ent(0) : (emit_mode == 1 ? ent(1) : tab(1));
    const uint32_t emit_lds = 8 * L + (emit_mode == 2 ? 2 * counts[1] * tmax : 0u);
    hipLaunchKernelGGL(k_plan_emit, dim3(nseg), dim3(256), emit_lds, c->stream, P,
                       (const uint16_t *)(emit_mode == 0 ? nullptr : pre(0)), up, emit_mode,
                       (unsigned long long *)c->plan_status.ptr, d_plan);
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
    uint32_t *d_order = nullptr, *d_unit_base = nullptr, *d_slot_base = nullptr;
    unsigned long long *d_agg = nullptr, *d_dtot = nullptr;
    std::vector<vr::FrameVariant> variants;
    bool index_error = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// The frame kernels: unit bases in variant order, one persistent kernel per
// variant, per-draw counters and (when total_inv is not NULL) the frame's
// invocation total.
struct FrameLaunch {
    const DrawDesc *draws;
    const uint32_t *order;
    uint32_t n;
    const vr_shader_params *shaders;
    uint32_t *unit_base, *slot_base;
    unsigned long long *agg, *dtot;
    const FrameVariant *variants;
    uint32_t num_variants;
    uint32_t *err;
    unsigned long long *total_inv;
};

template <int MODE, int KIND, bool OCC>
void launch_frame_variant(const FrameLaunch &L, const FrameVariant &v, hipStream_t s) {
    hipLaunchKernelGGL((k_frame<MODE, KIND, OCC>), dim3(v.grid), dim3(kFrameNT), v.lds_total, s, L.draws, L.order,
                       v.lo, v.hi, L.shaders, (const uint32_t *)L.unit_base, (const uint32_t *)L.slot_base, L.agg,
                       v.unit_lds, v.ballot_stride, L.err, L.total_inv);
}

template <int MODE, int KIND, bool OCC>
int frame_variant_occupancy(uint32_t lds) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_frame<MODE, KIND, OCC>, kFrameNT, lds) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu;
}

template <int MODE, int KIND, bool OCC>
int frame_variant_kind(const FrameLaunch *L, const FrameVariant &v, hipStream_t s, bool launch) {
    return launch ? (launch_frame_variant<MODE, KIND, OCC>(*L, v, s), 0)
                  : frame_variant_occupancy<MODE, KIND, OCC>(v.lds_total);
}

// Resident workgroups per CU of a variant's kernel (launch = false), or its
// launch (launch = true); mode, kind and the occupancy bound (hashing modes
// only) select the instantiation.
template <int MODE>
int frame_variant_mode(const FrameLaunch *L, const FrameVariant &v, hipStream_t s, bool launch) {
    constexpr bool kHashing = MODE == kFrameHash || MODE == kFramePHash;
    if (kHashing && v.occ) {
        switch (v.kind) {
        case 0: return frame_variant_kind<MODE, 0, kHashing>(L, v, s, launch);
        case 1: return frame_variant_kind<MODE, 1, kHashing>(L, v, s, launch);
        default: return frame_variant_kind<MODE, 2, kHashing>(L, v, s, launch);
        }
    }
    switch (v.kind) {
    case 0: return frame_variant_kind<MODE, 0, false>(L, v, s, launch);
    case 1: return frame_variant_kind<MODE, 1, false>(L, v, s, launch);
    default: return frame_variant_kind<MODE, 2, false>(L, v, s, launch);
    }
}

int frame_variant_dispatch(const FrameLaunch *L, const FrameVariant &v, hipStream_t s, bool launch) {
    switch (v.mode) {
    case kFrameSort: return frame_variant_mode<kFrameSort>(L, v, s, launch);
    case kFrameHash: return frame_variant_mode<kFrameHash>(L, v, s, launch);
    case kFramePHash: return frame_variant_mode<kFramePHash>(L, v, s, launch);
    case kFrameBallot: return frame_variant_mode<kFrameBallot>(L, v, s, launch);
    default: return frame_variant_mode<kFrameNaive>(L, v, s, launch);
    }
}

void enqueue_frame_kernels(const FrameLaunch &L, hipStream_t s) {
    if (L.n == 0) return;
    hipLaunchKernelGGL(k_frame_prepare, dim3(1), dim3(1024), 0, s, L.draws, L.order, L.n, L.unit_base, L.slot_base,
                       L.err);
    for (uint32_t i = 0; i < L.num_variants; ++i) frame_variant_dispatch(&L, L.variants[i], s, true);
    hipLaunchKernelGGL(k_frame_finish, dim3((L.n + 15) / 16), dim3(1024), 0, s, L.draws, L.order, L.n,
                       (const uint32_t *)L.slot_base, (const unsigned long long *)L.agg, L.dtot);
    if (L.total_inv)
        hipLaunchKernelGGL(k_frame_total, dim3(1), dim3(1024), 0, s, (const unsigned long long *)L.dtot, L.n,
                           L.total_inv);
}

void frame_enqueue(vr_frame *f, hipStream_t s) {
    vr_ctx *c = f->c;
    FrameLaunch L{f->d_draws, f->d_order, f->n, f->d_shaders, f->d_unit_base, f->d_slot_base, f->d_agg,
                  f->d_dtot, f->variants.data(), (uint32_t)f->variants.size(), &c->d_words->err,
                  &c->d_words->total_inv};
    enqueue_frame_kernels(L, s);
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

// Per-frame LDS and aggregate needs, accumulated over its draws.
struct FrameNeeds {
    uint64_t slots = 0, units = 0;
    uint32_t unit_lds = 256 * 48, ballot_stride = 0;
    bool index_error = false;
    uint32_t lds_total(uint32_t n) const {
        return align16(std::max(unit_lds, 4 * ballot_stride)) + 4 * (n + 1);
    }
    void merge(const FrameNeeds &o) {
        slots += o.slots;
        units += o.units;
        unit_lds = std::max(unit_lds, o.unit_lds);
        ballot_stride = std::max(ballot_stride, o.ballot_stride);
        index_error = index_error || o.index_error;
    }
};

// Validates one frame entry and fills its device descriptor.
vr_status describe_draw(vr_ctx *c, const vr_draw &D, const vr_shader_params &sh, uint32_t d, DrawDesc &X,
                        FrameNeeds &need) {
    vr_opts o{};
    o.max_unique = D.max_unique;
    o.d_plan = D.d_plan;
    vr_outputs ov{};
    ov.corners = D.d_corners;
    ov.counters = D.d_counters;
    Resolved r;
    vr_status st = check_args(c, D.num_indices, D.num_vertices, &sh, D.strategy, D.batch_tris, &o, &ov, &r);
    if (st != VR_OK) return fail(c, st, "draw %u: %s", d, c->error.c_str());
    if (D.strategy == VR_MULTI)
        return fail(c, VR_ERR_ARG, "draw %u: MULTI (two passes over the vertex buffer) cannot join a frame", d);
    const uint64_t T = D.num_indices / 3;
    if (T && (!D.d_indices || !D.d_vertices || !D.d_corners))
        return fail(c, VR_ERR_ARG, "draw %u: indices, vertices and corners are required", d);
    if (((uintptr_t)D.d_vertices & 15) || ((uintptr_t)D.d_corners & 15))
        return fail(c, VR_ERR_ARG, "draw %u: vertices and corners must be 16-byte aligned", d);
    if (is_dynamic(D.strategy) && T && !D.d_plan)
        return fail(c, VR_ERR_ARG, "draw %u: a dynamic draw in a frame needs its plan", d);
    if (T && D.num_vertices == 0) need.index_error = true;
    X = DrawDesc{};
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
    X.kind = sh.kind;
    X.max_idx = r.max_idx;
    X.max_uniq = r.max_uniq;
    X.hash_bits = r.hash_bits;
    X.probes = r.probes;
    if (X.mode == kFrameNaive) {
        need.slots += (3 * T + 255) / 256;
        need.units += (3 * T + 255) / 256;
    } else {
        const uint64_t nb = is_dynamic(D.strategy) ? dyn_batch_bound(T, r.nu, D.batch_tris) : X.num_batches;
        X.slot_cap = (uint32_t)std::min<uint64_t>(nb, 0xFFFFFFFFull);
        need.slots += nb;
        if (X.mode == kFrameBallot) {
            need.units += (nb + 3) / 4;
            need.ballot_stride = std::max(need.ballot_stride, align16(ballot_lds_bytes(D.batch_tris)));
        } else {
            need.units += nb;
            // the frame kernel runs every unit with kFrameNT threads
            const uint32_t per = X.mode == kFrameSort ? 8u : 32u;
            if (r.max_idx > per * kFrameNT)
                return fail(c, VR_ERR_ARG, "draw %u: batches of %u triangles are too large for a frame", d,
                            D.batch_tris);
            need.unit_lds = std::max(need.unit_lds, dedup_lds_layout((int)X.mode, r.max_idx, r.max_uniq, r.hash_bits,
                                                                     kFrameNT, r.max_uniq).total);
        }
    }
    return VR_OK;
}

// Groups the described draws by variant (dedup mode and vertex program):
// `order` lists the table positions variant by variant (stable), and every
// variant gets its kernel's LDS and a grid of at most one chunk of units per
// workgroup and the CUs' resident workgroups.  VR_ERR_ARG when a variant
// needs more LDS than a workgroup has.
vr_status frame_variants(vr_ctx *c, const DrawDesc *desc, const FrameNeeds *needs, uint32_t n,
                         std::vector<uint32_t> &order, std::vector<FrameVariant> &vars,
                         std::map<uint64_t, int> *occ_cache) {
    order.resize(n);
    for (uint32_t d = 0; d < n; ++d) order[d] = d;
    auto key = [&](uint32_t d) { return desc[d].mode * 3 + desc[d].kind; };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key(a) < key(b); });
    vars.clear();
    for (uint32_t lo = 0; lo < n;) {
        uint32_t hi = lo + 1;
        while (hi < n && key(order[hi]) == key(order[lo])) ++hi;
        FrameNeeds need;
        for (uint32_t k = lo; k < hi; ++k) need.merge(needs[order[k]]);
        FrameVariant v{};
        v.mode = desc[order[lo]].mode;
        v.kind = desc[order[lo]].kind;
        v.lo = lo;
        v.hi = hi;
        v.ballot_stride = need.ballot_stride;
        v.unit_lds = align16(std::max(need.unit_lds, 4 * need.ballot_stride));
        v.lds_total = need.lds_total(hi - lo);
        if (v.lds_total > c->lds_limit)
            return fail(c, VR_ERR_ARG, "frame variant needs %u B of LDS per workgroup (limit %zu)", v.lds_total,
                        c->lds_limit);
        // hashing variants take the occupancy-bound kernel when eight
        // workgroups (eight wavefronts per SIMD) fit in the LDS
        v.occ = (v.mode == kFrameHash || v.mode == kFramePHash) && 8ull * (v.lds_total + 64u) <= c->lds_limit;
        const uint64_t ck = ((uint64_t)(v.mode * 3 + v.kind) << 32) | v.lds_total;
        int per_cu;
        auto it = occ_cache ? occ_cache->find(ck) : std::map<uint64_t, int>::iterator();
        if (occ_cache && it != occ_cache->end()) {
            per_cu = it->second;
        } else {
            per_cu = frame_variant_dispatch(nullptr, v, nullptr, false);
            if (occ_cache) (*occ_cache)[ck] = per_cu;
        }
        const uint64_t want = std::max<uint64_t>(1, (need.units + frame_chunk(v.mode) - 1) / frame_chunk(v.mode));
        v.grid = (uint32_t)std::min<uint64_t>(want, (uint64_t)std::max(1, c->num_cus * per_cu));
        vars.push_back(v);
        lo = hi;
    }
    return VR_OK;
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
    scratch_setup(device);   // a failure is reported by vr_process_draw_noalloc
    *out = c;
    return VR_OK;
}

void vr_destroy(vr_ctx *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (Scratch *s : {&c->status, &c->agg, &c->plan, &c->plan_work, &c->tune, &c->shaded, &c->plan_status})
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
    return check_args(nullptr, num_indices, num_vertices, shader, strategy, batch_tris, opts, out, nullptr);
}

vr_status vr_plan_dynamic(vr_ctx *c, const uint32_t *d_indices, uint64_t num_indices, uint32_t num_vertices,
                          uint32_t max_unique, uint32_t max_tris, uint32_t *d_plan, uint64_t plan_cap) {
    if (!c) return VR_ERR_ARG;
    if (num_indices % 3 != 0 || num_indices > VR_MAX_INDICES)
        return fail(c, VR_ERR_ARG, "num_indices must be a multiple of 3 below 3*2^30");
    if (max_unique < 3 || max_unique > VR_MAX_UNIQUE)
        return fail(c, VR_ERR_ARG, "max_unique outside 3..%u", (unsigned)VR_MAX_UNIQUE);
    if (max_tris == 0 || max_tris > VR_MAX_BATCH_DYNAMIC)
        return fail(c, VR_ERR_ARG, "max_tris outside 1..%u", (unsigned)VR_MAX_BATCH_DYNAMIC);
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

}  // extern "C"

namespace {

// One draw (vr_process_draw).  With noalloc the per-batch aggregates and
// look-back words come from the static `scratch` array instead of context
// scratch, a dynamic draw must bring its plan, and nothing is allocated.
vr_status draw_impl(vr_ctx *c, const uint32_t *d_indices, uint64_t num_indices, const float *d_vertices,
                    uint32_t num_vertices, const vr_shader_params *shader, vr_strategy strategy, uint32_t batch_tris,
                    const vr_opts *opts, const vr_outputs *out, bool noalloc) {
    if (!c) return VR_ERR_ARG;
    Resolved r;
    vr_status st = check_args(c, num_indices, num_vertices, shader, strategy, batch_tris, opts, out, &r);
    if (st != VR_OK) return st;
    const uint64_t T = num_indices / 3;
    if (T && (!d_indices || !d_vertices)) return fail(c, VR_ERR_ARG, "indices or vertices are NULL");
    if (d_vertices && ((uintptr_t)d_vertices & 15)) return fail(c, VR_ERR_ARG, "vertices must be 16-byte aligned");
    if (out->corners && ((uintptr_t)out->corners & 15)) return fail(c, VR_ERR_ARG, "corners must be 16-byte aligned");
    if (out->verts && ((uintptr_t)out->verts & 15)) return fail(c, VR_ERR_ARG, "verts must be 16-byte aligned");
    // LDS of the dedup kernels: every unique vertex of a unit is kept when
    // corners are assembled, else an NT-row stage
    const int mode = (strategy == VR_STATIC_SORT || strategy == VR_DYN_SORT) ? kSort
                     : (strategy == VR_DYN_PHASH)                             ? kPHash
                                                                              : kHash;
    uint32_t lds = 0;
    bool stream = false;
    if (strategy != VR_NAIVE && strategy != VR_MULTI && !is_ballot(strategy)) {
        lds = dedup_lds_layout(mode, r.max_idx, r.max_uniq, r.hash_bits, r.nt, r.max_uniq).total;
        // indexed outputs only: shaded vertices stream out when keeping them all
        // would leave room for fewer than three workgroups per CU
        if (!out->corners && 3 * lds > c->lds_limit) {
            stream = true;
            lds = dedup_lds_layout(mode, r.max_idx, r.max_uniq, r.hash_bits, r.nt, r.nt).total;
        }
        if (lds > c->lds_limit)
            return fail(c, VR_ERR_ARG,
                        "LDS need %u B exceeds the %zu B limit (lower max_unique, batch_tris or hash_slots, or "
                        "request indexed outputs only)",
                        lds, c->lds_limit);
    }
    unsigned char *fixed = nullptr;   // the static scratch array on this device (noalloc)
    if (noalloc) {
        if (is_dynamic(strategy) && T && !(opts && opts->d_plan))
            return fail(c, VR_ERR_ARG, "an allocation-free dynamic draw needs opts->d_plan (vr_plan_dynamic)");
        if (strategy == VR_MULTI && T && !out->verts)
            return fail(c, VR_ERR_ARG, "an allocation-free MULTI draw needs out->verts for its shaded buffer");
        if (!is_dynamic(strategy) && strategy != VR_NAIVE && strategy != VR_MULTI &&
            (T + batch_tris - 1) / batch_tris > VR_NOALLOC_MAX_BATCHES)
            return fail(c, VR_ERR_CAPACITY, "%llu batches exceed the allocation-free limit of %u",
                        (unsigned long long)((T + batch_tris - 1) / batch_tris), (unsigned)VR_NOALLOC_MAX_BATCHES);
        if (is_dynamic(strategy) && dyn_batch_bound(T, r.nu, batch_tris) > VR_NOALLOC_MAX_BATCHES)
            return fail(c, VR_ERR_CAPACITY, "up to %llu dynamic batches exceed the allocation-free limit of %u",
                        (unsigned long long)dyn_batch_bound(T, r.nu, batch_tris), (unsigned)VR_NOALLOC_MAX_BATCHES);
        std::string why;
        fixed = scratch_ptr(c->device, &why);
        if (!fixed) return fail(c, VR_ERR_DEVICE, "allocation-free scratch unavailable: %s", why.c_str());
    }
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
    A.stream_verts = stream ? 1u : 0u;

    const vr_shader_params &sh = *shader;
    if (strategy == VR_MULTI) {
        f4 *shaded = (f4 *)out->verts;
        if (!shaded) {
            st = ensure(c, c->shaded, 48ull * num_vertices);
            if (st != VR_OK) return st;
            shaded = (f4 *)c->shaded.ptr;
        }
        TimedRegion timed(c, !noalloc);
        const dim3 gs((num_vertices + 255) / 256), ga((uint32_t)((3ull * T + 255) / 256));
        if (sh.kind == 0) hipLaunchKernelGGL(k_multi_shade<0>, gs, dim3(256), 0, c->stream, A, sh, shaded);
        else if (sh.kind == 1) hipLaunchKernelGGL(k_multi_shade<1>, gs, dim3(256), 0, c->stream, A, sh, shaded);
        else hipLaunchKernelGGL(k_multi_shade<2>, gs, dim3(256), 0, c->stream, A, sh, shaded);
        hipLaunchKernelGGL(k_multi_assemble, ga, dim3(256), 0, c->stream, A, (const f4 *)shaded);
        VR_HIP(c, hipGetLastError());
        return VR_OK;
    }
    if (strategy == VR_NAIVE) {
        TimedRegion timed(c, !noalloc);
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
    if (noalloc) {
        A.agg = (unsigned long long *)fixed;
        A.status = A.need_prefix ? (unsigned long long *)(fixed + 8ull * VR_NOALLOC_MAX_BATCHES) : nullptr;
        A.status_cap = (uint32_t)nb_bound;
    } else {
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
    }
    TimedRegion timed(c, !noalloc);
    if (is_ballot(strategy)) {
        const uint32_t lds = align16(ballot_lds_bytes(batch_tris));   // per wavefront
        if (sh.kind == 0) launch_ballot<0>(c, A, sh, lds, nb_bound);
        else if (sh.kind == 1) launch_ballot<1>(c, A, sh, lds, nb_bound);
        else launch_ballot<2>(c, A, sh, lds, nb_bound);
    } else {
        if (mode == kSort) dispatch_kind<kSort>(c, sh.kind, r.nt, A, sh, lds, nb_bound);
        else if (mode == kHash) dispatch_kind<kHash>(c, sh.kind, r.nt, A, sh, lds, nb_bound);
        else dispatch_kind<kPHash>(c, sh.kind, r.nt, A, sh, lds, nb_bound);
    }
    timed.done();
    const uint32_t fin = (uint32_t)std::min<uint64_t>(64, std::max<uint64_t>(1, (nb_bound + 2047) / 2048));
    hipLaunchKernelGGL(k_finish, dim3(fin), dim3(256), 0, c->stream, A.plan, A.num_batches, A.status_cap,
                       (const unsigned long long *)A.agg, A.status, A.counters, A.total_inv);
    VR_HIP(c, hipGetLastError());
    return VR_OK;
}

}  // namespace

extern "C" {

vr_status vr_process_draw(vr_ctx *c, const uint32_t *d_indices, uint64_t num_indices, const float *d_vertices,
                          uint32_t num_vertices, const vr_shader_params *shader, vr_strategy strategy,
                          uint32_t batch_tris, const vr_opts *opts, const vr_outputs *out) {
    return draw_impl(c, d_indices, num_indices, d_vertices, num_vertices, shader, strategy, batch_tris, opts, out,
                     false);
}

vr_status vr_process_draw_noalloc(vr_ctx *c, const uint32_t *d_indices, uint64_t num_indices,
                                  const float *d_vertices, uint32_t num_vertices, const vr_shader_params *shader,
                                  vr_strategy strategy, uint32_t batch_tris, const vr_opts *opts,
                                  const vr_outputs *out) {
    return draw_impl(c, d_indices, num_indices, d_vertices, num_vertices, shader, strategy, batch_tris, opts, out,
                     true);
}

// ---------------------------------------------------------------------------
// Streams: chunks drawn into a ring of corner slots, consumed by triangle
// setup on a second HIP stream; events order each slot's reuse.
// ---------------------------------------------------------------------------
struct vr_stream {
    vr_ctx *c = nullptr;
    hipStream_t cons = nullptr;
    uint32_t slots = 0, chunk_tris = 0, width = 0, height = 0;
    f4 *records = nullptr;
    uint64_t records_cap = 0;
    unsigned char *mem = nullptr;
    size_t slot_bytes = 0;
    unsigned long long *totals = nullptr;   // {visible, invocations, units, 0}
    std::vector<hipEvent_t> produced, consumed;
    std::vector<bool> used;
    uint64_t pushed = 0, next = 0;
};

namespace {
f4 *stream_corners(vr_stream *s, uint32_t k) { return (f4 *)(s->mem + k * s->slot_bytes); }
unsigned long long *stream_counters(vr_stream *s, uint32_t k) {
    return (unsigned long long *)(s->mem + k * s->slot_bytes + s->slot_bytes - 256);
}
void stream_release(vr_stream *s) {
    if (s->cons) (void)hipStreamSynchronize(s->cons);
    for (hipEvent_t e : s->produced) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->consumed) (void)hipEventDestroy(e);
    if (s->cons) (void)hipStreamDestroy(s->cons);
    if (s->mem) (void)hipFree(s->mem);
}
}  // namespace

vr_status vr_stream_create(vr_ctx *c, uint32_t slots, uint32_t chunk_tris, uint32_t width, uint32_t height,
                           float *d_records, uint64_t records_cap, vr_stream **out) {
    if (!c || !out) return VR_ERR_ARG;
    *out = nullptr;
    if (slots == 0 || slots > 8) return fail(c, VR_ERR_ARG, "slots %u outside 1..8", slots);
    if (chunk_tris == 0 || chunk_tris > (1u << 24)) return fail(c, VR_ERR_ARG, "chunk_tris outside 1..2^24");
    if (width == 0 || height == 0 || width > (1u << 24) || height > (1u << 24))
        return fail(c, VR_ERR_ARG, "viewport %ux%u outside 1..2^24", width, height);
    if (records_cap && (!d_records || ((uintptr_t)d_records & 15)))
        return fail(c, VR_ERR_ARG, "records must be a 16-byte aligned device buffer");
    DeviceGuard g(c->device);
    vr_stream *s = new vr_stream;
    s->c = c;
    s->slots = slots;
    s->chunk_tris = chunk_tris;
    s->width = width;
    s->height = height;
    s->records = (f4 *)d_records;
    s->records_cap = records_cap;
    s->slot_bytes = ((144ull * chunk_tris + 255) & ~(size_t)255) + 256;   // corners, then the draw's counters
    vr_status st = VR_OK;
    if (hipMalloc((void **)&s->mem, s->slot_bytes * slots + 256) != hipSuccess) {
        s->mem = nullptr;
        st = fail(c, VR_ERR_OOM, "stream slots: out of memory");
    } else if (hipStreamCreateWithFlags(&s->cons, hipStreamNonBlocking) != hipSuccess) {
        s->cons = nullptr;
        st = fail(c, VR_ERR_DEVICE, "stream: cannot create the consumer stream");
    }
    for (uint32_t k = 0; st == VR_OK && k < slots; ++k) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            st = fail(c, VR_ERR_DEVICE, "stream: cannot create events");
            break;
        }
        s->produced.push_back(a);
        s->consumed.push_back(b);
    }
    if (st == VR_OK) {
        s->totals = (unsigned long long *)(s->mem + s->slot_bytes * slots);
        if (hipMemsetAsync(s->totals, 0, 32, s->cons) != hipSuccess) st = fail(c, VR_ERR_DEVICE, "stream: memset");
    }
    if (st != VR_OK) {
        stream_release(s);
        delete s;
        return st;
    }
    s->used.assign(slots, false);
    *out = s;
    return VR_OK;
}

vr_status vr_stream_push(vr_stream *s, const uint32_t *d_indices, uint64_t num_indices, const float *d_vertices,
                         uint32_t num_vertices, const vr_shader_params *shader, vr_strategy strategy,
                         uint32_t batch_tris) {
    if (!s) return VR_ERR_ARG;
    vr_ctx *c = s->c;
    if (strategy != VR_NAIVE && strategy != VR_STATIC_BALLOT && strategy != VR_STATIC_SORT &&
        strategy != VR_STATIC_HASH)
        return fail(c, VR_ERR_ARG, "a stream takes NAIVE or STATIC_* (no analysis of the index buffer)");
    if (num_indices % 3) return fail(c, VR_ERR_ARG, "num_indices is not a multiple of 3");
    const uint64_t T = num_indices / 3;
    if (T > s->chunk_tris) return fail(c, VR_ERR_ARG, "chunk of %llu triangles above chunk_tris %u",
                                       (unsigned long long)T, s->chunk_tris);
    if (s->pushed + T > s->records_cap)
        return fail(c, VR_ERR_CAPACITY, "records_cap %llu below %llu triangles", (unsigned long long)s->records_cap,
                    (unsigned long long)(s->pushed + T));
    DeviceGuard g(c->device);
    const uint32_t k = (uint32_t)(s->next % s->slots);
    if (s->used[k]) VR_HIP(c, hipStreamWaitEvent(c->stream, s->consumed[k], 0));   // the consumer is done with it
    vr_outputs out{};
    out.corners = (float *)stream_corners(s, k);
    out.counters = (uint64_t *)stream_counters(s, k);
    vr_status st = vr_process_draw(c, d_indices, num_indices, d_vertices, num_vertices, shader, strategy, batch_tris,
                                   nullptr, &out);
    if (st != VR_OK) return st;
    VR_HIP(c, hipEventRecord(s->produced[k], c->stream));
    VR_HIP(c, hipStreamWaitEvent(s->cons, s->produced[k], 0));
    if (T)
        hipLaunchKernelGGL(k_setup, dim3((uint32_t)((T + 255) / 256)), dim3(256), 0, s->cons,
                           (const f4 *)stream_corners(s, k), (uint32_t)T, s->width, s->height,
                           s->records + 2 * s->pushed, (const unsigned long long *)stream_counters(s, k), s->totals);
    VR_HIP(c, hipGetLastError());
    VR_HIP(c, hipEventRecord(s->consumed[k], s->cons));
    s->used[k] = true;
    ++s->next;
    s->pushed += T;
    return VR_OK;
}

vr_status vr_stream_finish(vr_stream *s, uint64_t *h_triangles, uint64_t *h_visible, uint64_t *h_invocations) {
    if (!s) return VR_ERR_ARG;
    vr_ctx *c = s->c;
    DeviceGuard g(c->device);
    VR_HIP(c, hipStreamSynchronize(c->stream));
    VR_HIP(c, hipStreamSynchronize(s->cons));
    unsigned long long t[4] = {0, 0, 0, 0};
    VR_HIP(c, hipMemcpy(t, s->totals, sizeof t, hipMemcpyDeviceToHost));
    if (h_triangles) *h_triangles = s->pushed;
    if (h_visible) *h_visible = t[0];
    if (h_invocations) *h_invocations = t[1];
    return VR_OK;
}

void vr_stream_destroy(vr_stream *s) {
    if (!s) return;
    DeviceGuard g(s->c->device);
    (void)hipStreamSynchronize(s->c->stream);
    stream_release(s);
    delete s;
}

vr_status vr_walk_step(vr_ctx *c, const uint32_t *d_keys_in, uint32_t num_agents, const float *d_activity,
                       uint32_t grid, const int8_t *d_moves, const float *d_weights, uint32_t num_moves,
                       const float *d_uniforms, vr_strategy strategy, uint32_t batch_agents, uint32_t *d_keys_out,
                       uint64_t *d_counters) {
    if (!c) return VR_ERR_ARG;
    if (grid == 0 || grid > 32768) return fail(c, VR_ERR_ARG, "grid %u outside 1..32768", grid);
    if (num_moves == 0 || num_moves > 65535) return fail(c, VR_ERR_ARG, "num_moves %u outside 1..65535", num_moves);
    if (strategy != VR_NAIVE && strategy != VR_STATIC_HASH)
        return fail(c, VR_ERR_ARG, "a walk step takes NAIVE or STATIC_HASH");
    if (strategy == VR_STATIC_HASH && (batch_agents == 0 || batch_agents > kWalkMaxBatch))
        return fail(c, VR_ERR_ARG, "batch_agents %u outside 1..%u", batch_agents, kWalkMaxBatch);
    if (num_agents && (!d_keys_in || !d_keys_out || !d_activity || !d_moves || !d_weights || !d_uniforms))
        return fail(c, VR_ERR_ARG, "a walk buffer is NULL");
    DeviceGuard g(c->device);
    if (num_agents == 0) {
        hipLaunchKernelGGL(k_empty_draw, dim3(1), dim3(64), 0, c->stream, (unsigned long long *)d_counters,
                           (uint32_t *)nullptr);
        VR_HIP(c, hipGetLastError());
        return VR_OK;
    }
    WalkArgs W{};
    W.keys_in = d_keys_in;
    W.keys_out = d_keys_out;
    W.activity = d_activity;
    W.moves = d_moves;
    W.weights = d_weights;
    W.uniforms = d_uniforms;
    W.n = num_agents;
    W.grid = grid;
    W.num_moves = num_moves;
    W.batch = batch_agents;
    W.counters = (unsigned long long *)d_counters;
    W.total_inv = &c->d_words->total_inv;
    W.err = &c->d_words->err;
    if (strategy == VR_NAIVE) {
        TimedRegion timed(c);
        hipLaunchKernelGGL(k_walk_naive, dim3((num_agents + 255) / 256), dim3(256), 0, c->stream, W);
        VR_HIP(c, hipGetLastError());
        return VR_OK;
    }
    const uint32_t nb = (num_agents + batch_agents - 1) / batch_agents;
    vr_status st = ensure(c, c->agg, 8ull * nb);
    if (st != VR_OK) return st;
    W.agg = (unsigned long long *)c->agg.ptr;
    TimedRegion timed(c);
    hipLaunchKernelGGL(k_walk_hash<kWalkThreads>, dim3(nb), dim3(kWalkThreads), 0, c->stream, W);
    timed.done();
    const uint32_t fin = std::min<uint32_t>(64, std::max<uint32_t>(1, (nb + 2047) / 2048));
    hipLaunchKernelGGL(k_finish, dim3(fin), dim3(256), 0, c->stream, (const uint32_t *)nullptr, nb, nb,
                       (const unsigned long long *)W.agg, (unsigned long long *)nullptr, W.counters, W.total_inv);
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
    std::vector<FrameNeeds> needs(n);
    FrameNeeds need;
    for (uint32_t d = 0; d < n; ++d) {
        if (draws[d].shader >= ns) return fail(c, VR_ERR_ARG, "draw %u: shader %u out of range", d, draws[d].shader);
        vr_status st = describe_draw(c, draws[d], shaders[draws[d].shader], d, desc[d], needs[d]);
        if (st != VR_OK) return st;
        need.merge(needs[d]);
    }
    DeviceGuard g(c->device);
    std::vector<uint32_t> order;
    std::vector<FrameVariant> vars;
    vr_status vst = frame_variants(c, desc.data(), needs.data(), n, order, vars, nullptr);
    if (vst != VR_OK) return vst;
    const uint64_t slots = need.slots;
    const bool index_error = need.index_error;

    vr_frame *f = new vr_frame();
    f->c = c;
    f->n = n;
    f->variants = vars;
    f->index_error = index_error;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_draws = 0, o_sh = al(sizeof(DrawDesc) * n), o_ord = o_sh + al(sizeof(vr_shader_params) * ns),
                 o_ub = o_ord + al(4ull * n), o_sb = o_ub + al(4ull * (n + 1)), o_agg = o_sb + al(4ull * (n + 1)),
                 o_dt = o_agg + al(8 * (slots + 1)), total = o_dt + al(8ull * (n + 1));
    if (hipMalloc(&f->mem, total) != hipSuccess) {
        delete f;
        return fail(c, VR_ERR_OOM, "frame allocation of %zu bytes failed", total);
    }
    unsigned char *m = (unsigned char *)f->mem;
    f->d_draws = (DrawDesc *)(m + o_draws);
    f->d_shaders = (vr_shader_params *)(m + o_sh);
    f->d_order = (uint32_t *)(m + o_ord);
    f->d_unit_base = (uint32_t *)(m + o_ub);
    f->d_slot_base = (uint32_t *)(m + o_sb);
    f->d_agg = (unsigned long long *)(m + o_agg);
    f->d_dtot = (unsigned long long *)(m + o_dt);
    hipError_t e = hipSuccess;
    if (n) e = hipMemcpy(f->d_draws, desc.data(), sizeof(DrawDesc) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess && n) e = hipMemcpy(f->d_shaders, shaders, sizeof(vr_shader_params) * ns, hipMemcpyHostToDevice);
    if (e == hipSuccess && n) e = hipMemcpy(f->d_order, order.data(), 4ull * n, hipMemcpyHostToDevice);
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
        if (check_args(c, num_indices, V, sh, k.strategy, k.batch_tris, &o, &out, &r) != VR_OK) continue;
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
        // the fastest repetition: the least disturbed by other work on the device
        float fastest = -1.0f;
        for (size_t j = first; j < c->ev_used; ++j) {
            float ms = 0.0f;
            VR_HIP(c, hipEventElapsedTime(&ms, c->ev_pool[j].first, c->ev_pool[j].second));
            if (fastest < 0.0f || ms < fastest) fastest = ms;
        }
        const size_t timed = c->ev_used - first;
        c->ev_used = first;
        if (!ok || timed == 0) continue;
        VR_HIP(c, hipMemcpy(&k.invocations, counters, sizeof(uint64_t), hipMemcpyDeviceToHost));
        k.kernel_ms = fastest;
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

vr_status vr_math_selftest(vr_ctx *c, uint32_t fn, uint64_t first, uint64_t count, float *d_out,
                           uint64_t *h_mismatches) {
    if (!c) return VR_ERR_ARG;
    if (!h_mismatches || fn > 2 || first > (1ull << 32) || count > (1ull << 32) - first)
        return fail(c, VR_ERR_ARG, "math self-test: bad arguments (fn %u, first %llu, count %llu)", fn,
                    (unsigned long long)first, (unsigned long long)count);
    DeviceGuard g(c->device);
    vr_status st = ensure(c, c->selftest, sizeof(unsigned long long));
    if (st != VR_OK) return st;
    auto *d_cnt = (unsigned long long *)c->selftest.ptr;
    VR_HIP(c, hipMemsetAsync(d_cnt, 0, sizeof *d_cnt, c->stream));
    const uint64_t per = 1ull << 30;   // operands per launch
    for (uint64_t done = 0; done < count; done += per) {
        const uint64_t n = std::min(per, count - done);
        hipLaunchKernelGGL(k_math_selftest, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, fn,
                           first + done, n, d_out ? d_out + done : nullptr, d_cnt);
        VR_HIP(c, hipGetLastError());
    }
    unsigned long long h = 0;
    VR_HIP(c, hipMemcpyAsync(&h, d_cnt, sizeof h, hipMemcpyDeviceToHost, c->stream));
    VR_HIP(c, hipStreamSynchronize(c->stream));
    *h_mismatches = h;
    return VR_OK;
}

const char *vr_last_error(const vr_ctx *c) { return c ? c->error.c_str() : g_create_error.c_str(); }

}  // extern "C"

// ===========================================================================
// Request server
// ===========================================================================
namespace {

__global__ __launch_bounds__(256) void k_index_max(const uint32_t *idx, uint64_t n, uint32_t *out) {
    __shared__ uint32_t tmp[256 / kWave];
    uint32_t m = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        m = max(m, idx[i]);
    m = block_reduce_max<256>(m, tmp);
    if (threadIdx.x == 0) atomicMax(out, m);
}

struct ServerMesh {
    const uint32_t *idx = nullptr;
    const float *vtx = nullptr;
    uint32_t T = 0, V = 0;
    std::map<uint64_t, uint32_t *> plans;   // (max_unique << 32 | batch_tris) -> plan of the whole mesh
};

struct ServerReq {
    uint32_t mesh, num_tris, batch_tris, nu;
    vr_strategy strategy;
    vr_shader_params shader;
    uint64_t inv = 0, units = 0;   // from the tick's counters
};

// Byte offsets of a tick's staging for n draws.  The head [0, cnt) is
// uploaded (draw table, shader table, zeroed words), [words, end) is read
// back (error word and per-draw counters); bases and totals follow.
struct TickLayout {
    size_t sh, ord, words, cnt, end, ubase, sbase, dtot, total;
    explicit TickLayout(uint32_t n) {
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        sh = al(sizeof(DrawDesc) * n);
        ord = sh + al(sizeof(vr_shader_params) * n);
        words = ord + al(4ull * n);
        cnt = words + 256;
        end = cnt + al(32ull * n);
        ubase = end;
        sbase = ubase + al(4ull * (n + 1));
        dtot = sbase + al(4ull * (n + 1));
        total = dtot + al(8ull * n);
    }
};

// Staging of one tick; reused by the tick max_inflight later, which is only
// formed after this one retired.
struct TickSlot {
    hipEvent_t done = nullptr;
    unsigned char *host = nullptr;   // pinned
    unsigned char *dev = nullptr;
    unsigned long long *agg = nullptr;
    size_t agg_cap = 0;
    uint32_t n = 0;
    int launch_status = VR_OK;   // a tick that failed to launch retires with this
};

}  // namespace

struct vr_server {
    int device = 0;
    hipStream_t stream = nullptr;
    vr_ctx *ctx = nullptr;   // plans are built through it, on the server's stream
    vr_server_config cfg{};
    unsigned char *arena = nullptr;
    uint32_t *d_word = nullptr;
    std::vector<TickSlot> slots;
    std::map<uint64_t, int> per_cu;   // (variant, LDS bytes) -> resident frame workgroups per CU
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    sched::Scheduler *sch = nullptr;
    std::unordered_map<uint64_t, ServerReq> reqs;
    std::vector<ServerMesh> meshes;
    std::deque<uint64_t> done;   // finished, not yet polled
    uint64_t plan_bytes = 0;
    bool stop = false;
    std::string error;
    std::chrono::steady_clock::time_point t0;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

vr_status server_fail(vr_server *s, vr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s->error = buf;
    return st;
}

// Plan of the whole mesh for (nu, batch_tris), built on first use.  Called
// by the scheduler thread with the lock held.
uint32_t *server_plan(vr_server *s, ServerMesh &M, uint32_t nu, uint32_t bt) {
    const uint64_t key = (uint64_t)nu << 32 | bt;
    auto it = M.plans.find(key);
    if (it != M.plans.end()) return it->second;
    uint32_t *plan = nullptr;
    const size_t bytes = 4ull * (M.T + 2);
    if (hipMalloc((void **)&plan, bytes) != hipSuccess) return nullptr;
    if (vr_plan_dynamic(s->ctx, M.idx, 3ull * M.T, M.V, nu, bt, plan, M.T + 2) != VR_OK) {
        (void)hipFree(plan);
        return nullptr;
    }
    s->plan_bytes += bytes;
    M.plans[key] = plan;
    return plan;
}

// Enqueues one tick over `jobs` (lock held).  A job that cannot be described
// is finished with its error and processed as an empty draw.
vr_status server_launch(vr_server *s, uint32_t tick, const std::vector<uint64_t> &jobs) {
    vr_ctx *c = s->ctx;
    TickSlot &S = s->slots[tick % s->slots.size()];
    const uint32_t n = (uint32_t)jobs.size();
    const TickLayout L(n);
    DrawDesc *hd = (DrawDesc *)S.host;
    vr_shader_params *hs = (vr_shader_params *)(S.host + L.sh);
    memset(S.host + L.words, 0, 256);
    unsigned long long *dcnt = (unsigned long long *)(S.dev + L.cnt);
    FrameNeeds need;
    std::vector<FrameNeeds> needs(n);
    for (uint32_t d = 0; d < n; ++d) {
        sched::Job *j = s->sch->find(jobs[d]);
        const ServerReq &R = s->reqs[jobs[d]];
        ServerMesh &M = s->meshes[R.mesh];
        hs[d] = R.shader;
        vr_draw D{};
        D.d_indices = M.idx;
        D.num_indices = 3ull * R.num_tris;
        D.d_vertices = M.vtx;
        D.num_vertices = M.V;
        D.shader = d;
        D.strategy = R.strategy;
        D.batch_tris = R.batch_tris;
        D.max_unique = R.nu;
        D.d_corners = (float *)(s->arena + j->off);
        D.d_counters = (uint64_t *)(dcnt + 4ull * d);
        if (is_dynamic(R.strategy) && R.num_tris) {
            D.d_plan = server_plan(s, M, R.nu, R.batch_tris);
            if (!D.d_plan) {
                j->status = VR_ERR_OOM;
                D.num_indices = 0;
            }
        }
        if (describe_draw(c, D, hs[d], d, hd[d], needs[d]) != VR_OK) {
            if (j->status == VR_OK) j->status = VR_ERR_ARG;
            D.num_indices = 0;
            D.d_plan = nullptr;
            needs[d] = FrameNeeds();
            if (describe_draw(c, D, hs[d], d, hd[d], needs[d]) != VR_OK) return VR_ERR_ARG;
        }
        need.merge(needs[d]);
    }
    std::vector<uint32_t> order;
    std::vector<FrameVariant> vars;
    if (frame_variants(c, hd, needs.data(), n, order, vars, &s->per_cu) != VR_OK)
        return server_fail(s, VR_ERR_ARG, "%s", c->error.c_str());
    if (n) memcpy(S.host + L.ord, order.data(), 4ull * n);
    if (need.slots + 1 > S.agg_cap) {
        if (S.agg) (void)hipFree(S.agg);
        S.agg = nullptr;
        S.agg_cap = std::max<size_t>(need.slots + 1, 2 * S.agg_cap);
        if (hipMalloc((void **)&S.agg, 8 * S.agg_cap) != hipSuccess) {
            S.agg_cap = 0;
            return server_fail(s, VR_ERR_OOM, "tick aggregates: out of memory");
        }
    }
    CtxWords *dw = (CtxWords *)(S.dev + L.words);
    FrameLaunch F{(const DrawDesc *)S.dev, (const uint32_t *)(S.dev + L.ord), n,
                  (const vr_shader_params *)(S.dev + L.sh), (uint32_t *)(S.dev + L.ubase),
                  (uint32_t *)(S.dev + L.sbase), S.agg, (unsigned long long *)(S.dev + L.dtot), vars.data(),
                  (uint32_t)vars.size(), &dw->err, &dw->total_inv};
    S.n = n;
    hipError_t e = hipMemcpyAsync(S.dev, S.host, L.cnt, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
        enqueue_frame_kernels(F, s->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(S.host + L.words, S.dev + L.words, L.end - L.words, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipEventRecord(S.done, s->stream);
    if (e != hipSuccess) return server_fail(s, VR_ERR_DEVICE, "tick launch: %s", hipGetErrorString(e));
    return VR_OK;
}

// Retires finished ticks, oldest first (lock held).  Returns true if any.
bool server_retire(vr_server *s) {
    bool any = false;
    while (s->sch->inflight() > 0) {
        const uint32_t tick = s->sch->oldest_tick();
        TickSlot &S = s->slots[tick % s->slots.size()];
        const hipError_t q = S.launch_status == VR_OK ? hipEventQuery(S.done) : hipSuccess;
        if (q == hipErrorNotReady) break;
        const double t = s->now();
        const std::vector<uint64_t> jobs = s->sch->oldest_jobs();
        const TickLayout L(S.n);
        const CtxWords *hw = (const CtxWords *)(S.host + L.words);
        const unsigned long long *hc = (const unsigned long long *)(S.host + L.cnt);
        int status = VR_OK;
        if (S.launch_status != VR_OK) {
            status = S.launch_status;
        } else if (q != hipSuccess) {
            status = VR_ERR_DEVICE;
            s->error = std::string("tick failed: ") + hipGetErrorString(q);
        } else if (hw->err) {
            status = (int)hw->err;
        }
        for (uint32_t d = 0; d < jobs.size() && status == VR_OK; ++d) {
            ServerReq &R = s->reqs[jobs[d]];
            R.inv = hc[4ull * d];
            R.units = hc[4ull * d + 1];
        }
        s->sch->retire_oldest(t, status);
        for (uint32_t d = 0; d < jobs.size(); ++d) s->done.push_back(jobs[d]);
        any = true;
    }
    return any;
}

}  // namespace

namespace {

// The scheduler thread: retire finished ticks, admit, launch; sleeps on the
// condition variable, waking every 20 us while ticks are in flight.
void server_loop(vr_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->m);
    std::vector<uint64_t> jobs;
    for (;;) {
        if (server_retire(s)) s->cv_done.notify_all();
        if (s->stop && s->sch->idle()) break;
        const double t = s->now();
        s->sch->admit(t);
        bool launched = false;
        uint32_t tick = 0;
        while (s->sch->next_tick(t, jobs, &tick)) {
            TickSlot &S = s->slots[tick % s->slots.size()];
            S.launch_status = VR_OK;
            const vr_status st = server_launch(s, tick, jobs);
            if (st != VR_OK) S.launch_status = st;
            launched = true;
        }
        if (launched) continue;
        if (s->sch->inflight() > 0) s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        else s->cv_work.wait(lk);
    }
    s->cv_done.notify_all();
}

void server_free(vr_server *s) {
    for (TickSlot &S : s->slots) {
        if (S.done) (void)hipEventDestroy(S.done);
        if (S.host) (void)hipHostFree(S.host);
        if (S.dev) (void)hipFree(S.dev);
        if (S.agg) (void)hipFree(S.agg);
    }
    for (ServerMesh &M : s->meshes)
        for (auto &kv : M.plans) (void)hipFree(kv.second);
    if (s->arena) (void)hipFree(s->arena);
    if (s->d_word) (void)hipFree(s->d_word);
    if (s->ctx) vr_destroy(s->ctx);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s->sch;
    delete s;
}

sched::Policy server_policy(const vr_server_config &cfg) {
    sched::Policy p;
    p.budget = cfg.budget_bytes;
    p.max_inflight = cfg.max_inflight;
    p.max_tick_draws = cfg.max_tick_draws;
    p.max_tick_tris = cfg.max_tick_tris;
    return p;
}

vr_status check_server_config(const vr_server_config *in, vr_server_config &cfg, std::string &why) {
    if (!in) {
        why = "config is NULL";
        return VR_ERR_ARG;
    }
    cfg = *in;
    if (cfg.max_inflight == 0) cfg.max_inflight = 2;
    if (cfg.max_tick_draws == 0) cfg.max_tick_draws = 1024;
    if (cfg.max_inflight > 8) {
        why = "max_inflight must be 1..8";
        return VR_ERR_ARG;
    }
    if (cfg.max_tick_draws > VR_MAX_FRAME_DRAWS) {
        why = "max_tick_draws must be 1..4096";
        return VR_ERR_ARG;
    }
    if (cfg.budget_bytes < sched::Arena::kGranule) {
        why = "budget_bytes below 256";
        return VR_ERR_ARG;
    }
    return VR_OK;
}

}  // namespace

extern "C" {

vr_status vr_server_create(int device, const vr_server_config *cfg_in, vr_server **out) {
    if (!out) return fail(nullptr, VR_ERR_ARG, "server pointer is NULL");
    *out = nullptr;
    vr_server_config cfg;
    std::string why;
    if (check_server_config(cfg_in, cfg, why) != VR_OK) return fail(nullptr, VR_ERR_ARG, "%s", why.c_str());
    vr_server *s = new vr_server();
    s->device = device;
    s->cfg = cfg;
    s->t0 = std::chrono::steady_clock::now();
    s->sch = new sched::Scheduler(server_policy(cfg));
    if (vr_create(&s->ctx, device, nullptr) != VR_OK) {
        server_free(s);
        return fail(nullptr, VR_ERR_DEVICE, "%s", vr_last_error(nullptr));
    }
    DeviceGuard g(device);
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        s->stream = nullptr;
        server_free(s);
        return fail(nullptr, VR_ERR_DEVICE, "stream creation failed");
    }
    vr_set_stream(s->ctx, s->stream);
    if (hipMalloc((void **)&s->arena, cfg.budget_bytes) != hipSuccess) {
        s->arena = nullptr;
        server_free(s);
        return fail(nullptr, VR_ERR_OOM, "arena of %llu bytes: out of memory", (unsigned long long)cfg.budget_bytes);
    }
    bool ok = hipMalloc((void **)&s->d_word, 256) == hipSuccess;
    const TickLayout L(cfg.max_tick_draws);
    s->slots.resize(cfg.max_inflight);
    for (TickSlot &S : s->slots) {
        if (!ok) break;
        ok = hipEventCreateWithFlags(&S.done, hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc((void **)&S.host, L.end, hipHostMallocDefault) == hipSuccess &&
             hipMalloc((void **)&S.dev, L.total) == hipSuccess;
    }
    if (!ok) {
        server_free(s);
        return fail(nullptr, VR_ERR_OOM, "server staging allocation failed");
    }
    s->worker = std::thread(server_loop, s);
    *out = s;
    return VR_OK;
}

vr_status vr_server_add_mesh(vr_server *s, const uint32_t *d_idx, uint64_t num_indices, const float *d_vtx,
                             uint32_t V, uint32_t *mesh) {
    if (!s || !mesh) return VR_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->m);
    if (num_indices % 3 != 0 || num_indices > VR_MAX_INDICES)
        return server_fail(s, VR_ERR_ARG, "num_indices must be a multiple of 3 below 3*2^30");
    if (num_indices && (!d_idx || !d_vtx)) return server_fail(s, VR_ERR_ARG, "indices or vertices are NULL");
    if ((uintptr_t)d_vtx & 15) return server_fail(s, VR_ERR_ARG, "vertices must be 16-byte aligned");
    if (s->meshes.size() >= (1u << 20)) return server_fail(s, VR_ERR_ARG, "too many meshes");
    if (num_indices) {
        // every index below V, checked once so that no request can fault
        DeviceGuard g(s->device);
        hipStream_t st = nullptr;
        uint32_t mx = 0;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMemsetAsync(s->d_word, 0, 4, st);
        if (e == hipSuccess) {
            const uint64_t blocks = std::min<uint64_t>(4096, (num_indices + 255) / 256);
            hipLaunchKernelGGL(k_index_max, dim3((uint32_t)blocks), dim3(256), 0, st, d_idx, num_indices, s->d_word);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&mx, s->d_word, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (st) (void)hipStreamDestroy(st);
        if (e != hipSuccess) return server_fail(s, VR_ERR_DEVICE, "index check: %s", hipGetErrorString(e));
        if (mx >= V) return server_fail(s, VR_ERR_INDEX_RANGE, "index %u >= num_vertices %u", mx, V);
    }
    ServerMesh M;
    M.idx = d_idx;
    M.vtx = d_vtx;
    M.T = (uint32_t)(num_indices / 3);
    M.V = V;
    *mesh = (uint32_t)s->meshes.size();
    s->meshes.push_back(std::move(M));
    return VR_OK;
}

// Validates and queues one request; the caller holds s->m and wakes the
// scheduler.
static vr_status server_submit_locked(vr_server *s, const vr_request *r, uint64_t *ticket) {
    if (s->stop) return server_fail(s, VR_ERR_BUSY, "the server is shutting down");
    if (r->mesh >= s->meshes.size()) return server_fail(s, VR_ERR_ARG, "unknown mesh %u", r->mesh);
    const ServerMesh &M = s->meshes[r->mesh];
    if (r->num_tris > M.T) return server_fail(s, VR_ERR_ARG, "num_tris %u beyond the mesh (%u)", r->num_tris, M.T);
    // the same rules as vr_process_draw, and the request alone must fit a tick
    ServerReq R{};
    R.mesh = r->mesh;
    R.num_tris = r->num_tris;
    R.batch_tris = r->batch_tris;
    R.strategy = r->strategy;
    R.shader = r->shader;
    vr_opts o{};
    o.max_unique = r->max_unique;
    vr_outputs ov{};
    Resolved res;
    if (check_args(s->ctx, 3ull * r->num_tris, M.V, &r->shader, r->strategy, r->batch_tris, &o, &ov, &res) != VR_OK)
        return server_fail(s, VR_ERR_ARG, "%s", s->ctx->error.c_str());
    if (r->strategy == VR_MULTI)
        return server_fail(s, VR_ERR_ARG, "MULTI (two passes over the vertex buffer) is not served");
    R.nu = is_dynamic(r->strategy) ? res.nu : 0;
    FrameNeeds need;
    DrawDesc X;
    vr_draw D{};
    D.d_indices = M.idx;
    D.num_indices = 3ull * r->num_tris;
    D.d_vertices = M.vtx;
    D.num_vertices = M.V;
    D.strategy = r->strategy;
    D.batch_tris = r->batch_tris;
    D.max_unique = R.nu;
    D.d_plan = M.idx;          // stands in for the plan during validation
    D.d_corners = (float *)s->arena;
    if (describe_draw(s->ctx, D, r->shader, 0, X, need) != VR_OK)
        return server_fail(s, VR_ERR_ARG, "%s", s->ctx->error.c_str());
    if (need.lds_total(s->cfg.max_tick_draws) > s->ctx->lds_limit)
        return server_fail(s, VR_ERR_ARG, "the request needs more LDS than a tick allows");
    const uint64_t bytes = 144ull * r->num_tris;
    uint64_t t = 0;
    const int st = s->sch->submit(r->user, bytes, r->num_tris, s->now(), &t);
    if (st != sched::kOk)
        return server_fail(s, (vr_status)st, "the request's %llu output bytes exceed the budget",
                           (unsigned long long)bytes);
    s->reqs[t] = R;
    *ticket = t;
    return VR_OK;
}

vr_status vr_server_submit(vr_server *s, const vr_request *r, uint64_t *ticket) {
    if (!s || !r || !ticket) return VR_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->m);
    const vr_status st = server_submit_locked(s, r, ticket);
    if (st == VR_OK) s->cv_work.notify_one();
    return st;
}

vr_status vr_server_submit_many(vr_server *s, const vr_request *r, uint32_t n, uint64_t *tickets,
                                uint32_t *accepted) {
    if (!s || !accepted || (n && (!r || !tickets))) return VR_ERR_ARG;
    *accepted = 0;
    std::lock_guard<std::mutex> lk(s->m);
    vr_status st = VR_OK;
    for (uint32_t i = 0; i < n && st == VR_OK; ++i) {
        st = server_submit_locked(s, r + i, tickets + i);
        if (st == VR_OK) ++*accepted;
    }
    if (*accepted) s->cv_work.notify_one();
    return st;
}

vr_status vr_server_poll(vr_server *s, vr_completion *out, uint32_t cap, uint32_t *count, uint32_t timeout_ms) {
    if (!s || !count || (cap && !out)) return VR_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->m);
    if (s->done.empty() && timeout_ms)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [s] { return !s->done.empty(); });
    uint32_t k = 0;
    while (k < cap && !s->done.empty()) {
        const uint64_t t = s->done.front();
        s->done.pop_front();
        const sched::Job *j = s->sch->find(t);
        if (!j) continue;   // released before it was polled
        const ServerReq &R = s->reqs[t];
        vr_completion &c = out[k++];
        c.ticket = t;
        c.user = j->user;
        c.status = j->status;
        c.tick = j->tick;
        c.num_tris = R.num_tris;
        c.invocations = R.inv;
        c.units = R.units;
        c.d_corners = j->has_mem ? (const float *)(s->arena + j->off) : nullptr;
        c.t_submit = j->t_submit;
        c.t_admit = j->t_admit;
        c.t_launch = j->t_launch;
        c.t_done = j->t_done;
    }
    *count = k;
    return VR_OK;
}

vr_status vr_server_release(vr_server *s, uint64_t ticket) {
    if (!s) return VR_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->m);
    const int st = s->sch->release(ticket);
    if (st == sched::kArg) return server_fail(s, VR_ERR_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (st == sched::kBusy) return server_fail(s, VR_ERR_BUSY, "request %llu has not finished", (unsigned long long)ticket);
    s->reqs.erase(ticket);
    s->cv_work.notify_one();
    return VR_OK;
}

vr_status vr_server_fetch(vr_server *s, uint64_t ticket, void *dst, uint64_t bytes) {
    if (!s || (!dst && bytes)) return VR_ERR_ARG;
    const float *src = nullptr;
    uint64_t need = 0;
    {
        std::lock_guard<std::mutex> lk(s->m);
        const sched::Job *j = s->sch->find(ticket);
        if (!j) return server_fail(s, VR_ERR_ARG, "unknown ticket %llu", (unsigned long long)ticket);
        if (j->state != sched::State::Done) return server_fail(s, VR_ERR_BUSY, "request has not finished");
        need = 144ull * s->reqs[ticket].num_tris;
        if (bytes < need) return server_fail(s, VR_ERR_CAPACITY, "need %llu bytes", (unsigned long long)need);
        src = j->has_mem ? (const float *)(s->arena + j->off) : nullptr;
    }
    if (!src || need == 0) return VR_OK;
    // the request stays reserved until the caller releases it, so the copy
    // runs outside the lock
    DeviceGuard g(s->device);
    if (hipMemcpy(dst, src, need, hipMemcpyDeviceToHost) != hipSuccess) {
        std::lock_guard<std::mutex> lk(s->m);
        return server_fail(s, VR_ERR_DEVICE, "result copy failed");
    }
    return VR_OK;
}

vr_status vr_server_cancel(vr_server *s, uint64_t ticket) {
    if (!s) return VR_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->m);
    const int st = s->sch->cancel(ticket, s->now());
    if (st == sched::kArg) return server_fail(s, VR_ERR_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (st == sched::kBusy) return server_fail(s, VR_ERR_BUSY, "request %llu was launched", (unsigned long long)ticket);
    s->done.push_back(ticket);
    s->cv_done.notify_all();
    s->cv_work.notify_one();
    return VR_OK;
}

vr_status vr_server_stats_get(vr_server *s, vr_server_stats *o) {
    if (!s || !o) return VR_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->m);
    const sched::Counts &n = s->sch->counts();
    *o = vr_server_stats{};
    o->submitted = n.submitted;
    o->completed = n.completed;
    o->cancelled = n.cancelled;
    o->rejected = n.rejected;
    o->ticks = n.ticks;
    o->budget_bytes = s->sch->arena().capacity();
    o->reserved_bytes = s->sch->arena().used();
    o->peak_reserved_bytes = s->sch->arena().peak();
    o->pending = s->sch->pending();
    o->admitted = s->sch->admitted();
    o->inflight_ticks = s->sch->inflight();
    o->max_pending = n.max_pending;
    o->max_tick_draws = n.max_tick_draws;
    o->admission_blocked = n.admission_blocked;
    o->plan_bytes = s->plan_bytes;
    return VR_OK;
}

void vr_server_destroy(vr_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
        for (uint64_t t : s->sch->cancel_all(s->now())) s->done.push_back(t);
        s->cv_work.notify_one();
    }
    if (s->worker.joinable()) s->worker.join();
    DeviceGuard g(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    server_free(s);
}

const char *vr_server_last_error(const vr_server *s) { return s ? s->error.c_str() : g_create_error.c_str(); }

// The same policy on a simulated clock and device (host only).
vr_status vr_server_simulate(const vr_server_config *cfg_in, const vr_sim_request *rq, uint32_t n, double fixed_s,
                             double per_tri_s, vr_sim_result *res, vr_server_stats *stats) {
    vr_server_config cfg;
    std::string why;
    if (check_server_config(cfg_in, cfg, why) != VR_OK) return fail(nullptr, VR_ERR_ARG, "%s", why.c_str());
    if (n && (!rq || !res)) return fail(nullptr, VR_ERR_ARG, "requests and results must not be NULL");
    for (uint32_t i = 1; i < n; ++i)
        if (rq[i].arrival < rq[i - 1].arrival) return fail(nullptr, VR_ERR_ARG, "requests must be sorted by arrival");
    sched::Scheduler sch(server_policy(cfg));
    std::vector<uint64_t> ticket(n, 0);
    std::unordered_map<uint64_t, uint32_t> index;
    for (uint32_t i = 0; i < n; ++i) res[i] = vr_sim_result{VR_OK, 0, -1.0, -1.0, -1.0, -1.0, 0};
    std::deque<std::pair<double, uint32_t>> ticks;   // end time, tick id (device runs them in order)
    std::multimap<double, uint64_t> releases, cancels;
    double device_free = 0.0;
    uint32_t next = 0;
    std::vector<uint64_t> jobs;
    auto finish = [&](uint64_t t, double now) {
        const sched::Job *j = sch.find(t);
        vr_sim_result &r = res[index[t]];
        r.status = j->status;
        r.tick = j->tick;
        r.t_admit = j->t_admit;
        r.t_launch = j->t_launch;
        r.t_done = j->t_done;
        r.offset = j->off;
        const uint32_t i = index[t];
        releases.emplace(now + std::max(0.0, rq[i].hold), t);
    };
    const double inf = 1e300;
    for (;;) {
        const double ta = next < n ? rq[next].arrival : inf;
        const double tt = ticks.empty() ? inf : ticks.front().first;
        const double tr = releases.empty() ? inf : releases.begin()->first;
        const double tc = cancels.empty() ? inf : cancels.begin()->first;
        const double now = std::min(std::min(ta, tt), std::min(tr, tc));
        if (now >= inf) break;
        // events at `now`: tick ends, releases, cancellations, arrivals
        while (!ticks.empty() && ticks.front().first <= now) {
            const std::vector<uint64_t> done = sch.oldest_jobs();
            sch.retire_oldest(ticks.front().first, VR_OK);
            for (uint64_t t : done) finish(t, ticks.front().first);
            ticks.pop_front();
        }
        while (!releases.empty() && releases.begin()->first <= now) {
            const uint64_t t = releases.begin()->second;
            res[index[t]].t_release = releases.begin()->first;
            sch.release(t);
            releases.erase(releases.begin());
        }
        while (!cancels.empty() && cancels.begin()->first <= now) {
            const uint64_t t = cancels.begin()->second;
            if (sch.cancel(t, cancels.begin()->first) == sched::kOk) {
                const sched::Job *j = sch.find(t);
                vr_sim_result &r = res[index[t]];
                r.status = j->status;
                r.t_admit = j->t_admit;
                r.t_done = j->t_done;
                r.offset = j->off;
                res[index[t]].t_release = cancels.begin()->first;
                sch.release(t);
            }
            cancels.erase(cancels.begin());
        }
        while (next < n && rq[next].arrival <= now) {
            uint64_t t = 0;
            const int st = sch.submit(next, rq[next].bytes, rq[next].num_tris, rq[next].arrival, &t);
            if (st != sched::kOk) {
                res[next].status = st;
            } else {
                ticket[next] = t;
                index[t] = next;
                if (rq[next].cancel_at >= 0.0) cancels.emplace(std::max(rq[next].cancel_at, rq[next].arrival), t);
            }
            ++next;
        }
        sch.admit(now);
        uint32_t tick = 0;
        while (sch.next_tick(now, jobs, &tick)) {
            uint64_t tris = 0;
            for (uint64_t t : jobs) tris += sch.find(t)->tris;
            const double start = std::max(now, device_free);
            device_free = start + fixed_s + per_tri_s * (double)tris;
            ticks.push_back({device_free, tick});
        }
    }
    if (stats) {
        const sched::Counts &c = sch.counts();
        *stats = vr_server_stats{};
        stats->submitted = c.submitted;
        stats->completed = c.completed;
        stats->cancelled = c.cancelled;
        stats->rejected = c.rejected;
        stats->ticks = c.ticks;
        stats->budget_bytes = sch.arena().capacity();
        stats->reserved_bytes = sch.arena().used();
        stats->peak_reserved_bytes = sch.arena().peak();
        stats->max_pending = c.max_pending;
        stats->max_tick_draws = c.max_tick_draws;
        stats->admission_blocked = c.admission_blocked;
    }
    return VR_OK;
}

}  // extern "C"
