// Device-side building blocks of the geometry stage for gfx950 (wave64):
// vertex programs, wavefront and workgroup scans, look-back prefix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vr.h"

namespace vr {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;   // empty hash slot / no index
constexpr int kWave = 64;
constexpr int kOutF4 = 3;                  // a shaded vertex is 3 float4 (48 B)

// Multiplicative hashing of a vertex index into a table of 2^bits slots.
__device__ __forceinline__ uint32_t hash_slot(uint32_t key, uint32_t bits) {
    return (key * 0x9E3779B1u) >> (32u - bits);
}

// Kernel-side error bits (a vr_status value is stored, first one wins).
__device__ __forceinline__ void raise_error(uint32_t *err, uint32_t code) {
    atomicCAS(err, 0u, code);
}

// --------------------------------------------------------------------------
// Vertex programs.  Every operation is spelled out (fma = single rounding,
// '/' and sqrtf correctly rounded, contraction disabled at build time) so the
// FP32 results are the ones fixed by the written program.
// --------------------------------------------------------------------------
__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz) {
    return __builtin_fmaf(az, bz, __builtin_fmaf(ay, by, ax * bx));
}

// row r of a row-major matrix with 4 columns, applied to (x, y, z, 1)
__device__ __forceinline__ float xrow(const float *M, int r, float x, float y, float z) {
    return __builtin_fmaf(M[4 * r + 2], z,
                          __builtin_fmaf(M[4 * r + 1], y, __builtin_fmaf(M[4 * r + 0], x, M[4 * r + 3])));
}

// Correctly rounded reciprocal and square root.  The compiler's IEEE
// sequences scale their operands and test for special values; for operands
// whose intermediates all stay normal that is not needed, and a shorter
// sequence gives the same bits:
//  * 1/x for |x| in [2^-125, 2^125]: the hardware reciprocal (within one ulp)
//    and one Newton-Raphson step on the exact FMA residual 1 - x.y;
//  * sqrt(x) for x in [2^-96, 2^126]: s = x.y and h = y/2 from the hardware
//    reciprocal square root y, then one Newton step s + h.(x - s.s) on the
//    exact FMA residual.
// Every other operand (zero, denormal, huge, negative, inf, NaN) takes the
// compiler's sequence.  vr_math_selftest compares both against the
// compiler's sequences bit for bit over all 2^32 float32 operands
// (k_math_selftest).
__device__ __forceinline__ float recip_fast(float x) {
    const float y = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(__builtin_fmaf(-x, y, 1.0f), y, y);
}
__device__ __forceinline__ float sqrt_fast(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    const float s = x * y, h = 0.5f * y;
    return __builtin_fmaf(__builtin_fmaf(-s, s, x), h, s);
}

// Lanes whose operand lies outside [lo, hi] (NaN included), as a wavefront
// mask: one ballot per compare keeps the test on compare results in scalar
// registers.  The fallback below runs only when the mask is not empty (a
// scalar branch), under an execution mask of exactly those lanes.
__device__ __forceinline__ uint64_t lanes_outside(float x, float lo, float hi) {
    return __builtin_amdgcn_ballot_w64(!(x >= lo)) | __builtin_amdgcn_ballot_w64(!(x <= hi));
}

__device__ __forceinline__ float recip_rn(float x) {
    float y = recip_fast(x);
    const uint64_t other = lanes_outside(__builtin_fabsf(x), 0x1p-125f, 0x1p125f);
    if (__builtin_expect(other != 0, 0)) {
        if (__builtin_amdgcn_inverse_ballot_w64(other)) y = 1.0f / x;
    }
    return y;
}
__device__ __forceinline__ float sqrt_rn(float x) {
    float r = sqrt_fast(x);
    const uint64_t other = lanes_outside(x, 0x1p-96f, 0x1p126f);
    if (__builtin_expect(other != 0, 0)) {
        if (__builtin_amdgcn_inverse_ballot_w64(other)) r = __builtin_sqrtf(x);
    }
    return r;
}
// 1/sqrt(s) with both operations rounded: a square root of the fast range
// lies in [2^-48, 2^63], inside the reciprocal's, so one test covers both.
__device__ __forceinline__ float inv_sqrt_rn(float s) {
    float q = recip_fast(sqrt_fast(s));
    const uint64_t other = lanes_outside(s, 0x1p-96f, 0x1p126f);
    if (__builtin_expect(other != 0, 0)) {
        if (__builtin_amdgcn_inverse_ballot_w64(other)) q = 1.0f / __builtin_sqrtf(s);
    }
    return q;
}

__device__ __forceinline__ void normalize3(float &x, float &y, float &z) {
    float s = dot3(x, y, z, x, y, z);
    float q = inv_sqrt_rn(s);
    x = x * q;
    y = y * q;
    z = z * q;
}

// in: a = (px, py, pz, nx), b = (ny, nz, u, v); out: 3 float4 =
// (clip xyzw), (n'xyz, u), (v, rgb)
template <int KIND>
__device__ __forceinline__ void shade_vertex(const vr_shader_params &sh, float4 a, float4 b,
                                             float4 &o0, float4 &o1, float4 &o2) {
    float px = a.x, py = a.y, pz = a.z;
    const float nx = a.w, ny = b.x, nz = b.y;
    if (KIND == 2) {
        const float *c = sh.coef;
        const float ph = dot3(c[4], c[5], c[6], px, py, pz);
        float h = 0.0f;
        for (uint32_t it = 0; it < sh.iterations; ++it) {
            float g = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(c[3], h, c[2]), h, c[1]), h, ph);
            h = __builtin_fmaf(c[0], g - h, h);
        }
        px = __builtin_fmaf(h, nx, px);
        py = __builtin_fmaf(h, ny, py);
        pz = __builtin_fmaf(h, nz, pz);
    }
    o0.x = xrow(sh.mvp, 0, px, py, pz);
    o0.y = xrow(sh.mvp, 1, px, py, pz);
    o0.z = xrow(sh.mvp, 2, px, py, pz);
    o0.w = xrow(sh.mvp, 3, px, py, pz);
    float mx = dot3(sh.normal[0], sh.normal[1], sh.normal[2], nx, ny, nz);
    float my = dot3(sh.normal[3], sh.normal[4], sh.normal[5], nx, ny, nz);
    float mz = dot3(sh.normal[6], sh.normal[7], sh.normal[8], nx, ny, nz);
    normalize3(mx, my, mz);
    float cr = sh.ambient[0], cg = sh.ambient[1], cb = sh.ambient[2];
    if (KIND == 1) {
        const float wx = xrow(sh.model, 0, px, py, pz);
        const float wy = xrow(sh.model, 1, px, py, pz);
        const float wz = xrow(sh.model, 2, px, py, pz);
        float vx = sh.eye[0] - wx, vy = sh.eye[1] - wy, vz = sh.eye[2] - wz;
        normalize3(vx, vy, vz);
        // fma(2 ndl, n', -l) = fma(ndl, 2 n', -l) bit for bit: doubling is
        // exact, so both see the same exact product
        const float m2x = 2.0f * mx, m2y = 2.0f * my, m2z = 2.0f * mz;
        // with 0 <= katt <= 1/2, d2 in [2^-96, 2^126] gives katt.d2 + 1 in
        // [1, 2^125] (the fma rounds 2^125 + 1 down to 2^125), inside the
        // reciprocal's short range: its own range test is then not needed
        const bool katt_small = sh.katt >= 0.0f && sh.katt <= 0.5f;
        for (uint32_t l = 0; l < sh.num_lights; ++l) {
            const float *L = sh.lights[l];
            const float dx = L[0] - wx, dy = L[1] - wy, dz = L[2] - wz;
            const float d2 = dot3(dx, dy, dz, dx, dy, dz);
            const float ad = __builtin_fmaf(sh.katt, d2, 1.0f);
            // 1/sqrt(d2) and the attenuation 1/(katt.d2 + 1), one range test
            float inv = recip_fast(sqrt_fast(d2));
            float att = recip_fast(ad);
            uint64_t other = lanes_outside(d2, 0x1p-96f, 0x1p126f);
            if (!katt_small) other |= lanes_outside(__builtin_fabsf(ad), 0x1p-125f, 0x1p125f);
            if (__builtin_expect(other != 0, 0)) {
                if (__builtin_amdgcn_inverse_ballot_w64(other)) {
                    inv = 1.0f / __builtin_sqrtf(d2);
                    att = 1.0f / ad;
                }
            }
            const float lx = dx * inv, ly = dy * inv, lz = dz * inv;
            const float ndl = dot3(mx, my, mz, lx, ly, lz);
            // ndl > 0 ? ndl : 0 as one v_max_f32 with 0: ndl is an arithmetic
            // result (never a signalling NaN), NaN gives 0 and -0 gives +0, as
            // the select does; written out so that no canonicalising max precedes it
            float df;
            asm("v_max_f32 %0, 0, %1" : "=v"(df) : "v"(ndl));
            const float kdf = sh.kd * df;
            const float rx = __builtin_fmaf(ndl, m2x, -lx);
            const float ry = __builtin_fmaf(ndl, m2y, -ly);
            const float rz = __builtin_fmaf(ndl, m2z, -lz);
            const float rv = dot3(rx, ry, rz, vx, vy, vz);
            float sp = rv > 0.0f ? rv : 0.0f;
            for (uint32_t s = 0; s < sh.spec_squarings; ++s) sp = sp * sp;
            const float k = att * __builtin_fmaf(sh.ks, sp, kdf);
            cr = __builtin_fmaf(k, L[3], cr);
            cg = __builtin_fmaf(k, L[4], cg);
            cb = __builtin_fmaf(k, L[5], cb);
        }
    }
    o1 = make_float4(mx, my, mz, b.z);
    o2 = make_float4(b.w, cr, cg, cb);
}

// --------------------------------------------------------------------------
// Wavefront / workgroup helpers (wave64)
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Orders this wavefront's LDS accesses before and after the call.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive scan over the 64 lanes with DPP: Hillis-Steele steps of 1, 2, 4
// and 8 lanes inside each 16-lane row, then row 0's and row 2's totals are
// broadcast into rows 1 and 3 (row_bcast:15) and the total of rows 0-1 into
// rows 2 and 3 (row_bcast:31).  Lanes whose source is out of range add 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Minimum / maximum over the 64 lanes with DPP (row shifts, then row
// broadcasts; lanes without a source keep the identity), read from lane 63.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, kWave - 1);
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, kWave - 1);
}

// Exclusive scan over one value per thread of an NT-thread workgroup.
// `tmp` is LDS scratch of NT/64 words.  Contains barriers: call uniformly.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *tmp, uint32_t &total) {
    constexpr int NW = NT / kWave;
    const uint32_t tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    uint32_t incl = wave_incl_scan(v);
    if (NW == 1) {
        total = __builtin_amdgcn_readlane(incl, kWave - 1);
        return incl - v;
    }
    if (lane == kWave - 1) tmp[w] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        uint32_t t = tmp[i];
        before += (i < (int)w) ? t : 0u;
        all += t;
    }
    __syncthreads();
    total = all;
    return before + incl - v;
}

// Workgroup-wide min and max together; `tmp` holds 2*NT/64 words.  Contains
// barriers: call uniformly.
template <int NT>
__device__ __forceinline__ void block_reduce_minmax(uint32_t &mn, uint32_t &mx, uint32_t *tmp) {
    constexpr int NW = NT / kWave;
    mn = wave_min(mn);
    mx = wave_max(mx);
    __syncthreads();
    if (lane_id() == 0) {
        tmp[threadIdx.x / kWave] = mn;
        tmp[NW + threadIdx.x / kWave] = mx;
    }
    __syncthreads();
    mn = tmp[0];
    mx = tmp[NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
        mn = min(mn, tmp[i]);
        mx = max(mx, tmp[NW + i]);
    }
    __syncthreads();
}

// Workgroup-wide min / max (contain barriers: call uniformly).
template <int NT>
__device__ __forceinline__ uint32_t block_reduce_min(uint32_t v, uint32_t *tmp) {
    constexpr int NW = NT / kWave;
    v = wave_min(v);
    __syncthreads();
    if (lane_id() == 0) tmp[threadIdx.x / kWave] = v;
    __syncthreads();
    uint32_t r = tmp[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r = min(r, tmp[i]);
    __syncthreads();
    return r;
}

template <int NT>
__device__ __forceinline__ uint32_t block_reduce_max(uint32_t v, uint32_t *tmp) {
    constexpr int NW = NT / kWave;
    v = wave_max(v);
    __syncthreads();
    if (lane_id() == 0) tmp[threadIdx.x / kWave] = v;
    __syncthreads();
    uint32_t r = tmp[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r = max(r, tmp[i]);
    __syncthreads();
    return r;
}

// --------------------------------------------------------------------------
// Single-pass prefix over units (decoupled look-back).  A status word is
//   [63:62] flag (0 = not ready, 1 = aggregate, 2 = inclusive prefix)
//   [61:32] unit count, [31:0] invocation count
// so both prefixes travel in one 64-bit word; totals stay below 2^30 units
// and 2^32 invocations because a draw has fewer than 2^30 triangles.
// --------------------------------------------------------------------------
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

// The status words carry their whole payload, so they need no ordering
// with other memory: relaxed atomics at agent scope (coherent across the
// XCDs' L2s) suffice, and no release or acquire fence writes back or
// invalidates the L2.
__device__ __forceinline__ void status_store(unsigned long long *p, uint64_t v) {
    __hip_atomic_store(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_load(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes unit b's aggregate; called by one thread.
__device__ __forceinline__ void lookback_publish(unsigned long long *status, uint32_t b, uint64_t agg) {
    status_store(&status[b], (b == 0 ? kFlagInc : kFlagAgg) | agg);
}

// Returns the exclusive prefix of unit b (packed), called by every lane of
// one wavefront after lookback_publish.  The wavefront reads the status
// words of the 64 preceding units at once; when every unit down to the
// nearest inclusive prefix is ready, it adds their values, otherwise it
// reads the same window again.  Unit b is workgroup b.  Workgroups are
// dispatched in index order within each XCD (the grid is dealt round-robin
// over the XCDs), so when b runs, the lowest unfinished unit has been
// dispatched or its XCD holds only lower, finishing units: every wait ends.
// A bounded spin still turns a lost update into an error instead of a hang.
__device__ __forceinline__ uint64_t lookback_resolve(unsigned long long *status, uint32_t b, uint64_t agg,
                                                     uint32_t *err) {
    const uint32_t lane = lane_id();
    uint64_t excl = 0;
    int64_t hi = (int64_t)b;   // the window is units hi - 64 .. hi - 1, lane i reading hi - 1 - i
    uint32_t spins = 0;
    while (hi > 0) {
        const int64_t j = hi - 1 - (int64_t)lane;
        const uint64_t s = j >= 0 ? status_load(&status[j]) : kFlagInc;   // before unit 0: an empty prefix
        const uint64_t inc = ballot((s >> 62) == 2);
        // lanes up to and including the nearest inclusive prefix (all 64 when none)
        const uint64_t need = inc ? ((inc & (~inc + 1)) << 1) - 1 : ~0ull;
        if (ballot((s >> 62) == 0) & need) {
            if (++spins > (1u << 26)) {
                if (lane == 0) raise_error(err, VR_ERR_DEVICE);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const bool take = (need >> lane) & 1ull;
        const uint32_t lo = take ? (uint32_t)s : 0u, up = take ? (uint32_t)((s & kValMask) >> 32) : 0u;
        excl += ((uint64_t)__builtin_amdgcn_readlane(wave_incl_scan(up), kWave - 1) << 32) |
                __builtin_amdgcn_readlane(wave_incl_scan(lo), kWave - 1);
        if (inc) break;
        hi -= kWave;
    }
    if (lane == 0) status_store(&status[b], kFlagInc | (excl + agg));
    return excl;
}

}  // namespace vr
