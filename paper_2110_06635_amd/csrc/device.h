// Device-side building blocks of the one-pixel point rasterizer (gfx950).
//
// - ViewRec: the per-view record the kernels read (camera + pyramid layout).
// - project(): the FP32 projection of Sec. 3.1 Eq. 2 with pinhole +
//   Brown-Conrady distortion, written with explicit fused multiply-adds so
//   that the result does not depend on compiler contraction (the library is
//   also built with -ffp-contract=off).  Depth keys and pixel choices are
//   bit-exact functions of this arithmetic.
// - wave64 helpers built on DPP row shifts / row broadcasts and ballots.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include "launch.h"

namespace adop {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per workgroup for point kernels
constexpr int kMaxLayers = 8;
constexpr int kXcds = 8;             // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kMaxViewsBwd = 32;

// 256-byte per-view record staged into the workspace by the host.
struct alignas(16) ViewRec {
    float fx, fy, cx, cy;
    float k1, k2, k3, p1;
    float p2, znear, r2max, pad0;
    float R[9];
    float t[3];
    int32_t w, h, L, pad1;
    int32_t lw[kMaxLayers];
    int32_t lh[kMaxLayers];
    uint32_t base[kMaxLayers];       // first pixel of layer l of this view in the frame
    float pad2[12];
};
static_assert(sizeof(ViewRec) == 256, "ViewRec must be 256 bytes");

// The constants of one view as the kernels hold them (scalar registers when
// the view is wave-uniform); layer tables indexed with constant l only.
struct Cam {
    float fx, fy, cx, cy, k1, k2, k3, p1, p2, znear, r2max;
    float R[9];
    float t[3];
    int w, h;
    int lw[kMaxLayers];
    int lh[kMaxLayers];
    uint32_t base[kMaxLayers];
};

__device__ __forceinline__ Cam load_cam(const ViewRec* __restrict__ v) {
    Cam c;
    c.fx = v->fx; c.fy = v->fy; c.cx = v->cx; c.cy = v->cy;
    c.k1 = v->k1; c.k2 = v->k2; c.k3 = v->k3; c.p1 = v->p1; c.p2 = v->p2;
    c.znear = v->znear; c.r2max = v->r2max;
    c.w = v->w; c.h = v->h;
#pragma unroll
    for (int k = 0; k < 9; ++k) c.R[k] = v->R[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) c.t[k] = v->t[k];
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) {
        c.lw[l] = v->lw[l];
        c.lh[l] = v->lh[l];
        c.base[l] = v->base[l];
    }
    return c;
}

// Layer loops run to a compile-time bound: kernels are compiled for a fixed
// layer count LN (4 and 5, the pyramid depths of the paper's renders) and for
// any count (LN = 0: up to kMaxLayers with a run-time stop at L).  With a
// fixed count a point's per-layer work is straight-line code, its per-layer
// gathers stay in flight together and its layer arrays stay in registers.
template <int LN> struct Layers {
    static constexpr int max = LN > 0 ? LN : kMaxLayers;
    static __device__ __forceinline__ bool has(int l, int L) { return LN > 0 ? true : l < L; }
};

// Layer scale 2^-l as an exact constant.
__device__ __forceinline__ float layer_scale(int l) {
    return __int_as_float((127 - l) << 23);
}

struct Proj {
    float X, Y, Z;        // camera-space position
    float a, b, r2, D;    // normalised coordinates and radial factor
    float xd, yd;         // distorted normalised coordinates
    float u0, v0;         // layer-0 pixel coordinates
    bool ok;
};

// x_c = R x + t, a = X/Z, b = Y/Z, r2 = a^2 + b^2,
// D = 1 + k1 r2 + k2 r2^2 + k3 r2^3,
// x_d = a D + 2 p1 a b + p2 (r2 + 2a^2), y_d = b D + 2 p2 a b + p1 (r2 + 2b^2),
// u0 = fx x_d + cx, v0 = fy y_d + cy.
template <typename CamT>
__device__ __forceinline__ Proj project(const CamT& c, float x, float y, float z) {
    Proj p;
    float X = __fmaf_rn(c.R[0], x, __fmaf_rn(c.R[1], y, __fmaf_rn(c.R[2], z, c.t[0])));
    float Y = __fmaf_rn(c.R[3], x, __fmaf_rn(c.R[4], y, __fmaf_rn(c.R[5], z, c.t[1])));
    float Z = __fmaf_rn(c.R[6], x, __fmaf_rn(c.R[7], y, __fmaf_rn(c.R[8], z, c.t[2])));
    float a = __fdiv_rn(X, Z);
    float b = __fdiv_rn(Y, Z);
    float ab = __fmul_rn(a, b);
    float bb = __fmul_rn(b, b);
    float r2 = __fmaf_rn(a, a, bb);
    float D = __fmaf_rn(r2, __fmaf_rn(r2, __fmaf_rn(r2, c.k3, c.k2), c.k1), 1.0f);
    float tx = __fmul_rn(c.p2, __fmaf_rn(__fadd_rn(a, a), a, r2));
    float ty = __fmul_rn(c.p1, __fmaf_rn(__fadd_rn(b, b), b, r2));
    float xd = __fmaf_rn(a, D, __fmaf_rn(__fadd_rn(c.p1, c.p1), ab, tx));
    float yd = __fmaf_rn(b, D, __fmaf_rn(__fadd_rn(c.p2, c.p2), ab, ty));
    p.u0 = __fmaf_rn(c.fx, xd, c.cx);
    p.v0 = __fmaf_rn(c.fy, yd, c.cy);
    p.X = X; p.Y = Y; p.Z = Z;
    p.a = a; p.b = b; p.r2 = r2; p.D = D; p.xd = xd; p.yd = yd;
    p.ok = (Z > c.znear) && (r2 <= c.r2max) && __builtin_isfinite(p.u0) && __builtin_isfinite(p.v0);
    return p;
}

// Pixel of layer l (Eq. round + Eq. boundscheck): rint(u0 * 2^-l), in
// [0,w_l) x [0,h_l), for a point whose projection is valid (ok).  The
// rounded coordinate is an integer-valued float; clamped into [-1, 2^24] it
// converts exactly, and the float range test becomes one unsigned compare
// (-0 maps to 0 and stays inside, as the float test keeps it).  u0, v0 are
// finite whenever ok holds.  Lanes outside get px = py = 0, so *pix is the
// layer's first pixel: always a valid address to load from.
__device__ __forceinline__ bool layer_pixel_at(bool ok, int l, int lw, int lh, uint32_t base, float u0, float v0,
                                               int& px, int& py, uint32_t& pix) {
    float s = layer_scale(l);
    float fx = __builtin_rintf(__fmul_rn(u0, s));
    float fy = __builtin_rintf(__fmul_rn(v0, s));
    int ix = (int)__builtin_amdgcn_fmed3f(fx, -1.0f, 16777216.0f);
    int iy = (int)__builtin_amdgcn_fmed3f(fy, -1.0f, 16777216.0f);
    bool in = ok & ((uint32_t)ix < (uint32_t)lw) & ((uint32_t)iy < (uint32_t)lh);
    px = in ? ix : 0;
    py = in ? iy : 0;
    pix = base + (uint32_t)py * (uint32_t)lw + (uint32_t)px;
    return in;
}

template <typename CamT>
__device__ __forceinline__ bool layer_pixel(const CamT& c, bool ok, int l, float u0, float v0,
                                            int& px, int& py, uint32_t& pix) {
    return layer_pixel_at(ok, l, c.lw[l], c.lh[l], c.base[l], u0, v0, px, py, pix);
}

// Correctly rounded square root of a binary32 value.  The hardware square
// root is within one unit in the last place; the neighbour that is the
// correctly rounded result is found by comparing x with the squared
// midpoints between neighbouring floats, which are exact in binary64
// (25-bit midpoints, 50-bit squares); ties go to the even neighbour.
__device__ __forceinline__ float sqrt_rn(float x) {
    if (!(x > 0.0f) || !__builtin_isfinite(x)) return __builtin_sqrtf(x);
    float y = __builtin_sqrtf(x);
    const double xd = (double)x;
    for (int it = 0; it < 2; ++it) {
        const uint32_t b = __float_as_uint(y);
        const float up = __uint_as_float(b + 1u), dn = __uint_as_float(b - 1u);
        const double mh = 0.5 * ((double)y + (double)up), ml = 0.5 * ((double)dn + (double)y);
        const double h2 = mh * mh, l2 = ml * ml;
        if (xd > h2 || (xd == h2 && (b & 1u))) y = up;
        else if (xd < l2 || (xd == l2 && (b & 1u))) y = dn;
        else break;
    }
    return y;
}

// Optional per-point inputs of one point (loaded with the point's position,
// so that their latency hides behind the same wait).
struct PointExtra {
    float nx = 0.f, ny = 0.f, nz = 0.f, r = 0.f, beta = 0.f;
};

__device__ __forceinline__ void load_extra(const PointOpts& o, int64_t i, PointExtra& e) {
    if (o.flags & (kOptCullBack | kOptCullPrinted)) {
        e.nx = __builtin_nontemporal_load(o.nx + i);
        e.ny = __builtin_nontemporal_load(o.ny + i);
        e.nz = __builtin_nontemporal_load(o.nz + i);
    }
    if (o.flags & kOptDiscard) {
        e.r = __builtin_nontemporal_load(o.radius + i);
        e.beta = __builtin_nontemporal_load(o.beta + i);
    }
}

// Eq. normalculling (see kOptCull*): the sign of (R n) . x_c in FP32 with
// the nesting of the projection.
template <typename CamT>
__device__ __forceinline__ bool normal_kept(const PointOpts& o, const CamT& c, const Proj& p, const PointExtra& e) {
    if (!(o.flags & (kOptCullBack | kOptCullPrinted))) return true;
    const float m0 = __fmaf_rn(c.R[0], e.nx, __fmaf_rn(c.R[1], e.ny, __fmul_rn(c.R[2], e.nz)));
    const float m1 = __fmaf_rn(c.R[3], e.nx, __fmaf_rn(c.R[4], e.ny, __fmul_rn(c.R[5], e.nz)));
    const float m2 = __fmaf_rn(c.R[6], e.nx, __fmaf_rn(c.R[7], e.ny, __fmul_rn(c.R[8], e.nz)));
    const float d = __fmaf_rn(m0, p.X, __fmaf_rn(m1, p.Y, __fmul_rn(m2, p.Z)));
    return (o.flags & kOptCullBack) ? d < 0.0f : d > 0.0f;
}

// Eq. discard: bit l set when the point takes part in layer l, i.e.
// ((fx r / Z) 2^-l) gamma > sqrt(1 - beta) in FP32 (all bits without
// discarding).
template <typename CamT>
__device__ __forceinline__ uint32_t discard_mask(const PointOpts& o, const CamT& c, const Proj& p, const PointExtra& e,
                                                 int L) {
    if (!(o.flags & kOptDiscard)) return 0xffu;
    const float s0 = __fdiv_rn(__fmul_rn(c.fx, e.r), p.Z);
    const float rhs = sqrt_rn(__fsub_rn(1.0f, e.beta));
    uint32_t m = 0;
    for (int l = 0; l < L; ++l) m |= (uint32_t)(__fmul_rn(__fmul_rn(s0, layer_scale(l)), o.gamma) > rhs) << l;
    return m;
}

// ----------------------------------------------------------------------------
// environment map (Eq. blend: an empty pixel takes E(R^T C^-1(u, v)))
// ----------------------------------------------------------------------------
// Pixel (x, y) of layer l sits at layer-0 coordinates (x 2^l, y 2^l); C^-1
// inverts the pinhole and, with kUndistortIters fixed-point steps from the
// distorted coordinates, the Brown-Conrady map of project(); the world ray
// R^T (a, b, 1) is looked up in an equirectangular map of S x S texels
// (longitude atan2(d_x, d_z), colatitude arccos(d_y)), bilinearly between
// texel centres, wrapping in longitude and clamping in colatitude.
constexpr int kUndistortIters = 20;

struct EnvTaps {
    uint32_t idx[4];   // texel index r * S + c of the four taps
    float w[4];
};

template <typename CamT>
__device__ __forceinline__ EnvTaps env_taps(const CamT& c, int l, int x, int y, int S) {
    const float s2 = (float)(1 << l);
    const float xd = ((float)x * s2 - c.cx) / c.fx;
    const float yd = ((float)y * s2 - c.cy) / c.fy;
    float a = xd, b = yd;
    for (int it = 0; it < kUndistortIters; ++it) {
        const float r2 = a * a + b * b;
        const float D = 1.0f + r2 * (c.k1 + r2 * (c.k2 + r2 * c.k3));
        const float dx = 2.0f * c.p1 * a * b + c.p2 * (r2 + 2.0f * a * a);
        const float dy = 2.0f * c.p2 * a * b + c.p1 * (r2 + 2.0f * b * b);
        a = (xd - dx) / D;
        b = (yd - dy) / D;
    }
    float wx = c.R[0] * a + c.R[3] * b + c.R[6];
    float wy = c.R[1] * a + c.R[4] * b + c.R[7];
    float wz = c.R[2] * a + c.R[5] * b + c.R[8];
    const float inv = 1.0f / sqrtf(wx * wx + wy * wy + wz * wz);
    wx *= inv;
    wy *= inv;
    wz *= inv;
    const float kInv2Pi = 0.159154943091895336f, kInvPi = 0.318309886183790672f;
    const float sc = (atan2f(wx, wz) * kInv2Pi + 0.5f) * (float)S - 0.5f;
    const float tc = acosf(fminf(fmaxf(wy, -1.0f), 1.0f)) * kInvPi * (float)S - 0.5f;
    const float i0f = floorf(sc), j0f = floorf(tc);
    const float fx = sc - i0f, fy = tc - j0f;
    int i0 = (int)i0f % S;
    if (i0 < 0) i0 += S;
    const int i1 = i0 + 1 == S ? 0 : i0 + 1;
    const int j0 = (int)j0f;
    const int r0 = min(max(j0, 0), S - 1), r1 = min(max(j0 + 1, 0), S - 1);
    EnvTaps t;
    t.idx[0] = (uint32_t)(r0 * S + i0); t.w[0] = (1.0f - fx) * (1.0f - fy);
    t.idx[1] = (uint32_t)(r0 * S + i1); t.w[1] = fx * (1.0f - fy);
    t.idx[2] = (uint32_t)(r1 * S + i0); t.w[2] = (1.0f - fx) * fy;
    t.idx[3] = (uint32_t)(r1 * S + i1); t.w[3] = fx * fy;
    return t;
}

// ----------------------------------------------------------------------------
// wave64 helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <int CTRL, int ROWMASK, bool BOUND>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWMASK, 0xf, BOUND);
}

// Sum over all 64 lanes (every lane must be active); the total is returned
// to every lane.  Row shifts 1,2,4,8 build row sums in lane 15 of each row,
// row broadcasts 15 and 31 carry them to lane 63.
__device__ __forceinline__ float wave_sum(float v) {
    v += __uint_as_float(dpp_u32<0x111, 0xf, true>(0u, __float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x112, 0xf, true>(0u, __float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x114, 0xf, true>(0u, __float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x118, 0xf, true>(0u, __float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x142, 0xa, false>(0u, __float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x143, 0xc, false>(0u, __float_as_uint(v)));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// wave_sum of N values at once: the DPP steps of the N sums are interleaved,
// so no step waits on the one before it in the same chain.
template <int N>
__device__ __forceinline__ void wave_sum_n(float (&v)[N]) {
#define ADOP_SUM_STEP(CTRL, RM, BC)                                                              \
    _Pragma("unroll") for (int i = 0; i < N; ++i)                                               \
        v[i] += __uint_as_float(dpp_u32<CTRL, RM, BC>(0u, __float_as_uint(v[i])));
    ADOP_SUM_STEP(0x111, 0xf, true)
    ADOP_SUM_STEP(0x112, 0xf, true)
    ADOP_SUM_STEP(0x114, 0xf, true)
    ADOP_SUM_STEP(0x118, 0xf, true)
    ADOP_SUM_STEP(0x142, 0xa, false)
    ADOP_SUM_STEP(0x143, 0xc, false)
#undef ADOP_SUM_STEP
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[i]), 63));
}

// Segmented sums over runs of consecutive lanes that hold the same key
// (every lane must be active).  Lanes whose key is `none` carry zeros.  On
// return the last lane of each run holds the run's totals in v and the
// function returns true there (false on every other lane and on runs of
// `none`).  In-row Hillis-Steele steps (shift 1, 2, 4, 8) followed by the two
// row broadcasts, each combining (v, f) pairs as (f ? v : v + v_left,
// f | f_left) with f = "a run starts at or after the source lane".
template <int N>
__device__ __forceinline__ bool run_sums(uint32_t key, uint32_t none, float (&v)[N]) {
    const int lane = __lane_id();
    const uint32_t prev = (uint32_t)__builtin_amdgcn_ds_bpermute((lane - 1) << 2, (int)key);
    const uint32_t next = (uint32_t)__builtin_amdgcn_ds_bpermute((lane + 1) << 2, (int)key);
    uint32_t f = (lane == 0 || prev != key) ? 1u : 0u;
#define ADOP_RUN_STEP(CTRL, RM, BC)                                                            \
    {                                                                                        \
        const uint32_t fl = dpp_u32<CTRL, RM, BC>(0u, f);                                    \
        _Pragma("unroll") for (int i = 0; i < N; ++i) {                                      \
            const float vl = __uint_as_float(dpp_u32<CTRL, RM, BC>(0u, __float_as_uint(v[i]))); \
            v[i] = f ? v[i] : v[i] + vl;                                                     \
        }                                                                                    \
        f |= fl;                                                                             \
    }
    ADOP_RUN_STEP(0x111, 0xf, true)
    ADOP_RUN_STEP(0x112, 0xf, true)
    ADOP_RUN_STEP(0x114, 0xf, true)
    ADOP_RUN_STEP(0x118, 0xf, true)
    ADOP_RUN_STEP(0x142, 0xa, false)
    ADOP_RUN_STEP(0x143, 0xc, false)
#undef ADOP_RUN_STEP
    return key != none && (lane == 63 || next != key);
}

// Segmented minimum of 64-bit values over runs of equal keys, with the
// same steps as run_sums; lanes whose key is `none` carry ~0.  Returns true
// on the last lane of each run, which then holds the run's minimum.
__device__ __forceinline__ bool run_min_u64(uint32_t key, uint32_t none, uint64_t& v) {
    const int lane = __lane_id();
    const uint32_t prev = (uint32_t)__builtin_amdgcn_ds_bpermute((lane - 1) << 2, (int)key);
    const uint32_t next = (uint32_t)__builtin_amdgcn_ds_bpermute((lane + 1) << 2, (int)key);
    uint32_t f = (lane == 0 || prev != key) ? 1u : 0u;
#define ADOP_RUN_STEP(CTRL, RM, BC)                                                  \
    {                                                                              \
        const uint32_t fl = dpp_u32<CTRL, RM, BC>(0u, f);                          \
        const uint32_t lo = dpp_u32<CTRL, RM, BC>(0xffffffffu, (uint32_t)v);       \
        const uint32_t hi = dpp_u32<CTRL, RM, BC>(0xffffffffu, (uint32_t)(v >> 32)); \
        const uint64_t o = ((uint64_t)hi << 32) | lo;                              \
        v = (!f && o < v) ? o : v;                                                 \
        f |= fl;                                                                   \
    }
    ADOP_RUN_STEP(0x111, 0xf, false)
    ADOP_RUN_STEP(0x112, 0xf, false)
    ADOP_RUN_STEP(0x114, 0xf, false)
    ADOP_RUN_STEP(0x118, 0xf, false)
    ADOP_RUN_STEP(0x142, 0xa, false)
    ADOP_RUN_STEP(0x143, 0xc, false)
#undef ADOP_RUN_STEP
    return key != none && (lane == 63 || next != key);
}

template <int CTRL, int ROWMASK, bool BOUND>
__device__ __forceinline__ double dpp_f64(double v) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    uint32_t lo = dpp_u32<CTRL, ROWMASK, BOUND>(0u, (uint32_t)u);
    uint32_t hi = dpp_u32<CTRL, ROWMASK, BOUND>(0u, (uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// FP64 sum over all 64 lanes (fixed order), result valid in lane 63 and
// returned to every lane via readlane.
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0x111, 0xf, true>(v);
    v += dpp_f64<0x112, 0xf, true>(v);
    v += dpp_f64<0x114, 0xf, true>(v);
    v += dpp_f64<0x118, 0xf, true>(v);
    v += dpp_f64<0x142, 0xa, false>(v);
    v += dpp_f64<0x143, 0xc, false>(v);
    uint64_t u = (uint64_t)__double_as_longlong(v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Minimum of a u64 over all 64 lanes (every lane active), broadcast.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#define ADOP_MIN_STEP(CTRL, RM)                                                   \
    {                                                                             \
        uint32_t lo = dpp_u32<CTRL, RM, false>(0xffffffffu, (uint32_t)v);         \
        uint32_t hi = dpp_u32<CTRL, RM, false>(0xffffffffu, (uint32_t)(v >> 32)); \
        uint64_t o = ((uint64_t)hi << 32) | lo;                                   \
        v = o < v ? o : v;                                                        \
    }
    ADOP_MIN_STEP(0x111, 0xf)
    ADOP_MIN_STEP(0x112, 0xf)
    ADOP_MIN_STEP(0x114, 0xf)
    ADOP_MIN_STEP(0x118, 0xf)
    ADOP_MIN_STEP(0x142, 0xa)
    ADOP_MIN_STEP(0x143, 0xc)
#undef ADOP_MIN_STEP
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t load_relaxed_u64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t load_relaxed_u32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_min_u64(uint64_t* p, uint64_t v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_add_i32(int32_t* p, int32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------------------------------
// feature storage
// ----------------------------------------------------------------------------
struct F32 { using T = float; static constexpr int bytes = 4; };
struct BF16 { using T = uint16_t; static constexpr int bytes = 2; };
struct F16 { using T = uint16_t; static constexpr int bytes = 2; };

template <typename S> __device__ __forceinline__ float widen(typename S::T v);
template <> __device__ __forceinline__ float widen<F32>(float v) { return v; }
template <> __device__ __forceinline__ float widen<BF16>(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
template <> __device__ __forceinline__ float widen<F16>(uint16_t v) {
    _Float16 h = __builtin_bit_cast(_Float16, v);
    return (float)h;
}

// Streaming accesses to the point arrays (each element is touched once per
// pass) are non-temporal, so they do not push the gathered pixel data (keys,
// per-pixel records) out of the caches.
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef float vf2 __attribute__((ext_vector_type(2)));
typedef unsigned int vu4 __attribute__((ext_vector_type(4)));
typedef unsigned int vu2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int32_t ld_nt(const int32_t* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }

// A point's features as loaded: the raw 32-bit words of its row (one vector
// load per 16 or 8 bytes when the row allows it, else one element per word).
// Prefetches keep the raw words and widen them when the point is processed:
// a conversion right after the load would make the wave wait for it there.
template <int C, typename S>
struct FeatRaw {
    static constexpr int bytes = C * S::bytes;
    static constexpr bool vec = bytes % 8 == 0;
    static constexpr int words = vec ? bytes / 4 : C;
    uint32_t w[words];
};

template <int C, typename S>
__device__ __forceinline__ void load_feat_raw(const void* feat, int64_t i, FeatRaw<C, S>& r) {
    using T = typename S::T;
    const T* p = reinterpret_cast<const T*>(feat) + i * C;
    constexpr int bytes = C * S::bytes;
    if constexpr (bytes % 16 == 0) {
        const vu4* q = reinterpret_cast<const vu4*>(p);
#pragma unroll
        for (int k = 0; k < bytes / 16; ++k) {
            vu4 v = __builtin_nontemporal_load(q + k);
            r.w[4 * k] = v.x;
            r.w[4 * k + 1] = v.y;
            r.w[4 * k + 2] = v.z;
            r.w[4 * k + 3] = v.w;
        }
    } else if constexpr (bytes % 8 == 0) {
        const vu2* q = reinterpret_cast<const vu2*>(p);
#pragma unroll
        for (int k = 0; k < bytes / 8; ++k) {
            vu2 v = __builtin_nontemporal_load(q + k);
            r.w[2 * k] = v.x;
            r.w[2 * k + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if constexpr (S::bytes == 4)
                r.w[c] = __float_as_uint(p[c]);
            else
                r.w[c] = (uint32_t)p[c];
        }
    }
}

template <int C, typename S>
__device__ __forceinline__ void widen_feat(const FeatRaw<C, S>& r, float (&f)[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if constexpr (S::bytes == 4) {
            f[c] = __uint_as_float(r.w[c]);
        } else if constexpr (FeatRaw<C, S>::vec) {
            f[c] = widen<S>((uint16_t)(r.w[c >> 1] >> (16 * (c & 1))));   // little-endian pairs
        } else {
            f[c] = widen<S>((uint16_t)r.w[c]);
        }
    }
}

// Load the C features of point i (row-major [n][C]) widened to FP32.
template <int C, typename S>
__device__ __forceinline__ void load_feat(const void* feat, int64_t i, float (&f)[C]) {
    FeatRaw<C, S> r;
    load_feat_raw<C, S>(feat, i, r);
    widen_feat<C, S>(r, f);
}

template <int C>
__device__ __forceinline__ void store_f32_row(float* out, int64_t i, const float (&f)[C]) {
    float* p = out + i * C;
    if constexpr (C % 4 == 0) {
#pragma unroll
        for (int k = 0; k < C / 4; ++k) {
            vf4 v = {f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]};
            __builtin_nontemporal_store(v, reinterpret_cast<vf4*>(p) + k);
        }
    } else if constexpr (C % 2 == 0) {
#pragma unroll
        for (int k = 0; k < C / 2; ++k) {
            vf2 v = {f[2 * k], f[2 * k + 1]};
            __builtin_nontemporal_store(v, reinterpret_cast<vf2*>(p) + k);
        }
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) st_nt(p + c, f[c]);
    }
}

// Per-pixel record the backward pass gathers: upstream gradient G (C floats),
// gdot = <G, I> (or <G, background> for an empty pixel), the front depth
// min_z as float bits, and the blend count n.
// Per-pixel record of the backward pass: G (C floats), <G, I> (<G, b> for an
// empty pixel), min_z, (1+alpha) min_z and the count as a float; an empty
// pixel has min_z = (1+alpha) min_z = +inf, so the case tests need no
// separate emptiness check.
template <int C> struct PackLayout {
    static constexpr int used = C + 4;
    static constexpr int stride = (used + 3) / 4 * 4;   // floats, multiple of 4
    static constexpr int gdot = C, minz = C + 1, behind = C + 2, count = C + 3;
};

// Range mapping of the point kernels: the grid is persistent (a multiple of
// 8 workgroups) and workgroup b, which runs on XCD b % 8, owns one contiguous
// range of chunks.  Ranges are numbered so that the workgroups of XCD x own
// the x-th eighth of the (Morton-ordered) points: every workgroup renders a
// spatially compact part of the cloud and every XCD's L2 serves one region.
struct RangeMap {
    int64_t c0, c1;   // chunk indices [c0, c1)
};

__device__ __forceinline__ RangeMap range_map(int64_t n, int64_t chunk) {
    RangeMap m;
    const int64_t nc = (n + chunk - 1) / chunk;
    const int G = (int)gridDim.x;
    const int b = (int)blockIdx.x;
    const int64_t r = (int64_t)(b % kXcds) * (G / kXcds) + b / kXcds;
    m.c0 = nc * r / G;
    m.c1 = nc * (r + 1) / G;
    return m;
}

// Several views, one per workgroup.  The grid holds R point ranges for each
// of the V views (R a multiple of 8), dispatched in groups of VG views: the
// blocks of group g render views g VG .. g VG + VG - 1 (fewer in the last
// group), interleaved, so each view's blocks are spread evenly over the 8
// XCDs, and within a view the ranges of one XCD are a contiguous share of
// the Morton order.  The views of a group share the dispatch window, so the
// caches hold one group's per-pixel buffers while its points stream by.
__device__ __forceinline__ RangeMap view_range_map(int64_t n, int64_t chunk, int V, int VG, int& view) {
    RangeMap m;
    const int64_t nc = (n + chunk - 1) / chunk;
    const int64_t R = (int64_t)gridDim.x / V;
    const int64_t b = blockIdx.x;
    const int64_t g = b / (R * VG);
    const int64_t w = b - g * R * VG;
    const int64_t gs = (V - g * VG) < VG ? (V - g * VG) : VG;   // views in this group
    view = (int)(g * VG + w % gs);
    const int64_t rr = w / gs;                               // range index in dispatch order
    int64_t r = rr;
    if (gs <= kXcds && kXcds % gs == 0) {
        const int64_t per = kXcds / gs;                      // XCDs that share a view
        if (R % per == 0) r = (rr % per) * (R / per) + rr / per;
    }
    m.c0 = nc * r / R;
    m.c1 = nc * (r + 1) / R;
    return m;
}

// ----------------------------------------------------------------------------
// workgroup-private open-addressing tables in LDS (pixel -> partial result)
// ----------------------------------------------------------------------------
constexpr uint32_t kEmptySlot = 0xffffffffu;

template <int BITS>
__device__ __forceinline__ uint32_t hash_slot(uint32_t pix) {
    return (pix * 2654435761u) >> (32 - BITS);
}

// Find or claim the slot of `pix` with two fixed probes (home slot and its
// neighbour): no loop; -1 when both are taken by other pixels.
template <int BITS>
__device__ __forceinline__ int table_slot2(uint32_t* tkey, uint32_t pix) {
    constexpr uint32_t mask = (1u << BITS) - 1;
    uint32_t h = hash_slot<BITS>(pix);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        uint32_t k = __hip_atomic_load(&tkey[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == pix) return (int)h;
        if (k == kEmptySlot) {
            uint32_t old = atomicCAS(&tkey[h], kEmptySlot, pix);
            if (old == kEmptySlot || old == pix) return (int)h;
        }
        h = (h + 1) & mask;
    }
    return -1;
}

}  // namespace adop
