// Kernels and launchers of the rasterizer (templates); the instantiations
// are spread over render_*.hip so that they compile in parallel.
#pragma once
// HIP kernels of the one-pixel point rasterizer (ADOP Sec. 3.1) for gfx950.
//
// Forward (three passes over the points, as in "Implementation Details"):
//   k_clear      keys := empty, counts := 0, sums := 0
//   k_depth      project every point into every view and layer, 64-bit
//                atomic minimum of (depth bits << 32 | original index);
//                optionally marks each point's candidate layers (those where
//                its depth is within (1+alpha) of the front it read)
//   k_accum      fuzzy depth test z <= (1+alpha) min_z (Eq. depthtest) for
//                the candidates, FP32 sums of the features and an integer
//                count; optionally each point's blend-set bits (one byte per
//                point and view)
//   k_normalize  mean of the blend set, or for an empty pixel the constant
//                background or the environment map's sample (Eq. blend)
// Backward:
//   k_pack       per-pixel record {G, <G,I>, min_z, (1+alpha) min_z, n}
//   k_backward   re-render every point (the blend sets are not stored), or
//                take the forward's blend-set bits and skip the points
//                without any; feature gradient, approximate spatial gradient
//                (Eqs. induce, gradp, spatialderiv), chain to positions, pose
//                (Eq. tangent) and intrinsics; every per-point pose/intrinsics
//                term widened to FP64 before it is added, sums in a fixed order
//   k_env_grad   the environment map's gradient from the empty pixels
//   k_reduce_slices, k_reduce   fixed-order FP64 sum of the per-workgroup
//                partials (slices of workgroups, then the slices)
//
// Every workgroup of a point kernel owns one contiguous range of the
// Morton-ordered points (a compact region of space), so the 64 points of a
// wave usually land in one or a few pixels per layer.  The depth pass tests
// each point against the pixel's current front and combines the lanes that
// would lower a key with a wave minimum (one pixel) or segmented minima over
// runs of equal pixels; the accumulation pass combines passing lanes with a
// wave sum (one pixel) into a per-wave register cache of pixel sums, or with
// segmented sums over runs, in front of a workgroup table in LDS and the
// channel-last global sums (one L2 request per update: C lanes add its C
// channels in one instruction).
#include <type_traits>
#include "device.h"
#include "launch.h"

namespace adop {


// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------

#ifdef ADOP_RENDER_BASE
__global__ void __launch_bounds__(256) k_clear(uint64_t* __restrict__ keys, int32_t* __restrict__ counts,
                                               float* __restrict__ sums, int64_t pixels, int64_t nsum) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pixels; i += stride) {
        keys[i] = ~0ull;
        counts[i] = 0;
    }
    float4* s4 = reinterpret_cast<float4*>(sums);
    int64_t n4 = nsum / 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        s4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t i = n4 * 4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsum; i += stride)
        sums[i] = 0.f;
}
#endif  // ADOP_RENDER_BASE

// ---- depth pass -----------------------------------------------------------
// Returns the point's candidate layers: bit l is set when the point lies in
// layer l's bounds and is not yet behind the front depth read at its pixel
// by more than the fuzzy margin.  The front depth only falls, so a point
// with z > fl((1+alpha) z_read) >= fl((1+alpha) min_z) fails the fuzzy
// depth test of the accumulation pass there (Eq. depthtest, monotone FP32
// rounding): the bits are a superset of the layers where it blends.
template <bool OPTS, int LN>
__device__ __forceinline__ uint32_t depth_point(const Cam& c, int L, float fa, bool live, float x, float y, float z,
                                                const int32_t* __restrict__ orig, uint64_t i, uint32_t& oi,
                                                bool& have_oi, const PointOpts& o, const PointExtra& e,
                                                uint64_t* __restrict__ keys) {
    Proj p = project(c, x, y, z);
    bool ok = live && p.ok;
    uint32_t lmask = 0xffu;
    if (OPTS && o.flags != 0) {   // uniform: culling and discarding read per-point inputs
        ok = ok && normal_kept(o, c, p, e);
        if (ok) lmask = discard_mask(o, c, p, e, L);
    }
    // Only the depth word (the high half) of each current key is read: the
    // candidate test needs nothing else, and a point goes on to the atomic
    // when its depth is at most the front's (an equal depth may still win
    // the tie on its index; the 64-bit atomic minimum decides).
    const uint32_t* keys_hi = reinterpret_cast<const uint32_t*>(keys) + 1;
    const uint32_t zb = __float_as_uint(p.Z);
    uint32_t pix[Layers<LN>::max];
    bool in[Layers<LN>::max];
    uint32_t cur[Layers<LN>::max];
#pragma unroll
    for (int l = 0; l < Layers<LN>::max; ++l) {
        pix[l] = 0;
        in[l] = false;
        cur[l] = 0;
        if (Layers<LN>::has(l, L)) {
            int px = 0, py = 0;
            in[l] = layer_pixel(c, ok, l, p.u0, p.v0, px, py, pix[l]) && ((lmask >> l) & 1u);
            cur[l] = load_relaxed_u32(keys_hi + 2 * (uint64_t)pix[l]);   // pix is valid for every lane
        }
    }
    // keep the L gathers in flight together: nothing that uses them is
    // scheduled between them
    __builtin_amdgcn_sched_barrier(0);
    uint32_t cand = 0;
    bool any = false;
#pragma unroll
    for (int l = 0; l < Layers<LN>::max; ++l) {
        if (!Layers<LN>::has(l, L)) break;
        // an empty key reads as NaN depth: the point stays a candidate; a
        // visible depth is positive, so its bits order as the values do
        const float zr = __uint_as_float(cur[l]);
        cand |= (uint32_t)(in[l] && !(p.Z > __fmul_rn(zr, fa))) << l;
        any |= in[l] && zb <= cur[l];
    }
    if (ballot(any) == 0) return cand;
    // the original index is needed only for the atomics' keys
    if (!have_oi) {
        oi = live ? (uint32_t)ld_nt(orig + i) : 0u;
        have_oi = true;
    }
    const uint64_t key = ((uint64_t)zb << 32) | oi;
#pragma unroll
    for (int l = 0; l < Layers<LN>::max; ++l) {
        if (!Layers<LN>::has(l, L)) break;
        bool want = in[l] && zb <= cur[l];
        uint64_t m = ballot(want);
        if (m == 0) continue;
        int leader = __builtin_ctzll(m);
        uint32_t p0 = (uint32_t)__builtin_amdgcn_readlane((int)pix[l], leader);
        if (ballot(want && pix[l] != p0) == 0) {
            uint64_t k = wave_min_u64(want ? key : ~0ull);
            if (lane_id() == leader) atomic_min_u64(keys + p0, k);
        } else {
            // several pixels: segmented minima over runs of equal pixels
            uint64_t k = want ? key : ~0ull;
            if (run_min_u64(want ? pix[l] : kEmptySlot, kEmptySlot, k)) atomic_min_u64(keys + pix[l], k);
        }
    }
    return cand;
}

#ifdef ADOP_RENDER_BASE
#ifndef ADOP_DEPTH_SAMPLE
#define ADOP_DEPTH_SAMPLE 8
#endif
constexpr int64_t kDepthSample = ADOP_DEPTH_SAMPLE;   // sample stride of the depth pass's chunk order
static_assert(kDepthSample >= 2, "sample stride");
// OPTS: compiled with the optional per-point inputs (culling, discarding).
// cand (optional, [V][n]): the candidate layers of every point and view,
// read and overwritten by the accumulation pass.
template <bool SINGLE, bool OPTS, int LN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) k_depth(const float* __restrict__ xs, const float* __restrict__ ys,
                                               const float* __restrict__ zs, const int32_t* __restrict__ orig,
                                               int64_t n, const ViewRec* __restrict__ views, int V, int L,
                                               float fa, PointOpts o, uint64_t* __restrict__ keys,
                                               uint8_t* __restrict__ cand) {
    const Cam c0 = load_cam(views);
    RangeMap m = range_map(n, kBlock);
    // the next chunk's points are loaded while the current one is processed
    // (one view: the original index is loaded only by waves that reach an
    // atomic; several views, where nearly every wave does, prefetch it)
    float nx = 0.f, ny = 0.f, nz = 0.f;
    uint32_t noi = 0;
    bool nlive = false;
    PointExtra ne;
    // chunk and point numbers fit 32 bits (n < 2^31, so c * kBlock + 255 < 2^32)
    auto fetch = [&](uint32_t c) {
        const uint32_t i = c * (uint32_t)kBlock + threadIdx.x;
        nlive = (int64_t)i < n;
        if (nlive) {
            nx = ld_nt(xs + i);
            ny = ld_nt(ys + i);
            nz = ld_nt(zs + i);
            if (!SINGLE) noi = (uint32_t)ld_nt(orig + i);
            if (OPTS) load_extra(o, i, ne);
        }
    };
    // Chunk order: first every kDepthSample-th chunk of the range (a sample
    // spread over its region), then the others in order.  The minimum does
    // not depend on the order, but once every workgroup has done its sample
    // the keys hold nearly the final fronts, so the later points mostly find
    // themselves behind them: fewer atomics here and fewer candidates for the
    // accumulation pass.
    const uint32_t cs0 = (uint32_t)m.c0;
    const uint32_t len = (uint32_t)(m.c1 - m.c0);
    constexpr uint32_t kS = (uint32_t)kDepthSample;
    const uint32_t q = (len + kS - 1) / kS;
    auto chunk_at = [&](uint32_t j) -> uint32_t {
        if (j < q) return cs0 + j * kS;
        j -= q;   // j-th chunk whose offset is not a multiple of kDepthSample
        return cs0 + j + j / (kS - 1) + 1;
    };
    if (len > 0) fetch(chunk_at(0));
    for (uint32_t j = 0; j < len; ++j) {
        const uint32_t c = chunk_at(j);
        const bool live = nlive;
        const float x = nx, y = ny, z = nz;
        const uint32_t oi0 = noi;
        const PointExtra e = ne;
        if (j + 1 < len) fetch(chunk_at(j + 1));
        const uint64_t i = (uint64_t)(c * (uint32_t)kBlock + threadIdx.x);
        uint32_t oi = oi0;
        bool have_oi = !SINGLE;
        if (SINGLE) {
            const uint32_t cm = depth_point<OPTS, LN>(c0, L, fa, live, x, y, z, orig, i, oi, have_oi, o, e, keys);
            if (cand != nullptr && live) cand[i] = (uint8_t)cm;
        } else {
            for (int v = 0; v < V; ++v) {
                const uint32_t cm = depth_point<OPTS, LN>(load_cam(views + v), L, fa, live, x, y, z, orig, i, oi,
                                                          have_oi, o, e, keys);
                if (cand != nullptr && live) cand[(uint64_t)v * (uint64_t)n + i] = (uint8_t)cm;
            }
        }
    }
}
#endif  // ADOP_RENDER_BASE

// ---- accumulation pass ----------------------------------------------------

template <int C> struct AccTable {
    // slots of the per-workgroup LDS table: 1024 up to 4 channels (24 KB),
    // 128 above (more slots cost the 8-channel multi-view pass occupancy
    // and flush work than they save in global atomics)
    static constexpr int bits = C <= 4 ? 10 : 7;
    static constexpr int H = 1 << bits;
    uint32_t key[H];
    float sum[C][H];
    int32_t cnt[H];
};

// The global per-pixel FP32 sums of the accumulation, channel-last
// [pixels][C].  The L2 processes atomics per 64-byte request (measured on
// MI355X: FP32 adds of consecutive lanes to consecutive words run about 14
// times faster than one word per lane on separate lines), so a pixel's C
// sums are added with ONE instruction whose lanes 0..C-1 each take one
// channel of the same update, i.e. one request per update (plus one for
// the count), instead of C + 1 requests.
struct SumsRef {
    float* p;
};
template <int C>
__device__ __forceinline__ float* sum_at(const SumsRef& s, uint64_t pix, int c) {
    return s.p + pix * (uint64_t)C + (uint64_t)c;
}

// Adds the updates of the lanes where `has` holds to the global sums and
// counts, one update at a time: lanes 0..C-1 add its C sums with one
// lane-parallel instruction, lane C its count.  Every lane calls this.
template <int C>
__device__ __forceinline__ void global_add_coop(bool has, uint32_t pix, const float (&s)[C], int32_t k,
                                                const SumsRef& sums, int32_t* __restrict__ counts) {
    uint64_t m = ballot(has);
    const int lane = lane_id();
    while (m != 0) {
        const int src = __builtin_ctzll(m);
        m &= m - 1;
        const uint32_t p = (uint32_t)__builtin_amdgcn_readlane((int)pix, src);
        float val = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float t = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s[c]), src));
            val = lane == c ? t : val;
        }
        const int32_t kk = __builtin_amdgcn_readlane(k, src);
        if (lane < C) atomic_add_f32(sum_at<C>(sums, p, lane), val);
        else if (lane == C) atomic_add_i32(counts + p, kk);
    }
}

// Adds an update to the workgroup table; false when both probes of its
// pixel are taken by other pixels (the caller then adds it to the global
// sums).
template <int C>
__device__ __forceinline__ bool table_put(AccTable<C>& t, uint32_t pix, const float (&s)[C], int32_t k) {
    int slot = table_slot2<AccTable<C>::bits>(t.key, pix);
    if (slot < 0) return false;
#pragma unroll
    for (int c = 0; c < C; ++c)
        __hip_atomic_fetch_add(&t.sum[c][slot], s[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&t.cnt[slot], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return true;
}

// Per-wave cache of 64 pixel sums, one slot per lane (direct mapped by a
// hash of the pixel): a wave's group totals land in a register of the slot's
// lane; a slot taken by another pixel is first written to the workgroup
// table.  Consecutive Morton-ordered points hit the same pixels again, so
// most group totals never touch LDS.
template <int C> struct WaveCache {
    uint32_t key;
    float sum[C];
    int32_t cnt;
};

template <int C>
__device__ __forceinline__ void wcache_init(WaveCache<C>& w) {
    w.key = kEmptySlot;
#pragma unroll
    for (int c = 0; c < C; ++c) w.sum[c] = 0.f;
    w.cnt = 0;
}

// s and k are wave-uniform; every lane calls this.
template <int C>
__device__ __forceinline__ void wcache_add(WaveCache<C>& w, uint32_t p0, const float (&s)[C], int32_t k,
                                           AccTable<C>& t, const SumsRef& sums, int32_t* __restrict__ counts) {
    const int slot = (int)((p0 * 2654435761u) >> 26);
    const uint32_t ck = (uint32_t)__builtin_amdgcn_readlane((int)w.key, slot);
    const bool me = lane_id() == slot;
    if (ck != p0) {
        if (me) {
            // the slot's previous pixel goes to the table or, when the table
            // has no room for it (one lane, rarely), straight to the global sums
            if (ck != kEmptySlot && !table_put<C>(t, ck, w.sum, w.cnt)) {
#pragma unroll
                for (int c = 0; c < C; ++c) atomic_add_f32(sum_at<C>(sums, ck, c), w.sum[c]);
                atomic_add_i32(counts + ck, w.cnt);
            }
            w.key = p0;
#pragma unroll
            for (int c = 0; c < C; ++c) w.sum[c] = s[c];
            w.cnt = k;
        }
    } else if (me) {
#pragma unroll
        for (int c = 0; c < C; ++c) w.sum[c] += s[c];
        w.cnt += k;
    }
}

// Every lane calls this (end of a workgroup's range).
template <int C>
__device__ __forceinline__ void wcache_flush(WaveCache<C>& w, AccTable<C>& t, const SumsRef& sums,
                                             int32_t* __restrict__ counts) {
    bool spill = false;
    if (w.key != kEmptySlot) spill = !table_put<C>(t, w.key, w.sum, w.cnt);
    global_add_coop<C>(spill, w.key, w.sum, w.cnt, sums, counts);
    wcache_init<C>(w);
}

// Passing lanes that all fall into one pixel: one wave sum into the wave
// cache; otherwise segmented sums over runs of equal pixels (consecutive
// lanes), one table update per run.
template <int C>
__device__ __forceinline__ void accum_update(bool pass, uint32_t pix, const float (&f)[C], AccTable<C>& t,
                                             const SumsRef& sums, int32_t* __restrict__ counts,
                                             WaveCache<C>& w) {
    const uint64_t rem = ballot(pass);
    if (rem == 0) return;
    const int leader = __builtin_ctzll(rem);
    const uint32_t p0 = (uint32_t)__builtin_amdgcn_readlane((int)pix, leader);
    const uint64_t mm = ballot(pass && pix == p0);
    if (mm == rem) {
        float s[C];
#pragma unroll
        for (int c = 0; c < C; ++c) s[c] = pass ? f[c] : 0.0f;
        wave_sum_n<C>(s);
        wcache_add<C>(w, p0, s, __builtin_popcountll(mm), t, sums, counts);
        return;
    }
    float v[C + 1];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = pass ? f[c] : 0.0f;
    v[C] = pass ? 1.0f : 0.0f;
    const bool end = run_sums<C + 1>(pass ? pix : kEmptySlot, kEmptySlot, v);
    float s[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = v[c];
    bool spill = false;
    if (end) spill = !table_put<C>(t, pix, s, (int32_t)v[C]);
    global_add_coop<C>(spill, pix, s, (int32_t)v[C], sums, counts);
}

template <int C>
__device__ __forceinline__ void acc_table_clear(AccTable<C>& t) {
    for (int j = threadIdx.x; j < AccTable<C>::H; j += blockDim.x) {
        t.key[j] = kEmptySlot;
#pragma unroll
        for (int c = 0; c < C; ++c) t.sum[c][j] = 0.f;
        t.cnt[j] = 0;
    }
}

// Adds every occupied slot to the global sums and counts (end of the
// workgroup): the occupied slots are first listed in LDS (wave ballots and
// one LDS counter), then consecutive threads take consecutive channels of a
// listed slot, so each slot's C sums are one request.
template <int C>
__device__ __forceinline__ void acc_table_flush(AccTable<C>& t, const SumsRef& sums, int32_t* __restrict__ counts) {
    constexpr int H = AccTable<C>::H;
    __shared__ uint16_t occ[H];
    __shared__ uint32_t nocc;
    if (threadIdx.x == 0) nocc = 0;
    __syncthreads();
    for (int j0 = 0; j0 < H; j0 += blockDim.x) {
        const int j = j0 + (int)threadIdx.x;
        const bool used = j < H && t.key[j] != kEmptySlot;
        if (used) atomic_add_i32(counts + t.key[j], t.cnt[j]);
        const uint64_t m = ballot(used);
        if (m == 0) continue;
        const int lane = lane_id();
        const uint32_t before = (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1ull));
        uint32_t base = 0;
        if (lane == __builtin_ctzll(m))
            base = __hip_atomic_fetch_add(&nocc, (uint32_t)__builtin_popcountll(m), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
        base = (uint32_t)__builtin_amdgcn_readlane((int)base, __builtin_ctzll(m));
        if (used) occ[base + before] = (uint16_t)j;
    }
    __syncthreads();
    const int n = (int)nocc;
    for (int e = threadIdx.x; e < n * C; e += blockDim.x) {
        const int slot = occ[e / C], c = e - (e / C) * C;
        atomic_add_f32(sum_at<C>(sums, t.key[slot], c), t.sum[c][slot]);
    }
}

// Returns the blend-set bits of the point (bit l: it passed at layer l).
// cand: the point's candidate layers from the depth pass (0xff without).
template <int C, bool OPTS, int LN>
__device__ __forceinline__ uint32_t accum_point(const Cam& c, int L, float fa, bool live, uint32_t cand, float x,
                                                float y, float z, const float (&f)[C], const PointOpts& o,
                                                const PointExtra& e, const uint32_t* __restrict__ keys32,
                                                AccTable<C>& t, const SumsRef& sums, int32_t* __restrict__ counts,
                                                WaveCache<C>& w) {
    Proj p = project(c, x, y, z);
    bool ok = live && p.ok;
    uint32_t lmask = cand;
    if (OPTS && (o.flags & (kOptCullBack | kOptCullPrinted | kOptDiscard))) {
        ok = ok && normal_kept(o, c, p, e);
        if (ok) lmask &= discard_mask(o, c, p, e, L);
    }
    // all layers' front depths are gathered before any update, so the
    // gathers are in flight together; a lane outside a layer (or no
    // candidate there) loads nothing for it
    uint32_t pix[Layers<LN>::max];
    bool in[Layers<LN>::max];
    float mz[Layers<LN>::max];
#pragma unroll
    for (int l = 0; l < Layers<LN>::max; ++l) {
        pix[l] = 0;
        in[l] = false;
        mz[l] = 0.f;
        if (Layers<LN>::has(l, L)) {
            int px = 0, py = 0;
            in[l] = layer_pixel(c, ok, l, p.u0, p.v0, px, py, pix[l]) && ((lmask >> l) & 1u);
            if (in[l]) mz[l] = __uint_as_float(keys32[2 * (uint64_t)pix[l] + 1]);
        }
    }
    uint32_t seen = 0;
#pragma unroll
    for (int l = 0; l < Layers<LN>::max; ++l) {
        if (!Layers<LN>::has(l, L)) break;
        bool pass = in[l] && p.Z <= __fmul_rn(mz[l], fa);
        seen |= (uint32_t)pass << l;
        accum_update<C>(pass, pix[l], f, t, sums, counts, w);
    }
    return seen;
}

// One view per workgroup: with V views the grid holds one workgroup per
// point range and view (view_range_map, views dispatched in groups of
// kAccumViewGroup), so every workgroup's table and wave cache see one view's
// pixels, and the workgroups of a range in one group read its points while
// they are in the caches.
template <int C, typename S, bool OPTS, int LN>
__global__ void __launch_bounds__(256) k_accum(const float* __restrict__ xs, const float* __restrict__ ys,
                                               const float* __restrict__ zs, const void* __restrict__ feat,
                                               int64_t n, const ViewRec* __restrict__ views, int V, int L,
                                               int VG, float fa, PointOpts o, const uint32_t* __restrict__ keys32,
                                               float* __restrict__ sums_p, int64_t P, int32_t* __restrict__ counts,
                                               uint8_t* __restrict__ vis) {
    const SumsRef sums{sums_p};
    __shared__ AccTable<C> t;
    acc_table_clear<C>(t);
    __syncthreads();
    WaveCache<C> w;
    wcache_init<C>(w);
    int view = 0;
    RangeMap m = V > 1 ? view_range_map(n, kBlock, V, VG, view) : range_map(n, kBlock);
    const Cam c0 = load_cam(views + view);
    // With blend-set bits requested, vis holds the depth pass's candidate
    // layers on entry (read two chunks ahead): a point without any cannot
    // blend anywhere, so its position and features are not loaded, it is not
    // projected, and a wave without candidates only writes its zero bits.
    uint8_t* const vrow = vis != nullptr ? vis + (uint64_t)view * (uint64_t)n : nullptr;
    auto fetch_cand = [&](int64_t cc) -> uint32_t {
        const int64_t i = cc * kBlock + threadIdx.x;
        return (vrow != nullptr && i < n) ? (uint32_t)vrow[i] : 0xffu;
    };
    // the next chunk's points are loaded while the current one is processed
    float nx = 0.f, ny = 0.f, nz = 0.f;
    FeatRaw<C, S> nf;
#pragma unroll
    for (int k = 0; k < FeatRaw<C, S>::words; ++k) nf.w[k] = 0u;
    bool nlive = false;
    uint32_t ncand = 0xffu, ncand2 = 0xffu;   // candidates of chunks c + 1 and c + 2
    PointExtra ne;
    auto fetch = [&](int64_t c) {
        int64_t i = c * kBlock + threadIdx.x;
        nlive = i < n;
        if (nlive && ncand != 0) {
            nx = ld_nt(xs + i);
            ny = ld_nt(ys + i);
            nz = ld_nt(zs + i);
            load_feat_raw<C, S>(feat, i, nf);
            if (OPTS) load_extra(o, i, ne);
        }
    };
    if (m.c0 < m.c1) {
        ncand = fetch_cand(m.c0);
        fetch(m.c0);
    }
    if (m.c0 + 1 < m.c1) ncand2 = fetch_cand(m.c0 + 1);
    for (int64_t c = m.c0; c < m.c1; ++c) {
        const bool live = nlive;
        const uint32_t cand = ncand;
        const float x = nx, y = ny, z = nz;
        const FeatRaw<C, S> fr = nf;
        const PointExtra e = ne;
        ncand = ncand2;
        if (c + 1 < m.c1) fetch(c + 1);
        if (c + 2 < m.c1) ncand2 = fetch_cand(c + 2);
        const uint64_t i = (uint64_t)(c * kBlock + threadIdx.x);
        if (ballot(live && cand != 0) == 0) {
            if (vrow != nullptr && live) vrow[i] = 0;
            continue;
        }
        float f[C];
        widen_feat<C, S>(fr, f);
        if (OPTS && (o.flags & kOptLog)) {
#pragma unroll
            for (int ch = 0; ch < C; ++ch) f[ch] = expf(f[ch]);
        }
        const uint32_t seen = accum_point<C, OPTS, LN>(c0, L, fa, live && cand != 0, cand, x, y, z, f, o, e, keys32, t,
                                                   sums, counts, w);
        if (vrow != nullptr && live) vrow[i] = (uint8_t)seen;
    }
    wcache_flush<C>(w, t, sums, counts);
    __syncthreads();
    acc_table_flush<C>(t, sums, counts);
}

struct Background {
    float v[16];
};

template <int C>
__global__ void __launch_bounds__(256) k_normalize(const ViewRec* __restrict__ views, int L,
                                                   const float* __restrict__ sums, int64_t P,
                                                   const int32_t* __restrict__ counts,
                                                   float* __restrict__ images, Background bg,
                                                   const float* __restrict__ env, int S) {
    int vl = blockIdx.y;
    int v = vl / L, l = vl - (vl / L) * L;
    const ViewRec& c = views[v];
    int64_t npx = (int64_t)c.lw[l] * c.lh[l];
    uint64_t base = c.base[l];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < npx; j += (int64_t)gridDim.x * blockDim.x) {
        uint64_t p = base + (uint64_t)j;
        int32_t k = counts[p];
        const float* s = sums + p * (uint64_t)C;   // channel-last [pixels][C]
        float* out = images + (uint64_t)C * base + (uint64_t)j;
        if (k == 0 && env != nullptr) {
            const int lw = c.lw[l];
            const EnvTaps t = env_taps(c, l, (int)(j % lw), (int)(j / lw), S);
            const uint64_t plane = (uint64_t)S * (uint64_t)S;
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
                const float* e = env + (uint64_t)ch * plane;
                float val = t.w[0] * e[t.idx[0]];
                val = __fmaf_rn(t.w[1], e[t.idx[1]], val);
                val = __fmaf_rn(t.w[2], e[t.idx[2]], val);
                val = __fmaf_rn(t.w[3], e[t.idx[3]], val);
                out[(uint64_t)ch * (uint64_t)npx] = val;
            }
            continue;
        }
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
            float val = k > 0 ? __fdiv_rn(s[ch], (float)k) : bg.v[ch];
            out[(uint64_t)ch * (uint64_t)npx] = val;
        }
    }
}

// Gradient of the environment map (derivative of Eq. blend at the empty
// pixels): every empty pixel adds G(p) times its four bilinear weights to
// the texels it sampled (FP32 atomics; the order varies between runs).
template <int C>
__global__ void __launch_bounds__(256) k_env_grad(const ViewRec* __restrict__ views, int L,
                                                  const int32_t* __restrict__ counts,
                                                  const float* __restrict__ grad, float* __restrict__ env_grad,
                                                  int S) {
    int vl = blockIdx.y;
    int v = vl / L, l = vl - (vl / L) * L;
    const ViewRec& c = views[v];
    int64_t npx = (int64_t)c.lw[l] * c.lh[l];
    uint64_t base = c.base[l];
    const uint64_t plane = (uint64_t)S * (uint64_t)S;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < npx; j += (int64_t)gridDim.x * blockDim.x) {
        if (counts[base + (uint64_t)j] != 0) continue;
        const int lw = c.lw[l];
        const EnvTaps t = env_taps(c, l, (int)(j % lw), (int)(j / lw), S);
        const float* g = grad + (uint64_t)C * base + (uint64_t)j;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
            const float gc = g[(uint64_t)ch * (uint64_t)npx];
            if (gc == 0.0f) continue;
            float* e = env_grad + (uint64_t)ch * plane;
#pragma unroll
            for (int q = 0; q < 4; ++q) atomic_add_f32(e + t.idx[q], gc * t.w[q]);
        }
    }
}

#ifdef ADOP_RENDER_BASE
__global__ void __launch_bounds__(256) k_fill_zero(float* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}
#endif  // ADOP_RENDER_BASE

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------

template <int C>
__global__ void __launch_bounds__(256) k_pack(const ViewRec* __restrict__ views, int L,
                                              const uint64_t* __restrict__ keys,
                                              const int32_t* __restrict__ counts,
                                              const float* __restrict__ images,
                                              const float* __restrict__ grad,
                                              float* __restrict__ pack, float fa, Background bg, bool env) {
    using PL = PackLayout<C>;
    int vl = blockIdx.y;
    int v = vl / L, l = vl - (vl / L) * L;
    const ViewRec& c = views[v];
    int64_t npx = (int64_t)c.lw[l] * c.lh[l];
    uint64_t base = c.base[l];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < npx; j += (int64_t)gridDim.x * blockDim.x) {
        uint64_t p = base + (uint64_t)j;
        int32_t k = counts[p];
        uint32_t minz = (uint32_t)(keys[p] >> 32);
        const float* gi = grad + (uint64_t)C * base + (uint64_t)j;
        const float* ii = images + (uint64_t)C * base + (uint64_t)j;
        float rec[PL::stride];
        float gdot = 0.f;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
            float g = gi[(uint64_t)ch * (uint64_t)npx];
            // an empty pixel's value: the environment map's sample (written
            // by the forward into the image) or the constant background
            float I = (k > 0 || env) ? ii[(uint64_t)ch * (uint64_t)npx] : bg.v[ch];
            rec[ch] = g;
            gdot = __fmaf_rn(g, I, gdot);
        }
        const float inf = __builtin_inff();
        const float mzf = __uint_as_float(minz);
        rec[PL::gdot] = gdot;
        rec[PL::minz] = k > 0 ? mzf : inf;
        rec[PL::behind] = k > 0 ? __fmul_rn(mzf, fa) : inf;
        rec[PL::count] = (float)k;
#pragma unroll
        for (int q = PL::used; q < PL::stride; ++q) rec[q] = 0.f;
        float4* dst = reinterpret_cast<float4*>(pack + p * PL::stride);
#pragma unroll
        for (int q = 0; q < PL::stride / 4; ++q)
            dst[q] = make_float4(rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], rec[4 * q + 3]);
    }
}

// <G(q), dI> for the point virtually moved into neighbour q (Eq. spatialderiv):
// empty q -> tau - b; point hidden behind q (z > (1+alpha) min_z(q)) -> 0;
// point in front (z (1+alpha) < min_z(q)) -> tau - I(q); otherwise the point
// joins q's blend set -> (tau - I(q)) / (n+1).  With gdot = <G, I(q)> (or
// <G, b>), every case is factor * (<G(q), tau> - gdot).
template <int C>
__device__ __forceinline__ void load_rec(const float* __restrict__ pack, uint64_t q,
                                         float (&rec)[PackLayout<C>::stride]) {
    using PL = PackLayout<C>;
    const float4* r4 = reinterpret_cast<const float4*>(pack + q * PL::stride);
#pragma unroll
    for (int k = 0; k < PL::stride / 4; ++k) {
        float4 t4 = r4[k];
        rec[4 * k] = t4.x;
        rec[4 * k + 1] = t4.y;
        rec[4 * k + 2] = t4.z;
        rec[4 * k + 3] = t4.w;
    }
}

template <int C>
__device__ __forceinline__ float induced_rec(const float (&rec)[PackLayout<C>::stride], float Z, float Zfa,
                                             const float (&tau)[C]) {
    using PL = PackLayout<C>;
    float dot = 0.f;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) dot = __fmaf_rn(rec[ch], tau[ch], dot);
    float t = dot - rec[PL::gdot];
    float factor = __builtin_amdgcn_rcpf(rec[PL::count] + 1.0f);
    factor = (Zfa < rec[PL::minz]) ? 1.0f : factor;        // in front, or q empty
    factor = (Z > rec[PL::behind]) ? 0.0f : factor;        // hidden behind q
    return factor * t;
}

// A layer where the point is in its pixel's blend set (or every in-bounds
// point with SPATIAL_ALL): the own record and the four neighbour records are
// loaded together, then dtau += G/n (if vis) and dL/du, dL/dv.
template <int C, bool UNI>
__device__ __forceinline__ void layer_work(const float* __restrict__ pack, uint32_t pix, int qx, int qy, int lw,
                                           int lh, float Z, float fa, bool vis, const float (&tau)[C],
                                           float (&dt)[C], float& du, float& dv) {
    using PL = PackLayout<C>;
    float own[PL::stride], rr[PL::stride], rl[PL::stride], rd[PL::stride], ru[PL::stride];
    const uint32_t p0 = __builtin_amdgcn_readfirstlane(pix);
    if (UNI && ballot(pix != p0) == 0) {
        // every working lane is on one pixel (a wave's points share a
        // cluster): its five records are read once for the wave through
        // scalar loads instead of once per lane.  One view only: with several
        // views the branch costs the kernel a wave per SIMD.
        const int sx = __builtin_amdgcn_readfirstlane(qx), sy = __builtin_amdgcn_readfirstlane(qy);
        const uint64_t q = p0;
        load_rec<C>(pack, q, own);
        load_rec<C>(pack, sx + 1 < lw ? q + 1 : q, rr);
        load_rec<C>(pack, sx > 0 ? q - 1 : q, rl);
        load_rec<C>(pack, sy + 1 < lh ? q + (uint64_t)lw : q, rd);
        load_rec<C>(pack, sy > 0 ? q - (uint64_t)lw : q, ru);
    } else {
        load_rec<C>(pack, pix, own);
        load_rec<C>(pack, qx + 1 < lw ? (uint64_t)pix + 1 : (uint64_t)pix, rr);
        load_rec<C>(pack, qx > 0 ? (uint64_t)pix - 1 : (uint64_t)pix, rl);
        load_rec<C>(pack, qy + 1 < lh ? (uint64_t)pix + lw : (uint64_t)pix, rd);
        load_rec<C>(pack, qy > 0 ? (uint64_t)pix - lw : (uint64_t)pix, ru);
    }
    const bool hr = qx + 1 < lw, hl = qx > 0, hd = qy + 1 < lh, hu = qy > 0;
    if (vis) {
        float inv = __builtin_amdgcn_rcpf(own[PL::count]);
#pragma unroll
        for (int ch = 0; ch < C; ++ch) dt[ch] = __fmaf_rn(own[ch], inv, dt[ch]);
    }
    const float Zfa = __fmul_rn(Z, fa);
    float tr = hr ? induced_rec<C>(rr, Z, Zfa, tau) : 0.f;
    float tl = hl ? induced_rec<C>(rl, Z, Zfa, tau) : 0.f;
    float td = hd ? induced_rec<C>(rd, Z, Zfa, tau) : 0.f;
    float tu = hu ? induced_rec<C>(ru, Z, Zfa, tau) : 0.f;
    du = tr - tl;
    dv = td - tu;
}

// One point in one view: dL/du0, dL/dv0 summed over layers, then the chain
// through the projection; adds the 15 pose/intrinsics terms to acc (FP32).
// The layer loop is not unrolled (it keeps the kernel within the instruction
// cache); w_l = w >> l, h_l = h >> l and layer bases follow one another.
// `known`: the point's blend-set bits as the forward recorded them, or
// kVisUnknown to test the point against the records here.
constexpr uint32_t kVisUnknown = 0xffffffffu;

template <int C, bool OPTS, int LN, bool UNI, typename Terms>
__device__ __forceinline__ void point_view(const Cam& c, int L, float fa, bool spatial_all,
                                           const float* __restrict__ pack, bool live, float x, float y, float z,
                                           const float (&tau)[C], float (&dt)[C], float (&dp)[3], Terms& acc,
                                           bool& any, const PointOpts& o, const PointExtra& e, uint32_t known) {
    using PL = PackLayout<C>;
    if (known == 0) return;   // in no blend set: no gradient (known only without SPATIAL_ALL)
    Proj p = project(c, x, y, z);
    if (!(live && p.ok)) return;
    float gu = 0.f, gv = 0.f;
    // bit l of work: the layer needs the neighbour records; bit l of seen:
    // the point is in the layer's blend set
    uint32_t work = known, seen = known;
    if (known == kVisUnknown) {
        uint32_t lmask = 0xffu;
        if (OPTS && (o.flags & (kOptCullBack | kOptCullPrinted | kOptDiscard))) {
            if (!normal_kept(o, c, p, e)) return;
            lmask = discard_mask(o, c, p, e, L);
        }
        work = 0;
        seen = 0;
        float mz[Layers<LN>::max];
        bool in[Layers<LN>::max];
#pragma unroll
        for (int l = 0; l < Layers<LN>::max; ++l) {
            mz[l] = 0.f;
            in[l] = false;
            if (Layers<LN>::has(l, L)) {
                int qx = 0, qy = 0;
                uint32_t pix = 0;
                in[l] = layer_pixel(c, true, l, p.u0, p.v0, qx, qy, pix) && ((lmask >> l) & 1u);
                mz[l] = pack[(uint64_t)pix * PL::stride + PL::behind];   // pix is valid for every lane
            }
        }
#pragma unroll
        for (int l = 0; l < Layers<LN>::max; ++l) {
            const bool vis = in[l] && p.Z <= mz[l];   // Eq. depthtest against (1+alpha) min_z
            seen |= (uint32_t)vis << l;
            work |= (uint32_t)(vis || (spatial_all && in[l])) << l;
        }
    }
    uint32_t base = c.base[0];
#pragma unroll 1
    for (int l = 0; l < L; ++l) {
        const int lw = c.w >> l, lh = c.h >> l;
        const uint32_t lbase = base;
        base += (uint32_t)lw * (uint32_t)lh;
        if (!((work >> l) & 1u)) continue;
        int qx = 0, qy = 0;
        uint32_t pix = 0;
        layer_pixel_at(true, l, lw, lh, lbase, p.u0, p.v0, qx, qy, pix);
        const bool vis = (seen >> l) & 1u;
        float du = 0.f, dv = 0.f;
        layer_work<C, UNI>(pack, pix, qx, qy, lw, lh, p.Z, fa, vis, tau, dt, du, dv);
        const float s = 0.5f * layer_scale(l);
        gu = __fmaf_rn(du, s, gu);
        gv = __fmaf_rn(dv, s, gv);
    }
    if (gu == 0.f && gv == 0.f) return;
    any = true;
    const float a = p.a, b = p.b, r2 = p.r2, D = p.D;
    const float Dp = __fmaf_rn(r2, __fmaf_rn(r2, 3.0f * c.k3, 2.0f * c.k2), c.k1);
    const float xa = D + 2.0f * a * a * Dp + 2.0f * c.p1 * b + 6.0f * c.p2 * a;
    const float xb = 2.0f * a * b * Dp + 2.0f * c.p1 * a + 2.0f * c.p2 * b;
    const float yb = D + 2.0f * b * b * Dp + 6.0f * c.p1 * b + 2.0f * c.p2 * a;
    const float gux = gu * c.fx, gvy = gv * c.fy;
    const float ga = gux * xa + gvy * xb;
    const float gb = gux * xb + gvy * yb;
    const float iz = __builtin_amdgcn_rcpf(p.Z);
    const float gcx = ga * iz, gcy = gb * iz, gcz = -(a * ga + b * gb) * iz;
    dp[0] += c.R[0] * gcx + c.R[3] * gcy + c.R[6] * gcz;
    dp[1] += c.R[1] * gcx + c.R[4] * gcy + c.R[7] * gcz;
    dp[2] += c.R[2] * gcx + c.R[5] * gcy + c.R[8] * gcz;
    const float au = gux * a + gvy * b;
    const float r4 = r2 * r2;
    // the point's 15 pose/intrinsics terms in FP32, each widened to FP64
    // before it is added
    const float term[15] = {gcx, gcy, gcz,
                            p.Y * gcz - p.Z * gcy, p.Z * gcx - p.X * gcz, p.X * gcy - p.Y * gcx,
                            gu * p.xd, gv * p.yd, gu, gv,
                            au * r2, au * r4, au * r4 * r2,
                            gux * 2.0f * a * b + gvy * (r2 + 2.0f * b * b),
                            gux * (r2 + 2.0f * a * a) + gvy * 2.0f * a * b};
    acc.add(term);
}

// Where a point's 15 pose/intrinsics terms go (each widened to FP64 before
// it is added).  One view: the lane's own FP64 slots in LDS, a [15][256]
// array with one column per lane (consecutive lanes hit consecutive banks,
// no two lanes share a slot, and a lane adds its points in its own order).
// Several views: FP64 registers per view, summed over the wave afterwards.
struct LdsTerms {
    double* col;   // &slots[0][threadIdx.x]
    __device__ __forceinline__ void add(const float (&term)[15]) {
#pragma unroll
        for (int t = 0; t < 15; ++t)
            __hip_atomic_fetch_add(col + t * kBlock, (double)term[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
};
struct RegTerms {
    double v[15];
    __device__ __forceinline__ void add(const float (&term)[15]) {
#pragma unroll
        for (int t = 0; t < 15; ++t) v[t] += (double)term[t];
    }
};

// FP64 sums of the 15 terms over the wave, transposed through LDS: every
// lane writes its terms to the wave's [15][64] scratch, lane 4t + q adds
// entries 16q .. 16q + 15 of term t in order, the quarters are combined as
// (q0 + q1) + (q2 + q3), and lane 4t adds term t's sum to the wave's own
// slot.  The order is fixed, so for a fixed grid the result is too.  (The
// wave's LDS operations complete in issue order, so the reads see every
// lane's writes; the next call's writes follow these reads.)
__device__ __forceinline__ void reduce_terms(const RegTerms& acc, bool any, double* __restrict__ slot, int lane,
                                             double* __restrict__ scratch) {
    if (ballot(any) == 0) return;
#pragma unroll
    for (int t = 0; t < 15; ++t) scratch[t * kWave + lane] = acc.v[t];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int t = lane >> 2, q = lane & 3;
    double s = 0.0;
    if (lane < 60) {
        const double* col = scratch + t * kWave + q * 16;
#pragma unroll
        for (int k = 0; k < 16; ++k) s += col[k];
    }
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    if (lane < 60 && q == 0) slot[t] += s;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int C, typename S, int PPL, bool SINGLE, bool OPTS, int LN>
__global__ void __launch_bounds__(256) k_backward(const float* __restrict__ xs, const float* __restrict__ ys,
                                                  const float* __restrict__ zs, const void* __restrict__ feat,
                                                  int64_t n, const ViewRec* __restrict__ views, int V, int L,
                                                  float fa, uint32_t flags, PointOpts o,
                                                  const float* __restrict__ pack,
                                                  float* __restrict__ dfeat, float* __restrict__ dpos,
                                                  double* __restrict__ partials, const uint8_t* __restrict__ vis) {
    // one view: [15][256] per-lane FP64 slots; several views: [4 waves][V][16]
    // per-wave FP64 sums, then [4 waves][15][64] reduction scratch (dynamic LDS)
    extern __shared__ double acc_lds[];
    // When the next chunk's loads are issued (one view): 16-bit features
    // (half the bytes per load) measured faster with the loads issued before
    // this chunk's gathers (1.47 -> 1.45 ms at 100M points), FP32 features
    // faster with them issued after (1.50 -> 1.47 ms)
    constexpr bool kEarlyFetch = SINGLE && S::bytes < 4;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int slots = SINGLE ? 15 * kBlock : 4 * V * 16;
    for (int j = threadIdx.x; j < slots; j += blockDim.x) acc_lds[j] = 0.0;
    __syncthreads();
    const bool spatial_all = (flags & 1u) != 0;
    // the forward's blend-set bits replace the tests (not with SPATIAL_ALL,
    // which needs every in-bounds point)
    const bool use_vis = vis != nullptr && !spatial_all;
    const Cam c0 = load_cam(views);
    LdsTerms lterms{acc_lds + threadIdx.x};

    RangeMap m = range_map(n, (int64_t)kBlock * PPL);
    // chunk and point numbers fit 32 bits (n < 2^31, so the last chunk's
    // indices stay below 2^32)
    const uint32_t cb0 = (uint32_t)m.c0, cb1 = (uint32_t)m.c1;
    auto index = [&](uint32_t cc, int k) -> uint32_t {
        return cc * (uint32_t)(kBlock * PPL) + (uint32_t)(wave * kWave * PPL + k * kWave + lane);
    };
    // One view: the blend-set bits are loaded two chunks ahead and the
    // positions and features one chunk ahead (after the current chunk's
    // gathers), only for points with bits (a point that blends nowhere costs
    // its bit load and its zero stores).
    uint32_t kn1[PPL], kn2[PPL];   // bits of chunks c + 1 and c + 2
    float nx[PPL], ny[PPL], nz[PPL];
    FeatRaw<C, S> nf[PPL];
    PointExtra nex[PPL];
    auto bits = [&](uint32_t cc, int k) -> uint32_t {
        const uint32_t i = index(cc, k);
        return (SINGLE && use_vis && (int64_t)i < n) ? (uint32_t)vis[i] : kVisUnknown;
    };
    auto fetch = [&](uint32_t cc) {
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const uint32_t i = index(cc, k);
            if ((int64_t)i < n && kn1[k] != 0) {
                nx[k] = ld_nt(xs + i);
                ny[k] = ld_nt(ys + i);
                nz[k] = ld_nt(zs + i);
                load_feat_raw<C, S>(feat, i, nf[k]);
                if (OPTS) load_extra(o, i, nex[k]);
            }
        }
    };
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        kn1[k] = kn2[k] = kVisUnknown;
        nx[k] = ny[k] = nz[k] = 0.f;
#pragma unroll
        for (int q = 0; q < FeatRaw<C, S>::words; ++q) nf[k].w[q] = 0u;
    }
    if (cb0 < cb1) {
#pragma unroll
        for (int k = 0; k < PPL; ++k) kn1[k] = bits(cb0, k);
        fetch(cb0);
    }
    if (cb0 + 1 < cb1) {
#pragma unroll
        for (int k = 0; k < PPL; ++k) kn2[k] = bits(cb0 + 1, k);
    }
    for (uint32_t c = cb0; c < cb1; ++c) {
        float px_[PPL], py_[PPL], pz_[PPL];
        float tau[PPL][C], dt[PPL][C], dp[PPL][3];
        bool live[PPL];
        PointExtra ex[PPL];
        uint32_t known[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            known[k] = kn1[k];
            live[k] = (int64_t)index(c, k) < n;
            px_[k] = nx[k];
            py_[k] = ny[k];
            pz_[k] = nz[k];
            ex[k] = nex[k];
            widen_feat<C, S>(nf[k], tau[k]);
#pragma unroll
            for (int ch = 0; ch < C; ++ch) dt[k][ch] = 0.f;
            dp[k][0] = dp[k][1] = dp[k][2] = 0.f;
            kn1[k] = kn2[k];
        }
        if (c + 2 < cb1) {
#pragma unroll
            for (int k = 0; k < PPL; ++k) kn2[k] = bits(c + 2, k);
        }
        if (kEarlyFetch && c + 1 < cb1) fetch(c + 1);
        if (OPTS && (o.flags & kOptLog)) {   // logarithmic descriptors render as exp(f)
#pragma unroll
            for (int k = 0; k < PPL; ++k)
#pragma unroll
                for (int ch = 0; ch < C; ++ch) tau[k][ch] = expf(tau[k][ch]);
        }
        if (SINGLE) {
            bool any = false;
#pragma unroll
            for (int k = 0; k < PPL; ++k)
                point_view<C, OPTS, LN, true>(c0, L, fa, spatial_all, pack, live[k], px_[k], py_[k], pz_[k],
                                              tau[k], dt[k], dp[k], lterms, any, o, ex[k], known[k]);
        } else {
            for (int v = 0; v < V; ++v) {
                const Cam cv = load_cam(views + v);
                RegTerms acc;
#pragma unroll
                for (int t = 0; t < 15; ++t) acc.v[t] = 0.0;
                bool any = false;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    const uint32_t i = index(c, k);
                    const uint32_t kn = (use_vis && live[k]) ? (uint32_t)vis[(uint64_t)v * (uint64_t)n + (uint64_t)i]
                                                             : kVisUnknown;
                    point_view<C, OPTS, LN, false>(cv, L, fa, spatial_all, pack, live[k], px_[k], py_[k],
                                                   pz_[k], tau[k], dt[k], dp[k], acc, any, o, ex[k], kn);
                }
                reduce_terms(acc, any, acc_lds + (wave * V + v) * 16, lane,
                             acc_lds + 4 * V * 16 + wave * 15 * kWave);
            }
        }
        // FP32 features or several views: the next chunk's positions and
        // features are requested only now, as a wave's loads complete in
        // issue order and loads issued before this chunk's record gathers
        // would hold up every wait on those gathers.
        if (!kEarlyFetch && c + 1 < cb1) fetch(c + 1);
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            if (!live[k]) continue;
            const int64_t i = index(c, k);
            if (OPTS && (o.flags & kOptLog)) {   // d exp(f) / df = exp(f)
#pragma unroll
                for (int ch = 0; ch < C; ++ch) dt[k][ch] *= tau[k][ch];
            }
            store_f32_row<C>(dfeat, i, dt[k]);
            st_nt(dpos + i, dp[k][0]);
            st_nt(dpos + n + i, dp[k][1]);
            st_nt(dpos + 2 * n + i, dp[k][2]);
        }
    }
    __syncthreads();
    if (SINGLE) {
        // fixed-order FP64 sums: each wave's 64 lane columns (DPP tree),
        // then the four waves in order
        __shared__ double wsum[4][16];
#pragma unroll
        for (int t = 0; t < 15; ++t) {
            const double s = wave_sum_f64(acc_lds[t * kBlock + threadIdx.x]);
            if (lane == 0) wsum[wave][t] = s;
        }
        __syncthreads();
        if (threadIdx.x < 16) {
            const int t = threadIdx.x;
            partials[(uint64_t)blockIdx.x * 16 + t] =
                t < 15 ? ((wsum[0][t] + wsum[1][t]) + wsum[2][t]) + wsum[3][t] : 0.0;
        }
    } else {
        for (int j = threadIdx.x; j < V * 16; j += blockDim.x) {
            double s = 0.0;
            for (int w = 0; w < 4; ++w) s += acc_lds[w * V * 16 + j];
            partials[(uint64_t)blockIdx.x * V * 16 + j] = s;
        }
    }
}

// Fixed-order FP64 sums over the workgroup partials, in two stages.
// Stage 1: block (s, v) sums groups [s G / S, (s+1) G / S) of view v
// (S = kReduceSlices): each thread a strided subset in order, then a tree
// over the threads.
#ifdef ADOP_RENDER_BASE
__global__ void __launch_bounds__(256) k_reduce_slices(const double* __restrict__ partials, int groups, int V,
                                                       double* __restrict__ slices) {
    __shared__ double red[256][16];
    const int sl = blockIdx.x, v = blockIdx.y;
    const int g0 = (int)((int64_t)groups * sl / kReduceSlices);
    const int g1 = (int)((int64_t)groups * (sl + 1) / kReduceSlices);
    double s[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) s[t] = 0.0;
    for (int g = g0 + (int)threadIdx.x; g < g1; g += blockDim.x) {
        const double2* p = reinterpret_cast<const double2*>(partials + ((uint64_t)g * V + v) * 16);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const double2 d = p[t];
            s[2 * t] += d.x;
            s[2 * t + 1] += d.y;
        }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) red[threadIdx.x][t] = s[t];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int t = 0; t < 16; ++t) red[threadIdx.x][t] += red[threadIdx.x + w][t];
        }
        __syncthreads();
    }
    if (threadIdx.x < 16) slices[((uint64_t)v * kReduceSlices + sl) * 16 + threadIdx.x] = red[0][threadIdx.x];
}

// Stage 2: block v sums its slices in order; writes dpose[v], dintr[v].
__global__ void __launch_bounds__(64) k_reduce(const double* __restrict__ slices, double* __restrict__ dpose,
                                               double* __restrict__ dintr) {
    const int v = blockIdx.x, t = threadIdx.x;
    if (t >= 15) return;
    double r = 0.0;
    for (int sl = 0; sl < kReduceSlices; ++sl) r += slices[((uint64_t)v * kReduceSlices + sl) * 16 + t];
    if (t < 6) dpose[v * 6 + t] = r;
    else dintr[v * 9 + t - 6] = r;
}
#endif  // ADOP_RENDER_BASE

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline Background make_bg(const float* bg, int C) {
    Background b;
    for (int c = 0; c < 16; ++c) b.v[c] = (bg && c < C) ? bg[c] : 0.0f;
    return b;
}

static inline unsigned grid_for(int64_t items, int64_t per_group, int cap) {
    int64_t g = (items + per_group - 1) / per_group;
    g = (g + kXcds - 1) / kXcds * kXcds;
    if (g < kXcds) g = kXcds;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Resident workgroups per CU of a kernel (persistent grids).
template <typename K>
static int resident(K kernel, size_t dyn_lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, dyn_lds) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

// Persistent grid: every CU full once, a multiple of 8 (one range per
// workgroup, XCD-major), and no more workgroups than chunks.
static inline unsigned persistent_grid(int64_t n, int64_t chunk, int cus, int per_cu, int cap) {
    int64_t g = (int64_t)cus * per_cu;
    g = g / kXcds * kXcds;
    int64_t need = (n + chunk - 1) / chunk;
    need = (need + kXcds - 1) / kXcds * kXcds;
    g = std::min<int64_t>(g, need);
    g = std::min<int64_t>(g, cap);
    if (g < kXcds) g = kXcds;
    return (unsigned)g;
}

// Points per workgroup (one contiguous range of the Morton order each).
// The cost of a point varies by orders of magnitude across the scene (a
// dense cluster front blends and gathers at every layer, empty space only
// projects), so an even split over the resident workgroups leaves a long
// tail; ranges far smaller than that split let the hardware dispatcher
// balance the load.  The single-view depth pass, whose cost per point is
// nearly uniform, keeps the persistent split.
constexpr int64_t kAccumRange = 4096;       // accumulation, one view
constexpr int64_t kAccumViewRange = 2048;   // accumulation, per workgroup of one of several views
constexpr int64_t kDepthViewRange = 4096;   // depth pass, several views
// Views per dispatch group of the multi-view accumulation
constexpr int kAccumViewGroup = 4;
constexpr int64_t kBackwardRange = 4096;    // backward
// Points per lane and chunk of the backward (their loads are issued
// together, one chunk ahead).  One view: two (112 VGPRs at C = 4, 4 waves
// per SIMD; one point per lane gives 5 waves per SIMD but is slower: the two
// points' gathers are independent work for the same wave).  Several views:
// one (the per-view FP64 sums take registers of their own).
template <bool SINGLE> constexpr int bwd_points_per_lane() { return SINGLE ? 2 : 1; }

// Grid of ranges of `range` points, a multiple of 8 and at least at_least.
static inline unsigned range_grid(int64_t n, int64_t range, unsigned at_least) {
    int64_t g = (n + range - 1) / range;
    g = (g + kXcds - 1) / kXcds * kXcds;
    return (unsigned)std::max<int64_t>(g, at_least);
}

// Kernels that do not depend on the channel count or storage type are
// compiled once (render.hip); the channel-specific translation units launch
// them through these functions.
void launch_clear(const FwdArgs& a, int64_t nsums, hipStream_t st);
void launch_depth(const FwdArgs& a, hipStream_t st);
void launch_reduce(const BwdArgs& a, unsigned groups, hipStream_t st);
void launch_fill_zero(float* p, int64_t n, hipStream_t st);

template <int C, typename S, bool SINGLE, bool OPTS, int LN>
static void accum_pass(const FwdArgs& a, hipStream_t st) {
    static const int occ_accum = resident(k_accum<C, S, OPTS, LN>, 0);
    unsigned ga;
    int vg = a.V;
    if (SINGLE) {
        ga = range_grid(a.n, kAccumRange, persistent_grid(a.n, kBlock, a.cus, occ_accum, 1 << 20));
    } else {
        // R point ranges (a multiple of 8) for each view
        const unsigned per_view = persistent_grid(a.n, kBlock, a.cus, occ_accum, 1 << 20) / (unsigned)a.V;
        int64_t ranges = range_grid(a.n, kAccumViewRange, per_view);
        ranges = std::max<int64_t>(kXcds, std::min<int64_t>(ranges, (a.n + kBlock - 1) / kBlock) / kXcds * kXcds);
        ga = (unsigned)(ranges * a.V);
        vg = std::min(a.V, kAccumViewGroup);
    }
    a.timer.mark(kKAccum, 0, st);
    k_accum<C, S, OPTS, LN><<<ga, kBlock, 0, st>>>(a.x, a.y, a.z, a.feat, a.n, a.views, a.V, a.L, vg, a.fa, a.opts,
                                                      reinterpret_cast<const uint32_t*>(a.keys), a.sums, a.pixels,
                                                      a.counts, a.vis);
    a.timer.mark(kKAccum, 1, st);
}

// Fixed layer counts 4 and 5 for the plain path; the optional per-point
// inputs take the any-count kernel.
template <int C, typename S, bool SINGLE, bool OPTS>
static void forward_points(const FwdArgs& a, hipStream_t st) {
    launch_depth(a, st);
    if (!OPTS && a.L == 4) accum_pass<C, S, SINGLE, OPTS, 4>(a, st);
    else if (!OPTS && a.L == 5) accum_pass<C, S, SINGLE, OPTS, 5>(a, st);
    else accum_pass<C, S, SINGLE, OPTS, 0>(a, st);
}

template <int C, typename S>
static hipError_t forward_impl(const FwdArgs& a, hipStream_t st) {
    launch_clear(a, a.pixels * C, st);
    if (a.n > 0) {
        const bool opts = a.opts.flags != 0;
        if (a.V == 1) opts ? forward_points<C, S, true, true>(a, st) : forward_points<C, S, true, false>(a, st);
        else opts ? forward_points<C, S, false, true>(a, st) : forward_points<C, S, false, false>(a, st);
    }
    dim3 gn((unsigned)std::min<int64_t>((a.max_layer_pixels + 255) / 256, 1024), (unsigned)(a.V * a.L));
    a.timer.mark(kKNormalize, 0, st);
    k_normalize<C><<<gn, 256, 0, st>>>(a.views, a.L, a.sums, a.pixels, a.counts, a.images, make_bg(a.background, C),
                                       a.env, a.env_size);
    a.timer.mark(kKNormalize, 1, st);
    return hipGetLastError();
}

template <int C, typename S, bool SINGLE, bool OPTS, int LN>
static unsigned backward_pass(const BwdArgs& a, hipStream_t st) {
    constexpr int PPL = bwd_points_per_lane<SINGLE>();
    // several views: the per-wave view sums and the reduction scratch
    constexpr size_t kScratch = (size_t)4 * 15 * kWave * sizeof(double);
    const size_t lds = SINGLE ? (size_t)15 * kBlock * sizeof(double)
                              : (size_t)4 * a.V * 16 * sizeof(double) + kScratch;
    static const int occ = resident(k_backward<C, S, PPL, SINGLE, OPTS, LN>,
                                    SINGLE ? lds : (size_t)4 * kMaxViewsBwd * 16 * sizeof(double) + kScratch);
    unsigned g = persistent_grid(a.n, (int64_t)kBlock * PPL, a.cus, occ, a.groups);
    g = std::min<unsigned>(range_grid(a.n, kBackwardRange, g), (unsigned)a.groups / kXcds * kXcds);
    a.timer.mark(kKBackward, 0, st);
    k_backward<C, S, PPL, SINGLE, OPTS, LN><<<g, kBlock, lds, st>>>(a.x, a.y, a.z, a.feat, a.n, a.views, a.V, a.L,
                                                                     a.fa, a.flags, a.opts, a.pack, a.dfeat, a.dpos,
                                                                     a.partials, a.vis);
    a.timer.mark(kKBackward, 1, st);
    return g;
}

template <int C, typename S, bool SINGLE, bool OPTS>
static unsigned backward_points(const BwdArgs& a, hipStream_t st) {
    if (!OPTS && a.L == 4) return backward_pass<C, S, SINGLE, OPTS, 4>(a, st);
    if (!OPTS && a.L == 5) return backward_pass<C, S, SINGLE, OPTS, 5>(a, st);
    return backward_pass<C, S, SINGLE, OPTS, 0>(a, st);
}

template <int C, typename S>
static hipError_t backward_impl(const BwdArgs& a, hipStream_t st) {
    dim3 gn((unsigned)std::min<int64_t>((a.max_layer_pixels + 255) / 256, 1024), (unsigned)(a.V * a.L));
    a.timer.mark(kKPack, 0, st);
    k_pack<C><<<gn, 256, 0, st>>>(a.views, a.L, a.keys, a.counts, a.images, a.grad, a.pack, a.fa,
                                 make_bg(a.background, C), a.env != nullptr);
    if (a.env != nullptr && a.env_grad != nullptr) {
        launch_fill_zero(a.env_grad, (int64_t)C * a.env_size * a.env_size, st);
        k_env_grad<C><<<gn, 256, 0, st>>>(a.views, a.L, a.counts, a.grad, a.env_grad, a.env_size);
    }
    a.timer.mark(kKPack, 1, st);
    const bool opts = a.opts.flags != 0;
    unsigned g = a.V == 1 ? (opts ? backward_points<C, S, true, true>(a, st) : backward_points<C, S, true, false>(a, st))
                          : (opts ? backward_points<C, S, false, true>(a, st) : backward_points<C, S, false, false>(a, st));
    launch_reduce(a, g, st);
    return hipGetLastError();
}

// Channel-count groups: render_c<g>.hip instantiates the kernels of group g
// (C in 4g-3 .. 4g) for every storage type.
hipError_t forward_group(int group, const FwdArgs& a, hipStream_t st);
hipError_t backward_group(int group, const BwdArgs& a, hipStream_t st);

#define ADOP_GROUP_DISPATCH(FN, ARGS, ST, C0)                                               \
    switch (ARGS.dtype * 100 + ARGS.C) {                                                   \
        case 0 + C0: return FN<C0, F32>(ARGS, ST);                                         \
        case 0 + C0 + 1: return FN<C0 + 1, F32>(ARGS, ST);                                 \
        case 0 + C0 + 2: return FN<C0 + 2, F32>(ARGS, ST);                                 \
        case 0 + C0 + 3: return FN<C0 + 3, F32>(ARGS, ST);                                 \
        case 100 + C0: return FN<C0, BF16>(ARGS, ST);                                      \
        case 100 + C0 + 1: return FN<C0 + 1, BF16>(ARGS, ST);                              \
        case 100 + C0 + 2: return FN<C0 + 2, BF16>(ARGS, ST);                              \
        case 100 + C0 + 3: return FN<C0 + 3, BF16>(ARGS, ST);                              \
        case 200 + C0: return FN<C0, F16>(ARGS, ST);                                       \
        case 200 + C0 + 1: return FN<C0 + 1, F16>(ARGS, ST);                               \
        case 200 + C0 + 2: return FN<C0 + 2, F16>(ARGS, ST);                               \
        case 200 + C0 + 3: return FN<C0 + 3, F16>(ARGS, ST);                               \
        default: return hipErrorInvalidValue;                                              \
    }

#define ADOP_DEFINE_GROUP(G)                                                                \
    hipError_t forward_group_##G(const FwdArgs& a, hipStream_t st);                          \
    hipError_t backward_group_##G(const BwdArgs& a, hipStream_t st);

ADOP_DEFINE_GROUP(1)
ADOP_DEFINE_GROUP(2)
ADOP_DEFINE_GROUP(3)
ADOP_DEFINE_GROUP(4)

}  // namespace adop
