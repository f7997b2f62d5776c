// World radius of stochastic point discarding (Sec. 3.1, "Stochastic Point
// Discarding"): for every point, the distance to its 4th-nearest other point.
//
// Exact for the stated FP32 formula (d = p_j - p_i, squared distance
// fma(dx, dx, fma(dy, dy, dz dz)), radius = correctly rounded square root of
// the 4th smallest).  The points are sorted by a 63-bit Morton code, so the
// cells of every level of the implied octree are contiguous runs.  Level by
// level (cells of 2^k quanta), every cell that still holds an unresolved
// point searches its 3x3x3 block of cells; a point is resolved once its 4th
// distance is below the block's inner margin (one cell minus two quanta), so
// the block holds every point that could be nearer.  Points of dense regions
// resolve at fine levels, isolated ones at coarse levels; the top level (one
// cell) resolves everything left.  Work per cell is (points) x (points of its
// block); large groups of coincident points make that quadratic.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "device.h"
#include "launch.h"

namespace adop {

namespace {

constexpr int kBits = 21;                       // quanta per axis: 2^21
constexpr float kQuanta = 2097151.0f;           // 2^21 - 1
constexpr uint64_t kNonFinite = ~0ull >> 1;     // code of points with a non-finite coordinate

// float <-> int mapping that preserves the order (for atomic min / max)
__device__ __forceinline__ int key_of(float f) {
    int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float float_of(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff); }

__global__ void k_knn_init(int* bb, unsigned long long* counters) {
    if (threadIdx.x < 3) bb[threadIdx.x] = 0x7fffffff;
    else if (threadIdx.x < 6) bb[threadIdx.x] = (int)0x80000000;
    if (threadIdx.x < 2) counters[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256) k_knn_bbox(const float* __restrict__ x, const float* __restrict__ y,
                                                  const float* __restrict__ z, int64_t n, int* bb) {
    __shared__ int s[6][256];
    int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff};
    int hi[3] = {(int)0x80000000, (int)0x80000000, (int)0x80000000};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float p[3] = {x[i], y[i], z[i]};
        if (!(__builtin_isfinite(p[0]) && __builtin_isfinite(p[1]) && __builtin_isfinite(p[2]))) continue;
        for (int k = 0; k < 3; ++k) {
            lo[k] = min(lo[k], key_of(p[k]));
            hi[k] = max(hi[k], key_of(p[k]));
        }
    }
    for (int k = 0; k < 3; ++k) {
        s[k][threadIdx.x] = lo[k];
        s[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) {
                s[k][threadIdx.x] = min(s[k][threadIdx.x], s[k][threadIdx.x + w]);
                s[3 + k][threadIdx.x] = max(s[3 + k][threadIdx.x], s[3 + k][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) {
            atomicMin(&bb[k], s[k][0]);
            atomicMax(&bb[3 + k], s[3 + k][0]);
        }
}

// Quantisation of the bounding box: lo, quanta per unit length (0 on a
// degenerate axis) and the length of one quantum.
struct Grid {
    float lo[3], scale[3], unit[3];
};

__device__ __forceinline__ Grid grid_of(const int* __restrict__ bb) {
    Grid g;
    for (int k = 0; k < 3; ++k) {
        const float a = float_of(bb[k]), b = float_of(bb[3 + k]);
        const float ext = b - a;
        const bool ok = ext > 0.0f && __builtin_isfinite(ext);
        g.lo[k] = a;
        g.scale[k] = ok ? kQuanta / ext : 0.0f;
        g.unit[k] = ok ? ext / kQuanta : 0.0f;
    }
    return g;
}

__device__ __forceinline__ uint64_t spread(uint32_t v) {
    uint64_t x = v & 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t compact(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

__global__ void __launch_bounds__(256) k_knn_codes(const float* __restrict__ x, const float* __restrict__ y,
                                                   const float* __restrict__ z, int64_t n,
                                                   const int* __restrict__ bb, uint64_t* __restrict__ codes,
                                                   int32_t* __restrict__ idx, unsigned long long* counters) {
    const Grid g = grid_of(bb);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float p[3] = {x[i], y[i], z[i]};
        uint64_t code = kNonFinite;
        if (__builtin_isfinite(p[0]) && __builtin_isfinite(p[1]) && __builtin_isfinite(p[2])) {
            uint32_t q[3];
            for (int k = 0; k < 3; ++k) {
                float t = (p[k] - g.lo[k]) * g.scale[k];
                t = fminf(fmaxf(t, 0.0f), kQuanta);
                q[k] = (uint32_t)t;
            }
            code = spread(q[0]) | (spread(q[1]) << 1) | (spread(q[2]) << 2);
        } else {
            atomicAdd(&counters[0], 1ull);
        }
        codes[i] = code;
        idx[i] = (int32_t)i;
    }
}

__global__ void __launch_bounds__(256) k_knn_sorted_points(const float* __restrict__ x, const float* __restrict__ y,
                                                           const float* __restrict__ z, int64_t n,
                                                           const int32_t* __restrict__ idx, float* __restrict__ xs,
                                                           float* __restrict__ ys, float* __restrict__ zs,
                                                           float* __restrict__ radius,
                                                           uint8_t* __restrict__ resolved) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = idx[s];
        xs[s] = x[i];
        ys[s] = y[i];
        zs[s] = z[i];
        radius[i] = __builtin_inff();   // non-finite points (and too few others) keep +inf
        resolved[s] = 0;
    }
}

// head[s] = 1 where a level-`shift` cell starts (nf finite points, sorted)
__global__ void __launch_bounds__(256) k_knn_heads(const uint64_t* __restrict__ codes, int64_t nf, int shift,
                                                   int32_t* __restrict__ head) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nf; s += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = shift >= 64 ? 0 : codes[s] >> shift;
        const uint64_t p = s == 0 ? ~c : (shift >= 64 ? 0 : codes[s - 1] >> shift);
        head[s] = (s == 0 || c != p) ? 1 : 0;
    }
}

// cells in order: code (level-`shift` cell index) and first point; start[U] = nf
__global__ void __launch_bounds__(256) k_knn_cells(const uint64_t* __restrict__ codes, const int32_t* __restrict__ head,
                                                   const int32_t* __restrict__ cellid, int64_t nf, int shift,
                                                   uint64_t* __restrict__ cell_code, int32_t* __restrict__ cell_start) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nf; s += (int64_t)gridDim.x * blockDim.x) {
        if (head[s]) {
            const int32_t c = cellid[s] - 1;   // inclusive scan of the heads
            cell_code[c] = shift >= 64 ? 0 : codes[s] >> shift;
            cell_start[c] = (int32_t)s;
        }
        if (s == nf - 1) cell_start[cellid[s]] = (int32_t)nf;
    }
}

// One wave per cell of level k (2^k quanta per side) that holds an
// unresolved point.  Lanes 0..26 find the cells of the 3x3x3 block by binary
// search; then each lane takes one unresolved point of the cell and scans the
// block's points (all lanes read the same candidate, so loads are shared),
// skipping cells whose box is farther than its current 4th distance.
__global__ void __launch_bounds__(256) k_knn_search(const float* __restrict__ xs, const float* __restrict__ ys,
                                                    const float* __restrict__ zs, const int32_t* __restrict__ idx,
                                                    const uint64_t* __restrict__ cell_code,
                                                    const int32_t* __restrict__ cell_start, int64_t ncells, int k,
                                                    const int* __restrict__ bb, uint8_t* __restrict__ resolved,
                                                    float* __restrict__ radius, unsigned long long* counters) {
    const Grid g = grid_of(bb);
    const int lane = threadIdx.x % 64;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    const bool top = k >= kBits;
    const uint32_t side = top ? 1u : (1u << (kBits - k));   // cells per axis at this level
    // inner margin of the block: one cell less two quanta of the widest axis
    float hmin = __builtin_inff(), umax = 0.0f;
    for (int a = 0; a < 3; ++a) {
        if (g.unit[a] > 0.0f) hmin = fminf(hmin, g.unit[a] * (float)(1u << min(k, 30)));
        umax = fmaxf(umax, g.unit[a]);
    }
    const float margin = hmin - 2.0f * umax;
    const float accept = margin > 0.0f ? margin * margin * 0.999999f : -1.0f;
    for (int64_t c = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; c < ncells; c += waves) {
        const int32_t s0 = cell_start[c], s1 = cell_start[c + 1];
        // any unresolved point here?
        bool pending = false;
        for (int32_t b = s0; b < s1; b += 64) {
            const int32_t s = b + lane;
            pending |= s < s1 && !resolved[s];
        }
        if (__ballot(pending) == 0) continue;
        // block cells: lane j < 27 -> offsets (j % 3 - 1, j / 3 % 3 - 1, j / 9 - 1)
        const uint64_t cc = cell_code[c];
        const int cx = (int)compact(cc), cy = (int)compact(cc >> 1), cz = (int)compact(cc >> 2);
        int32_t rs = 0, re = 0;
        float blo[3] = {0.f, 0.f, 0.f}, bhi[3] = {0.f, 0.f, 0.f};
        if (lane < 27) {
            const int nxc = cx + lane % 3 - 1, nyc = cy + lane / 3 % 3 - 1, nzc = cz + lane / 9 - 1;
            const bool inside = top ? (nxc == 0 && nyc == 0 && nzc == 0)
                                    : (nxc >= 0 && nyc >= 0 && nzc >= 0 && nxc < (int)side &&
                                       nyc < (int)side && nzc < (int)side);
            if (inside) {
                const uint64_t want = top ? 0 : (spread((uint32_t)nxc) | (spread((uint32_t)nyc) << 1) |
                                                 (spread((uint32_t)nzc) << 2));
                int64_t lo = 0, hi = ncells;   // first cell with code >= want
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (cell_code[mid] < want) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < ncells && cell_code[lo] == want) {
                    rs = cell_start[lo];
                    re = cell_start[lo + 1];
                }
            }
            // the cell's box, widened by two quanta for the quantisation
            const int nc[3] = {nxc, nyc, nzc};
            for (int a = 0; a < 3; ++a) {
                const float q = g.unit[a] * (float)(1u << min(k, 30));
                blo[a] = g.lo[a] + (float)nc[a] * q - 2.0f * g.unit[a];
                bhi[a] = g.lo[a] + (float)(nc[a] + 1) * q + 2.0f * g.unit[a];
            }
        }
        for (int32_t b = s0; b < s1; b += 64) {
            const int32_t s = b + lane;
            const bool mine = s < s1 && !resolved[s];
            if (__ballot(mine) == 0) continue;
            const float px = mine ? xs[s] : 0.f, py = mine ? ys[s] : 0.f, pz = mine ? zs[s] : 0.f;
            float best0 = __builtin_inff(), best1 = best0, best2 = best0, best3 = best0;
            for (int t = 0; t < 27; ++t) {
                const int j = t == 0 ? 13 : (t <= 13 ? t - 1 : t);   // own cell first
                const int32_t a0 = __shfl(rs, j), a1 = __shfl(re, j);
                if (a0 >= a1) continue;
                float d2box = 0.f;
                {
                    const float l0 = __shfl(blo[0], j), l1 = __shfl(blo[1], j), l2 = __shfl(blo[2], j);
                    const float h0 = __shfl(bhi[0], j), h1 = __shfl(bhi[1], j), h2 = __shfl(bhi[2], j);
                    const float ex = fmaxf(fmaxf(l0 - px, px - h0), 0.f);
                    const float ey = fmaxf(fmaxf(l1 - py, py - h1), 0.f);
                    const float ez = fmaxf(fmaxf(l2 - pz, pz - h2), 0.f);
                    d2box = ex * ex + ey * ey + ez * ez;
                }
                const bool use = mine && (top || !(d2box > best3 * 1.000001f));
                if (__ballot(use) == 0) continue;
                for (int32_t q = a0; q < a1; ++q) {
                    const float qx = xs[q], qy = ys[q], qz = zs[q];
                    if (!use || q == s) continue;
                    const float dx = __fsub_rn(qx, px), dy = __fsub_rn(qy, py), dz = __fsub_rn(qz, pz);
                    const float d2 = __fmaf_rn(dx, dx, __fmaf_rn(dy, dy, __fmul_rn(dz, dz)));
                    if (!(d2 < best3)) continue;
                    if (d2 < best2) {
                        best3 = best2;
                        if (d2 < best1) {
                            best2 = best1;
                            if (d2 < best0) {
                                best1 = best0;
                                best0 = d2;
                            } else {
                                best1 = d2;
                            }
                        } else {
                            best2 = d2;
                        }
                    } else {
                        best3 = d2;
                    }
                }
            }
            if (mine) {
                if (top || best3 <= accept) {
                    radius[idx[s]] = sqrt_rn(best3);
                    resolved[s] = 1;
                } else {
                    atomicAdd(&counters[1], 1ull);
                }
            }
        }
    }
}

struct Buf {
    void* p = nullptr;
    ~Buf() { if (p) (void)hipFree(p); }
};

}  // namespace

hipError_t knn_radius(const float* x, const float* y, const float* z, int64_t n, float* radius, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipError_t e;
#define ADOP_CK(call) do { e = (call); if (e != hipSuccess) return e; } while (0)
    Buf bb, cnt, codes, codes2, idx, idx2, xs, ys, zs, res, head, cellid, ccode, cstart, tmp;
    ADOP_CK(hipMalloc(&bb.p, 6 * sizeof(int)));
    ADOP_CK(hipMalloc(&cnt.p, 2 * sizeof(unsigned long long)));
    ADOP_CK(hipMalloc(&codes.p, n * sizeof(uint64_t)));
    ADOP_CK(hipMalloc(&codes2.p, n * sizeof(uint64_t)));
    ADOP_CK(hipMalloc(&idx.p, n * sizeof(int32_t)));
    ADOP_CK(hipMalloc(&idx2.p, n * sizeof(int32_t)));
    ADOP_CK(hipMalloc(&xs.p, n * sizeof(float)));
    ADOP_CK(hipMalloc(&ys.p, n * sizeof(float)));
    ADOP_CK(hipMalloc(&zs.p, n * sizeof(float)));
    ADOP_CK(hipMalloc(&res.p, n));
    ADOP_CK(hipMalloc(&head.p, n * sizeof(int32_t)));
    ADOP_CK(hipMalloc(&cellid.p, n * sizeof(int32_t)));
    ADOP_CK(hipMalloc(&ccode.p, n * sizeof(uint64_t)));
    ADOP_CK(hipMalloc(&cstart.p, (n + 1) * sizeof(int32_t)));
    unsigned long long* counters = (unsigned long long*)cnt.p;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    k_knn_init<<<1, 64, 0, st>>>((int*)bb.p, counters);
    k_knn_bbox<<<g, 256, 0, st>>>(x, y, z, n, (int*)bb.p);
    k_knn_codes<<<g, 256, 0, st>>>(x, y, z, n, (const int*)bb.p, (uint64_t*)codes.p, (int32_t*)idx.p, counters);
    ADOP_CK(hipGetLastError());
    size_t tb = 0, tb2 = 0;
    ADOP_CK(rocprim::radix_sort_pairs(nullptr, tb, (uint64_t*)codes.p, (uint64_t*)codes2.p, (int32_t*)idx.p,
                                      (int32_t*)idx2.p, (size_t)n, 0, 63, st));
    ADOP_CK(rocprim::inclusive_scan(nullptr, tb2, (const int32_t*)head.p, (int32_t*)cellid.p, (size_t)n,
                                    rocprim::plus<int32_t>(), st));
    ADOP_CK(hipMalloc(&tmp.p, std::max(tb, tb2)));
    size_t tbytes = std::max(tb, tb2);
    ADOP_CK(rocprim::radix_sort_pairs(tmp.p, tbytes, (uint64_t*)codes.p, (uint64_t*)codes2.p, (int32_t*)idx.p,
                                      (int32_t*)idx2.p, (size_t)n, 0, 63, st));
    k_knn_sorted_points<<<g, 256, 0, st>>>(x, y, z, n, (const int32_t*)idx2.p, (float*)xs.p, (float*)ys.p,
                                           (float*)zs.p, radius, (uint8_t*)res.p);
    ADOP_CK(hipGetLastError());
    unsigned long long host_cnt[2] = {0, 0};
    ADOP_CK(hipMemcpyAsync(host_cnt, counters, sizeof(host_cnt), hipMemcpyDeviceToHost, st));
    int host_bb[6];
    ADOP_CK(hipMemcpyAsync(host_bb, bb.p, sizeof(host_bb), hipMemcpyDeviceToHost, st));
    ADOP_CK(hipStreamSynchronize(st));
    const int64_t nf = n - (int64_t)host_cnt[0];   // finite points come first in the sorted order
    if (nf <= 0) return hipSuccess;
    // first level: cells of about a quarter of the mean spacing
    double ext[3], vol = 1.0, emax = 0.0, umin = 0.0, umax = 0.0;
    int ndim = 0;
    for (int a = 0; a < 3; ++a) {
        const int lo = host_bb[a], hi = host_bb[3 + a];
        float flo, fhi;
        const int ulo = lo >= 0 ? lo : lo ^ 0x7fffffff, uhi = hi >= 0 ? hi : hi ^ 0x7fffffff;
        std::memcpy(&flo, &ulo, 4);
        std::memcpy(&fhi, &uhi, 4);
        ext[a] = (double)fhi - (double)flo;
        if (ext[a] > 0.0 && std::isfinite(ext[a])) {
            vol *= ext[a];
            ++ndim;
            emax = std::max(emax, ext[a]);
            const double u = ext[a] / (double)kQuanta;
            umin = umin == 0.0 ? u : std::min(umin, u);
            umax = std::max(umax, u);
        }
    }
    int k0 = 0;
    if (ndim > 0 && umin > 0.0) {
        const double spacing = std::pow(vol / (double)nf, 1.0 / ndim);
        const double want = 0.25 * spacing / umin;
        k0 = want > 1.0 ? std::min(kBits, (int)std::floor(std::log2(want))) : 0;
    }
    for (int k = k0; k <= kBits; ++k) {
        // a level whose cells are not wider than the quantisation margin
        // cannot resolve anything
        if (k < kBits && umin > 0.0 && umin * std::ldexp(1.0, k) <= 2.5 * umax) continue;
        const int shift = k >= kBits ? 64 : 3 * k;
        k_knn_heads<<<g, 256, 0, st>>>((const uint64_t*)codes2.p, nf, shift, (int32_t*)head.p);
        ADOP_CK(hipGetLastError());
        size_t tbytes2 = std::max(tb, tb2);
        ADOP_CK(rocprim::inclusive_scan(tmp.p, tbytes2, (const int32_t*)head.p, (int32_t*)cellid.p, (size_t)nf,
                                        rocprim::plus<int32_t>(), st));
        k_knn_cells<<<g, 256, 0, st>>>((const uint64_t*)codes2.p, (const int32_t*)head.p, (const int32_t*)cellid.p,
                                       nf, shift, (uint64_t*)ccode.p, (int32_t*)cstart.p);
        ADOP_CK(hipGetLastError());
        int32_t ncells = 0;
        ADOP_CK(hipMemcpyAsync(&ncells, (const int32_t*)cellid.p + (nf - 1), sizeof(int32_t), hipMemcpyDeviceToHost,
                               st));
        ADOP_CK(hipMemsetAsync(counters + 1, 0, sizeof(unsigned long long), st));
        ADOP_CK(hipStreamSynchronize(st));
        const unsigned gs = (unsigned)std::min<int64_t>((ncells + 3) / 4, 65536);
        k_knn_search<<<gs, 256, 0, st>>>((const float*)xs.p, (const float*)ys.p, (const float*)zs.p,
                                         (const int32_t*)idx2.p, (const uint64_t*)ccode.p, (const int32_t*)cstart.p,
                                         ncells, k, (const int*)bb.p, (uint8_t*)res.p, radius, counters);
        ADOP_CK(hipGetLastError());
        unsigned long long left = 0;
        ADOP_CK(hipMemcpyAsync(&left, counters + 1, sizeof(left), hipMemcpyDeviceToHost, st));
        ADOP_CK(hipStreamSynchronize(st));
        if (left == 0) break;
    }
#undef ADOP_CK
    return hipSuccess;
}

}  // namespace adop
