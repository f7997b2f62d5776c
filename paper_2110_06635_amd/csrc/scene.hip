// Scene preparation: the blocked Morton shuffle of the point cloud (ADOP
// Sec. 3.1, "Implementation Details", after Schuetz et al. 2021).
//
// 1. bounding box of the finite positions
// 2. 63-bit Morton code (21 bits per axis) per point; non-finite points sort last
// 3. radix sort of (code, index) pairs (rocPRIM)
// 4. optionally, the sorted order is cut into 8 segments and blocks of
//    `block` points are shuffled inside each segment with a seeded
//    permutation (the shuffle of Schuetz et al.; the render kernels here give
//    every workgroup a contiguous range instead, so the default is none)
// 5. gather into SoA position planes, the feature array and orig_index.
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cstring>
#include <vector>

#include "launch.h"

namespace adop {

namespace {

__device__ __forceinline__ int ordered(float f) {
    int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float unordered(int i) {
    return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff);
}

__global__ void k_bbox_init(int* bb) {
    if (threadIdx.x < 3) bb[threadIdx.x] = 0x7fffffff;
    else if (threadIdx.x < 6) bb[threadIdx.x] = (int)0x80000000;
}

__global__ void __launch_bounds__(256) k_bbox(const float* __restrict__ pos, int64_t n, int* bb) {
    __shared__ int s[6][256];
    int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff};
    int hi[3] = {(int)0x80000000, (int)0x80000000, (int)0x80000000};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float p0 = pos[3 * i], p1 = pos[3 * i + 1], p2 = pos[3 * i + 2];
        if (!(__builtin_isfinite(p0) && __builtin_isfinite(p1) && __builtin_isfinite(p2))) continue;
        int q[3] = {ordered(p0), ordered(p1), ordered(p2)};
        for (int k = 0; k < 3; ++k) {
            lo[k] = min(lo[k], q[k]);
            hi[k] = max(hi[k], q[k]);
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

__device__ __forceinline__ uint64_t spread21(uint32_t v) {
    uint64_t x = v & 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ void __launch_bounds__(256) k_morton(const float* __restrict__ pos, int64_t n, const int* __restrict__ bb,
                                                uint64_t* __restrict__ codes, int32_t* __restrict__ idx) {
    float lo[3], scale[3];
    for (int k = 0; k < 3; ++k) {
        float a = unordered(bb[k]), b = unordered(bb[3 + k]);
        lo[k] = a;
        float ext = b - a;
        scale[k] = (ext > 0.0f && __builtin_isfinite(ext)) ? 2097151.0f / ext : 0.0f;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        uint64_t code;
        if (__builtin_isfinite(p[0]) && __builtin_isfinite(p[1]) && __builtin_isfinite(p[2])) {
            uint32_t q[3];
            for (int k = 0; k < 3; ++k) {
                float t = (p[k] - lo[k]) * scale[k];
                t = fminf(fmaxf(t, 0.0f), 2097151.0f);
                q[k] = (uint32_t)t;
            }
            code = spread21(q[0]) | (spread21(q[1]) << 1) | (spread21(q[2]) << 2);
        } else {
            code = ~0ull >> 1;
        }
        codes[i] = code;
        idx[i] = (int32_t)i;
    }
}

// out position of sorted element s: its block (inside its segment) is moved
// to out_off[block id].
__global__ void __launch_bounds__(256) k_gather(const float* __restrict__ pos, const unsigned char* __restrict__ feat,
                                                int64_t n, int rowbytes, const int32_t* __restrict__ sorted_idx,
                                                const int64_t* __restrict__ seg, const int64_t* __restrict__ blk_base,
                                                const int64_t* __restrict__ out_off, int block,
                                                float* __restrict__ x, float* __restrict__ y, float* __restrict__ z,
                                                unsigned char* __restrict__ feat_out, int32_t* __restrict__ orig) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        int xsg = 0;
        while (xsg < 7 && s >= seg[xsg + 1]) ++xsg;
        int64_t local = s - seg[xsg];
        int64_t b = blk_base[xsg] + local / block;
        int64_t o = out_off[b] + local % block;
        int32_t src = sorted_idx[s];
        x[o] = pos[3 * (int64_t)src];
        y[o] = pos[3 * (int64_t)src + 1];
        z[o] = pos[3 * (int64_t)src + 2];
        orig[o] = src;
        const unsigned char* fs = feat + (int64_t)src * rowbytes;
        unsigned char* fo = feat_out + o * rowbytes;
        if ((rowbytes & 3) == 0) {
            for (int k = 0; k < rowbytes; k += 4)
                *reinterpret_cast<uint32_t*>(fo + k) = *reinterpret_cast<const uint32_t*>(fs + k);
        } else {
            for (int k = 0; k < rowbytes; k += 2)
                *reinterpret_cast<uint16_t*>(fo + k) = *reinterpret_cast<const uint16_t*>(fs + k);
        }
    }
}

uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

int64_t host_segment_bound(int64_t n, int x) {
    if (x >= 8) return n;
    int64_t b = (n * x) / 8;
    return b / kSegAlign * kSegAlign;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

__global__ void __launch_bounds__(256) k_scene_gather(const float* __restrict__ src, int comp, int64_t n,
                                                      const int32_t* __restrict__ orig, float* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = orig[i];
        for (int k = 0; k < comp; ++k) dst[(int64_t)k * n + i] = src[o * comp + k];
    }
}

}  // namespace

hipError_t scene_gather(const float* src, int comp, int64_t n, const int32_t* orig, float* dst, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    k_scene_gather<<<g, 256, 0, st>>>(src, comp, n, orig, dst);
    return hipGetLastError();
}

hipError_t scene_prepare(const PrepArgs& a, hipStream_t st) {
    const int64_t n = a.n;
    if (n == 0) return hipSuccess;
    const int esize = a.dtype == 0 ? 4 : 2;
    const int rowbytes = a.C * esize;
    hipError_t e;
    DevBuf bb, codes, codes2, idx, idx2, tmp, meta;
#define ADOP_CK(x) do { e = (x); if (e != hipSuccess) return e; } while (0)
    ADOP_CK(hipMalloc(&bb.p, 6 * sizeof(int)));
    ADOP_CK(hipMalloc(&codes.p, n * sizeof(uint64_t)));
    ADOP_CK(hipMalloc(&codes2.p, n * sizeof(uint64_t)));
    ADOP_CK(hipMalloc(&idx.p, n * sizeof(int32_t)));
    ADOP_CK(hipMalloc(&idx2.p, n * sizeof(int32_t)));
    unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    k_bbox_init<<<1, 64, 0, st>>>((int*)bb.p);
    k_bbox<<<g, 256, 0, st>>>(a.pos, n, (int*)bb.p);
    k_morton<<<g, 256, 0, st>>>(a.pos, n, (const int*)bb.p, (uint64_t*)codes.p, (int32_t*)idx.p);
    ADOP_CK(hipGetLastError());
    size_t tmp_bytes = 0;
    ADOP_CK(rocprim::radix_sort_pairs(nullptr, tmp_bytes, (uint64_t*)codes.p, (uint64_t*)codes2.p,
                                      (int32_t*)idx.p, (int32_t*)idx2.p, (size_t)n, 0, 63, st));
    ADOP_CK(hipMalloc(&tmp.p, tmp_bytes));
    ADOP_CK(rocprim::radix_sort_pairs(tmp.p, tmp_bytes, (uint64_t*)codes.p, (uint64_t*)codes2.p,
                                      (int32_t*)idx.p, (int32_t*)idx2.p, (size_t)n, 0, 63, st));

    // block permutation inside each segment (host); block == 0 keeps the
    // plain Morton order
    const bool shuffle = a.block > 0;
    const int block = shuffle ? a.block : 1024;
    std::vector<int64_t> seg(9), blk_base(9);
    for (int x = 0; x <= 8; ++x) seg[x] = host_segment_bound(n, x);
    int64_t nblocks = 0;
    for (int x = 0; x < 8; ++x) {
        blk_base[x] = nblocks;
        nblocks += (seg[x + 1] - seg[x] + block - 1) / block;
    }
    blk_base[8] = nblocks;
    std::vector<int64_t> out_off(std::max<int64_t>(nblocks, 1));
    uint64_t rs = a.seed;
    for (int x = 0; x < 8; ++x) {
        int64_t nb = blk_base[x + 1] - blk_base[x];
        if (nb == 0) continue;
        std::vector<int64_t> order(nb);
        for (int64_t k = 0; k < nb; ++k) order[k] = k;
        for (int64_t k = nb - 1; shuffle && k > 0; --k) {
            int64_t j = (int64_t)(splitmix64(rs) % (uint64_t)(k + 1));
            std::swap(order[k], order[j]);
        }
        int64_t len = seg[x + 1] - seg[x];
        int64_t off = seg[x];
        for (int64_t k = 0; k < nb; ++k) {
            int64_t b = order[k];
            int64_t sz = std::min<int64_t>(block, len - b * block);
            out_off[blk_base[x] + b] = off;
            off += sz;
        }
    }
    size_t meta_bytes = (9 + 9 + out_off.size()) * sizeof(int64_t);
    ADOP_CK(hipMalloc(&meta.p, meta_bytes));
    std::vector<int64_t> host_meta;
    host_meta.insert(host_meta.end(), seg.begin(), seg.end());
    host_meta.insert(host_meta.end(), blk_base.begin(), blk_base.end());
    host_meta.insert(host_meta.end(), out_off.begin(), out_off.end());
    ADOP_CK(hipMemcpyAsync(meta.p, host_meta.data(), meta_bytes, hipMemcpyHostToDevice, st));
    const int64_t* dm = (const int64_t*)meta.p;
    k_gather<<<g, 256, 0, st>>>(a.pos, (const unsigned char*)a.feat, n, rowbytes, (const int32_t*)idx2.p, dm, dm + 9,
                                dm + 18, block, a.x, a.y, a.z, (unsigned char*)a.feat_out, a.orig);
    ADOP_CK(hipGetLastError());
    ADOP_CK(hipStreamSynchronize(st));
#undef ADOP_CK
    return hipSuccess;
}

}  // namespace adop
