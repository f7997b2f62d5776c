// Host-side launch interface between the C-ABI layer (api.cpp) and the
// kernels (render.hip, scene.hip).  Plain structs of device pointers and sizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adop {

struct ViewRec;

// Points are processed in 8 segments (one per XCD) whose boundaries are
// multiples of this many points; scene preparation shuffles blocks inside
// the same segments.
constexpr int64_t kSegAlign = 1024;

// Optional per-kernel timing: the launchers call fn(self, kernel, 0, stream)
// before and fn(self, kernel, 1, stream) after each kernel they enqueue.
enum KernelId { kKClear = 0, kKDepth, kKAccum, kKNormalize, kKPack, kKBackward, kKReduce, kKernelCount };
struct Timer {
    void (*fn)(void* self, int kernel, int end, hipStream_t st) = nullptr;
    void* self = nullptr;
    void mark(int k, int end, hipStream_t st) const {
        if (fn) fn(self, k, end, st);
    }
};

// Optional per-point inputs and switches of the point kernels (normal
// culling, logarithmic features, stochastic discarding).
struct PointOpts {
    uint32_t flags;        // kOpt* bits
    float gamma;
    const float *nx, *ny, *nz;
    const float *radius, *beta;
};
constexpr uint32_t kOptCullBack = 2u, kOptCullPrinted = 4u, kOptLog = 8u, kOptDiscard = 16u;

struct FwdArgs {
    int dtype, C, V, L, cus;
    int64_t n, pixels, max_layer_pixels;
    float fa;
    const float *x, *y, *z;
    const void* feat;
    const int32_t* orig;
    const ViewRec* views;
    uint64_t* keys;
    int32_t* counts;
    float* sums;       // workspace [pixels][C]
    float* images;
    const float* background;   // host [C] or null
    const float* env = nullptr;   // optional environment map [C][S][S] (empty pixels sample it)
    int env_size = 0;
    PointOpts opts;
    uint8_t* vis = nullptr;   // optional [V][n] blend-set bits per point and view
    Timer timer;
};

// The FP64 pose/intrinsics partials of the backward workgroups are summed
// in two fixed-order stages: kReduceSlices contiguous slices per view, then
// the slices.
constexpr int kReduceSlices = 64;
// Largest backward grid per CU (the partials buffer is sized for it).
constexpr int kBwdGroupsPerCu = 128;

struct BwdArgs {
    int dtype, C, V, L, cus, groups;   // groups: largest backward grid the partials buffer holds
    uint32_t flags;
    int64_t n, pixels, max_layer_pixels;
    float fa;
    const float *x, *y, *z;
    const void* feat;
    const ViewRec* views;
    const uint64_t* keys;
    const int32_t* counts;
    const float* images;
    const float* grad;
    PointOpts opts;
    float* pack;       // workspace [pixels][stride]
    double* partials;  // workspace [groups][V][16]
    double* slices;    // workspace [V][kReduceSlices][16]
    float* dfeat;
    float* dpos;
    double* dpose;
    double* dintr;
    const float* background;
    const float* env = nullptr;     // environment map of the forward, if any
    int env_size = 0;
    float* env_grad = nullptr;      // optional [C][S][S] output: the map's gradient
    const uint8_t* vis = nullptr;   // optional [V][n], written by the forward
    Timer timer;
};

hipError_t launch_forward(const FwdArgs& a, hipStream_t st);
hipError_t launch_backward(const BwdArgs& a, hipStream_t st);
inline int pack_stride(int C) { return (C + 4 + 3) / 4 * 4; }

// Atomic-throughput probe: `ops` atomics of one kind (0: u64 minimum, 1: FP32
// add) on words (i * stride) mod footprint of `buf`.
hipError_t atomic_probe(int kind, int64_t ops, int64_t footprint, int64_t stride, void* buf, int cus,
                        hipStream_t st);

// Photometric tone mapper (Sec. 3.3) of V 3-channel images [V][3][h][w].
struct TonemapArgs {
    int V, w, h, K;
    float leak;                 // >= 0 leaky response, < 0 clamp
    const float* hdr;
    const float* ev;            // [V]
    const float* white;         // [V][3]
    const float* vig;           // [5] a2, a4, a6, cx, cy
    const float* crf;           // [3][K]
    float* ldr;                 // forward output
    const float* grad;          // backward: dL/dldr
    float* d_hdr;
    double *d_ev, *d_white, *d_vig, *d_crf;
    double* partials;           // workspace [V][kTonemapBlocks][16]
};
constexpr int kTonemapBlocks = 128;     // blocks per view (grid-stride over its pixels)
constexpr int kTonemapMaxTable = 1024;  // largest response table (LDS gradient table of 3 K doubles)
hipError_t tonemap_forward(const TonemapArgs& a, hipStream_t st);
hipError_t tonemap_backward(const TonemapArgs& a, hipStream_t st);

struct PrepArgs {
    int64_t n;
    int C, dtype, block;
    uint64_t seed;
    const float* pos;
    const void* feat;
    float *x, *y, *z;
    void* feat_out;
    int32_t* orig;
};
// Returns hipSuccess or the first HIP error; allocates temporaries.
hipError_t scene_prepare(const PrepArgs& a, hipStream_t st);
// dst[k * n + i] = src[orig[i] * comp + k]
hipError_t scene_gather(const float* src, int comp, int64_t n, const int32_t* orig, float* dst, hipStream_t st);
// distance of every point to its 4th-nearest other point (allocates; synchronises st)
hipError_t knn_radius(const float* x, const float* y, const float* z, int64_t n, float* radius, hipStream_t st);

}  // namespace adop
