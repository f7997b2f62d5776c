// Channel-independent kernels of the rasterizer (clear, depth pass, FP64
// reduction) and the dispatch of render calls to the channel-count groups
// compiled in render_c1.hip .. render_c4.hip.
#define ADOP_RENDER_BASE 1
#include "render_impl.h"

namespace adop {

void launch_clear(const FwdArgs& a, int64_t nsums, hipStream_t st) {
    unsigned gp = grid_for(a.pixels, 256 * 4, a.cus * 8);
    a.timer.mark(kKClear, 0, st);
    k_clear<<<gp, 256, 0, st>>>(a.keys, a.counts, a.sums, a.pixels, nsums);
    a.timer.mark(kKClear, 1, st);
}

template <bool SINGLE, bool OPTS, int LN>
static void depth_pass(const FwdArgs& a, hipStream_t st) {
    static const int occ = resident(k_depth<SINGLE, OPTS, LN>, 0);
    unsigned gd = persistent_grid(a.n, kBlock, a.cus, occ, 1 << 20);
    if (!SINGLE) gd = range_grid(a.n, kDepthViewRange, gd);
    k_depth<SINGLE, OPTS, LN><<<gd, kBlock, 0, st>>>(a.x, a.y, a.z, a.orig, a.n, a.views, a.V, a.L, a.fa, a.opts,
                                                    a.keys, a.vis);
}

template <bool SINGLE, bool OPTS>
static void depth_layers(const FwdArgs& a, hipStream_t st) {
    switch (a.L) {
        case 4: return depth_pass<SINGLE, OPTS, 4>(a, st);
        case 5: return depth_pass<SINGLE, OPTS, 5>(a, st);
        default: return depth_pass<SINGLE, OPTS, 0>(a, st);
    }
}

void launch_depth(const FwdArgs& a, hipStream_t st) {
    const bool opts = a.opts.flags & (kOptCullBack | kOptCullPrinted | kOptDiscard);
    a.timer.mark(kKDepth, 0, st);
    if (a.V == 1) opts ? depth_layers<true, true>(a, st) : depth_layers<true, false>(a, st);
    else opts ? depth_layers<false, true>(a, st) : depth_layers<false, false>(a, st);
    a.timer.mark(kKDepth, 1, st);
}

void launch_fill_zero(float* p, int64_t n, hipStream_t st) {
    k_fill_zero<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, st>>>(p, n);
}

void launch_reduce(const BwdArgs& a, unsigned groups, hipStream_t st) {
    a.timer.mark(kKReduce, 0, st);
    k_reduce_slices<<<dim3(kReduceSlices, (unsigned)a.V), 256, 0, st>>>(a.partials, (int)groups, a.V, a.slices);
    k_reduce<<<a.V, 64, 0, st>>>(a.slices, a.dpose, a.dintr);
    a.timer.mark(kKReduce, 1, st);
}

// Atomic-throughput probe (diagnostic): op i targets word (i * stride) mod
// footprint; consecutive lanes take consecutive ops.
__global__ void __launch_bounds__(256) k_atomic_probe(int kind, int64_t ops, int64_t footprint, int64_t stride,
                                                      void* __restrict__ buf) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ops; i += step) {
        const int64_t w = (i * stride) % footprint;
        if (kind == 0)
            atomic_min_u64(static_cast<uint64_t*>(buf) + w, (uint64_t)(ops - i));
        else
            atomic_add_f32(static_cast<float*>(buf) + w, 1.0f);
    }
}

hipError_t atomic_probe(int kind, int64_t ops, int64_t footprint, int64_t stride, void* buf, int cus,
                        hipStream_t st) {
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((ops + 255) / 256, (int64_t)cus * 32));
    k_atomic_probe<<<g, 256, 0, st>>>(kind, ops, footprint, stride, buf);
    return hipGetLastError();
}

hipError_t launch_forward(const FwdArgs& a, hipStream_t st) {
    if (a.C < 1 || a.C > 16) return hipErrorInvalidValue;
    switch ((a.C - 1) / 4) {
        case 0: return forward_group_1(a, st);
        case 1: return forward_group_2(a, st);
        case 2: return forward_group_3(a, st);
        default: return forward_group_4(a, st);
    }
}

hipError_t launch_backward(const BwdArgs& a, hipStream_t st) {
    if (a.C < 1 || a.C > 16) return hipErrorInvalidValue;
    switch ((a.C - 1) / 4) {
        case 0: return backward_group_1(a, st);
        case 1: return backward_group_2(a, st);
        case 2: return backward_group_3(a, st);
        default: return backward_group_4(a, st);
    }
}

}  // namespace adop
