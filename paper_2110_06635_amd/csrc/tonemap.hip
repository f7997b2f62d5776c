// Photometric tone mapper of ADOP Sec. 3.3 ("Differentiable Tone Mapping")
// for V 3-channel images [V][3][h][w] FP32, forward and backward (gfx950).
//
// Per image i and pixel (u, v):
//   I_e = I_hdr * 2^-EV_i                          (exposure)
//   I_w[c] = I_e[c] * W_i[c]                       (white point)
//   I_v = I_w * (1 + a2 r^2 + a4 r^4 + a6 r^6),    r = |p - c_v|,
//       p = ((u + 0.5) / w, (v + 0.5) / h)         (vignette, normalised coordinates)
//   I_ldr[c] = R_t(I_v[c])                         (response, Eq. resonseleak)
// R on [0, 1] is a table of K entries per channel sampled at k / (K - 1) and
// linearly interpolated; R_t(x) = leak x below 0 and -leak / sqrt(x) + leak + 1
// above 1; a negative leak clamps the input to [0, 1] instead (inference).
//
// Backward: dL/dI_hdr per pixel; the per-image exposure and white-point
// gradients and the vignette gradients are FP64 sums in a fixed order
// (wave DPP tree, the block's four waves, then the blocks of a view in
// order, then the views); the table gradient is summed per block in LDS and
// added to the output with FP64 atomics (its order varies between runs).
#include <hip/hip_runtime.h>
#include "device.h"
#include "launch.h"

namespace adop {

namespace {

constexpr float kLn2 = 0.693147180559945309f;

struct Px {
    float r2, dx, dy, vf, dvdr2;
};

__device__ __forceinline__ Px pixel_geom(int j, int w, int h, const float* __restrict__ vig) {
    const int u = j % w, v = j / w;
    Px g;
    const float px = ((float)u + 0.5f) / (float)w, py = ((float)v + 0.5f) / (float)h;
    g.dx = px - vig[3];
    g.dy = py - vig[4];
    g.r2 = g.dx * g.dx + g.dy * g.dy;
    const float a2 = vig[0], a4 = vig[1], a6 = vig[2];
    g.vf = 1.0f + g.r2 * (a2 + g.r2 * (a4 + g.r2 * a6));
    g.dvdr2 = a2 + g.r2 * (2.0f * a4 + 3.0f * a6 * g.r2);
    return g;
}

// R_t(x) of one channel; slope = dR_t/dx, (i, f, used) the table weights.
__device__ __forceinline__ float response(const float* __restrict__ T, int K, float x, float leak, float& slope,
                                          int& i, float& f, bool& used) {
    const float xc = fminf(fmaxf(x, 0.0f), 1.0f);
    const float pos = xc * (float)(K - 1);
    i = min((int)floorf(pos), K - 2);
    f = pos - (float)i;
    const float t0 = T[i], t1 = T[i + 1];
    const float mid = (1.0f - f) * t0 + f * t1;
    const float tslope = (t1 - t0) * (float)(K - 1);
    if (leak < 0.0f) {
        used = true;
        slope = (x >= 0.0f && x <= 1.0f) ? tslope : 0.0f;
        return mid;
    }
    if (x < 0.0f) {
        used = false;
        slope = leak;
        return leak * x;
    }
    if (x > 1.0f) {
        used = false;
        const float s = sqrtf(x);
        slope = 0.5f * leak / (x * s);
        return -leak / s + leak + 1.0f;
    }
    used = true;
    slope = tslope;
    return mid;
}

__global__ void __launch_bounds__(256) k_tm_fwd(TonemapArgs a) {
    const int view = blockIdx.y;
    const int64_t P = (int64_t)a.w * a.h;
    const float scale = exp2f(-a.ev[view]);
    const float* src = a.hdr + (int64_t)view * 3 * P;
    float* dst = a.ldr + (int64_t)view * 3 * P;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P; j += (int64_t)gridDim.x * blockDim.x) {
        const Px g = pixel_geom((int)j, a.w, a.h, a.vig);
        for (int c = 0; c < 3; ++c) {
            const float x = src[c * P + j] * scale * a.white[3 * view + c] * g.vf;
            float slope, f;
            int i;
            bool used;
            dst[c * P + j] = response(a.crf + c * a.K, a.K, x, a.leak, slope, i, f, used);
        }
    }
}

__global__ void __launch_bounds__(256) k_tm_zero(double* __restrict__ p, int n) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) p[j] = 0.0;
}

__global__ void __launch_bounds__(256) k_tm_bwd(TonemapArgs a) {
    __shared__ double table[3 * kTonemapMaxTable];
    __shared__ double wsum[4][9];
    const int view = blockIdx.y;
    const int64_t P = (int64_t)a.w * a.h;
    for (int j = threadIdx.x; j < 3 * a.K; j += blockDim.x) table[j] = 0.0;
    __syncthreads();
    const float scale = exp2f(-a.ev[view]);
    const float* src = a.hdr + (int64_t)view * 3 * P;
    const float* gin = a.grad + (int64_t)view * 3 * P;
    float* dh = a.d_hdr + (int64_t)view * 3 * P;
    double s[9];   // ev, white r g b, a2, a4, a6, cx, cy
    for (int k = 0; k < 9; ++k) s[k] = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P; j += (int64_t)gridDim.x * blockDim.x) {
        const Px g = pixel_geom((int)j, a.w, a.h, a.vig);
        float tv = 0.0f, tev = 0.0f;
        for (int c = 0; c < 3; ++c) {
            const float wc = a.white[3 * view + c];
            const float ie = src[c * P + j] * scale;
            const float iw = ie * wc;
            const float x = iw * g.vf;
            float slope, f;
            int i;
            bool used;
            response(a.crf + c * a.K, a.K, x, a.leak, slope, i, f, used);
            const float gl = gin[c * P + j];
            const float gv = gl * slope;
            dh[c * P + j] = gv * g.vf * wc * scale;
            s[1 + c] += (double)(gv * g.vf * ie);
            tv += gv * iw;
            tev += gv * x;
            if (used) {
                __hip_atomic_fetch_add(&table[c * a.K + i], (double)(gl * (1.0f - f)), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(&table[c * a.K + i + 1], (double)(gl * f), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        s[0] += (double)(-kLn2 * tev);
        s[4] += (double)(tv * g.r2);
        s[5] += (double)(tv * g.r2 * g.r2);
        s[6] += (double)(tv * g.r2 * g.r2 * g.r2);
        s[7] += (double)(tv * g.dvdr2 * (-2.0f * g.dx));
        s[8] += (double)(tv * g.dvdr2 * (-2.0f * g.dy));
    }
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int k = 0; k < 9; ++k) {
        const double t = wave_sum_f64(s[k]);
        if (lane == 0) wsum[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        const int k = threadIdx.x;
        a.partials[((uint64_t)view * kTonemapBlocks + blockIdx.x) * 16 + k] =
            ((wsum[0][k] + wsum[1][k]) + wsum[2][k]) + wsum[3][k];
    }
    for (int j = threadIdx.x; j < 3 * a.K; j += blockDim.x)
        if (table[j] != 0.0) atomicAdd(a.d_crf + j, table[j]);
}

// Fixed-order sums of the block partials: thread t < V sums view t's
// exposure, t < 4V the white points, then the five vignette entries over
// every view and block.
__global__ void __launch_bounds__(256) k_tm_reduce(TonemapArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int V = a.V;
    auto sum_view = [&](int v, int k) {
        double r = 0.0;
        for (int b = 0; b < kTonemapBlocks; ++b) r += a.partials[((uint64_t)v * kTonemapBlocks + b) * 16 + k];
        return r;
    };
    if (t < V) {
        a.d_ev[t] = sum_view(t, 0);
    } else if (t < 4 * V) {
        const int v = (t - V) / 3, c = (t - V) % 3;
        a.d_white[3 * v + c] = sum_view(v, 1 + c);
    } else if (t < 4 * V + 5) {
        const int k = 4 + (t - 4 * V);
        double r = 0.0;
        for (int v = 0; v < V; ++v) r += sum_view(v, k);
        a.d_vig[t - 4 * V] = r;
    }
}

}  // namespace

hipError_t tonemap_forward(const TonemapArgs& a, hipStream_t st) {
    const int64_t P = (int64_t)a.w * a.h;
    const unsigned gx = (unsigned)std::min<int64_t>((P + 255) / 256, 1024);
    k_tm_fwd<<<dim3(gx, (unsigned)a.V), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t tonemap_backward(const TonemapArgs& a, hipStream_t st) {
    k_tm_zero<<<(3 * a.K + 255) / 256, 256, 0, st>>>(a.d_crf, 3 * a.K);
    k_tm_bwd<<<dim3(kTonemapBlocks, (unsigned)a.V), 256, 0, st>>>(a);
    k_tm_reduce<<<(4 * a.V + 5 + 255) / 256, 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace adop
