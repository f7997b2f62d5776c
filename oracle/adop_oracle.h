/*
 * CPU oracle for the ADOP one-pixel point rasterizer (Rueckert, Franke,
 * Stamminger, "ADOP: Approximate Differentiable One-Pixel Point Rendering",
 * ACM TOG 41(4) 2022, Sec. 3.1).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded
 * implementation used to check the GPU path.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code
 * with the HIP library.
 *
 * Parity status of each function is listed in oracle/README.md.
 *
 * Buffer layout of a rendered frame (an interface format both sides agree on):
 *   views are stored one after another; inside a view, layer l (l = 0..L-1,
 *   w_l = w >> l, h_l = h >> l) follows layer l-1.
 *   keys / counts : [sum_v P_v] with P_v = sum_l w_l*h_l, pixel (l,x,y) of
 *                   view v at viewbase_v + layeroff_l + y*w_l + x.
 *   images        : [C * sum_v P_v]; view v, layer l occupies C*w_l*h_l
 *                   floats at C*(viewbase_v + layeroff_l), channel-major
 *                   ([C][h_l][w_l]).
 */
#ifndef ADOP_ORACLE_H
#define ADOP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Pinhole + Brown-Conrady camera, world->camera pose x_c = R x + t.
 * Same byte layout as the library's camera record (100 bytes). */
typedef struct oracle_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float k1, k2, k3, p1, p2;
    float znear;    /* points with z_c <= znear are culled (znear >= 0) */
    float r2_max;   /* points with a^2+b^2 > r2_max are culled */
    float R[9];     /* row-major */
    float t[3];
} oracle_camera;

#define ORACLE_SPATIAL_ALL 1u   /* spatial gradient for every in-bounds point */
/* Eq. normalculling: with n the point's normal and x_c = R x + t, the sign
 * of d = (R n) . x_c decides (dividing by |x_c| > 0 does not change it).
 * CULL_BACKFACE keeps points whose normal faces the camera (d < 0);
 * CULL_PRINTED keeps d > 0, the inequality as printed.  R n and d are
 * evaluated in binary32 with the nesting of the projection:
 *   m_k = fmaf(R[3k], nx, fmaf(R[3k+1], ny, R[3k+2] * nz)),
 *   d = fmaf(m_0, X, fmaf(m_1, Y, m_2 * Z)). */
#define ORACLE_CULL_BACKFACE 2u
#define ORACLE_CULL_PRINTED 4u
/* Logarithmic descriptors (Sec. 4, network architecture): features are
 * stored as log values and rendered as exp(feat); dL/dfeat is the gradient
 * with respect to the linear value times exp(feat). */
#define ORACLE_LOG_FEATURES 8u
/* Stochastic point discarding (Eq. discard): a point is rendered at layer l
 * only if r_screen / sqrt(1 - beta) > 1 / gamma, with the world radius
 * projected as r_screen = (fx r_world / Z) 2^-l; evaluated in binary32 as
 *   (((fx * r) / Z) * 2^-l) * gamma > sqrtf(1 - beta). */
#define ORACLE_DISCARD 16u

/* Options of the extended passes.  normals [n][3] (culling), radius [n] and
 * beta [n] (discarding) may be NULL when the matching flag is off.
 * bg_image (optional, float64 in the image layout [C * pixels]): the value
 * of every pixel where Lambda is empty -- the environment map sampled
 * through the inverse camera, E(R^T C^-1(u, v)) of Eq. blend -- used by the
 * blend and by case 1 of Eq. spatialderiv; NULL: the constant background. */
typedef struct oracle_options {
    uint32_t flags;
    const float* normals;
    const float* radius;
    const float* beta;
    float gamma;
    const double* bg_image;
} oracle_options;

/* Projection of one point (FP32 arithmetic, stated formula).  Returns 1 and
 * writes depth Z and layer-0 pixel coordinates (u0, v0) if the point is not
 * culled by the near plane, the distortion limit or non-finite values. */
int oracle_project(const oracle_camera* cam, float x, float y, float z,
                   float* Z, float* u0, float* v0);

/* Batch form of oracle_project; pos is [n][3]. */
void oracle_project_points(const oracle_camera* cam, int64_t n, const float* pos,
                           float* Z, float* u0, float* v0, int32_t* valid);

/* Pixel of a projected point at layer l: returns 1 if in bounds, with the
 * integer pixel in (*px,*py). */
int oracle_layer_pixel(const oracle_camera* cam, float u0, float v0, int l,
                       int32_t* px, int32_t* py);

/* Total pyramid pixels of V views with L layers. */
int64_t oracle_total_pixels(const oracle_camera* cams, int32_t V, int32_t L);

/* Forward pass (Eqs. render, round, boundscheck, depthtest, blend).
 *   pos [n][3], feat [n][c] (float; narrower storage is widened by the caller)
 *   outputs: keys, counts, images (float), images64 (double, may be NULL).
 * Returns 0 on success, nonzero on invalid arguments. */
int oracle_forward(int64_t n, int32_t c, const float* pos, const float* feat,
                   int32_t V, const oracle_camera* cams, int32_t L, float alpha,
                   const float* background, uint64_t* keys, int32_t* counts,
                   float* images, double* images64);

/* Backward pass (Eqs. partial, induce, gradp, spatialderiv; tangent-space
 * pose of Eq. tangent).  grad is dL/dI in the image layout above.
 * Outputs (double): dfeat [n][c], dpos [3][n], dpose [V][6] = (rho, omega),
 * dintr [V][9] = (fx, fy, cx, cy, k1, k2, k3, p1, p2).
 * Optional (may be NULL): *_abs = sum of |terms| forming each output entry,
 * gu/gv [V][n] = dL/du0, dL/dv0 per point and view. */
int oracle_backward(int64_t n, int32_t c, const float* pos, const float* feat,
                    int32_t V, const oracle_camera* cams, int32_t L, float alpha,
                    uint32_t flags, const float* background, const float* grad,
                    double* dfeat, double* dpos, double* dpose, double* dintr,
                    double* dfeat_abs, double* dpos_abs, double* dpose_abs,
                    double* dintr_abs, double* gu, double* gv);

/* The forward and backward passes with options (flags of the backward's
 * SPATIAL_ALL included in opt->flags). */
int oracle_forward_ex(int64_t n, int32_t c, const float* pos, const float* feat,
                      int32_t V, const oracle_camera* cams, int32_t L, float alpha,
                      const oracle_options* opt, const float* background, uint64_t* keys,
                      int32_t* counts, float* images, double* images64);
int oracle_backward_ex(int64_t n, int32_t c, const float* pos, const float* feat,
                       int32_t V, const oracle_camera* cams, int32_t L, float alpha,
                       const oracle_options* opt, const float* background, const float* grad,
                       double* dfeat, double* dpos, double* dpose, double* dintr,
                       double* dfeat_abs, double* dpos_abs, double* dpose_abs,
                       double* dintr_abs, double* gu, double* gv);

/* Stochastic discarding preprocess: r_world[i] = distance from point i to its
 * 4th-nearest other point (brute force), with squared distances in binary32
 * as fmaf(dx, dx, fmaf(dy, dy, dz * dz)), d = x_j - x_i, and r the correctly
 * rounded square root of the 4th smallest.  n >= 5. */
int oracle_knn_radius(int64_t n, const float* pos, float* radius);

#ifdef __cplusplus
}
#endif
#endif
