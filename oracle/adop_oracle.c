/*
 * CPU oracle for the ADOP one-pixel point rasterizer -- TEST INFRASTRUCTURE.
 *
 * Plain single-threaded C, written from Sec. 3.1 of Rueckert et al. (ADOP,
 * TOG 2022).  Discrete decisions (projection, rounding, bounds, depth keys,
 * fuzzy depth test, backward case selection) are taken in IEEE binary32
 * exactly as the stated formula below prescribes; every accumulation and all
 * gradient arithmetic is binary64.  Build with -ffp-contract=off and without
 * fast-math (the build script does this) so that no multiply-add is fused
 * implicitly and x86 uses SSE arithmetic.
 *
 * Only tests, the smoke check and the benchmark's CPU baseline may call this.
 */
#include "adop_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define EMPTY_KEY 0xFFFFFFFFFFFFFFFFull

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* ------------------------------------------------------------------------ */
/* Projection P_0 = C(R x + t) of Sec. 3.1 (Eq. 2 at l = 0) for a pinhole     */
/* camera with Brown-Conrady radial (k1,k2,k3) and tangential (p1,p2) terms.  */
/* The paper names the model "Pinhole + Dist." without a formula; this is the  */
/* OpenCV form, written with explicit fused multiply-adds:                    */
/*   x_c = R x + t, a = X/Z, b = Y/Z, r2 = a^2 + b^2,                         */
/*   D = 1 + k1 r2 + k2 r2^2 + k3 r2^3,                                       */
/*   x_d = a D + 2 p1 a b + p2 (r2 + 2 a^2),  y_d = b D + 2 p2 a b + p1 (r2 + 2 b^2),
 *   u0 = fx x_d + cx,  v0 = fy y_d + cy.                                     */
/* ------------------------------------------------------------------------ */
static int project_full(const oracle_camera* cam, float x, float y, float z,
                        float* Xo, float* Yo, float* Zo, float* u0o, float* v0o)
{
    const float* R = cam->R;
    float X = fmaf(R[0], x, fmaf(R[1], y, fmaf(R[2], z, cam->t[0])));
    float Y = fmaf(R[3], x, fmaf(R[4], y, fmaf(R[5], z, cam->t[1])));
    float Z = fmaf(R[6], x, fmaf(R[7], y, fmaf(R[8], z, cam->t[2])));
    if (!(Z > cam->znear)) return 0;             /* near plane; NaN fails */
    float a = X / Z;
    float b = Y / Z;
    float ab = a * b;
    float bb = b * b;
    float r2 = fmaf(a, a, bb);
    if (!(r2 <= cam->r2_max)) return 0;          /* distortion fold-over */
    float D = fmaf(r2, fmaf(r2, fmaf(r2, cam->k3, cam->k2), cam->k1), 1.0f);
    float tx = cam->p2 * fmaf(a + a, a, r2);
    float ty = cam->p1 * fmaf(b + b, b, r2);
    float xd = fmaf(a, D, fmaf(cam->p1 + cam->p1, ab, tx));
    float yd = fmaf(b, D, fmaf(cam->p2 + cam->p2, ab, ty));
    float u0 = fmaf(cam->fx, xd, cam->cx);
    float v0 = fmaf(cam->fy, yd, cam->cy);
    if (!isfinite(u0) || !isfinite(v0)) return 0;
    *Xo = X; *Yo = Y; *Zo = Z; *u0o = u0; *v0o = v0;
    return 1;
}

int oracle_project(const oracle_camera* cam, float x, float y, float z,
                   float* Zo, float* u0o, float* v0o)
{
    float X, Y;
    return project_full(cam, x, y, z, &X, &Y, Zo, u0o, v0o);
}

static const oracle_options no_options = { 0u, NULL, NULL, NULL, 0.0f, NULL };

/* Eq. normalculling for point i in a view (see ORACLE_CULL_*). */
static int kept_by_normal(const oracle_camera* cam, const oracle_options* opt, int64_t i,
                          float X, float Y, float Z)
{
    if (!(opt->flags & (ORACLE_CULL_BACKFACE | ORACLE_CULL_PRINTED))) return 1;
    const float* R = cam->R;
    const float* nv = &opt->normals[3 * i];
    float m0 = fmaf(R[0], nv[0], fmaf(R[1], nv[1], R[2] * nv[2]));
    float m1 = fmaf(R[3], nv[0], fmaf(R[4], nv[1], R[5] * nv[2]));
    float m2 = fmaf(R[6], nv[0], fmaf(R[7], nv[1], R[8] * nv[2]));
    float d = fmaf(m0, X, fmaf(m1, Y, m2 * Z));
    if (opt->flags & ORACLE_CULL_BACKFACE) return d < 0.0f;
    return d > 0.0f;
}

/* Eq. discard for point i at layer l. */
static int kept_at_layer(const oracle_camera* cam, const oracle_options* opt, int64_t i, float Z, int l)
{
    if (!(opt->flags & ORACLE_DISCARD)) return 1;
    float s0 = (cam->fx * opt->radius[i]) / Z;
    float lhs = ldexpf(s0, -l) * opt->gamma;
    float rhs = sqrtf(1.0f - opt->beta[i]);
    return lhs > rhs;
}

/* Feature channel ch of point i as rendered (exp of a logarithmic one). */
static double feat_val(const oracle_options* opt, const float* feat, int64_t i, int c, int ch)
{
    double f = (double)feat[i * c + ch];
    return (opt->flags & ORACLE_LOG_FEATURES) ? exp(f) : f;
}

void oracle_project_points(const oracle_camera* cam, int64_t n, const float* pos,
                           float* Z, float* u0, float* v0, int32_t* valid)
{
    for (int64_t i = 0; i < n; ++i) {
        float zz = 0.f, uu = 0.f, vv = 0.f;
        valid[i] = oracle_project(cam, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], &zz, &uu, &vv);
        Z[i] = zz; u0[i] = uu; v0[i] = vv;
    }
}

/* Eq. round + Eq. boundscheck: layer l scales by 2^-l (exact), rounds to the
 * nearest integer with ties to even, and keeps p in [0,w_l[ x [0,h_l[ with
 * w_l = w >> l, h_l = h >> l (integers are pixel centres). */
int oracle_layer_pixel(const oracle_camera* cam, float u0, float v0, int l,
                       int32_t* px, int32_t* py)
{
    int wl = cam->width >> l, hl = cam->height >> l;
    float fx = rintf(ldexpf(u0, -l));
    float fy = rintf(ldexpf(v0, -l));
    if (!(fx >= 0.0f && fx < (float)wl && fy >= 0.0f && fy < (float)hl)) return 0;
    *px = (int32_t)fx;
    *py = (int32_t)fy;
    return 1;
}

static int64_t view_pixels(const oracle_camera* cam, int L)
{
    int64_t p = 0;
    for (int l = 0; l < L; ++l) p += (int64_t)(cam->width >> l) * (int64_t)(cam->height >> l);
    return p;
}

int64_t oracle_total_pixels(const oracle_camera* cams, int32_t V, int32_t L)
{
    int64_t s = 0;
    for (int v = 0; v < V; ++v) s += view_pixels(&cams[v], L);
    return s;
}

/* offset of layer l's first pixel inside a view */
static int64_t layer_offset(const oracle_camera* cam, int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += (int64_t)(cam->width >> k) * (int64_t)(cam->height >> k);
    return o;
}

static int check_args(int64_t n, int32_t c, int32_t V, const oracle_camera* cams, int32_t L)
{
    if (n < 0 || c < 1 || c > 16 || V < 1 || L < 1 || L > 8) return 1;
    for (int v = 0; v < V; ++v) {
        if (cams[v].width < 1 || cams[v].height < 1) return 1;
        if ((cams[v].width >> (L - 1)) < 1 || (cams[v].height >> (L - 1)) < 1) return 1;
        if (!(cams[v].znear >= 0.0f)) return 1;
    }
    return 0;
}

/* The per-pixel state after the two point passes. */
typedef struct {
    int64_t total;       /* pixels over all views */
    int64_t* vbase;      /* [V] first pixel of each view */
    uint64_t* keys;      /* min depth|index key */
    int32_t* counts;     /* |Lambda| */
    double* sums;        /* [total][c] sum of features over Lambda */
} raster_state;

/* Depth pass and accumulation pass of the three-pass rasterizer (Sec. 3.1,
 * "Implementation Details"), computed as the plain definition:
 *   min_z(p) is the smallest key (depth bits, then original index) over the
 *   points landing in p;  Lambda(p) = { i landing in p : z_i <= (1+alpha) min_z(p) }
 *   (Eq. depthtest, evaluated in binary32 with fa = 1 + alpha). */
static int rasterize(int64_t n, int32_t c, const float* pos, const float* feat,
                     int32_t V, const oracle_camera* cams, int32_t L, float alpha,
                     const oracle_options* opt, uint64_t* keys_out, int32_t* counts_out, raster_state* st)
{
    const float fa = 1.0f + alpha;
    st->total = oracle_total_pixels(cams, V, L);
    st->vbase = (int64_t*)malloc(sizeof(int64_t) * (size_t)V);
    st->keys = keys_out;
    st->counts = counts_out;
    st->sums = (double*)calloc((size_t)(st->total * c) + 1, sizeof(double));
    if (!st->vbase || !st->sums) return 1;
    int64_t acc = 0;
    for (int v = 0; v < V; ++v) { st->vbase[v] = acc; acc += view_pixels(&cams[v], L); }
    for (int64_t p = 0; p < st->total; ++p) { st->keys[p] = EMPTY_KEY; st->counts[p] = 0; }

    /* pass 1: per-pixel minimum of (depth bits << 32 | original index) */
    for (int v = 0; v < V; ++v) {
        const oracle_camera* cam = &cams[v];
        for (int64_t i = 0; i < n; ++i) {
            float X, Y, Z, u0, v0;
            if (!project_full(cam, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], &X, &Y, &Z, &u0, &v0)) continue;
            if (!kept_by_normal(cam, opt, i, X, Y, Z)) continue;
            uint64_t key = ((uint64_t)f2u(Z) << 32) | (uint64_t)(uint32_t)i;
            for (int l = 0; l < L; ++l) {
                int32_t px, py;
                if (!oracle_layer_pixel(cam, u0, v0, l, &px, &py)) continue;
                if (!kept_at_layer(cam, opt, i, Z, l)) continue;
                int64_t idx = st->vbase[v] + layer_offset(cam, l) + (int64_t)py * (cam->width >> l) + px;
                if (key < st->keys[idx]) st->keys[idx] = key;
            }
        }
    }
    /* pass 2: fuzzy depth test against the final minimum, count and sum */
    for (int v = 0; v < V; ++v) {
        const oracle_camera* cam = &cams[v];
        for (int64_t i = 0; i < n; ++i) {
            float X, Y, Z, u0, v0;
            if (!project_full(cam, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], &X, &Y, &Z, &u0, &v0)) continue;
            if (!kept_by_normal(cam, opt, i, X, Y, Z)) continue;
            for (int l = 0; l < L; ++l) {
                int32_t px, py;
                if (!oracle_layer_pixel(cam, u0, v0, l, &px, &py)) continue;
                if (!kept_at_layer(cam, opt, i, Z, l)) continue;
                int64_t idx = st->vbase[v] + layer_offset(cam, l) + (int64_t)py * (cam->width >> l) + px;
                float minz = u2f((uint32_t)(st->keys[idx] >> 32));
                float thr = minz * fa;
                if (Z <= thr) {
                    st->counts[idx] += 1;
                    for (int ch = 0; ch < c; ++ch) st->sums[idx * c + ch] += feat_val(opt, feat, i, c, ch);
                }
            }
        }
    }
    return 0;
}

/* image index of (view v, layer l, channel ch, pixel (px,py)) */
static int64_t img_index(const raster_state* st, const oracle_camera* cam, int v, int l,
                         int c, int ch, int32_t px, int32_t py)
{
    int64_t wl = cam->width >> l, hl = cam->height >> l;
    return (int64_t)c * (st->vbase[v] + layer_offset(cam, l)) + (int64_t)ch * wl * hl + (int64_t)py * wl + px;
}

/* Eq. blend: the mean of the features over Lambda, or the background where
 * Lambda is empty: the environment map's value at this pixel (bg_image, at
 * image index o) or a constant background standing in for it. */
static double blended(const raster_state* st, int64_t idx, int c, int ch, const float* background,
                      const double* bg_image, int64_t o)
{
    int32_t k = st->counts[idx];
    if (k == 0) return bg_image ? bg_image[o] : (double)background[ch];
    return st->sums[idx * c + ch] / (double)k;
}

static int check_options(int64_t n, const oracle_options* opt)
{
    uint32_t f = opt->flags;
    if ((f & ORACLE_CULL_BACKFACE) && (f & ORACLE_CULL_PRINTED)) return 1;
    if ((f & (ORACLE_CULL_BACKFACE | ORACLE_CULL_PRINTED)) && n > 0 && !opt->normals) return 1;
    if ((f & ORACLE_DISCARD) && n > 0 && (!opt->radius || !opt->beta || !(opt->gamma > 0.0f))) return 1;
    return 0;
}

int oracle_forward(int64_t n, int32_t c, const float* pos, const float* feat,
                   int32_t V, const oracle_camera* cams, int32_t L, float alpha,
                   const float* background, uint64_t* keys, int32_t* counts,
                   float* images, double* images64)
{
    return oracle_forward_ex(n, c, pos, feat, V, cams, L, alpha, &no_options, background, keys, counts,
                             images, images64);
}

int oracle_forward_ex(int64_t n, int32_t c, const float* pos, const float* feat,
                      int32_t V, const oracle_camera* cams, int32_t L, float alpha,
                      const oracle_options* opt, const float* background, uint64_t* keys,
                      int32_t* counts, float* images, double* images64)
{
    if (check_args(n, c, V, cams, L) || check_options(n, opt)) return 1;
    raster_state st;
    if (rasterize(n, c, pos, feat, V, cams, L, alpha, opt, keys, counts, &st)) return 2;
    for (int v = 0; v < V; ++v) {
        const oracle_camera* cam = &cams[v];
        for (int l = 0; l < L; ++l) {
            int32_t wl = cam->width >> l, hl = cam->height >> l;
            for (int32_t py = 0; py < hl; ++py)
                for (int32_t px = 0; px < wl; ++px) {
                    int64_t idx = st.vbase[v] + layer_offset(cam, l) + (int64_t)py * wl + px;
                    for (int ch = 0; ch < c; ++ch) {
                        int64_t o = img_index(&st, cam, v, l, c, ch, px, py);
                        double m = blended(&st, idx, c, ch, background, opt->bg_image, o);
                        images[o] = (float)m;
                        if (images64) images64[o] = m;
                    }
                }
        }
    }
    free(st.vbase);
    free(st.sums);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Backward pass.                                                            */
/* ------------------------------------------------------------------------ */

/* Induced change at neighbour q when the point (depth Z, features tau) is
 * virtually shifted into q -- the four cases of Eq. spatialderiv, with the
 * readings: case 1 tests the neighbour's Lambda (background), cases 2/3 use
 * the neighbour's min_z, comparisons in binary32.  Returns <G(q), dI> and
 * writes a magnitude bound of that dot product into *mag. */
static double induced(const raster_state* st, const oracle_camera* cam, int v, int l, int c,
                      int32_t qx, int32_t qy, float Z, float fa, const double* tau,
                      const float* background, const double* bg_image, const float* grad, double* mag)
{
    int32_t wl = cam->width >> l, hl = cam->height >> l;
    *mag = 0.0;
    if (qx < 0 || qx >= wl || qy < 0 || qy >= hl) return 0.0;   /* off the image */
    int64_t q = st->vbase[v] + layer_offset(cam, l) + (int64_t)qy * wl + qx;
    int32_t nq = st->counts[q];
    double dot = 0.0, m = 0.0;
    if (nq == 0) {
        /* case 1: background is replaced by the point's texture */
        for (int ch = 0; ch < c; ++ch) {
            int64_t o = img_index(st, cam, v, l, c, ch, qx, qy);
            double g = (double)grad[o];
            double b = bg_image ? bg_image[o] : (double)background[ch];
            double dI = tau[ch] - b;
            dot += g * dI;
            m += fabs(g) * (fabs(tau[ch]) + fabs(b));
        }
        *mag = m;
        return dot;
    }
    float minz = u2f((uint32_t)(st->keys[q] >> 32));
    float behind = minz * fa;
    float front = Z * fa;
    if (Z > behind) return 0.0;                      /* case 2: hidden behind q */
    if (front < minz) {                              /* case 3: replaces q's colour */
        for (int ch = 0; ch < c; ++ch) {
            int64_t o = img_index(st, cam, v, l, c, ch, qx, qy);
            double g = (double)grad[o];
            double I = blended(st, q, c, ch, background, bg_image, o);
            dot += g * (tau[ch] - I);
            m += fabs(g) * (fabs(tau[ch]) + fabs(I));
        }
        *mag = m;
        return dot;
    }
    /* case 4: joins q's blend set; new mean minus old mean */
    for (int ch = 0; ch < c; ++ch) {
        int64_t o = img_index(st, cam, v, l, c, ch, qx, qy);
        double g = (double)grad[o];
        double I = blended(st, q, c, ch, background, bg_image, o);
        double Inew = ((double)nq * I + tau[ch]) / (double)(nq + 1);
        dot += g * (Inew - I);
        m += fabs(g) * (fabs(tau[ch]) + fabs(I)) / (double)(nq + 1);
    }
    *mag = m;
    return dot;
}

int oracle_backward(int64_t n, int32_t c, const float* pos, const float* feat,
                    int32_t V, const oracle_camera* cams, int32_t L, float alpha,
                    uint32_t flags, const float* background, const float* grad,
                    double* dfeat, double* dpos, double* dpose, double* dintr,
                    double* dfeat_abs, double* dpos_abs, double* dpose_abs,
                    double* dintr_abs, double* gu_out, double* gv_out)
{
    oracle_options opt = no_options;
    opt.flags = flags & ORACLE_SPATIAL_ALL;
    return oracle_backward_ex(n, c, pos, feat, V, cams, L, alpha, &opt, background, grad, dfeat, dpos,
                              dpose, dintr, dfeat_abs, dpos_abs, dpose_abs, dintr_abs, gu_out, gv_out);
}

int oracle_backward_ex(int64_t n, int32_t c, const float* pos, const float* feat,
                       int32_t V, const oracle_camera* cams, int32_t L, float alpha,
                       const oracle_options* opt, const float* background, const float* grad,
                       double* dfeat, double* dpos, double* dpose, double* dintr,
                       double* dfeat_abs, double* dpos_abs, double* dpose_abs,
                       double* dintr_abs, double* gu_out, double* gv_out)
{
    if (check_args(n, c, V, cams, L) || check_options(n, opt)) return 1;
    const uint32_t flags = opt->flags;
    const float fa = 1.0f + alpha;
    int64_t total = oracle_total_pixels(cams, V, L);
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(total + 1));
    int32_t* counts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total + 1));
    if (!keys || !counts) { free(keys); free(counts); return 2; }
    raster_state st;
    if (rasterize(n, c, pos, feat, V, cams, L, alpha, opt, keys, counts, &st)) { free(keys); free(counts); return 2; }

    memset(dfeat, 0, sizeof(double) * (size_t)(n * c));
    memset(dpos, 0, sizeof(double) * (size_t)(3 * n));
    memset(dpose, 0, sizeof(double) * (size_t)(6 * V));
    memset(dintr, 0, sizeof(double) * (size_t)(9 * V));
    if (dfeat_abs) memset(dfeat_abs, 0, sizeof(double) * (size_t)(n * c));
    if (dpos_abs) memset(dpos_abs, 0, sizeof(double) * (size_t)(3 * n));
    if (dpose_abs) memset(dpose_abs, 0, sizeof(double) * (size_t)(6 * V));
    if (dintr_abs) memset(dintr_abs, 0, sizeof(double) * (size_t)(9 * V));

    for (int v = 0; v < V; ++v) {
        const oracle_camera* cam = &cams[v];
        const double fx = cam->fx, fy = cam->fy;
        const double k1 = cam->k1, k2 = cam->k2, k3 = cam->k3, p1 = cam->p1, p2 = cam->p2;
        for (int64_t i = 0; i < n; ++i) {
            float X, Y, Z, u0, v0;
            if (gu_out) { gu_out[(int64_t)v * n + i] = 0.0; gv_out[(int64_t)v * n + i] = 0.0; }
            if (!project_full(cam, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], &X, &Y, &Z, &u0, &v0)) continue;
            if (!kept_by_normal(cam, opt, i, X, Y, Z)) continue;
            double tau[16];
            for (int ch = 0; ch < c; ++ch) tau[ch] = feat_val(opt, feat, i, c, ch);
            double gu = 0.0, gv = 0.0, gu_m = 0.0, gv_m = 0.0;
            for (int l = 0; l < L; ++l) {
                int32_t px, py;
                if (!oracle_layer_pixel(cam, u0, v0, l, &px, &py)) continue;
                if (!kept_at_layer(cam, opt, i, Z, l)) continue;
                int32_t wl = cam->width >> l;
                int64_t idx = st.vbase[v] + layer_offset(cam, l) + (int64_t)py * wl + px;
                float minz = u2f((uint32_t)(st.keys[idx] >> 32));
                float thr = minz * fa;
                int visible = (Z <= thr);
                if (visible) {
                    /* derivative of Eq. blend w.r.t. each feature in Lambda */
                    double k = (double)st.counts[idx];
                    for (int ch = 0; ch < c; ++ch) {
                        double g = (double)grad[img_index(&st, cam, v, l, c, ch, px, py)];
                        /* logarithmic descriptors: d exp(f) / df = exp(f) */
                        double chain = (flags & ORACLE_LOG_FEATURES) ? tau[ch] : 1.0;
                        dfeat[i * c + ch] += g / k * chain;
                        if (dfeat_abs) dfeat_abs[i * c + ch] += fabs(g) / k * chain;
                    }
                }
                if (!visible && !(flags & ORACLE_SPATIAL_ALL)) continue;
                /* Eq. gradp: average of the induced changes of a shift by +1 and
                 * by -1 pixel; the -1 shift divides by Delta u = -1. */
                double mr, ml, md, mu;
                double right = induced(&st, cam, v, l, c, px + 1, py, Z, fa, tau, background, opt->bg_image, grad, &mr);
                double left = induced(&st, cam, v, l, c, px - 1, py, Z, fa, tau, background, opt->bg_image, grad, &ml);
                double down = induced(&st, cam, v, l, c, px, py + 1, Z, fa, tau, background, opt->bg_image, grad, &md);
                double up = induced(&st, cam, v, l, c, px, py - 1, Z, fa, tau, background, opt->bg_image, grad, &mu);
                double du = 0.5 * (right - left);
                double dv = 0.5 * (down - up);
                /* u_l = 2^-l u0: chain to layer-0 pixel coordinates */
                gu += ldexp(du, -l);
                gv += ldexp(dv, -l);
                gu_m += ldexp(0.5 * (mr + ml), -l);
                gv_m += ldexp(0.5 * (md + mu), -l);
            }
            if (gu_out) { gu_out[(int64_t)v * n + i] = gu; gv_out[(int64_t)v * n + i] = gv; }
            if (gu == 0.0 && gv == 0.0 && gu_m == 0.0 && gv_m == 0.0) continue;

            /* smooth part of the projection in binary64 */
            const float* Rf = cam->R;
            double xw = pos[3 * i], yw = pos[3 * i + 1], zw = pos[3 * i + 2];
            double Xd = (double)Rf[0] * xw + (double)Rf[1] * yw + (double)Rf[2] * zw + (double)cam->t[0];
            double Yd = (double)Rf[3] * xw + (double)Rf[4] * yw + (double)Rf[5] * zw + (double)cam->t[1];
            double Zd = (double)Rf[6] * xw + (double)Rf[7] * yw + (double)Rf[8] * zw + (double)cam->t[2];
            double a = Xd / Zd, b = Yd / Zd;
            double r2 = a * a + b * b, r4 = r2 * r2, r6 = r4 * r2;
            double D = 1.0 + k1 * r2 + k2 * r4 + k3 * r6;
            double Dp = k1 + 2.0 * k2 * r2 + 3.0 * k3 * r4;
            double xd = a * D + 2.0 * p1 * a * b + p2 * (r2 + 2.0 * a * a);
            double yd = b * D + 2.0 * p2 * a * b + p1 * (r2 + 2.0 * b * b);
            /* d(x_d, y_d) / d(a, b) */
            double xa = D + 2.0 * a * a * Dp + 2.0 * p1 * b + 6.0 * p2 * a;
            double xb = 2.0 * a * b * Dp + 2.0 * p1 * a + 2.0 * p2 * b;
            double ya = xb;
            double yb = D + 2.0 * b * b * Dp + 6.0 * p1 * b + 2.0 * p2 * a;
            double ga = gu * fx * xa + gv * fy * ya;
            double gb = gu * fx * xb + gv * fy * yb;
            double ga_m = gu_m * fabs(fx * xa) + gv_m * fabs(fy * ya);
            double gb_m = gu_m * fabs(fx * xb) + gv_m * fabs(fy * yb);
            /* a = X/Z, b = Y/Z */
            double gc[3] = { ga / Zd, gb / Zd, -(a * ga + b * gb) / Zd };
            double gc_m[3] = { ga_m / fabs(Zd), gb_m / fabs(Zd), (fabs(a) * ga_m + fabs(b) * gb_m) / fabs(Zd) };
            /* world position: x_c = R x + t */
            for (int k = 0; k < 3; ++k) {
                double s = 0.0, sm = 0.0;
                for (int j = 0; j < 3; ++j) { s += (double)Rf[3 * j + k] * gc[j]; sm += fabs((double)Rf[3 * j + k]) * gc_m[j]; }
                dpos[(int64_t)k * n + i] += s;
                if (dpos_abs) dpos_abs[(int64_t)k * n + i] += sm;
            }
            /* pose tangent xi = (rho, omega), left-multiplied exp(xi) at xi = 0:
             * d x_c / d rho = I,  d x_c / d omega = -[x_c]_x */
            double xc[3] = { Xd, Yd, Zd };
            double cr[3] = { xc[1] * gc[2] - xc[2] * gc[1], xc[2] * gc[0] - xc[0] * gc[2], xc[0] * gc[1] - xc[1] * gc[0] };
            double cr_m[3] = { fabs(xc[1]) * gc_m[2] + fabs(xc[2]) * gc_m[1], fabs(xc[2]) * gc_m[0] + fabs(xc[0]) * gc_m[2],
                               fabs(xc[0]) * gc_m[1] + fabs(xc[1]) * gc_m[0] };
            for (int k = 0; k < 3; ++k) {
                dpose[6 * v + k] += gc[k];
                dpose[6 * v + 3 + k] += cr[k];
                if (dpose_abs) { dpose_abs[6 * v + k] += gc_m[k]; dpose_abs[6 * v + 3 + k] += cr_m[k]; }
            }
            /* intrinsics (fx, fy, cx, cy, k1, k2, k3, p1, p2) */
            double au = gu * fx * a + gv * fy * b;
            double au_m = gu_m * fabs(fx * a) + gv_m * fabs(fy * b);
            double di[9] = { gu * xd, gv * yd, gu, gv, au * r2, au * r4, au * r6,
                             gu * fx * 2.0 * a * b + gv * fy * (r2 + 2.0 * b * b),
                             gu * fx * (r2 + 2.0 * a * a) + gv * fy * 2.0 * a * b };
            double di_m[9] = { gu_m * fabs(xd), gv_m * fabs(yd), gu_m, gv_m, au_m * r2, au_m * r4, au_m * r6,
                               gu_m * fabs(fx * 2.0 * a * b) + gv_m * fabs(fy * (r2 + 2.0 * b * b)),
                               gu_m * fabs(fx * (r2 + 2.0 * a * a)) + gv_m * fabs(fy * 2.0 * a * b) };
            for (int k = 0; k < 9; ++k) {
                dintr[9 * v + k] += di[k];
                if (dintr_abs) dintr_abs[9 * v + k] += di_m[k];
            }
        }
    }
    free(st.vbase);
    free(st.sums);
    free(keys);
    free(counts);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Stochastic discarding preprocess: distance to the 4th-nearest other point */
/* (Sec. 3.1, "Stochastic Point Discarding"), by brute force.                */
/* ------------------------------------------------------------------------ */
int oracle_knn_radius(int64_t n, const float* pos, float* radius)
{
    if (n < 5 || !pos || !radius) return 1;
    for (int64_t i = 0; i < n; ++i) {
        float best[4] = { INFINITY, INFINITY, INFINITY, INFINITY };   /* ascending */
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            float dx = pos[3 * j] - pos[3 * i];
            float dy = pos[3 * j + 1] - pos[3 * i + 1];
            float dz = pos[3 * j + 2] - pos[3 * i + 2];
            float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            if (!(d2 < best[3])) continue;
            int k = 3;
            while (k > 0 && d2 < best[k - 1]) { best[k] = best[k - 1]; --k; }
            best[k] = d2;
        }
        radius[i] = sqrtf(best[3]);
    }
    return 0;
}
