/*
 * adop.h -- C ABI of the MI355X (gfx950) differentiable one-pixel point
 * rasterizer.
 *
 * Method: Rueckert, Franke, Stamminger, "ADOP: Approximate Differentiable
 * One-Pixel Point Rendering", ACM TOG 41(4), 2022, Sec. 3.1.  The forward
 * pass is the render function of Eq. render, I_l = Phi_l(C, R, t, x, n, E, tau),
 * for pyramid layers l = 0..L-1; the backward pass returns the partials of
 * Eq. partial (camera C, pose (R,t) in the tangent space of Eq. tangent,
 * positions x, features tau).  The environment map E is replaced by a
 * constant background and normals are not used.
 *
 * Conventions
 *   - All device buffers are caller-owned.  Render calls never allocate
 *     device memory; scene preparation allocates temporary device memory for
 *     its sort and frees it before returning.
 *   - Every call that takes a `stream` (a hipStream_t passed as void*, NULL =
 *     the default stream) is asynchronous on that stream.  All arguments are
 *     validated on the host before anything is enqueued; on error nothing is
 *     enqueued and the context's last-error message says why.  A failure of
 *     the HIP runtime is reported as ADOP_E_DEVICE with the HIP error text.
 *   - A context is used by one host thread at a time.
 *   - The library is built for gfx950 only.
 *
 * Frame layout (images, keys, counts of V views with L layers):
 *   views follow one another; inside view v, layer l (w_l = w >> l,
 *   h_l = h >> l) follows layer l-1.  Pixel (x, y) of layer l of view v is
 *   element  o(v,l) + y*w_l + x  of keys and counts, where o(v,l) is given by
 *   adop_views_layout.  Images hold C channels per pixel in channel-major
 *   blocks: channel c of that pixel is element  C*o(v,l) + c*w_l*h_l + y*w_l + x,
 *   so each (view, layer) is a contiguous [C][h_l][w_l] FP32 image.
 */
#ifndef ADOP_H
#define ADOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef int32_t adop_status;
#define ADOP_OK             0
#define ADOP_E_INVALID      1   /* an argument is out of range or inconsistent */
#define ADOP_E_UNSUPPORTED  2   /* valid request the library does not implement */
#define ADOP_E_WORKSPACE    3   /* workspace smaller than adop_workspace_bytes */
#define ADOP_E_DEVICE       4   /* HIP runtime error (text in adop_last_error) */
#define ADOP_E_STATE        5   /* call out of order (e.g. graph in use) */

/* feature storage types; rendering always accumulates in FP32 */
typedef int32_t adop_dtype;
#define ADOP_F32   0
#define ADOP_BF16  1
#define ADOP_F16   2

#define ADOP_MAX_LAYERS     8
#define ADOP_MAX_CHANNELS  16
#define ADOP_MAX_VIEWS    256   /* per forward call */
#define ADOP_MAX_VIEWS_BWD 32   /* per backward call */
#define ADOP_MAX_SIZE   65536   /* camera width and height (and a frame below 2^31 pixels) */

/* render flags */
#define ADOP_FLAG_SPATIAL_ALL 1u  /* spatial gradient for every in-bounds point,
                                     not only points in the blend set */
/* Normal culling (Eq. normalculling) needs scene normals.  With n the point's
 * normal and x_c = R x + t, the sign of d = (R n) . x_c decides (the printed
 * division by |x_c| > 0 does not change it), in FP32 with the nesting of the
 * projection: m_k = fma(R[3k], nx, fma(R[3k+1], ny, R[3k+2] nz)),
 * d = fma(m_0, X, fma(m_1, Y, m_2 Z)).  A culled point takes no part in any
 * pass of that view.  At most one of the two flags may be set. */
#define ADOP_FLAG_CULL_BACKFACE 2u   /* keep d < 0: the normal faces the camera */
#define ADOP_FLAG_CULL_PRINTED 4u    /* keep d > 0: the inequality as printed */
/* Logarithmic descriptors (Sec. 4, network architecture): the stored
 * features are log values; every pass uses exp(feat) and dfeat is the
 * gradient with respect to the stored (log) values. */
#define ADOP_FLAG_LOG_FEATURES 8u
/* Stochastic point discarding (Eq. discard) needs scene radius and beta: a
 * point takes part in layer l only if, in FP32,
 *   (((fx * radius) / Z) * 2^-l) * gamma > sqrt(1 - beta)
 * i.e. r_screen / sqrt(1 - beta) > 1 / gamma with the world radius (the
 * distance to the 4th-nearest point, adop_knn_radius) projected to layer-l
 * pixels; gamma = params->gamma. */
#define ADOP_FLAG_DISCARD 16u

/* Camera: pinhole with Brown-Conrady radial (k1,k2,k3) and tangential
 * (p1,p2) distortion, world->camera pose x_c = R x + t (R row-major, OpenCV
 * axes: x right, y down, z forward).  The paper names the model
 * "Pinhole + Dist." (scene table, Sec. 4) without a formula; the projection
 * evaluated in FP32 is
 *   a = X/Z, b = Y/Z, r2 = a^2 + b^2, D = 1 + k1 r2 + k2 r2^2 + k3 r2^3,
 *   x_d = a D + 2 p1 a b + p2 (r2 + 2 a^2), y_d = b D + 2 p2 a b + p1 (r2 + 2 b^2),
 *   u0 = fx x_d + cx, v0 = fy y_d + cy,
 * and layer l uses (u0, v0) * 2^-l (Eq. 2) rounded to the nearest integer,
 * ties to even (Eq. round).  A point is culled when Z <= znear, when
 * r2 > r2_max (distortion fold-over limit), or when anything is non-finite.
 * Requirements: width, height >= 1; znear >= 0.  100 bytes. */
struct adop_camera;
typedef struct adop_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float k1, k2, k3, p1, p2;
    float znear;
    float r2_max;
    float R[9];
    float t[3];
} adop_camera;

typedef struct adop_render_params {
    int32_t layers;            /* L, 1..ADOP_MAX_LAYERS; every view needs w>>(L-1) >= 1 and h>>(L-1) >= 1 */
    float alpha;               /* fuzzy depth test z <= (1+alpha) min_z (Eq. depthtest); >= 0 */
    uint32_t flags;            /* ADOP_FLAG_* */
    const float* background;   /* host, [channels] colour of empty pixels; NULL = zeros */
    float gamma;               /* ADOP_FLAG_DISCARD: > 0 (the paper uses 1.5) */
    /* Optional device camera table of the V views (adop_cameras_upload, or
     * written by device code): when not NULL the render call reads each
     * view's intrinsics (fx .. p2), znear, r2_max and pose (R, t) from it on
     * the device when the call executes; the host array `cams` of the call
     * then only supplies the image sizes (which must match the table's) and
     * its other fields are validated but not used.  NULL: the host cameras. */
    const struct adop_camera* cameras_device;
    /* Optional environment map (Eq. blend: a pixel no point hits takes
     * E(R^T C^-1(u, v))): device [C][S][S] FP32 of S x S texels, S >= 2.
     * Pixel (x, y) of layer l is unprojected at layer-0 coordinates
     * (x 2^l, y 2^l) through the pinhole and the distortion of the camera
     * (the Brown-Conrady map inverted by 20 fixed-point steps from the
     * distorted coordinates); the world ray d = R^T (a, b, 1) / |.| is looked
     * up at longitude atan2(d_x, d_z) and colatitude arccos(d_y), i.e. texel
     * coordinates s = (atan2(d_x, d_z) / 2pi + 1/2) S, t = arccos(d_y) / pi S
     * with texel (i, j) centred at (i + 1/2, j + 1/2), bilinearly, wrapping
     * in longitude and clamping in colatitude.  The same map must be given
     * to the backward of the frame (empty neighbours of Eq. spatialderiv's
     * case 1 then take its values).  NULL: the constant background. */
    const float* env_map;
    int32_t env_size;          /* S */
    /* backward, with env_map: device [C][S][S] FP32 output, overwritten
     * with dL/dE (the derivative of Eq. blend at the empty pixels, summed
     * with FP32 atomics in an order that varies between runs); NULL: not
     * computed.  No gradient reaches the pose or intrinsics through the
     * lookup. */
    float* env_grad;
} adop_render_params;

/* A prepared scene (see adop_scene_prepare).  The SoA position planes and the
 * feature array are the trainable parameters; gradients are returned in the
 * same (prepared) order.  orig_index[i] is the caller's index of point i and
 * breaks depth ties (smaller original index wins). */
typedef struct adop_scene {
    int64_t n;                 /* number of points, 0 .. 2^31-1 */
    int32_t channels;          /* C, 1..ADOP_MAX_CHANNELS */
    adop_dtype dtype;          /* storage type of feat */
    const float* x;            /* device [n] */
    const float* y;            /* device [n] */
    const float* z;            /* device [n] */
    const void* feat;          /* device [n][C] of dtype, 16-byte aligned */
    const int32_t* orig_index; /* device [n] */
    const float* nx;           /* device [n] normals (ADOP_FLAG_CULL_*), else may be NULL */
    const float* ny;
    const float* nz;
    const float* radius;       /* device [n] world radius (ADOP_FLAG_DISCARD), else may be NULL */
    const float* beta;         /* device [n] U[0,1) per point (ADOP_FLAG_DISCARD), else may be NULL */
} adop_scene;

/* Rendered frame buffers (device, caller-owned), layout in the file comment. */
typedef struct adop_frame {
    float* images;             /* [C * pixels] FP32 */
    uint64_t* keys;            /* [pixels] (bits(z) << 32 | orig_index), empty = ~0 */
    int32_t* counts;           /* [pixels] number of blended points |Lambda| */
    int64_t pixels;            /* must equal the total of adop_views_layout */
    uint8_t* visible;          /* optional, [V][n]: the forward sets bit l of visible[v * n + i]
                                  when point i is in the blend set of layer l of view v (Eq.
                                  depthtest, after culling and discarding), and clears the other
                                  bits; the backward of the same frame then reads the bits
                                  instead of testing every point against the pixel records, and
                                  skips points without any (not with ADOP_FLAG_SPATIAL_ALL, which
                                  needs every in-bounds point).  NULL: not written; the backward
                                  re-renders every point. */
} adop_frame;

typedef struct adop_context adop_context;
typedef struct adop_graph adop_graph;

/* ------------------------------------------------------------ context */
/* Create a context on HIP device `device` (makes it current on this thread).
 * Allocates a small pinned staging ring for camera uploads. */
adop_status adop_context_create(int32_t device, adop_context** out);
void adop_context_destroy(adop_context* ctx);
/* Message of the last failed call on this context ("" if none); valid until
 * the next call on the context. */
const char* adop_last_error(const adop_context* ctx);
const char* adop_status_string(adop_status s);
/* Library version string. */
const char* adop_version(void);

/* --------------------------------------------------- host-only queries */
/* Pyramid layout of V views with L layers (no device access).  Writes the
 * total pixel count, and if `offsets` is not NULL, o(v,l) at offsets[v*L+l]. */
adop_status adop_views_layout(const adop_camera* cams, int32_t V, int32_t layers,
                              int64_t* total_pixels, int64_t* offsets);

/* Workspace bytes needed by render calls with C channels, V views and
 * `pixels` pyramid pixels (the same workspace serves forward and backward). */
size_t adop_workspace_bytes(const adop_context* ctx, int32_t channels, int32_t V,
                            int64_t pixels);

/* Bytes of the prepared feature array for n points, C channels, dtype. */
size_t adop_feature_bytes(int64_t n, int32_t channels, adop_dtype dtype);

/* Layout of one view's pyramid (Eq. 2: layer l is (w >> l) x (h >> l)) in the
 * frame buffers, for w x h pixels, L layers and C channels: layer sizes, the
 * first pixel of each layer in keys and counts (pixel_offset; images hold
 * C * pixel_offset floats before the layer), and the bytes of the view's
 * images (FP32), keys (u64) and counts (int32).  Host only; ADOP_E_INVALID
 * when w >> (L-1) or h >> (L-1) is 0 or L is outside 1..ADOP_MAX_LAYERS. */
typedef struct adop_layout {
    int32_t layers, channels;
    int32_t width[ADOP_MAX_LAYERS];
    int32_t height[ADOP_MAX_LAYERS];
    int64_t pixel_offset[ADOP_MAX_LAYERS];
    int64_t pixels;            /* sum of the layers' pixels */
    int64_t image_bytes;       /* C * pixels * 4 */
    int64_t key_bytes;         /* pixels * 8 */
    int64_t count_bytes;       /* pixels * 4 */
} adop_layout;
adop_status adop_pyramid_layout(int32_t width, int32_t height, int32_t layers, int32_t channels,
                                adop_layout* out);

/* A prepared scene in ONE caller-owned device buffer: the planes x, y, z
 * (FP32 [n] each), the features [n][C] of dtype and orig_index (int32 [n]),
 * in this order, each part starting on a 256-byte boundary.
 * adop_scene_bytes gives the buffer size (0 for invalid arguments);
 * adop_scene_bind fills `out` with pointers into `scene_mem` (which must be
 * 256-byte aligned; nothing is read or copied, so it needs no context and
 * no device), sets n, channels and dtype, and leaves the optional per-point
 * planes (normals, radius, beta) NULL.  adop_scene_prepare can then write
 * the prepared points through those pointers. */
size_t adop_scene_bytes(int64_t n, int32_t channels, adop_dtype dtype);
adop_status adop_scene_bind(void* scene_mem, int64_t n, int32_t channels, adop_dtype dtype,
                            adop_scene* out);

/* Copy V host cameras into a device camera table (caller-owned device memory
 * of V * sizeof(adop_camera) bytes, 4-byte aligned) for
 * adop_render_params.cameras_device.  The cameras are validated like those of
 * a render call (sizes, znear >= 0) and staged through a pinned slot of the
 * context, so `host` may be reused as soon as the call returns; the copy is
 * asynchronous on `stream`. */
adop_status adop_cameras_upload(adop_context* ctx, const adop_camera* host, int32_t V,
                                adop_camera* dev_table, void* stream);

/* ------------------------------------------------------- scene upload */
/* Reorder a point cloud for rendering (Sec. 3.1, "Implementation Details":
 * Morton order of the cloud).  Points are sorted by a 63-bit Morton code over
 * their bounding box (21 bits per axis; non-finite points last).  The render
 * kernels give every workgroup a contiguous range of this order, i.e. a
 * compact region of space.  With block > 0 (a multiple of 256) the order is
 * additionally cut into 8 segments and blocks of `block` points are shuffled
 * inside each segment with a permutation drawn from `seed` (the blocked
 * Morton shuffle); block == 0 keeps the plain Morton order (default).
 *   pos       device [n][3] FP32, caller's order
 *   feat      device [n][C] of dtype, caller's order
 *   x,y,z     device [n] FP32 outputs (SoA positions)
 *   feat_out  device [n][C] of dtype output
 *   orig_index device [n] output: caller's index of each prepared point
 * Allocates and frees temporary device memory (about 24 bytes per point);
 * synchronises `stream` before returning. */
adop_status adop_scene_prepare(adop_context* ctx, const float* pos, const void* feat,
                               int64_t n, int32_t channels, adop_dtype dtype,
                               int32_t block, uint64_t seed,
                               float* x, float* y, float* z, void* feat_out,
                               int32_t* orig_index, void* stream);

/* Gather per-point values of the caller's order into the prepared order:
 * dst[k * n + i] = src[orig_index[i] * components + k] for k < components
 * (so normals [n][3] become the planes nx, ny, nz).  Device pointers, FP32,
 * 1 <= components <= 4.  Asynchronous on `stream`. */
adop_status adop_scene_gather(adop_context* ctx, const float* src, int32_t components, int64_t n,
                              const int32_t* orig_index, float* dst, void* stream);

/* World radius of stochastic discarding (Sec. 3.1, "Stochastic Point
 * Discarding"): radius[i] = distance from point i to its 4th-nearest other
 * point, over the SoA positions x, y, z (any order; duplicates count at
 * distance 0).  Squared distances are evaluated in FP32 as
 * fma(dx, dx, fma(dy, dy, dz dz)) with d = p_j - p_i and the radius is the
 * correctly rounded square root of the 4th smallest, so the result is exact
 * for the stated formula.  n >= 5.  Allocates and frees temporary device
 * memory (about 40 bytes per point); synchronises `stream` before returning. */
adop_status adop_knn_radius(adop_context* ctx, const float* x, const float* y, const float* z,
                            int64_t n, float* radius, void* stream);

/* ---------------------------------------------------------- rendering */
/* Forward pass (Eqs. render, round, boundscheck, depthtest, blend): the
 * depth pass writes per-pixel keys with a 64-bit atomic minimum, the
 * accumulation pass sums the features of every point passing the fuzzy
 * depth test and counts them, and the normalisation writes the means (or the
 * background) into `frame->images`.  `cams` is a host array of V cameras,
 * staged to the workspace by the call.  Keys and counts are exact (they do
 * not depend on the order of floating-point operations). */
adop_status adop_render_forward(adop_context* ctx, const adop_scene* scene,
                                const adop_camera* cams, int32_t V,
                                const adop_render_params* params,
                                const adop_frame* frame,
                                void* workspace, size_t workspace_bytes, void* stream);

/* Backward pass (Eqs. partial, induce, gradp, spatialderiv, tangent).
 * Inputs: the frame written by adop_render_forward with the same scene,
 * cameras and params (including frame->visible when it is set), and
 * grad_images = dL/dI in the image layout.  Outputs
 * (device, overwritten):
 *   dfeat [n][C] FP32   -- derivative of Eq. blend (points in the blend set)
 *   dpos  [3][n] FP32   -- dL/dx, dL/dy, dL/dz from the approximate spatial
 *                          gradient chained through the projection
 *   dpose [V][6] FP64   -- dL/dxi, xi = (rho, omega) applied as exp(xi)*(R,t)
 *                          on the left, at xi = 0
 *   dintr [V][9] FP64   -- dL/d(fx, fy, cx, cy, k1, k2, k3, p1, p2)
 * The FP64 sums are reduced in a fixed order (run-to-run deterministic). */
/* Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same pass as adop_render_forward, with the same frame
 * outputs, but without a workspace argument: the per-view records and the
 * FP32 sums live in a fixed array of ADOP_NOALLOC_SCRATCH_BYTES bytes that
 * the library holds on every GPU it runs on until the process ends.  The
 * call needs  256*V (rounded up to a multiple of 256)  +  pixels*C*4 (rounded
 * up to a multiple of 256)  bytes of it, e.g. 44.2 MB at 1920x1080 with 5
 * layers and 4 channels; a larger request fails with ADOP_E_WORKSPACE before
 * anything is enqueued.  The call allocates nothing (no hipMalloc, no
 * library allocation); the sums are cleared by the call itself.
 * `stream` must belong to the context's device.  Every call on one GPU uses
 * that GPU's single array: calls that overlap in time on one GPU (other
 * streams, other contexts or threads) race and give wrong results; calls
 * ordered on one stream are safe. */
#define ADOP_NOALLOC_SCRATCH_BYTES (64u << 20)
adop_status adop_render_forward_noalloc(adop_context* ctx, const adop_scene* scene,
                                        const adop_camera* cams, int32_t V,
                                        const adop_render_params* params,
                                        const adop_frame* frame, void* stream);

adop_status adop_render_backward(adop_context* ctx, const adop_scene* scene,
                                 const adop_camera* cams, int32_t V,
                                 const adop_render_params* params,
                                 const adop_frame* frame, const float* grad_images,
                                 float* dfeat, float* dpos, double* dpose, double* dintr,
                                 void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------- photometric tone mapper */
/* Differentiable tone mapping of Sec. 3.3 for V 3-channel HDR images
 * [V][3][h][w] FP32 (device), per image i and pixel (u, v):
 *   I_e = I_hdr * 2^-EV_i                          exposure
 *   I_w[c] = I_e[c] * white_i[c]                   white point (multiplies)
 *   I_v = I_w * (1 + a2 r^2 + a4 r^4 + a6 r^6)     vignette, r = |p - c_v|,
 *       p = ((u + 0.5) / w, (v + 0.5) / h) and c_v = (cx, cy) in the same
 *       normalised coordinates (pixel centres at integer u, v)
 *   I_ldr[c] = R_t(I_v[c])                          response (Eq. resonseleak)
 * R on [0, 1] is a table of K entries per channel sampled at k / (K - 1)
 * and linearly interpolated (the paper's 1D texture, initialised to x^0.45);
 * R_t(x) = leak x for x < 0 and -leak / sqrt(x) + leak + 1 for x > 1
 * (training; the paper uses leak = 0.01); leak < 0 clamps x to [0, 1]
 * (inference).  Every parameter is a device array, so a training loop can
 * update them without host round trips. */
typedef struct adop_tonemap {
    const float* ev;           /* device [V] exposure values EV_i */
    const float* white;        /* device [V][3] white points */
    const float* vignette;     /* device [5]: a2, a4, a6, cx, cy */
    const float* crf;          /* device [3][K] response tables */
    int32_t crf_size;          /* K, 2..1024 */
    float leak;                /* >= 0: leaky response; < 0: clamp */
} adop_tonemap;

/* ldr [V][3][h][w] FP32 (device); asynchronous on `stream`. */
adop_status adop_tonemap_forward(adop_context* ctx, const float* hdr, int32_t V, int32_t width,
                                 int32_t height, const adop_tonemap* tm, float* ldr, void* stream);

/* Workspace bytes of adop_tonemap_backward for V images. */
size_t adop_tonemap_workspace_bytes(int32_t V);

/* Gradients of L given grad_ldr = dL/dI_ldr [V][3][h][w] FP32 (device
 * outputs, overwritten): grad_hdr [V][3][h][w] FP32, d_ev [V], d_white [V][3]
 * (the paper keeps the green entry constant: the caller ignores it),
 * d_vignette [5] (summed over the V images, which share the camera) and
 * d_crf [3][K] FP64.  The exposure, white-point and vignette sums are FP64
 * in a fixed order; the table sums are FP64 in an order that varies between
 * runs.  Asynchronous on `stream`. */
adop_status adop_tonemap_backward(adop_context* ctx, const float* hdr, int32_t V, int32_t width,
                                  int32_t height, const adop_tonemap* tm, const float* grad_ldr,
                                  float* grad_hdr, double* d_ev, double* d_white, double* d_vignette,
                                  double* d_crf, void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------ atomic throughput */
/* Diagnostic (Sec. 3.1 "Implementation Details": the depth pass and the
 * accumulation pass are built on atomics): times `ops` device atomics of one
 * kind on the caller's device buffer -- kind 0: 64-bit unsigned minimum (the
 * depth pass's key update), kind 1: FP32 add (the accumulation's sums).  Op i
 * targets word (i * stride) mod footprint (8-byte words for kind 0, 4-byte
 * for kind 1; consecutive lanes take consecutive ops), so stride 32 with a
 * large footprint scatters every lane to its own cache line, a small
 * footprint stays in the caches and footprint 1 contends on one word.  The
 * buffer's contents are overwritten.  Enqueues the kernel between two events
 * on `stream`, waits for them and writes the kernel's duration in
 * milliseconds to *ms. */
adop_status adop_atomic_probe(adop_context* ctx, int32_t kind, int64_t ops, int64_t footprint, int64_t stride,
                              void* buffer, size_t buffer_bytes, double* ms, void* stream);

/* ------------------------------------------------ per-kernel timing */
/* When enabled, every kernel a render call enqueues is bracketed by HIP
 * events recorded on the same stream.  adop_timing_read waits for the
 * recorded events, writes for each kernel id k < nkernels the summed
 * duration in milliseconds and the number of launches since the previous
 * read, and clears the records.  Kernel ids: 0 k_clear, 1 k_depth,
 * 2 k_accum, 3 k_normalize, 4 k_pack, 5 k_backward, 6 k_reduce.  Not used
 * inside captured graphs. */
#define ADOP_TIMING_KERNELS 7
adop_status adop_timing_enable(adop_context* ctx, int32_t on);
adop_status adop_timing_read(adop_context* ctx, int32_t nkernels, double* total_ms, int64_t* launches);
const char* adop_timing_kernel_name(int32_t kernel);

/* ------------------------------------------- captured forward (serving) */
/* Capture the forward pass for V cameras of fixed sizes into a HIP graph
 * bound to the given scene, frame and workspace.  The graph holds kernels
 * only; adop_forward_graph_launch stages new cameras (same widths and
 * heights as `cams`) into the workspace and replays it.  The cameras go
 * through a ring of four pinned staging slots: a launch blocks the host only
 * while the copy of four launches earlier is still pending.  The view
 * records, frame and workspace are shared by all launches of one graph, so
 * its launches must be ordered on one stream (or by the caller). */
adop_status adop_forward_graph_create(adop_context* ctx, const adop_scene* scene,
                                      const adop_camera* cams, int32_t V,
                                      const adop_render_params* params,
                                      const adop_frame* frame,
                                      void* workspace, size_t workspace_bytes,
                                      adop_graph** out);
adop_status adop_forward_graph_launch(adop_graph* g, const adop_camera* cams, void* stream);
void adop_graph_destroy(adop_graph* g);

#ifdef __cplusplus
}
#endif
#endif /* ADOP_H */
