// C-ABI layer of the one-pixel point rasterizer: argument validation,
// pyramid layout, camera staging and kernel launches.  Declarations and the
// contract of every entry point are in include/adop.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "adop.h"
#include "device.h"
#include "launch.h"

using adop::ViewRec;

namespace {

constexpr int kSlots = 32;
constexpr size_t kSlotBytes = (size_t)ADOP_MAX_VIEWS * sizeof(ViewRec);

}  // namespace

// Fixed scratch of adop_render_forward_noalloc: the per-view records and the
// FP32 sums of the forward pass, one copy per GPU (each device that loads
// the library holds its own instance until the process ends).  In host code
// `scratch` only names the symbol; the device address of a GPU's instance
// comes from hipGetSymbolAddress with that GPU current (scratch_setup).
static_assert(ADOP_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must be a multiple of 256");
static __device__ __align__(256) unsigned char scratch[ADOP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current: looked up
// once per device, then reused by every context on it.
hipError_t scratch_setup(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255) != 0) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

struct adop_context {
    int device = 0;
    int cus = 256;
    std::string err;
    unsigned char* pinned = nullptr;
    hipEvent_t ev[kSlots] = {};
    bool used[kSlots] = {};
    int next = 0;
    // per-kernel timing (adop_timing_enable / adop_timing_read)
    bool timing = false;
    struct Mark { int kernel; hipEvent_t start, end; };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> pool;
    hipError_t timing_error = hipSuccess;
    // device address of this GPU's instance of `scratch` (null if the lookup failed)
    void* scratch_dev = nullptr;
    hipError_t scratch_error = hipSuccess;
};

// Camera staging of a captured graph: a ring of pinned slots, each reused
// only after the copy that last read it has completed.
constexpr int kGraphStaging = 4;

struct adop_graph {
    adop_context* ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned char* pinned = nullptr;           // kGraphStaging slots of V view records
    hipEvent_t ev[kGraphStaging] = {};
    bool used[kGraphStaging] = {};
    int64_t launches = 0;
    int V = 0;
    int layers = 0;
    std::vector<int32_t> wh;
    ViewRec* views_dev = nullptr;
    int64_t pixels = 0;
};

namespace {

adop_status fail(adop_context* ctx, adop_status s, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return s;
}

adop_status hip_fail(adop_context* ctx, hipError_t e, const char* where) {
    return fail(ctx, ADOP_E_DEVICE, "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
}

int64_t view_pixels(const adop_camera& c, int L) {
    int64_t p = 0;
    for (int l = 0; l < L; ++l) p += (int64_t)(c.width >> l) * (int64_t)(c.height >> l);
    return p;
}

adop_status check_cameras(adop_context* ctx, const adop_camera* cams, int32_t V, int32_t L, int32_t vmax) {
    if (!cams) return fail(ctx, ADOP_E_INVALID, "cams is NULL");
    if (V < 1 || V > vmax) return fail(ctx, ADOP_E_INVALID, "number of views %d outside [1,%d]", V, vmax);
    if (L < 1 || L > ADOP_MAX_LAYERS) return fail(ctx, ADOP_E_INVALID, "layers %d outside [1,%d]", L, ADOP_MAX_LAYERS);
    for (int v = 0; v < V; ++v) {
        const adop_camera& c = cams[v];
        if (c.width < 1 || c.height < 1) return fail(ctx, ADOP_E_INVALID, "camera %d: size %dx%d", v, c.width, c.height);
        if (c.width > ADOP_MAX_SIZE || c.height > ADOP_MAX_SIZE)
            return fail(ctx, ADOP_E_UNSUPPORTED, "camera %d: size %dx%d above %d", v, c.width, c.height, ADOP_MAX_SIZE);
        if ((c.width >> (L - 1)) < 1 || (c.height >> (L - 1)) < 1)
            return fail(ctx, ADOP_E_INVALID, "camera %d: %dx%d too small for %d layers", v, c.width, c.height, L);
        if (!(c.znear >= 0.0f)) return fail(ctx, ADOP_E_INVALID, "camera %d: znear must be >= 0", v);
    }
    return ADOP_OK;
}

adop_status layout(const adop_camera* cams, int32_t V, int32_t L, int64_t* total, int64_t* offsets) {
    int64_t acc = 0;
    for (int v = 0; v < V; ++v) {
        for (int l = 0; l < L; ++l) {
            if (offsets) offsets[(int64_t)v * L + l] = acc;
            acc += (int64_t)(cams[v].width >> l) * (int64_t)(cams[v].height >> l);
        }
    }
    *total = acc;
    return ADOP_OK;
}

void make_views(const adop_camera* cams, int32_t V, int32_t L, ViewRec* out) {
    int64_t acc = 0;
    for (int v = 0; v < V; ++v) {
        const adop_camera& c = cams[v];
        ViewRec r;
        std::memset(&r, 0, sizeof r);
        r.fx = c.fx; r.fy = c.fy; r.cx = c.cx; r.cy = c.cy;
        r.k1 = c.k1; r.k2 = c.k2; r.k3 = c.k3; r.p1 = c.p1; r.p2 = c.p2;
        r.znear = c.znear; r.r2max = c.r2_max;
        for (int k = 0; k < 9; ++k) r.R[k] = c.R[k];
        for (int k = 0; k < 3; ++k) r.t[k] = c.t[k];
        r.w = c.width; r.h = c.height; r.L = L;
        for (int l = 0; l < L; ++l) {
            r.lw[l] = c.width >> l;
            r.lh[l] = c.height >> l;
            r.base[l] = (uint32_t)acc;
            acc += (int64_t)r.lw[l] * r.lh[l];
        }
        out[v] = r;
    }
}

int64_t max_layer_pixels(const adop_camera* cams, int32_t V) {
    int64_t m = 0;
    for (int v = 0; v < V; ++v) m = std::max<int64_t>(m, (int64_t)cams[v].width * cams[v].height);
    return m;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int bwd_group_cap(int cus) { return std::max(8, cus * adop::kBwdGroupsPerCu / 8 * 8); }

size_t views_region(int32_t V) { return align256((size_t)std::max(V, 1) * sizeof(ViewRec)); }

// Workspace of a forward pass alone: view records, then the FP32 sums.
size_t forward_workspace_bytes(int32_t C, int32_t V, int64_t pixels) {
    return views_region(V) + align256((size_t)pixels * C * sizeof(float));
}

size_t workspace_bytes(int cus, int32_t C, int32_t V, int64_t pixels) {
    size_t fwd = (size_t)pixels * C * sizeof(float);
    size_t bwd = align256((size_t)pixels * adop::pack_stride(C) * sizeof(float)) +
                 (size_t)(bwd_group_cap(cus) + adop::kReduceSlices) * std::max(V, 1) * 16 * sizeof(double);
    return views_region(V) + align256(std::max(fwd, bwd));
}

adop_status check_scene(adop_context* ctx, const adop_scene* s) {
    if (!s) return fail(ctx, ADOP_E_INVALID, "scene is NULL");
    if (s->n < 0 || s->n > 0x7fffffffLL) return fail(ctx, ADOP_E_INVALID, "n=%lld outside [0, 2^31-1]", (long long)s->n);
    if (s->channels < 1 || s->channels > ADOP_MAX_CHANNELS)
        return fail(ctx, ADOP_E_UNSUPPORTED, "channels=%d outside [1,%d]", s->channels, ADOP_MAX_CHANNELS);
    if (s->dtype < ADOP_F32 || s->dtype > ADOP_F16) return fail(ctx, ADOP_E_UNSUPPORTED, "dtype %d", s->dtype);
    if (s->n > 0) {
        if (!s->x || !s->y || !s->z || !s->feat || !s->orig_index)
            return fail(ctx, ADOP_E_INVALID, "scene has a NULL device pointer");
        if (((uintptr_t)s->feat & 15) != 0) return fail(ctx, ADOP_E_INVALID, "scene feat must be 16-byte aligned");
    }
    return ADOP_OK;
}

adop_status check_common(adop_context* ctx, const adop_scene* scene, const adop_camera* cams, int32_t V,
                         const adop_render_params* params, const adop_frame* frame, void* ws, size_t ws_bytes,
                         int32_t vmax, int64_t* total, bool forward_only = false) {
    if (!ctx) return ADOP_E_INVALID;
    ctx->err.clear();
    adop_status s = check_scene(ctx, scene);
    if (s) return s;
    if (!params) return fail(ctx, ADOP_E_INVALID, "params is NULL");
    if (!(params->alpha >= 0.0f) || !std::isfinite(params->alpha))
        return fail(ctx, ADOP_E_INVALID, "alpha must be finite and >= 0");
    s = check_cameras(ctx, cams, V, params->layers, vmax);
    if (s) return s;
    const uint32_t known = ADOP_FLAG_SPATIAL_ALL | ADOP_FLAG_CULL_BACKFACE | ADOP_FLAG_CULL_PRINTED |
                           ADOP_FLAG_LOG_FEATURES | ADOP_FLAG_DISCARD;
    if (params->flags & ~known) return fail(ctx, ADOP_E_INVALID, "unknown flags 0x%x", params->flags);
    if ((params->flags & ADOP_FLAG_CULL_BACKFACE) && (params->flags & ADOP_FLAG_CULL_PRINTED))
        return fail(ctx, ADOP_E_INVALID, "at most one of the normal-culling flags may be set");
    if ((params->flags & (ADOP_FLAG_CULL_BACKFACE | ADOP_FLAG_CULL_PRINTED)) && scene->n > 0 &&
        (!scene->nx || !scene->ny || !scene->nz))
        return fail(ctx, ADOP_E_INVALID, "normal culling needs scene normals nx, ny, nz");
    if (params->flags & ADOP_FLAG_DISCARD) {
        if (scene->n > 0 && (!scene->radius || !scene->beta))
            return fail(ctx, ADOP_E_INVALID, "stochastic discarding needs scene radius and beta");
        if (!(params->gamma > 0.0f) || !std::isfinite(params->gamma))
            return fail(ctx, ADOP_E_INVALID, "stochastic discarding needs a finite gamma > 0");
    }
    if (params->env_map && params->env_size < 2)
        return fail(ctx, ADOP_E_INVALID, "env_size=%d must be >= 2 with an environment map", params->env_size);
    if (params->env_map && (int64_t)params->env_size * params->env_size >= ((int64_t)1 << 31))
        return fail(ctx, ADOP_E_UNSUPPORTED, "env_size=%d too large", params->env_size);
    if (!frame || !frame->images || !frame->keys || !frame->counts) return fail(ctx, ADOP_E_INVALID, "frame has a NULL buffer");
    layout(cams, V, params->layers, total, nullptr);
    if (frame->pixels != *total)
        return fail(ctx, ADOP_E_INVALID, "frame->pixels=%lld but the cameras need %lld", (long long)frame->pixels,
                    (long long)*total);
    if (*total >= 0x7fffffffLL || (*total) * scene->channels >= (int64_t)1 << 40)
        return fail(ctx, ADOP_E_UNSUPPORTED, "frame of %lld pixels is too large", (long long)*total);
    if (!ws) return fail(ctx, ADOP_E_WORKSPACE, "workspace is NULL");
    size_t need = forward_only ? forward_workspace_bytes(scene->channels, V, *total)
                               : workspace_bytes(ctx->cus, scene->channels, V, *total);
    if (ws_bytes < need) return fail(ctx, ADOP_E_WORKSPACE, "workspace %zu bytes < %zu", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return fail(ctx, ADOP_E_INVALID, "workspace must be 256-byte aligned");
    return ADOP_OK;
}

// Copy V view records into the workspace through a pinned staging slot.
adop_status stage_views(adop_context* ctx, const adop_camera* cams, int32_t V, int32_t L, void* ws, hipStream_t st) {
    int slot = ctx->next;
    ctx->next = (ctx->next + 1) % kSlots;
    hipError_t e;
    if (ctx->used[slot]) {
        e = hipEventSynchronize(ctx->ev[slot]);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
    }
    ViewRec* host = reinterpret_cast<ViewRec*>(ctx->pinned + (size_t)slot * kSlotBytes);
    make_views(cams, V, L, host);
    e = hipMemcpyAsync(ws, host, (size_t)V * sizeof(ViewRec), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(views)");
    e = hipEventRecord(ctx->ev[slot], st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    ctx->used[slot] = true;
    return ADOP_OK;
}

// Intrinsics, near plane, fold-over limit and pose of V views from a device
// camera table into the staged view records (sizes and the layer table stay
// those of the host cameras).
__global__ void k_views_from_table(const adop_camera* __restrict__ cams, int V, ViewRec* __restrict__ views) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const adop_camera c = cams[v];
    ViewRec& r = views[v];
    r.fx = c.fx; r.fy = c.fy; r.cx = c.cx; r.cy = c.cy;
    r.k1 = c.k1; r.k2 = c.k2; r.k3 = c.k3; r.p1 = c.p1; r.p2 = c.p2;
    r.znear = c.znear; r.r2max = c.r2_max;
    for (int k = 0; k < 9; ++k) r.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) r.t[k] = c.t[k];
}

// Stage the host cameras' view records, then (with a device camera table)
// overwrite their camera fields on the device.
adop_status stage_cameras(adop_context* ctx, const adop_camera* cams, int32_t V, const adop_render_params* params,
                          void* ws, hipStream_t st) {
    adop_status s = stage_views(ctx, cams, V, params->layers, ws, st);
    if (s || !params->cameras_device) return s;
    k_views_from_table<<<(V + 63) / 64, 64, 0, st>>>(params->cameras_device, V, static_cast<ViewRec*>(ws));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "camera table");
    return ADOP_OK;
}

hipEvent_t take_event(adop_context* ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void timer_mark(void* self, int kernel, int end, hipStream_t st) {
    adop_context* ctx = static_cast<adop_context*>(self);
    hipEvent_t e = take_event(ctx);
    if (!e) {
        ctx->timing_error = hipErrorOutOfMemory;
        return;
    }
    hipError_t r = hipEventRecord(e, st);
    if (r != hipSuccess) ctx->timing_error = r;
    if (!end) {
        ctx->marks.push_back({kernel, e, nullptr});
    } else {
        for (auto it = ctx->marks.rbegin(); it != ctx->marks.rend(); ++it)
            if (it->kernel == kernel && it->end == nullptr) {
                it->end = e;
                return;
            }
        ctx->pool.push_back(e);
    }
}

adop::Timer timer_of(adop_context* ctx) {
    adop::Timer t;
    if (ctx->timing) {
        t.fn = timer_mark;
        t.self = ctx;
    }
    return t;
}

adop::PointOpts point_opts(const adop_scene* scene, const adop_render_params* params) {
    adop::PointOpts o;
    o.flags = params->flags & (ADOP_FLAG_CULL_BACKFACE | ADOP_FLAG_CULL_PRINTED | ADOP_FLAG_LOG_FEATURES |
                               ADOP_FLAG_DISCARD);
    o.gamma = (params->flags & ADOP_FLAG_DISCARD) ? params->gamma : 0.0f;
    o.nx = scene->nx; o.ny = scene->ny; o.nz = scene->nz;
    o.radius = scene->radius; o.beta = scene->beta;
    return o;
}

adop::FwdArgs fwd_args(adop_context* ctx, const adop_scene* scene, const adop_camera* cams, int32_t V,
                       const adop_render_params* params, const adop_frame* frame, void* ws, int64_t total) {
    adop::FwdArgs a;
    a.dtype = scene->dtype;
    a.C = scene->channels;
    a.V = V;
    a.L = params->layers;
    a.cus = ctx->cus;
    a.n = scene->n;
    a.pixels = total;
    a.max_layer_pixels = max_layer_pixels(cams, V);
    a.fa = 1.0f + params->alpha;
    a.x = scene->x; a.y = scene->y; a.z = scene->z;
    a.feat = scene->feat;
    a.orig = scene->orig_index;
    a.views = reinterpret_cast<const ViewRec*>(ws);
    a.keys = frame->keys;
    a.counts = frame->counts;
    a.sums = reinterpret_cast<float*>(static_cast<unsigned char*>(ws) + views_region(V));
    a.images = frame->images;
    a.background = params->background;
    a.env = params->env_map;
    a.env_size = params->env_map ? params->env_size : 0;
    a.opts = point_opts(scene, params);
    a.timer = timer_of(ctx);
    a.vis = frame->visible;
    return a;
}

}  // namespace

extern "C" {

const char* adop_version(void) { return "adop-mi355x 0.1.0 (gfx950)"; }

const char* adop_status_string(adop_status s) {
    switch (s) {
        case ADOP_OK: return "ok";
        case ADOP_E_INVALID: return "invalid argument";
        case ADOP_E_UNSUPPORTED: return "unsupported";
        case ADOP_E_WORKSPACE: return "workspace too small";
        case ADOP_E_DEVICE: return "device error";
        case ADOP_E_STATE: return "invalid state";
        default: return "unknown status";
    }
}

adop_status adop_context_create(int32_t device, adop_context** out) {
    if (!out) return ADOP_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return ADOP_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return ADOP_E_DEVICE;
    adop_context* ctx = new adop_context();
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->cus = prop.multiProcessorCount;
    ctx->scratch_error = scratch_setup(device, &ctx->scratch_dev);
    if (hipHostMalloc((void**)&ctx->pinned, kSlots * kSlotBytes, hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return ADOP_E_DEVICE;
    }
    for (int i = 0; i < kSlots; ++i) {
        if (hipEventCreateWithFlags(&ctx->ev[i], hipEventDisableTiming) != hipSuccess) {
            adop_context_destroy(ctx);
            return ADOP_E_DEVICE;
        }
    }
    *out = ctx;
    return ADOP_OK;
}

void adop_context_destroy(adop_context* ctx) {
    if (!ctx) return;
    for (auto& m : ctx->marks) {
        if (m.start) { (void)hipEventSynchronize(m.start); (void)hipEventDestroy(m.start); }
        if (m.end) { (void)hipEventSynchronize(m.end); (void)hipEventDestroy(m.end); }
    }
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    for (int i = 0; i < kSlots; ++i) {
        if (ctx->ev[i]) {
            if (ctx->used[i]) (void)hipEventSynchronize(ctx->ev[i]);
            (void)hipEventDestroy(ctx->ev[i]);
        }
    }
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

adop_status adop_timing_enable(adop_context* ctx, int32_t on) {
    if (!ctx) return ADOP_E_INVALID;
    ctx->timing = on != 0;
    return ADOP_OK;
}

const char* adop_timing_kernel_name(int32_t kernel) {
    static const char* names[] = {"k_clear", "k_depth", "k_accum", "k_normalize", "k_pack", "k_backward", "k_reduce"};
    if (kernel < 0 || kernel >= adop::kKernelCount) return "";
    return names[kernel];
}

adop_status adop_timing_read(adop_context* ctx, int32_t nkernels, double* total_ms, int64_t* launches) {
    if (!ctx || !total_ms || !launches || nkernels < 1) return ADOP_E_INVALID;
    ctx->err.clear();
    for (int k = 0; k < nkernels; ++k) { total_ms[k] = 0.0; launches[k] = 0; }
    hipError_t first = ctx->timing_error;
    ctx->timing_error = hipSuccess;
    for (auto& m : ctx->marks) {
        if (m.end) {
            hipError_t e = hipEventSynchronize(m.end);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.start, m.end);
            if (e != hipSuccess && first == hipSuccess) first = e;
            if (e == hipSuccess && m.kernel < nkernels) {
                total_ms[m.kernel] += ms;
                launches[m.kernel] += 1;
            }
            ctx->pool.push_back(m.end);
        }
        ctx->pool.push_back(m.start);
    }
    ctx->marks.clear();
    if (first != hipSuccess) return hip_fail(ctx, first, "timing events");
    return ADOP_OK;
}

const char* adop_last_error(const adop_context* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

adop_status adop_views_layout(const adop_camera* cams, int32_t V, int32_t layers, int64_t* total_pixels,
                              int64_t* offsets) {
    if (!total_pixels) return ADOP_E_INVALID;
    adop_status s = check_cameras(nullptr, cams, V, layers, ADOP_MAX_VIEWS);
    if (s) return s;
    return layout(cams, V, layers, total_pixels, offsets);
}

size_t adop_workspace_bytes(const adop_context* ctx, int32_t channels, int32_t V, int64_t pixels) {
    if (channels < 1 || channels > ADOP_MAX_CHANNELS || V < 1 || pixels < 0) return 0;
    return workspace_bytes(ctx ? ctx->cus : 256, channels, V, pixels);
}

size_t adop_feature_bytes(int64_t n, int32_t channels, adop_dtype dtype) {
    if (n < 0 || channels < 1 || dtype < ADOP_F32 || dtype > ADOP_F16) return 0;
    return (size_t)n * channels * (dtype == ADOP_F32 ? 4 : 2);
}

adop_status adop_pyramid_layout(int32_t width, int32_t height, int32_t layers, int32_t channels, adop_layout* out) {
    if (!out) return ADOP_E_INVALID;
    std::memset(out, 0, sizeof *out);
    if (layers < 1 || layers > ADOP_MAX_LAYERS || channels < 1 || channels > ADOP_MAX_CHANNELS || width < 1 ||
        height < 1 || (width >> (layers - 1)) < 1 || (height >> (layers - 1)) < 1)
        return ADOP_E_INVALID;
    out->layers = layers;
    out->channels = channels;
    int64_t acc = 0;
    for (int l = 0; l < layers; ++l) {
        out->width[l] = width >> l;
        out->height[l] = height >> l;
        out->pixel_offset[l] = acc;
        acc += (int64_t)out->width[l] * out->height[l];
    }
    out->pixels = acc;
    out->image_bytes = acc * channels * 4;
    out->key_bytes = acc * 8;
    out->count_bytes = acc * 4;
    return ADOP_OK;
}

size_t adop_scene_bytes(int64_t n, int32_t channels, adop_dtype dtype) {
    if (n < 0 || n > 0x7fffffffLL || channels < 1 || channels > ADOP_MAX_CHANNELS || dtype < ADOP_F32 ||
        dtype > ADOP_F16)
        return 0;
    const size_t plane = align256((size_t)n * sizeof(float));
    const size_t fb = align256((size_t)n * channels * (dtype == ADOP_F32 ? 4 : 2));
    return 3 * plane + fb + align256((size_t)n * sizeof(int32_t));
}

adop_status adop_scene_bind(void* scene_mem, int64_t n, int32_t channels, adop_dtype dtype, adop_scene* out) {
    if (!out) return ADOP_E_INVALID;
    std::memset(out, 0, sizeof *out);
    if (adop_scene_bytes(n, channels, dtype) == 0) return ADOP_E_INVALID;
    if (!scene_mem || ((uintptr_t)scene_mem & 255) != 0) return ADOP_E_INVALID;
    unsigned char* p = static_cast<unsigned char*>(scene_mem);
    const size_t plane = align256((size_t)n * sizeof(float));
    const size_t fb = align256((size_t)n * channels * (dtype == ADOP_F32 ? 4 : 2));
    out->n = n;
    out->channels = channels;
    out->dtype = dtype;
    out->x = reinterpret_cast<const float*>(p);
    out->y = reinterpret_cast<const float*>(p + plane);
    out->z = reinterpret_cast<const float*>(p + 2 * plane);
    out->feat = p + 3 * plane;
    out->orig_index = reinterpret_cast<const int32_t*>(p + 3 * plane + fb);
    return ADOP_OK;
}

adop_status adop_cameras_upload(adop_context* ctx, const adop_camera* host, int32_t V, adop_camera* dev_table,
                                void* stream) {
    if (!ctx) return ADOP_E_INVALID;
    ctx->err.clear();
    adop_status s = check_cameras(ctx, host, V, 1, ADOP_MAX_VIEWS);
    if (s) return s;
    if (!dev_table || ((uintptr_t)dev_table & 3) != 0)
        return fail(ctx, ADOP_E_INVALID, "dev_table must be a 4-byte aligned device pointer");
    int slot = ctx->next;
    ctx->next = (ctx->next + 1) % kSlots;
    hipError_t e;
    if (ctx->used[slot] && (e = hipEventSynchronize(ctx->ev[slot])) != hipSuccess)
        return hip_fail(ctx, e, "hipEventSynchronize");
    unsigned char* staging = ctx->pinned + (size_t)slot * kSlotBytes;
    static_assert((size_t)ADOP_MAX_VIEWS * sizeof(adop_camera) <= kSlotBytes, "staging slot");
    std::memcpy(staging, host, (size_t)V * sizeof(adop_camera));
    hipStream_t st = (hipStream_t)stream;
    if ((e = hipMemcpyAsync(dev_table, staging, (size_t)V * sizeof(adop_camera), hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return hip_fail(ctx, e, "hipMemcpyAsync(cameras)");
    if ((e = hipEventRecord(ctx->ev[slot], st)) != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    ctx->used[slot] = true;
    return ADOP_OK;
}

adop_status adop_atomic_probe(adop_context* ctx, int32_t kind, int64_t ops, int64_t footprint, int64_t stride,
                              void* buffer, size_t buffer_bytes, double* ms, void* stream) {
    if (!ctx) return ADOP_E_INVALID;
    ctx->err.clear();
    if (kind != 0 && kind != 1) return fail(ctx, ADOP_E_INVALID, "kind %d is not 0 (u64 min) or 1 (f32 add)", kind);
    if (ops < 1 || footprint < 1 || stride < 1 || !buffer || !ms)
        return fail(ctx, ADOP_E_INVALID, "ops, footprint, stride must be >= 1 and pointers non-NULL");
    const size_t word = kind == 0 ? 8 : 4;
    if ((size_t)footprint > buffer_bytes / word)
        return fail(ctx, ADOP_E_INVALID, "footprint %lld words exceeds the buffer", (long long)footprint);
    if (((uintptr_t)buffer & (word - 1)) != 0) return fail(ctx, ADOP_E_INVALID, "buffer misaligned");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    auto done = [&](adop_status s) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return s;
    };
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        return done(hip_fail(ctx, e, "hipEventCreate"));
    if ((e = hipEventRecord(e0, st)) != hipSuccess) return done(hip_fail(ctx, e, "hipEventRecord"));
    if ((e = adop::atomic_probe(kind, ops, footprint, stride, buffer, ctx->cus, st)) != hipSuccess)
        return done(hip_fail(ctx, e, "atomic probe"));
    if ((e = hipEventRecord(e1, st)) != hipSuccess) return done(hip_fail(ctx, e, "hipEventRecord"));
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return done(hip_fail(ctx, e, "hipEventSynchronize"));
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return done(hip_fail(ctx, e, "hipEventElapsedTime"));
    *ms = t;
    return done(ADOP_OK);
}

size_t adop_tonemap_workspace_bytes(int32_t V) {
    if (V < 1 || V > ADOP_MAX_VIEWS) return 0;
    return (size_t)V * adop::kTonemapBlocks * 16 * sizeof(double);
}

static adop_status check_tonemap(adop_context* ctx, const float* hdr, int32_t V, int32_t w, int32_t h,
                                 const adop_tonemap* tm, adop::TonemapArgs* a) {
    if (!ctx) return ADOP_E_INVALID;
    ctx->err.clear();
    if (V < 1 || V > ADOP_MAX_VIEWS) return fail(ctx, ADOP_E_INVALID, "V=%d outside [1,%d]", V, ADOP_MAX_VIEWS);
    if (w < 1 || h < 1 || (int64_t)w * h >= ((int64_t)1 << 31))
        return fail(ctx, ADOP_E_INVALID, "image size %dx%d", w, h);
    if (!hdr || !tm || !tm->ev || !tm->white || !tm->vignette || !tm->crf)
        return fail(ctx, ADOP_E_INVALID, "NULL pointer");
    if (tm->crf_size < 2 || tm->crf_size > adop::kTonemapMaxTable)
        return fail(ctx, ADOP_E_INVALID, "crf_size=%d outside [2,%d]", tm->crf_size, adop::kTonemapMaxTable);
    if (!std::isfinite(tm->leak)) return fail(ctx, ADOP_E_INVALID, "leak must be finite");
    std::memset(a, 0, sizeof *a);
    a->V = V; a->w = w; a->h = h; a->K = tm->crf_size; a->leak = tm->leak;
    a->hdr = hdr; a->ev = tm->ev; a->white = tm->white; a->vig = tm->vignette; a->crf = tm->crf;
    return ADOP_OK;
}

adop_status adop_tonemap_forward(adop_context* ctx, const float* hdr, int32_t V, int32_t width, int32_t height,
                                 const adop_tonemap* tm, float* ldr, void* stream) {
    adop::TonemapArgs a;
    adop_status s = check_tonemap(ctx, hdr, V, width, height, tm, &a);
    if (s) return s;
    if (!ldr) return fail(ctx, ADOP_E_INVALID, "ldr is NULL");
    a.ldr = ldr;
    hipError_t e = adop::tonemap_forward(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "tone mapper forward");
    return ADOP_OK;
}

adop_status adop_tonemap_backward(adop_context* ctx, const float* hdr, int32_t V, int32_t width, int32_t height,
                                  const adop_tonemap* tm, const float* grad_ldr, float* grad_hdr, double* d_ev,
                                  double* d_white, double* d_vignette, double* d_crf, void* workspace,
                                  size_t workspace_bytes_, void* stream) {
    adop::TonemapArgs a;
    adop_status s = check_tonemap(ctx, hdr, V, width, height, tm, &a);
    if (s) return s;
    if (!grad_ldr || !grad_hdr || !d_ev || !d_white || !d_vignette || !d_crf)
        return fail(ctx, ADOP_E_INVALID, "NULL gradient buffer");
    if (!workspace) return fail(ctx, ADOP_E_WORKSPACE, "workspace is NULL");
    if (workspace_bytes_ < adop_tonemap_workspace_bytes(V))
        return fail(ctx, ADOP_E_WORKSPACE, "workspace %zu bytes < %zu", workspace_bytes_,
                    adop_tonemap_workspace_bytes(V));
    if (((uintptr_t)workspace & 15) != 0) return fail(ctx, ADOP_E_INVALID, "workspace must be 16-byte aligned");
    a.grad = grad_ldr; a.d_hdr = grad_hdr; a.d_ev = d_ev; a.d_white = d_white; a.d_vig = d_vignette; a.d_crf = d_crf;
    a.partials = static_cast<double*>(workspace);
    hipError_t e = adop::tonemap_backward(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "tone mapper backward");
    return ADOP_OK;
}

adop_status adop_scene_prepare(adop_context* ctx, const float* pos, const void* feat, int64_t n, int32_t channels,
                               adop_dtype dtype, int32_t block, uint64_t seed, float* x, float* y, float* z,
                               void* feat_out, int32_t* orig_index, void* stream) {
    if (!ctx) return ADOP_E_INVALID;
    ctx->err.clear();
    if (n < 0 || n > 0x7fffffffLL) return fail(ctx, ADOP_E_INVALID, "n=%lld outside [0, 2^31-1]", (long long)n);
    if (channels < 1 || channels > ADOP_MAX_CHANNELS) return fail(ctx, ADOP_E_UNSUPPORTED, "channels=%d", channels);
    if (dtype < ADOP_F32 || dtype > ADOP_F16) return fail(ctx, ADOP_E_UNSUPPORTED, "dtype %d", dtype);
    if (block < 0 || block % 256 != 0) return fail(ctx, ADOP_E_INVALID, "block=%d must be 0 or a positive multiple of 256", block);
    if (n > 0 && (!pos || !feat || !x || !y || !z || !feat_out || !orig_index))
        return fail(ctx, ADOP_E_INVALID, "NULL pointer");
    if (n > 0 && ((uintptr_t)feat_out & 15) != 0) return fail(ctx, ADOP_E_INVALID, "feat_out must be 16-byte aligned");
    adop::PrepArgs a;
    a.n = n; a.C = channels; a.dtype = dtype; a.block = block; a.seed = seed;
    a.pos = pos; a.feat = feat; a.x = x; a.y = y; a.z = z; a.feat_out = feat_out; a.orig = orig_index;
    hipError_t e = adop::scene_prepare(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "scene_prepare");
    return ADOP_OK;
}

adop_status adop_scene_gather(adop_context* ctx, const float* src, int32_t components, int64_t n,
                              const int32_t* orig_index, float* dst, void* stream) {
    if (!ctx) return ADOP_E_INVALID;
    ctx->err.clear();
    if (n < 0 || n > 0x7fffffffLL) return fail(ctx, ADOP_E_INVALID, "n=%lld outside [0, 2^31-1]", (long long)n);
    if (components < 1 || components > 4) return fail(ctx, ADOP_E_INVALID, "components=%d outside [1,4]", components);
    if (n > 0 && (!src || !orig_index || !dst)) return fail(ctx, ADOP_E_INVALID, "NULL pointer");
    hipError_t e = adop::scene_gather(src, components, n, orig_index, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "scene_gather");
    return ADOP_OK;
}

adop_status adop_knn_radius(adop_context* ctx, const float* x, const float* y, const float* z, int64_t n,
                            float* radius, void* stream) {
    if (!ctx) return ADOP_E_INVALID;
    ctx->err.clear();
    if (n < 5 || n > 0x7fffffffLL) return fail(ctx, ADOP_E_INVALID, "n=%lld outside [5, 2^31-1]", (long long)n);
    if (!x || !y || !z || !radius) return fail(ctx, ADOP_E_INVALID, "NULL pointer");
    hipError_t e = adop::knn_radius(x, y, z, n, radius, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "knn_radius");
    return ADOP_OK;
}

adop_status adop_render_forward(adop_context* ctx, const adop_scene* scene, const adop_camera* cams, int32_t V,
                                const adop_render_params* params, const adop_frame* frame, void* workspace,
                                size_t workspace_bytes_, void* stream) {
    int64_t total = 0;
    adop_status s = check_common(ctx, scene, cams, V, params, frame, workspace, workspace_bytes_, ADOP_MAX_VIEWS, &total);
    if (s) return s;
    hipStream_t st = (hipStream_t)stream;
    s = stage_cameras(ctx, cams, V, params, workspace, st);
    if (s) return s;
    adop::FwdArgs a = fwd_args(ctx, scene, cams, V, params, frame, workspace, total);
    hipError_t e = adop::launch_forward(a, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "forward launch");
    return ADOP_OK;
}

adop_status adop_render_forward_noalloc(adop_context* ctx, const adop_scene* scene, const adop_camera* cams,
                                        int32_t V, const adop_render_params* params, const adop_frame* frame,
                                        void* stream) {
    if (!ctx) return ADOP_E_INVALID;
    ctx->err.clear();
    if (!ctx->scratch_dev)
        return fail(ctx, ADOP_E_DEVICE, "no scratch array on device %d: %s (%d)", ctx->device,
                    hipGetErrorString(ctx->scratch_error), (int)ctx->scratch_error);
    hipStream_t st = (hipStream_t)stream;
    int sdev = -1;
    hipError_t e = st ? hipStreamGetDevice(st, &sdev) : hipGetDevice(&sdev);
    if (e != hipSuccess) return hip_fail(ctx, e, "stream device");
    if (sdev != ctx->device)
        return fail(ctx, ADOP_E_INVALID, "stream is on device %d, the context on device %d", sdev, ctx->device);
    if (scene && params && check_cameras(nullptr, cams, V, params->layers, ADOP_MAX_VIEWS) == ADOP_OK &&
        scene->channels >= 1 && scene->channels <= ADOP_MAX_CHANNELS) {
        int64_t total = 0;
        layout(cams, V, params->layers, &total, nullptr);
        const size_t need = forward_workspace_bytes(scene->channels, V, total);
        if (need > (size_t)ADOP_NOALLOC_SCRATCH_BYTES)
            return fail(ctx, ADOP_E_WORKSPACE,
                        "allocation-free forward: %lld pyramid pixels x %d channels need %zu scratch bytes, "
                        "more than the fixed %zu",
                        (long long)total, scene->channels, need, (size_t)ADOP_NOALLOC_SCRATCH_BYTES);
    }
    int64_t total = 0;
    adop_status s = check_common(ctx, scene, cams, V, params, frame, ctx->scratch_dev, ADOP_NOALLOC_SCRATCH_BYTES,
                                 ADOP_MAX_VIEWS, &total, true);
    if (s) return s;
    s = stage_cameras(ctx, cams, V, params, ctx->scratch_dev, st);
    if (s) return s;
    adop::FwdArgs a = fwd_args(ctx, scene, cams, V, params, frame, ctx->scratch_dev, total);
    e = adop::launch_forward(a, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "forward launch");
    return ADOP_OK;
}

adop_status adop_render_backward(adop_context* ctx, const adop_scene* scene, const adop_camera* cams, int32_t V,
                                 const adop_render_params* params, const adop_frame* frame, const float* grad_images,
                                 float* dfeat, float* dpos, double* dpose, double* dintr, void* workspace,
                                 size_t workspace_bytes_, void* stream) {
    int64_t total = 0;
    adop_status s = check_common(ctx, scene, cams, V, params, frame, workspace, workspace_bytes_, ADOP_MAX_VIEWS_BWD,
                                 &total);
    if (s) return s;
    if (!grad_images || !dpose || !dintr) return fail(ctx, ADOP_E_INVALID, "NULL gradient buffer");
    if (scene->n > 0 && (!dfeat || !dpos)) return fail(ctx, ADOP_E_INVALID, "NULL dfeat/dpos");
    if (scene->n > 0 && ((uintptr_t)dfeat & 15) != 0) return fail(ctx, ADOP_E_INVALID, "dfeat must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    s = stage_cameras(ctx, cams, V, params, workspace, st);
    if (s) return s;
    adop::BwdArgs a;
    a.dtype = scene->dtype;
    a.C = scene->channels;
    a.V = V;
    a.L = params->layers;
    a.cus = ctx->cus;
    a.groups = bwd_group_cap(ctx->cus);   // upper bound of the backward grid (partials buffer)
    a.flags = params->flags;
    a.n = scene->n;
    a.pixels = total;
    a.max_layer_pixels = max_layer_pixels(cams, V);
    a.fa = 1.0f + params->alpha;
    a.x = scene->x; a.y = scene->y; a.z = scene->z;
    a.feat = scene->feat;
    a.views = reinterpret_cast<const ViewRec*>(workspace);
    a.keys = frame->keys;
    a.counts = frame->counts;
    a.images = frame->images;
    a.grad = grad_images;
    unsigned char* wsb = static_cast<unsigned char*>(workspace) + views_region(V);
    a.pack = reinterpret_cast<float*>(wsb);
    a.partials = reinterpret_cast<double*>(wsb + align256((size_t)total * adop::pack_stride(a.C) * sizeof(float)));
    a.slices = a.partials + (size_t)a.groups * V * 16;
    a.dfeat = dfeat;
    a.dpos = dpos;
    a.dpose = dpose;
    a.dintr = dintr;
    a.background = params->background;
    a.env = params->env_map;
    a.env_size = params->env_map ? params->env_size : 0;
    a.env_grad = params->env_map ? params->env_grad : nullptr;
    a.opts = point_opts(scene, params);
    a.timer = timer_of(ctx);
    a.vis = frame->visible;
    hipError_t e = adop::launch_backward(a, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "backward launch");
    return ADOP_OK;
}

adop_status adop_forward_graph_create(adop_context* ctx, const adop_scene* scene, const adop_camera* cams, int32_t V,
                                      const adop_render_params* params, const adop_frame* frame, void* workspace,
                                      size_t workspace_bytes_, adop_graph** out) {
    if (!out) return fail(ctx, ADOP_E_INVALID, "out is NULL");
    *out = nullptr;
    int64_t total = 0;
    adop_status s = check_common(ctx, scene, cams, V, params, frame, workspace, workspace_bytes_, ADOP_MAX_VIEWS, &total);
    if (s) return s;
    adop_graph* g = new adop_graph();
    g->ctx = ctx;
    g->V = V;
    g->layers = params->layers;
    g->pixels = total;
    g->views_dev = reinterpret_cast<ViewRec*>(workspace);
    for (int v = 0; v < V; ++v) {
        g->wh.push_back(cams[v].width);
        g->wh.push_back(cams[v].height);
    }
    hipError_t e;
    hipStream_t cs = nullptr;
    auto cleanup = [&](adop_status st) {
        if (cs) (void)hipStreamDestroy(cs);
        adop_graph_destroy(g);
        return st;
    };
    if ((e = hipHostMalloc((void**)&g->pinned, (size_t)kGraphStaging * V * sizeof(ViewRec), hipHostMallocDefault)) !=
        hipSuccess)
        return cleanup(hip_fail(ctx, e, "hipHostMalloc"));
    for (int k = 0; k < kGraphStaging; ++k)
        if ((e = hipEventCreateWithFlags(&g->ev[k], hipEventDisableTiming)) != hipSuccess)
            return cleanup(hip_fail(ctx, e, "hipEventCreate"));
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
        return cleanup(hip_fail(ctx, e, "hipStreamCreate"));
    adop::FwdArgs a = fwd_args(ctx, scene, cams, V, params, frame, workspace, total);
    a.timer = adop::Timer();
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return cleanup(hip_fail(ctx, e, "hipStreamBeginCapture"));
    hipError_t le = hipSuccess;
    if (params->cameras_device) {
        k_views_from_table<<<(V + 63) / 64, 64, 0, cs>>>(params->cameras_device, V, g->views_dev);
        le = hipGetLastError();
    }
    if (le == hipSuccess) le = adop::launch_forward(a, cs);
    e = hipStreamEndCapture(cs, &g->graph);
    if (le != hipSuccess) return cleanup(hip_fail(ctx, le, "forward launch (capture)"));
    if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "hipStreamEndCapture"));
    if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
        return cleanup(hip_fail(ctx, e, "hipGraphInstantiate"));
    (void)hipStreamDestroy(cs);
    *out = g;
    return ADOP_OK;
}

adop_status adop_forward_graph_launch(adop_graph* g, const adop_camera* cams, void* stream) {
    if (!g) return ADOP_E_INVALID;
    adop_context* ctx = g->ctx;
    ctx->err.clear();
    adop_status s = check_cameras(ctx, cams, g->V, g->layers, ADOP_MAX_VIEWS);
    if (s) return s;
    for (int v = 0; v < g->V; ++v)
        if (cams[v].width != g->wh[2 * v] || cams[v].height != g->wh[2 * v + 1])
            return fail(ctx, ADOP_E_INVALID, "camera %d size differs from the captured graph", v);
    hipError_t e;
    const int k = (int)(g->launches % kGraphStaging);
    // the slot's previous copy (kGraphStaging launches ago) must have read it
    if (g->used[k] && (e = hipEventSynchronize(g->ev[k])) != hipSuccess)
        return hip_fail(ctx, e, "hipEventSynchronize");
    hipStream_t st = (hipStream_t)stream;
    ViewRec* host = reinterpret_cast<ViewRec*>(g->pinned) + (size_t)k * g->V;
    make_views(cams, g->V, g->layers, host);
    if ((e = hipMemcpyAsync(g->views_dev, host, (size_t)g->V * sizeof(ViewRec), hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return hip_fail(ctx, e, "hipMemcpyAsync(views)");
    if ((e = hipEventRecord(g->ev[k], st)) != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    g->used[k] = true;
    ++g->launches;
    if ((e = hipGraphLaunch(g->exec, st)) != hipSuccess) return hip_fail(ctx, e, "hipGraphLaunch");
    return ADOP_OK;
}

void adop_graph_destroy(adop_graph* g) {
    if (!g) return;
    for (int k = 0; k < kGraphStaging; ++k)
        if (g->used[k] && g->ev[k]) (void)hipEventSynchronize(g->ev[k]);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (int k = 0; k < kGraphStaging; ++k)
        if (g->ev[k]) (void)hipEventDestroy(g->ev[k]);
    if (g->pinned) (void)hipHostFree(g->pinned);
    delete g;
}

}  // extern "C"
