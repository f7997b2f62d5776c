"""ctypes binding of libadop.so (include/adop.h).

Argument marshalling only: device memory comes from torch tensors, streams
from torch's current stream, and every step of rendering runs in the HIP
kernels of libadop.so.  There is no CPU fallback: if the library is missing,
loading it raises.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# ADOP_LIB selects another build of the same library (e.g. one compiled with
# different tuning macros); the default is the in-tree libadop.so.
LIB_PATH = os.environ.get("ADOP_LIB", os.path.join(HERE, "libadop.so"))

OK, E_INVALID, E_UNSUPPORTED, E_WORKSPACE, E_DEVICE, E_STATE = range(6)
F32, BF16, F16 = 0, 1, 2
FLAG_SPATIAL_ALL = 1
MAX_LAYERS, MAX_CHANNELS, MAX_VIEWS, MAX_VIEWS_BWD = 8, 16, 256, 32

DTYPES = {"f32": F32, "bf16": BF16, "f16": F16}
TORCH_STORAGE = {F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}


class AdopError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"adop status {status}: {msg}")
        self.status = status


class Camera(ct.Structure):
    _fields_ = [("width", ct.c_int32), ("height", ct.c_int32),
                ("fx", ct.c_float), ("fy", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float),
                ("k1", ct.c_float), ("k2", ct.c_float), ("k3", ct.c_float),
                ("p1", ct.c_float), ("p2", ct.c_float),
                ("znear", ct.c_float), ("r2_max", ct.c_float),
                ("R", ct.c_float * 9), ("t", ct.c_float * 3)]


class RenderParams(ct.Structure):
    _fields_ = [("layers", ct.c_int32), ("alpha", ct.c_float), ("flags", ct.c_uint32),
                ("background", ct.c_void_p), ("gamma", ct.c_float), ("cameras_device", ct.c_void_p),
                ("env_map", ct.c_void_p), ("env_size", ct.c_int32), ("env_grad", ct.c_void_p)]


MAX_LAYERS_ = 8


class Layout(ct.Structure):
    _fields_ = [("layers", ct.c_int32), ("channels", ct.c_int32),
                ("width", ct.c_int32 * MAX_LAYERS_), ("height", ct.c_int32 * MAX_LAYERS_),
                ("pixel_offset", ct.c_int64 * MAX_LAYERS_), ("pixels", ct.c_int64),
                ("image_bytes", ct.c_int64), ("key_bytes", ct.c_int64), ("count_bytes", ct.c_int64)]


class SceneDesc(ct.Structure):
    _fields_ = [("n", ct.c_int64), ("channels", ct.c_int32), ("dtype", ct.c_int32),
                ("x", ct.c_void_p), ("y", ct.c_void_p), ("z", ct.c_void_p),
                ("feat", ct.c_void_p), ("orig_index", ct.c_void_p),
                ("nx", ct.c_void_p), ("ny", ct.c_void_p), ("nz", ct.c_void_p),
                ("radius", ct.c_void_p), ("beta", ct.c_void_p)]


class FrameDesc(ct.Structure):
    _fields_ = [("images", ct.c_void_p), ("keys", ct.c_void_p), ("counts", ct.c_void_p),
                ("pixels", ct.c_int64), ("visible", ct.c_void_p)]


_LIB = None


def lib():
    """Load libadop.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2110_06635_amd/build.py "
                               "(or __graft_entry__.build()); there is no fallback")
        L = ct.CDLL(LIB_PATH)
        P, S, I32, I64 = ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int64
        L.adop_version.restype = ct.c_char_p
        L.adop_status_string.restype = ct.c_char_p
        L.adop_status_string.argtypes = [S]
        L.adop_context_create.restype = S
        L.adop_context_create.argtypes = [I32, ct.POINTER(P)]
        L.adop_context_destroy.restype = None
        L.adop_context_destroy.argtypes = [P]
        L.adop_last_error.restype = ct.c_char_p
        L.adop_last_error.argtypes = [P]
        L.adop_views_layout.restype = S
        L.adop_views_layout.argtypes = [P, I32, I32, ct.POINTER(I64), P]
        L.adop_workspace_bytes.restype = ct.c_size_t
        L.adop_workspace_bytes.argtypes = [P, I32, I32, I64]
        L.adop_feature_bytes.restype = ct.c_size_t
        L.adop_feature_bytes.argtypes = [I64, I32, I32]
        L.adop_pyramid_layout.restype = S
        L.adop_pyramid_layout.argtypes = [I32, I32, I32, I32, P]
        L.adop_scene_bytes.restype = ct.c_size_t
        L.adop_scene_bytes.argtypes = [I64, I32, I32]
        L.adop_scene_bind.restype = S
        L.adop_scene_bind.argtypes = [P, I64, I32, I32, P]
        L.adop_cameras_upload.restype = S
        L.adop_cameras_upload.argtypes = [P, P, I32, P, P]
        L.adop_atomic_probe.restype = S
        L.adop_atomic_probe.argtypes = [P, I32, I64, I64, I64, P, ct.c_size_t, P, P]
        L.adop_tonemap_forward.restype = S
        L.adop_tonemap_forward.argtypes = [P, P, I32, I32, I32, P, P, P]
        L.adop_tonemap_workspace_bytes.restype = ct.c_size_t
        L.adop_tonemap_workspace_bytes.argtypes = [I32]
        L.adop_tonemap_backward.restype = S
        L.adop_tonemap_backward.argtypes = [P, P, I32, I32, I32, P, P, P, P, P, P, P, P, ct.c_size_t, P]
        L.adop_scene_prepare.restype = S
        L.adop_scene_prepare.argtypes = [P, P, P, I64, I32, I32, I32, ct.c_uint64, P, P, P, P, P, P]
        L.adop_scene_gather.restype = S
        L.adop_scene_gather.argtypes = [P, P, I32, I64, P, P, P]
        L.adop_knn_radius.restype = S
        L.adop_knn_radius.argtypes = [P, P, P, P, I64, P, P]
        L.adop_render_forward.restype = S
        L.adop_render_forward.argtypes = [P, P, P, I32, P, P, P, ct.c_size_t, P]
        L.adop_render_forward_noalloc.restype = S
        L.adop_render_forward_noalloc.argtypes = [P, P, P, I32, P, P, P]
        L.adop_render_backward.restype = S
        L.adop_render_backward.argtypes = [P, P, P, I32, P, P, P, P, P, P, P, P, ct.c_size_t, P]
        L.adop_forward_graph_create.restype = S
        L.adop_forward_graph_create.argtypes = [P, P, P, I32, P, P, P, ct.c_size_t, ct.POINTER(P)]
        L.adop_forward_graph_launch.restype = S
        L.adop_forward_graph_launch.argtypes = [P, P, P]
        L.adop_graph_destroy.restype = None
        L.adop_graph_destroy.argtypes = [P]
        L.adop_timing_enable.restype = S
        L.adop_timing_enable.argtypes = [P, I32]
        L.adop_timing_read.restype = S
        L.adop_timing_read.argtypes = [P, I32, P, P]
        L.adop_timing_kernel_name.restype = ct.c_char_p
        L.adop_timing_kernel_name.argtypes = [I32]
        _LIB = L
    return _LIB


EXPORTS = ["adop_version", "adop_status_string", "adop_context_create", "adop_context_destroy",
           "adop_last_error", "adop_views_layout", "adop_workspace_bytes", "adop_feature_bytes",
           "adop_pyramid_layout", "adop_scene_bytes", "adop_scene_bind", "adop_cameras_upload",
           "adop_tonemap_forward", "adop_tonemap_workspace_bytes", "adop_tonemap_backward",
           "adop_atomic_probe",
           "adop_scene_prepare", "adop_scene_gather", "adop_knn_radius",
           "adop_render_forward", "adop_render_forward_noalloc", "adop_render_backward",
           "adop_forward_graph_create", "adop_forward_graph_launch", "adop_graph_destroy",
           "adop_timing_enable", "adop_timing_read", "adop_timing_kernel_name"]
TIMING_KERNELS = 7


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _stream(stream) -> ct.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


def make_cameras(cams: Sequence) -> ct.Array:
    """synth.Camera-like objects (or Camera structs) -> adop_camera array."""
    arr = (Camera * len(cams))()
    for k, c in enumerate(cams):
        if isinstance(c, Camera):
            ct.memmove(ct.byref(arr[k]), ct.byref(c), ct.sizeof(Camera))
            continue
        o = arr[k]
        o.width, o.height = int(c.width), int(c.height)
        for f in ("fx", "fy", "cx", "cy", "k1", "k2", "k3", "p1", "p2", "znear"):
            setattr(o, f, float(np.float32(getattr(c, f))))
        o.r2_max = float(np.float32(c.r2_max)) if math.isfinite(c.r2_max) else math.inf
        R = np.asarray(c.R, dtype=np.float32).reshape(9)
        t = np.asarray(c.t, dtype=np.float32).reshape(3)
        for j in range(9):
            o.R[j] = float(R[j])
        for j in range(3):
            o.t[j] = float(t[j])
    return arr


def views_layout(cams, layers: int):
    """Total pyramid pixels and offsets o(v,l) (numpy [V,L])."""
    arr = cams if isinstance(cams, ct.Array) else make_cameras(cams)
    V = len(arr)
    total = ct.c_int64()
    offs = np.zeros((V, layers), dtype=np.int64)
    st = lib().adop_views_layout(arr, V, layers, ct.byref(total), offs.ctypes.data_as(ct.c_void_p))
    if st != OK:
        raise AdopError(st, "invalid cameras/layers")
    return int(total.value), offs


def pyramid_layout(width: int, height: int, layers: int, channels: int) -> dict:
    """adop_pyramid_layout as a dict (host only)."""
    out = Layout()
    st = lib().adop_pyramid_layout(width, height, layers, channels, ct.byref(out))
    if st != OK:
        raise AdopError(st, "invalid pyramid")
    return {"layers": out.layers, "channels": out.channels,
            "width": list(out.width[:layers]), "height": list(out.height[:layers]),
            "pixel_offset": list(out.pixel_offset[:layers]), "pixels": out.pixels,
            "image_bytes": out.image_bytes, "key_bytes": out.key_bytes, "count_bytes": out.count_bytes}


CAMERA_FLOATS = 25   # sizeof(adop_camera) / 4


def cameras_upload(ctx: "Context", cams, stream=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Device camera table [V, 25] (the adop_camera records as 4-byte words)."""
    arr = cams if isinstance(cams, ct.Array) else make_cameras(cams)
    V = len(arr)
    if out is None:
        out = torch.empty((V, CAMERA_FLOATS), dtype=torch.float32, device=f"cuda:{ctx.device}")
    assert out.is_cuda and out.is_contiguous() and out.numel() == V * CAMERA_FLOATS
    ctx.check(lib().adop_cameras_upload(ctx.handle, arr, V, _ptr(out), _stream(stream)), "adop_cameras_upload")
    return out


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        torch.cuda.init()
        with torch.cuda.device(device):
            h = ct.c_void_p()
            st = lib().adop_context_create(device, ct.byref(h))
            if st != OK:
                raise AdopError(st, "adop_context_create failed")
        self.handle = h
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.adop_context_destroy(h)
            self.handle = None

    def check(self, st: int, what: str):
        if st != OK:
            msg = lib().adop_last_error(self.handle).decode()
            raise AdopError(st, f"{what}: {msg}")

    def workspace(self, channels: int, views: int, pixels: int) -> torch.Tensor:
        need = int(lib().adop_workspace_bytes(self.handle, channels, views, pixels))
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def timing(self, on: bool):
        self.check(lib().adop_timing_enable(self.handle, 1 if on else 0), "adop_timing_enable")

    def timing_read(self):
        """{kernel name: (total ms, launches)} since the previous read."""
        ms = np.zeros(TIMING_KERNELS, np.float64)
        cnt = np.zeros(TIMING_KERNELS, np.int64)
        st = lib().adop_timing_read(self.handle, TIMING_KERNELS, ms.ctypes.data_as(ct.c_void_p),
                                    cnt.ctypes.data_as(ct.c_void_p))
        self.check(st, "adop_timing_read")
        return {lib().adop_timing_kernel_name(k).decode(): (float(ms[k]), int(cnt[k]))
                for k in range(TIMING_KERNELS)}

    def workspace_bytes(self, channels: int, views: int, pixels: int) -> int:
        return int(lib().adop_workspace_bytes(self.handle, channels, views, pixels))


class Scene:
    """A prepared point cloud resident in device memory (SoA positions,
    features in storage dtype, original indices)."""

    def __init__(self, x, y, z, feat, orig, dtype: int):
        self.x, self.y, self.z, self.feat, self.orig = x, y, z, feat, orig
        self.dtype = dtype
        self.normals = None    # [3, n] planes (normal culling)
        self.radius = None     # [n] world radius (stochastic discarding)
        self.beta = None       # [n] U[0,1) per point (stochastic discarding)

    @property
    def n(self) -> int:
        return int(self.x.numel())

    @property
    def channels(self) -> int:
        return int(self.feat.shape[1])

    def desc(self) -> SceneDesc:
        nrm = self.normals
        return SceneDesc(self.n, self.channels, self.dtype, _ptr(self.x), _ptr(self.y), _ptr(self.z),
                         _ptr(self.feat), _ptr(self.orig),
                         _ptr(nrm[0]) if nrm is not None else None, _ptr(nrm[1]) if nrm is not None else None,
                         _ptr(nrm[2]) if nrm is not None else None, _ptr(self.radius), _ptr(self.beta))

    def gather(self, ctx: "Context", values: torch.Tensor, stream=None) -> torch.Tensor:
        """Per-point values in the caller's order ([n] or [n, k], k <= 4,
        FP32 device) -> planes [k, n] (or [n]) in the prepared order."""
        v = values.contiguous()
        assert v.is_cuda and v.dtype == torch.float32 and v.shape[0] == self.n
        k = 1 if v.dim() == 1 else int(v.shape[1])
        out = torch.empty((k, self.n), dtype=torch.float32, device=v.device)
        st = lib().adop_scene_gather(ctx.handle, _ptr(v), k, self.n, _ptr(self.orig), _ptr(out), _stream(stream))
        ctx.check(st, "adop_scene_gather")
        return out[0] if v.dim() == 1 else out

    def set_normals(self, ctx: "Context", normals: torch.Tensor, stream=None):
        """Normals [n, 3] in the caller's order (normal culling)."""
        self.normals = self.gather(ctx, normals, stream)

    def set_discard(self, ctx: "Context", beta: torch.Tensor, radius: Optional[torch.Tensor] = None,
                    stream=None):
        """Stochastic discarding inputs: beta [n] in the caller's order and
        the world radius (computed with adop_knn_radius when not given)."""
        self.beta = self.gather(ctx, beta, stream)
        self.radius = self.gather(ctx, radius, stream) if radius is not None else knn_radius(ctx, self, stream)

    @staticmethod
    def prepare(ctx: Context, pos: torch.Tensor, feat: torch.Tensor, dtype: int = F32,
                block: int = 0, seed: int = 1, stream=None) -> "Scene":
        """Morton order (and optional block shuffle, block > 0) of a device
        point cloud (pos [n,3] FP32, feat [n,C] in the storage dtype)."""
        dev = pos.device
        n = int(pos.shape[0])
        C = int(feat.shape[1])
        assert pos.is_cuda and feat.is_cuda and pos.dtype == torch.float32
        assert feat.dtype == TORCH_STORAGE[dtype]
        pos = pos.contiguous()
        feat = feat.contiguous()
        x = torch.empty(n, dtype=torch.float32, device=dev)
        y = torch.empty(n, dtype=torch.float32, device=dev)
        z = torch.empty(n, dtype=torch.float32, device=dev)
        fo = torch.empty((n, C), dtype=TORCH_STORAGE[dtype], device=dev)
        orig = torch.empty(n, dtype=torch.int32, device=dev)
        st = lib().adop_scene_prepare(ctx.handle, _ptr(pos), _ptr(feat), n, C, dtype, block, seed,
                                      _ptr(x), _ptr(y), _ptr(z), _ptr(fo), _ptr(orig), _stream(stream))
        ctx.check(st, "adop_scene_prepare")
        return Scene(x, y, z, fo, orig, dtype)

    @staticmethod
    def identity(pos: torch.Tensor, feat: torch.Tensor, dtype: int = F32) -> "Scene":
        """Use the points in the given order (no Morton shuffle)."""
        n = int(pos.shape[0])
        p = pos.contiguous()
        return Scene(p[:, 0].contiguous(), p[:, 1].contiguous(), p[:, 2].contiguous(),
                     feat.contiguous(), torch.arange(n, dtype=torch.int32, device=pos.device), dtype)


def knn_radius(ctx: "Context", scene: Scene, stream=None) -> torch.Tensor:
    """Distance of every point of the scene to its 4th-nearest other point
    (prepared order)."""
    out = torch.empty(scene.n, dtype=torch.float32, device=scene.x.device)
    st = lib().adop_knn_radius(ctx.handle, _ptr(scene.x), _ptr(scene.y), _ptr(scene.z), scene.n, _ptr(out),
                               _stream(stream))
    ctx.check(st, "adop_knn_radius")
    return out


FLAG_SPATIAL_ALL = 1
FLAG_CULL_BACKFACE = 2
FLAG_CULL_PRINTED = 4
FLAG_LOG_FEATURES = 8
FLAG_DISCARD = 16
GAMMA = 1.5   # the paper's discarding parameter


def _params(layers: int, alpha: float, flags: int, background, C: int, gamma: float = GAMMA,
            cams_device: Optional[torch.Tensor] = None, V: int = 0, env_map: Optional[torch.Tensor] = None,
            env_grad: Optional[torch.Tensor] = None):
    bg = None
    if background is not None:
        bg = (ct.c_float * C)(*[float(b) for b in np.asarray(background, np.float32).reshape(C)])
    if cams_device is not None:
        assert cams_device.is_cuda and cams_device.is_contiguous() and cams_device.dtype == torch.float32
        assert cams_device.numel() == V * CAMERA_FLOATS, "camera table must hold the views' cameras"
    S = 0
    if env_map is not None:
        assert env_map.is_cuda and env_map.dtype == torch.float32 and env_map.is_contiguous()
        assert env_map.dim() == 3 and env_map.shape[0] == C and env_map.shape[1] == env_map.shape[2]
        S = int(env_map.shape[1])
        if env_grad is not None:
            assert env_grad.shape == env_map.shape and env_grad.dtype == torch.float32 and env_grad.is_contiguous()
    p = RenderParams(layers, float(np.float32(alpha)), flags, ct.cast(bg, ct.c_void_p) if bg is not None else None,
                     float(np.float32(gamma)), _ptr(cams_device), _ptr(env_map), S, _ptr(env_grad))
    return p, bg


class Frame:
    def __init__(self, cams, layers: int, channels: int, device):
        self.cams = cams if isinstance(cams, ct.Array) else make_cameras(cams)
        self.layers = layers
        self.channels = channels
        self.pixels, self.offsets = views_layout(self.cams, layers)
        self.images = torch.empty(channels * self.pixels, dtype=torch.float32, device=device)
        self.keys = torch.empty(self.pixels, dtype=torch.int64, device=device)
        self.counts = torch.empty(self.pixels, dtype=torch.int32, device=device)
        # [V, n] blend-set bits per point and view, written by a forward that
        # records them and read by the backward of the same frame
        self.visible: Optional[torch.Tensor] = None

    def desc(self) -> FrameDesc:
        return FrameDesc(_ptr(self.images), _ptr(self.keys), _ptr(self.counts), self.pixels,
                         _ptr(self.visible) if self.visible is not None else None)

    def layer_image(self, v: int, l: int) -> torch.Tensor:
        cam = self.cams[v]
        w, h = cam.width >> l, cam.height >> l
        o = int(self.offsets[v, l])
        C = self.channels
        return self.images[C * o: C * (o + w * h)].view(C, h, w)

    def layer_images(self, l: int) -> torch.Tensor:
        """Layer l of all views as a strided [V, C, h_l, w_l] view (views of equal size)."""
        V = len(self.cams)
        w, h = self.cams[0].width >> l, self.cams[0].height >> l
        for v in range(V):
            assert (self.cams[v].width >> l) == w and (self.cams[v].height >> l) == h
        C = self.channels
        o0 = int(self.offsets[0, l])
        stride_v = C * (int(self.offsets[1, l]) - o0) if V > 1 else C * w * h
        return self.images.as_strided((V, C, h, w), (stride_v, h * w, w, 1), C * o0)


def render_forward(ctx: Context, scene: Scene, cams, layers: int, alpha: float = 0.01, flags: int = 0,
                   background=None, frame: Optional[Frame] = None, stream=None,
                   workspace: Optional[torch.Tensor] = None, gamma: float = GAMMA,
                   record_visibility: bool = True, cams_device: Optional[torch.Tensor] = None,
                   env_map: Optional[torch.Tensor] = None) -> Frame:
    """record_visibility: also write frame.visible ([V, n] uint8, bit l =
    the point is in layer l's blend set), which lets render_backward skip
    the points that blend nowhere; False leaves frame.visible unset.
    cams_device: a device camera table ([V, 25], cameras_upload) whose
    intrinsics and poses replace those of `cams` (which give the sizes).
    env_map: [C, S, S] FP32 environment map sampled by the empty pixels."""
    C = scene.channels
    if frame is None:
        frame = Frame(cams, layers, C, scene.x.device)
    else:
        arr = cams if isinstance(cams, ct.Array) else make_cameras(cams)
        if len(arr) != len(frame.cams) or frame.layers != layers or frame.channels != C or any(
                (arr[v].width, arr[v].height) != (frame.cams[v].width, frame.cams[v].height)
                for v in range(len(arr))):
            raise ValueError("cameras, layers or channels do not match the given frame")
        frame.cams = arr
    ws = workspace if workspace is not None else ctx.workspace(C, len(frame.cams), frame.pixels)
    if record_visibility:
        shape = (len(frame.cams), scene.n)
        if frame.visible is None or tuple(frame.visible.shape) != shape or frame.visible.device != scene.x.device:
            frame.visible = torch.empty(shape, dtype=torch.uint8, device=scene.x.device)
    else:
        frame.visible = None
    p, keep = _params(layers, alpha, flags, background, C, gamma, cams_device, len(frame.cams), env_map)
    sd = scene.desc()
    fd = frame.desc()
    st = lib().adop_render_forward(ctx.handle, ct.byref(sd), frame.cams, len(frame.cams), ct.byref(p),
                                   ct.byref(fd), _ptr(ws), ws.numel(), _stream(stream))
    ctx.check(st, "adop_render_forward")
    return frame


NOALLOC_SCRATCH_BYTES = 64 << 20   # ADOP_NOALLOC_SCRATCH_BYTES


def render_forward_noalloc(ctx: Context, scene: Scene, frame: Frame, alpha: float = 0.01, flags: int = 0,
                           background=None, stream=None, gamma: float = GAMMA) -> Frame:
    """The forward pass into an existing frame (with frame.visible, if set)
    through adop_render_forward_noalloc: no workspace, nothing allocated by
    this call; the library's fixed per-GPU array holds the sums."""
    C = scene.channels
    if frame.channels != C:
        raise ValueError("frame channels do not match the scene")
    if frame.visible is not None and tuple(frame.visible.shape) != (len(frame.cams), scene.n):
        raise ValueError("frame.visible does not match the scene and views")
    p, keep = _params(frame.layers, alpha, flags, background, C, gamma)
    sd = scene.desc()
    fd = frame.desc()
    st = lib().adop_render_forward_noalloc(ctx.handle, ct.byref(sd), frame.cams, len(frame.cams), ct.byref(p),
                                           ct.byref(fd), _stream(stream))
    ctx.check(st, "adop_render_forward_noalloc")
    return frame


def render_backward(ctx: Context, scene: Scene, frame: Frame, grad: torch.Tensor, alpha: float = 0.01,
                    flags: int = 0, background=None, stream=None, out=None,
                    workspace: Optional[torch.Tensor] = None, gamma: float = GAMMA,
                    cams_device: Optional[torch.Tensor] = None, env_map: Optional[torch.Tensor] = None,
                    env_grad: Optional[torch.Tensor] = None):
    """Returns (dfeat [n,C] f32, dpos [3,n] f32, dpose [V,6] f64, dintr [V,9] f64).
    cams_device: the camera table the forward of this frame used, if any.
    env_map: the forward's environment map; env_grad: [C, S, S] FP32 output
    for its gradient (or None)."""
    C = scene.channels
    V = len(frame.cams)
    dev = scene.x.device
    assert grad.is_cuda and grad.dtype == torch.float32 and grad.numel() == C * frame.pixels
    grad = grad.contiguous()
    if out is None:
        out = (torch.empty((scene.n, C), dtype=torch.float32, device=dev),
               torch.empty((3, scene.n), dtype=torch.float32, device=dev),
               torch.empty((V, 6), dtype=torch.float64, device=dev),
               torch.empty((V, 9), dtype=torch.float64, device=dev))
    dfeat, dpos, dpose, dintr = out
    if frame.visible is not None and tuple(frame.visible.shape) != (V, scene.n):
        raise ValueError("frame.visible was recorded for another scene")
    ws = workspace if workspace is not None else ctx.workspace(C, V, frame.pixels)
    p, keep = _params(frame.layers, alpha, flags, background, C, gamma, cams_device, V, env_map, env_grad)
    sd = scene.desc()
    fd = frame.desc()
    st = lib().adop_render_backward(ctx.handle, ct.byref(sd), frame.cams, V, ct.byref(p), ct.byref(fd),
                                    _ptr(grad), _ptr(dfeat), _ptr(dpos), _ptr(dpose), _ptr(dintr),
                                    _ptr(ws), ws.numel(), _stream(stream))
    ctx.check(st, "adop_render_backward")
    return dfeat, dpos, dpose, dintr


class ForwardGraph:
    """A captured forward render (kernels only) bound to fixed buffers; new
    cameras of the same sizes are staged on every launch."""

    def __init__(self, ctx: Context, scene: Scene, cams, layers: int, alpha: float = 0.01, flags: int = 0,
                 background=None, gamma: float = GAMMA, record_visibility: bool = False):
        """record_visibility: the frame carries a [V, n] byte buffer, so the
        depth pass's candidate layers let the accumulation skip points that
        cannot blend (and the blend-set bits are left in frame.visible)."""
        self.ctx = ctx
        self.scene = scene
        C = scene.channels
        self.frame = Frame(cams, layers, C, scene.x.device)
        V = len(self.frame.cams)
        if record_visibility:
            self.frame.visible = torch.empty((V, scene.n), dtype=torch.uint8, device=scene.x.device)
        need = ctx.workspace_bytes(C, V, self.frame.pixels)
        self.ws = torch.empty(need, dtype=torch.uint8, device=scene.x.device)
        p, keep = _params(layers, alpha, flags, background, C, gamma)
        sd = scene.desc()
        fd = self.frame.desc()
        h = ct.c_void_p()
        st = lib().adop_forward_graph_create(ctx.handle, ct.byref(sd), self.frame.cams, V, ct.byref(p),
                                             ct.byref(fd), _ptr(self.ws), need, ct.byref(h))
        ctx.check(st, "adop_forward_graph_create")
        self.handle = h

    def launch(self, cams, stream=None):
        arr = cams if isinstance(cams, ct.Array) else make_cameras(cams)
        st = lib().adop_forward_graph_launch(self.handle, arr, _stream(stream))
        self.ctx.check(st, "adop_forward_graph_launch")
        return self.frame

    def close(self):
        """Destroy the graph (waits for its last launch) and drop its buffers."""
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.adop_graph_destroy(h)
        self.handle = None
        self.frame = None
        self.ws = None

    def __del__(self):
        self.close()


# ---------------------------------------------------------------------------
# photometric tone mapper
# ---------------------------------------------------------------------------

class TonemapDesc(ct.Structure):
    _fields_ = [("ev", ct.c_void_p), ("white", ct.c_void_p), ("vignette", ct.c_void_p), ("crf", ct.c_void_p),
                ("crf_size", ct.c_int32), ("leak", ct.c_float)]


class Tonemapper:
    """Parameters of the tone mapper as device FP32 tensors: ev [V],
    white [V, 3], vignette [5] = (a2, a4, a6, cx, cy), crf [3, K]."""

    def __init__(self, ev: torch.Tensor, white: torch.Tensor, vignette: torch.Tensor, crf: torch.Tensor,
                 leak: float = 0.01):
        for t in (ev, white, vignette, crf):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        self.ev, self.white, self.vignette, self.crf, self.leak = ev, white, vignette, crf, leak

    def desc(self) -> TonemapDesc:
        return TonemapDesc(_ptr(self.ev), _ptr(self.white), _ptr(self.vignette), _ptr(self.crf),
                           int(self.crf.shape[1]), float(np.float32(self.leak)))


def tonemap_forward(ctx: Context, hdr: torch.Tensor, tm: Tonemapper, stream=None) -> torch.Tensor:
    """hdr [V, 3, h, w] FP32 device -> ldr of the same shape."""
    assert hdr.is_cuda and hdr.dtype == torch.float32 and hdr.dim() == 4 and hdr.shape[1] == 3
    hdr = hdr.contiguous()
    V, _, h, w = hdr.shape
    out = torch.empty_like(hdr)
    d = tm.desc()
    ctx.check(lib().adop_tonemap_forward(ctx.handle, _ptr(hdr), V, w, h, ct.byref(d), _ptr(out), _stream(stream)),
              "adop_tonemap_forward")
    return out


def tonemap_backward(ctx: Context, hdr: torch.Tensor, tm: Tonemapper, grad: torch.Tensor, stream=None):
    """(d_hdr [V,3,h,w] f32, d_ev [V], d_white [V,3], d_vignette [5], d_crf [3,K]) (f64)."""
    hdr = hdr.contiguous()
    grad = grad.contiguous()
    V, _, h, w = hdr.shape
    dev = hdr.device
    K = int(tm.crf.shape[1])
    d_hdr = torch.empty_like(hdr)
    d_ev = torch.empty(V, dtype=torch.float64, device=dev)
    d_white = torch.empty((V, 3), dtype=torch.float64, device=dev)
    d_vig = torch.empty(5, dtype=torch.float64, device=dev)
    d_crf = torch.empty((3, K), dtype=torch.float64, device=dev)
    nb = int(lib().adop_tonemap_workspace_bytes(V))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    d = tm.desc()
    st = lib().adop_tonemap_backward(ctx.handle, _ptr(hdr), V, w, h, ct.byref(d), _ptr(grad), _ptr(d_hdr),
                                     _ptr(d_ev), _ptr(d_white), _ptr(d_vig), _ptr(d_crf), _ptr(ws), nb,
                                     _stream(stream))
    ctx.check(st, "adop_tonemap_backward")
    return d_hdr, d_ev, d_white, d_vig, d_crf


def atomic_probe(ctx: Context, kind: int, ops: int, footprint: int, stride: int, buffer: torch.Tensor,
                 stream=None) -> float:
    """Duration in ms of `ops` device atomics (kind 0: u64 minimum, 1: FP32
    add) on words (i * stride) mod footprint of `buffer` (adop_atomic_probe)."""
    ms = ct.c_double()
    st = lib().adop_atomic_probe(ctx.handle, kind, ops, footprint, stride, _ptr(buffer),
                                 buffer.numel() * buffer.element_size(), ct.byref(ms), _stream(stream))
    ctx.check(st, "adop_atomic_probe")
    return float(ms.value)
