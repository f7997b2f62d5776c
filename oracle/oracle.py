"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It loads oracle/liboracle.so (built by oracle/build.py) and
exposes NumPy-facing functions.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

SPATIAL_ALL = 1
CULL_BACKFACE = 2
CULL_PRINTED = 4
LOG_FEATURES = 8
DISCARD = 16


class OracleOptions(ct.Structure):
    _fields_ = [("flags", ct.c_uint32), ("normals", ct.c_void_p), ("radius", ct.c_void_p),
                ("beta", ct.c_void_p), ("gamma", ct.c_float), ("bg_image", ct.c_void_p)]


class OracleCamera(ct.Structure):
    _fields_ = [("width", ct.c_int32), ("height", ct.c_int32),
                ("fx", ct.c_float), ("fy", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float),
                ("k1", ct.c_float), ("k2", ct.c_float), ("k3", ct.c_float),
                ("p1", ct.c_float), ("p2", ct.c_float),
                ("znear", ct.c_float), ("r2_max", ct.c_float),
                ("R", ct.c_float * 9), ("t", ct.c_float * 3)]


def load(path: str):
    """Load an oracle shared library and declare its entry points."""
    L = ct.CDLL(path)
    P = ct.c_void_p
    L.oracle_project.restype = ct.c_int
    L.oracle_project.argtypes = [P, ct.c_float, ct.c_float, ct.c_float, P, P, P]
    L.oracle_project_points.restype = None
    L.oracle_project_points.argtypes = [P, ct.c_int64, P, P, P, P, P]
    L.oracle_layer_pixel.restype = ct.c_int
    L.oracle_layer_pixel.argtypes = [P, ct.c_float, ct.c_float, ct.c_int, P, P]
    L.oracle_total_pixels.restype = ct.c_int64
    L.oracle_total_pixels.argtypes = [P, ct.c_int32, ct.c_int32]
    L.oracle_forward.restype = ct.c_int
    L.oracle_forward.argtypes = [ct.c_int64, ct.c_int32, P, P, ct.c_int32, P, ct.c_int32,
                                 ct.c_float, P, P, P, P, P]
    L.oracle_backward.restype = ct.c_int
    L.oracle_backward.argtypes = [ct.c_int64, ct.c_int32, P, P, ct.c_int32, P, ct.c_int32,
                                  ct.c_float, ct.c_uint32, P, P, P, P, P, P, P, P, P, P, P, P]
    L.oracle_forward_ex.restype = ct.c_int
    L.oracle_forward_ex.argtypes = [ct.c_int64, ct.c_int32, P, P, ct.c_int32, P, ct.c_int32,
                                    ct.c_float, P, P, P, P, P, P]
    L.oracle_backward_ex.restype = ct.c_int
    L.oracle_backward_ex.argtypes = [ct.c_int64, ct.c_int32, P, P, ct.c_int32, P, ct.c_int32,
                                     ct.c_float, P, P, P, P, P, P, P, P, P, P, P, P, P]
    L.oracle_knn_radius.restype = ct.c_int
    L.oracle_knn_radius.argtypes = [ct.c_int64, P, P]
    return L


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # type: ignore
            _b.build()
        _LIB = load(path)
    return _LIB


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def cameras(cams: Sequence) -> ct.Array:
    """Pack synth.Camera objects into the oracle's camera records (float32)."""
    arr = (OracleCamera * len(cams))()
    for k, c in enumerate(cams):
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


def project_points(cam, pos: np.ndarray):
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    n = pos.shape[0]
    Z = np.empty(n, np.float32)
    u0 = np.empty(n, np.float32)
    v0 = np.empty(n, np.float32)
    valid = np.empty(n, np.int32)
    cc = cameras([cam])
    lib().oracle_project_points(ct.byref(cc[0]), n, _p(pos), _p(Z), _p(u0), _p(v0), _p(valid))
    return Z, u0, v0, valid.astype(bool)


def layer_pixel(cam, u0: float, v0: float, l: int):
    cc = cameras([cam])
    px = ct.c_int32()
    py = ct.c_int32()
    ok = lib().oracle_layer_pixel(ct.byref(cc[0]), ct.c_float(u0), ct.c_float(v0), l,
                                  ct.byref(px), ct.byref(py))
    return bool(ok), px.value, py.value


def total_pixels(cams, layers: int) -> int:
    cc = cameras(cams)
    return int(lib().oracle_total_pixels(cc, len(cams), layers))


def _options(flags, normals, radius, beta, gamma, bg_image=None):
    """Options record plus the arrays it points to (kept alive by the caller)."""
    keep = []
    o = OracleOptions()
    o.flags = int(flags)
    for name, arr, shape in (("normals", normals, 3), ("radius", radius, 1), ("beta", beta, 1)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=np.float32)
            keep.append(a)
            setattr(o, name, a.ctypes.data)
    o.gamma = float(gamma)
    if bg_image is not None:
        b = np.ascontiguousarray(bg_image, dtype=np.float64)
        keep.append(b)
        o.bg_image = b.ctypes.data
    return o, keep


def knn_radius(pos):
    """Distance of each point to its 4th-nearest other point (brute force)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    out = np.empty(pos.shape[0], np.float32)
    if lib().oracle_knn_radius(pos.shape[0], _p(pos), _p(out)) != 0:
        raise ValueError("oracle_knn_radius needs at least 5 points")
    return out


def forward(pos, feat, cams, layers: int, alpha: float = 0.01, background=None,
            want64: bool = False, flags: int = 0, normals=None, radius=None, beta=None,
            gamma: float = 0.0, bg_image=None):
    """Returns dict(keys uint64, counts int32, images float32[, images64]).
    flags: CULL_BACKFACE / CULL_PRINTED (normals [n,3]), LOG_FEATURES,
    DISCARD (radius [n], beta [n], gamma).  bg_image: float64 values of
    empty pixels in the image layout (the environment map's samples,
    oracle.envmap.background_image); None: the constant background."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    feat = np.ascontiguousarray(feat, dtype=np.float32)
    n, c = feat.shape
    assert pos.shape == (n, 3)
    cc = cameras(cams)
    total = int(lib().oracle_total_pixels(cc, len(cams), layers))
    bg = np.zeros(c, np.float32) if background is None else np.ascontiguousarray(background, np.float32)
    keys = np.empty(total, np.uint64)
    counts = np.empty(total, np.int32)
    images = np.empty(total * c, np.float32)
    images64 = np.empty(total * c, np.float64) if want64 else None
    if bg_image is not None:
        assert np.asarray(bg_image).size == total * c
    opt, keep = _options(flags, normals, radius, beta, gamma, bg_image)
    rc = lib().oracle_forward_ex(n, c, _p(pos), _p(feat), len(cams), cc, layers,
                                 ct.c_float(alpha), ct.byref(opt), _p(bg), _p(keys), _p(counts),
                                 _p(images), _p(images64))
    if rc != 0:
        raise ValueError(f"oracle_forward failed ({rc})")
    out = dict(keys=keys, counts=counts, images=images)
    if want64:
        out["images64"] = images64
    return out


def backward(pos, feat, cams, layers: int, grad, alpha: float = 0.01, background=None,
             flags: int = 0, want_abs: bool = True, want_g: bool = False, normals=None,
             radius=None, beta=None, gamma: float = 0.0, bg_image=None):
    """Returns dict(dfeat [n,c], dpos [3,n], dpose [V,6], dintr [V,9]) in float64,
    plus *_abs magnitude bounds and per-point gu/gv [V,n] on request."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    feat = np.ascontiguousarray(feat, dtype=np.float32)
    grad = np.ascontiguousarray(grad, dtype=np.float32)
    n, c = feat.shape
    V = len(cams)
    cc = cameras(cams)
    total = int(lib().oracle_total_pixels(cc, V, layers))
    assert grad.size == total * c
    bg = np.zeros(c, np.float32) if background is None else np.ascontiguousarray(background, np.float32)
    out = dict(dfeat=np.empty((n, c)), dpos=np.empty((3, n)), dpose=np.empty((V, 6)),
               dintr=np.empty((V, 9)))
    if want_abs:
        out.update(dfeat_abs=np.empty((n, c)), dpos_abs=np.empty((3, n)),
                   dpose_abs=np.empty((V, 6)), dintr_abs=np.empty((V, 9)))
    if want_g:
        out.update(gu=np.empty((V, n)), gv=np.empty((V, n)))
    g = out.get
    if bg_image is not None:
        assert np.asarray(bg_image).size == total * c
    opt, keep = _options(flags, normals, radius, beta, gamma, bg_image)
    rc = lib().oracle_backward_ex(n, c, _p(pos), _p(feat), V, cc, layers, ct.c_float(alpha),
                               ct.byref(opt), _p(bg), _p(grad), _p(out["dfeat"]), _p(out["dpos"]),
                               _p(out["dpose"]), _p(out["dintr"]), _p(g("dfeat_abs")),
                               _p(g("dpos_abs")), _p(g("dpose_abs")), _p(g("dintr_abs")),
                               _p(g("gu")), _p(g("gv")))
    if rc != 0:
        raise ValueError(f"oracle_backward failed ({rc})")
    return out


def layer_slices(cams, layers: int, c: int):
    """Per (view, layer): (key offset, w_l, h_l, image offset) in the shared layout."""
    res = []
    base = 0
    for cam in cams:
        off = base
        row = []
        for l in range(layers):
            wl, hl = cam.width >> l, cam.height >> l
            row.append((off, wl, hl, c * off))
            off += wl * hl
        res.append(row)
        base = off
    return res
