"""Seeded synthetic inputs for the one-pixel point rasterizer.

This module is shared by the HIP path's tests/benchmarks and by the CPU
oracle's tests.  It holds no arithmetic of the rendering method itself: it
only draws point clouds, features, cameras and upstream gradients from
seeded NumPy generators (PCG64 via ``numpy.random.default_rng``).  Values are
drawn in float64 and cast to float32; BF16/FP16 copies are made from the same
float32 values with round-to-nearest-even.

The scene shapes stand in for the paper's MVS/LiDAR reconstructions
(9.7M-72.9M surface points, 1920x1080 and larger, 4-element descriptors,
4-layer pyramids; ADOP Table "scenes" and the runtime table in Appendix B),
which are not available here.

Camera convention (shared interface format): world->camera x_c = R x + t,
OpenCV axes (x right, y down, z forward), R row-major 3x3.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Generation happens in fixed-size chunks so that 100M-point scenes stay within
# a bounded amount of host memory; the chunk size is part of the recipe.
CHUNK = 1 << 22


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    k1: float = 0.0
    k2: float = 0.0
    k3: float = 0.0
    p1: float = 0.0
    p2: float = 0.0
    znear: float = 0.01
    r2_max: float = math.inf
    R: np.ndarray = dataclasses.field(default_factory=lambda: np.eye(3))
    t: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))

    def copy(self) -> "Camera":
        return dataclasses.replace(self, R=np.array(self.R, dtype=np.float64),
                                   t=np.array(self.t, dtype=np.float64))


@dataclasses.dataclass
class Scene:
    pos: np.ndarray                # [N,3] float32, user order (= original index)
    feat: np.ndarray               # [N,C] float32
    cams: List[Camera]
    layers: int
    alpha: float = 0.01
    background: Optional[np.ndarray] = None   # [C] float32
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def c(self) -> int:
        return int(self.feat.shape[1])

    def bg(self) -> np.ndarray:
        if self.background is None:
            return np.zeros(self.c, dtype=np.float32)
        return np.asarray(self.background, dtype=np.float32)


# ---------------------------------------------------------------------------
# storage-precision helpers (round-to-nearest-even, exact widening)
# ---------------------------------------------------------------------------

def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round to nearest even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    rounding = ((u >> 16) & 1) + np.uint32(0x7FFF)
    r = ((u + rounding) >> 16).astype(np.uint16)
    r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def to_f16_bits(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float16).view(np.uint16)


def f16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return np.asarray(b, dtype=np.uint16).view(np.float16).astype(np.float32)


def storage(feat: np.ndarray, dtype: str):
    """Return (raw storage array, its exact float32 widening) for dtype in
    {'f32','bf16','f16'}."""
    if dtype == "f32":
        f = np.ascontiguousarray(feat, dtype=np.float32)
        return f, f
    if dtype == "bf16":
        b = to_bf16_bits(feat)
        return b, bf16_bits_to_f32(b)
    if dtype == "f16":
        b = to_f16_bits(feat)
        return b, f16_bits_to_f32(b)
    raise ValueError(dtype)


# ---------------------------------------------------------------------------
# camera helpers
# ---------------------------------------------------------------------------

def r2_max_for(k1: float, k2: float, k3: float, p1: float = 0.0, p2: float = 0.0) -> float:
    """Per-camera fold-over limit on r^2 = a^2 + b^2 (a reading of the paper,
    which does not say how far off-axis a distorted pinhole stays valid).

    Radial map r -> r*D(r^2) stops being monotonic where
    1 + 3 k1 r^2 + 5 k2 r^4 + 7 k3 r^6 <= 0.  Scan r^2 in (0, 4] with step 1e-4
    in float64 and return the first such r^2; 4.0 if none; +inf without any
    distortion.  The value is rounded to float32 by whoever stores it."""
    if k1 == 0.0 and k2 == 0.0 and k3 == 0.0 and p1 == 0.0 and p2 == 0.0:
        return math.inf
    r2 = np.arange(1, 40001, dtype=np.float64) * 1e-4
    d = 1.0 + 3.0 * k1 * r2 + 5.0 * k2 * r2 ** 2 + 7.0 * k3 * r2 ** 3
    bad = np.nonzero(d <= 0.0)[0]
    if bad.size:
        return float(r2[bad[0]])
    return 4.0


def rodrigues(w: np.ndarray) -> np.ndarray:
    """Rotation matrix exp([w]_x) for an axis-angle vector (float64)."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.linalg.norm(w))
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]], dtype=np.float64)
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * (K @ K)


def look_at(centre: np.ndarray, target: np.ndarray, up=(0.0, 1.0, 0.0)):
    """World->camera (R, t) for a camera at `centre` looking at `target`,
    OpenCV axes: z forward, y down (opposite to `up`), x = y cross z."""
    c = np.asarray(centre, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    u = np.asarray(up, dtype=np.float64)
    y = -(u - np.dot(u, f) * f)
    y /= np.linalg.norm(y)
    x = np.cross(y, f)
    R = np.stack([x, y, f])
    t = -R @ c
    return R, t


# ---------------------------------------------------------------------------
# point-cloud generators
# ---------------------------------------------------------------------------

def _streams(seed: int, k: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def uniform_box(n: int, half: float, c: int, seed: int):
    rp, rf = _streams(seed, 2)
    pos = np.empty((n, 3), dtype=np.float32)
    feat = np.empty((n, c), dtype=np.float32)
    for s in range(0, n, CHUNK):
        m = min(CHUNK, n - s)
        pos[s:s + m] = rp.uniform(-half, half, size=(m, 3))
        feat[s:s + m] = rf.random((m, c))
    return pos, feat


def planes(n_planes: int, per_plane: int, c: int, seed: int, box: float = 5.0,
           half_lo: float = 0.5, half_hi: float = 2.0, sigma: float = 0.01, with_normals: bool = False):
    """Points on seeded random squares: centre U[-box,box]^3, random unit
    normal, half-extent U[half_lo,half_hi], in-plane U, normal offset N(0,sigma^2).
    with_normals: also return each point's plane normal [n,3] float32."""
    rg, rp, rf = _streams(seed, 3)
    centres = rg.uniform(-box, box, size=(n_planes, 3))
    normals = rg.normal(size=(n_planes, 3))
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    halves = rg.uniform(half_lo, half_hi, size=n_planes)
    n = n_planes * per_plane
    pos = np.empty((n, 3), dtype=np.float32)
    feat = np.empty((n, c), dtype=np.float32)
    for k in range(n_planes):
        nrm = normals[k]
        a = np.cross(nrm, [1.0, 0.0, 0.0] if abs(nrm[0]) < 0.9 else [0.0, 1.0, 0.0])
        a /= np.linalg.norm(a)
        b = np.cross(nrm, a)
        st = rp.uniform(-halves[k], halves[k], size=(per_plane, 2))
        off = rp.normal(0.0, sigma, size=per_plane)
        p = centres[k] + st[:, :1] * a + st[:, 1:] * b + off[:, None] * nrm
        pos[k * per_plane:(k + 1) * per_plane] = p
    for s in range(0, n, CHUNK):
        m = min(CHUNK, n - s)
        feat[s:s + m] = rf.random((m, c))
    if with_normals:
        return pos, feat, np.repeat(normals, per_plane, axis=0).astype(np.float32)
    return pos, feat


def unit_vectors(n: int, seed: int) -> np.ndarray:
    """Seeded random unit vectors [n,3] float32 (per-point normals)."""
    (r,) = _streams(seed, 1)
    v = np.empty((n, 3), np.float32)
    for s in range(0, n, CHUNK):
        m = min(CHUNK, n - s)
        w = r.normal(size=(m, 3))
        v[s:s + m] = w / np.linalg.norm(w, axis=1, keepdims=True)
    return v


def uniform01(n: int, seed: int) -> np.ndarray:
    """Seeded U[0,1) float32 [n] (the per-point beta of stochastic discarding)."""
    (r,) = _streams(seed, 1)
    out = np.empty(n, np.float32)
    for s in range(0, n, CHUNK):
        m = min(CHUNK, n - s)
        out[s:s + m] = r.random(m, dtype=np.float32)
    return out


def gaussian_mixture(n: int, k: int, box: float, sigma: float, c: int, seed: int):
    """k centres U[-box,box]^3, uniform cluster id per point, offset N(0,sigma^2)."""
    rg, rp, rf = _streams(seed, 3)
    centres = rg.uniform(-box, box, size=(k, 3))
    pos = np.empty((n, 3), dtype=np.float32)
    feat = np.empty((n, c), dtype=np.float32)
    for s in range(0, n, CHUNK):
        m = min(CHUNK, n - s)
        ids = rp.integers(0, k, size=m)
        pos[s:s + m] = centres[ids] + rp.normal(0.0, sigma, size=(m, 3))
        feat[s:s + m] = rf.random((m, c))
    return pos, feat


# ---------------------------------------------------------------------------
# the five workloads (sizes may be scaled down for tests via `n`)
# ---------------------------------------------------------------------------

def config1(n: int = 100_000, seed: int = 1001) -> Scene:
    """Forward only: uniform 10x10x10 box, C=4 FP32 U[0,1], 640x480 pinhole
    fx=fy=500 at identity rotation looking down +z from z=-15, L=4, alpha=0.01."""
    pos, feat = uniform_box(n, 5.0, 4, seed)
    cam = Camera(640, 480, 500.0, 500.0, 320.0, 240.0, t=np.array([0.0, 0.0, 15.0]))
    return Scene(pos, feat, [cam], layers=4, name="uniform-box-100k-640x480-L4")


DIST2 = dict(k1=-0.1, k2=0.02, k3=0.0, p1=1e-4, p2=1e-4)


def config2(n_planes: int = 200, per_plane: int = 50_000, seed: int = 1002) -> Scene:
    """Forward+backward FP32: points on 200 random planes, sigma 0.01, C=4,
    1920x1080 fx=fy=1500 with k1=-0.1 k2=0.02 p1=p2=1e-4, L=5."""
    pos, feat = planes(n_planes, per_plane, 4, seed)
    cam = Camera(1920, 1080, 1500.0, 1500.0, 960.0, 540.0, **DIST2,
                 r2_max=r2_max_for(**DIST2), t=np.array([0.0, 0.0, 15.0]))
    return Scene(pos, feat, [cam], layers=5,
                 name=f"planes-{n_planes * per_plane}-1920x1080-L5")


def config3(n: int = 100_000_000, seed: int = 1003) -> Scene:
    """Precision scale-up: 64-cluster Gaussian mixture (sigma 0.5) in a 100 m
    box, C=4, 1920x1080 fx=fy=1600 with the config-2 distortion, camera at
    z=-150 (depths 100-200), L=5."""
    pos, feat = gaussian_mixture(n, 64, 50.0, 0.5, 4, seed)
    cam = Camera(1920, 1080, 1600.0, 1600.0, 960.0, 540.0, **DIST2,
                 r2_max=r2_max_for(**DIST2), t=np.array([0.0, 0.0, 150.0]))
    return Scene(pos, feat, [cam], layers=5, name=f"gmm64-{n}-1920x1080-L5")


def orbit_cameras(v: int, radius: float, seed: int, width=1920, height=1080,
                  f=1500.0, kmax=0.1) -> List[Camera]:
    rng = np.random.default_rng(seed)
    cams = []
    for k in range(v):
        th = 2.0 * math.pi * k / v
        centre = radius * np.array([math.cos(th), 0.0, math.sin(th)]) + rng.normal(0.0, 0.25, 3)
        R, _ = look_at(centre, np.zeros(3))
        R = rodrigues(rng.normal(0.0, math.radians(1.0), 3)) @ R
        t = -R @ centre
        k1, k2, k3 = rng.uniform(-kmax, kmax, 3)
        cams.append(Camera(width, height, f, f, width / 2.0, height / 2.0,
                           k1=float(k1), k2=float(k2), k3=float(k3),
                           r2_max=r2_max_for(k1, k2, k3), R=R, t=t))
    return cams


def config4(n: int = 30_000_000, views: int = 16, seed: int = 1004) -> Scene:
    """Batched training step: 30M points (64-cluster mixture in a 16 m box),
    C=8, 16 orbit cameras (radius 20) with jitter and per-camera k1..k3,
    1920x1080, L=5."""
    pos, feat = gaussian_mixture(n, 64, 8.0, 0.5, 8, seed)
    cams = orbit_cameras(views, 20.0, seed + 100)
    return Scene(pos, feat, cams, layers=5, name=f"gmm64-{n}-16views-1920x1080-L5")


SERVE_CLASSES = [(640, 480), (1280, 720), (1920, 1080), (3840, 2160)]
SERVE_WEIGHTS = [4, 3, 2, 1]


def config5_scene(n: int = 50_000_000, seed: int = 1005) -> Scene:
    pos, feat = gaussian_mixture(n, 64, 50.0, 0.5, 4, seed)
    return Scene(pos, feat, [], layers=4, name=f"gmm64-{n}-serving-L4")


def serve_camera(rng: np.random.Generator, width: int, height: int,
                 radius: float = 150.0) -> Camera:
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    centre = radius * d
    up = (0.0, 1.0, 0.0) if abs(d[1]) < 0.95 else (1.0, 0.0, 0.0)
    R, _ = look_at(centre, np.zeros(3), up)
    roll = math.radians(rng.uniform(-10.0, 10.0))
    R = rodrigues(np.array([0.0, 0.0, roll])) @ R
    t = -R @ centre
    f = 0.8 * width
    return Camera(width, height, f, f, width / 2.0, height / 2.0, R=R, t=t)


def config5_requests(count: int, rate: float = 200.0, seed: int = 2005):
    """Poisson arrivals (rate req/s) of novel views; resolution drawn 4:3:2:1
    over SERVE_CLASSES.  Returns a list of (arrival_time_s, Camera)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    times = np.cumsum(gaps) - gaps[0]
    w = np.array(SERVE_WEIGHTS, dtype=np.float64)
    cls = rng.choice(len(SERVE_CLASSES), size=count, p=w / w.sum())
    out = []
    for k in range(count):
        wd, ht = SERVE_CLASSES[cls[k]]
        out.append((float(times[k]), serve_camera(rng, wd, ht)))
    return out


def upstream_grad(total: int, seed: int) -> np.ndarray:
    """Seeded upstream gradient dL/dI (float32 U[-1,1]) for parity runs, fed
    identically to both sides."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=total).astype(np.float32)


def target_values(total: int, seed: int = 1102) -> np.ndarray:
    """Seeded L1 target T ~ U[0,1] (float32)."""
    rng = np.random.default_rng(seed)
    return rng.random(total, dtype=np.float32)
