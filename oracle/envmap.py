"""CPU oracle of the environment-map background (TEST INFRASTRUCTURE ONLY).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  Plain float64 NumPy written from Sec. 3.1: a pixel that no
point hits takes the environment map's value in the direction of its ray,
E(R^T C^-1(u, v)) (Eq. blend), where E is a spherical map of S x S texels
holding C feature channels (1024^2 in the paper, "Environment Map").  The
gradient of the map is the derivative of Eq. blend with respect to E.

Readings (the paper gives no formula for them):
  * pixel centres: pixel (x, y) of layer l sits at layer-0 coordinates
    (x 2^l, y 2^l) (the inverse of Eq. 2's scaling by 2^-l);
  * C^-1: x_d = (u0 - cx) / fx, y_d = (v0 - cy) / fy, then the Brown-Conrady
    map of the projection is inverted by UNDISTORT_ITERS fixed-point steps
    a <- (x_d - dx(a, b)) / D(r^2), b <- (y_d - dy(a, b)) / D(r^2) from
    (x_d, y_d); the camera ray is (a, b, 1), the world ray R^T (a, b, 1)
    (normalised; the map is at infinity, so t does not enter);
  * the map is equirectangular: longitude phi = atan2(d_x, d_z) in
    (-pi, pi], colatitude theta = arccos(d_y) in [0, pi]; texel (i, j)
    covers s in [i, i+1) x t in [j, j+1) of s = (phi / 2pi + 0.5) S,
    t = (theta / pi) S, with its centre at (i + 0.5, j + 0.5);
  * sampling is bilinear between texel centres, wrapping in longitude and
    clamping in colatitude;
  * only the map texels receive a gradient through the background (no pose or
    intrinsics gradient through the lookup).
"""
from __future__ import annotations

import numpy as np

UNDISTORT_ITERS = 20


def distort(a, b, k1, k2, k3, p1, p2):
    """The projection's Brown-Conrady map (float64 textbook form)."""
    r2 = a * a + b * b
    D = 1.0 + k1 * r2 + k2 * r2 ** 2 + k3 * r2 ** 3
    return (a * D + 2.0 * p1 * a * b + p2 * (r2 + 2.0 * a * a),
            b * D + 2.0 * p2 * a * b + p1 * (r2 + 2.0 * b * b))


def undistort(xd, yd, k1, k2, k3, p1, p2, iters: int = UNDISTORT_ITERS):
    a = np.array(xd, dtype=np.float64, copy=True)
    b = np.array(yd, dtype=np.float64, copy=True)
    for _ in range(iters):
        r2 = a * a + b * b
        D = 1.0 + k1 * r2 + k2 * r2 ** 2 + k3 * r2 ** 3
        dx = 2.0 * p1 * a * b + p2 * (r2 + 2.0 * a * a)
        dy = 2.0 * p2 * a * b + p1 * (r2 + 2.0 * b * b)
        a, b = (xd - dx) / D, (yd - dy) / D
    return a, b


def ray(cam, u0, v0):
    """Unit world directions [..., 3] of layer-0 pixel coordinates (u0, v0)."""
    f = lambda k: float(np.float32(getattr(cam, k)))
    xd = (np.asarray(u0, np.float64) - f("cx")) / f("fx")
    yd = (np.asarray(v0, np.float64) - f("cy")) / f("fy")
    a, b = undistort(xd, yd, f("k1"), f("k2"), f("k3"), f("p1"), f("p2"))
    R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
    dc = np.stack([a, b, np.ones_like(a)], axis=-1)
    d = dc @ R          # R^T (a, b, 1) for every ray
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def layer_rays(cam, l: int):
    """Directions [h_l, w_l, 3] of layer l's pixel centres."""
    wl, hl = cam.width >> l, cam.height >> l
    u0 = np.arange(wl, dtype=np.float64) * 2.0 ** l
    v0 = np.arange(hl, dtype=np.float64) * 2.0 ** l
    U, Vv = np.meshgrid(u0, v0)
    return ray(cam, U, Vv)


def texcoords(d, S: int):
    """Continuous texel coordinates (s, t) of directions d [..., 3]."""
    phi = np.arctan2(d[..., 0], d[..., 2])
    theta = np.arccos(np.clip(d[..., 1], -1.0, 1.0))
    return (phi / (2.0 * np.pi) + 0.5) * S, theta / np.pi * S


def bilinear(S: int, s, t):
    """Four (row, column, weight) triples per sample, between texel centres."""
    x = s - 0.5
    y = t - 0.5
    i0 = np.floor(x).astype(np.int64)
    j0 = np.floor(y).astype(np.int64)
    fx, fy = x - i0, y - j0
    c0, c1 = np.mod(i0, S), np.mod(i0 + 1, S)
    r0, r1 = np.clip(j0, 0, S - 1), np.clip(j0 + 1, 0, S - 1)
    return [(r0, c0, (1 - fx) * (1 - fy)), (r0, c1, fx * (1 - fy)),
            (r1, c0, (1 - fx) * fy), (r1, c1, fx * fy)]


def sample(E, d):
    """E [C, S, S] at directions d [..., 3] -> [C, ...] (float64)."""
    E = np.asarray(E, np.float64)
    S = E.shape[1]
    s, t = texcoords(d, S)
    out = 0.0
    for r, c, w in bilinear(S, s, t):
        out = out + E[:, r, c] * w
    return out


def background_image(cams, layers: int, E):
    """The map's value at every pixel of the frame, float64, in the image
    layout of the library (views, then layers, each [C][h_l][w_l])."""
    E = np.asarray(E, np.float64)
    parts = []
    for cam in cams:
        for l in range(layers):
            parts.append(sample(E, layer_rays(cam, l)).reshape(-1))
    return np.concatenate(parts)


def map_gradient(cams, layers: int, E_shape, counts, grad):
    """dL/dE [C, S, S] from dL/dI = grad (image layout) through the pixels
    whose blend set is empty (counts == 0), with its sum of |terms|."""
    C, S, _ = E_shape
    dE = np.zeros((C, S, S))
    aE = np.zeros((C, S, S))
    grad = np.asarray(grad, np.float64)
    off = 0
    for cam in cams:
        for l in range(layers):
            wl, hl = cam.width >> l, cam.height >> l
            n = wl * hl
            empty = (np.asarray(counts[off:off + n]) == 0).reshape(hl, wl)
            g = grad[C * off: C * (off + n)].reshape(C, hl, wl)
            if empty.any():
                s, t = texcoords(layer_rays(cam, l), S)
                for r, c, w in bilinear(S, s, t):
                    for ch in range(C):
                        term = (g[ch] * w)[empty]
                        np.add.at(dE[ch], (r[empty], c[empty]), term)
                        np.add.at(aE[ch], (r[empty], c[empty]), np.abs(term))
            off += n
    return dE, aE
