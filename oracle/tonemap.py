"""CPU oracle of the photometric tone mapper (TEST INFRASTRUCTURE ONLY).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  Plain float64 NumPy, written from the paper's Sec. 3.3
("Differentiable Tone Mapping"); the derivatives are written out by hand
(not taken from an automatic differentiator) and pinned by finite
differences of the forward in tests/test_oracle_tonemap.py.

Stages, per image i and pixel (u, v) of a w x h image with 3 channels:
  exposure (Eq. ev's brightness correction):  I_e = I_hdr / 2^EV_i
  white balance (per-image white point W_i):  I_w[c] = I_e[c] * W_i[c]
  vignette (polynomial in r, Sec. 3.3):        I_v = I_w * (1 + a2 r^2 + a4 r^4 + a6 r^6)
      r = |p - c_v| with p = ((u + 0.5) / w, (v + 0.5) / h) and the centre c_v
      in the same normalised coordinates
  response (Eq. resonseleak):                  I_ldr = R_t(I_v)
      R(x) on [0, 1]: a table T[c][K] sampled at x = k / (K - 1), linearly
      interpolated; R_t(x) = leak * x for x < 0, R(x) on [0, 1],
      -leak / sqrt(x) + leak + 1 for x > 1.  With leak < 0 (inference) the
      input is clamped to [0, 1] instead.
Readings (the paper gives no formula for them): the white point multiplies
the image; pixel centres sit at integer coordinates, so the image extent
[-0.5, w - 0.5] maps to [0, 1].
"""
from __future__ import annotations

import numpy as np

LN2 = np.log(2.0)


def _coords(w: int, h: int):
    px = (np.arange(w, dtype=np.float64) + 0.5) / w
    py = (np.arange(h, dtype=np.float64) + 0.5) / h
    return np.meshgrid(px, py)          # [h, w] each


def response(x: np.ndarray, table: np.ndarray, leak: float) -> np.ndarray:
    """R_t for one channel: x any shape, table [K]."""
    K = table.shape[0]
    xc = np.clip(x, 0.0, 1.0)
    pos = xc * (K - 1)
    i = np.minimum(np.floor(pos).astype(np.int64), K - 2)
    f = pos - i
    mid = (1.0 - f) * table[i] + f * table[i + 1]
    if leak < 0:
        return mid
    out = np.where(x < 0, leak * x, mid)
    with np.errstate(divide="ignore", invalid="ignore"):
        hi = -leak / np.sqrt(np.where(x > 1, x, 1.0)) + leak + 1.0
    return np.where(x > 1, hi, out)


def vignette_factor(w: int, h: int, vig: np.ndarray) -> np.ndarray:
    a2, a4, a6, cx, cy = (float(t) for t in vig)
    px, py = _coords(w, h)
    r2 = (px - cx) ** 2 + (py - cy) ** 2
    return 1.0 + a2 * r2 + a4 * r2 ** 2 + a6 * r2 ** 3


def forward(hdr: np.ndarray, ev: np.ndarray, white: np.ndarray, vig: np.ndarray, crf: np.ndarray,
            leak: float = 0.01):
    """hdr [V, 3, h, w], ev [V], white [V, 3], vig [5] = (a2, a4, a6, cx, cy),
    crf [3, K] -> ldr [V, 3, h, w] (float64)."""
    hdr = np.asarray(hdr, np.float64)
    V, C, h, w = hdr.shape
    assert C == 3
    Ie = hdr / (2.0 ** np.asarray(ev, np.float64))[:, None, None, None]
    Iw = Ie * np.asarray(white, np.float64)[:, :, None, None]
    Iv = Iw * vignette_factor(w, h, vig)[None, None]
    out = np.empty_like(Iv)
    for c in range(3):
        out[:, c] = response(Iv[:, c], np.asarray(crf[c], np.float64), leak)
    return out


def backward(hdr, ev, white, vig, crf, grad, leak: float = 0.01):
    """Gradients of L with dL/dI_ldr = grad [V, 3, h, w]:
    (d_hdr [V,3,h,w], d_ev [V], d_white [V,3], d_vig [5], d_crf [3,K]).
    Each entry's sum of |terms| (the yardstick of the GPU tolerances) is
    returned as well: (..., abs) with the same shapes."""
    hdr = np.asarray(hdr, np.float64)
    grad = np.asarray(grad, np.float64)
    V, C, h, w = hdr.shape
    crf = np.asarray(crf, np.float64)
    K = crf.shape[1]
    a2, a4, a6, cx, cy = (float(t) for t in vig)
    px, py = _coords(w, h)
    dx, dy = px - cx, py - cy
    r2 = dx * dx + dy * dy
    Vf = 1.0 + a2 * r2 + a4 * r2 ** 2 + a6 * r2 ** 3
    dVdr2 = a2 + 2.0 * a4 * r2 + 3.0 * a6 * r2 ** 2
    scale = 2.0 ** -np.asarray(ev, np.float64)
    Ie = hdr * scale[:, None, None, None]
    Wt = np.asarray(white, np.float64)
    Iw = Ie * Wt[:, :, None, None]
    Iv = Iw * Vf[None, None]
    # dR_t/dx and the table weights
    gv = np.empty_like(Iv)
    d_crf = np.zeros((3, K))
    d_crf_abs = np.zeros((3, K))
    for c in range(3):
        x = Iv[:, c]
        T = crf[c]
        xc = np.clip(x, 0.0, 1.0)
        pos = xc * (K - 1)
        i = np.minimum(np.floor(pos).astype(np.int64), K - 2)
        f = pos - i
        slope = (T[i + 1] - T[i]) * (K - 1)
        inside = (x >= 0) & (x <= 1) if leak >= 0 else np.ones_like(x, bool)
        if leak >= 0:
            with np.errstate(divide="ignore", invalid="ignore"):
                hi = 0.5 * leak * np.where(x > 1, x, 1.0) ** -1.5
            dR = np.where(x < 0, leak, np.where(x > 1, hi, slope))
        else:
            dR = np.where((x >= 0) & (x <= 1), slope, 0.0)
        g = grad[:, c]
        gv[:, c] = g * dR
        # table: R = (1 - f) T[i] + f T[i + 1] where the table is used
        gi = np.where(inside, g, 0.0)
        np.add.at(d_crf[c], i.ravel(), ((1.0 - f) * gi).ravel())
        np.add.at(d_crf[c], i.ravel() + 1, (f * gi).ravel())
        np.add.at(d_crf_abs[c], i.ravel(), np.abs((1.0 - f) * gi).ravel())
        np.add.at(d_crf_abs[c], i.ravel() + 1, np.abs(f * gi).ravel())
    # I_v = I_w * Vf
    gw = gv * Vf[None, None]
    t_vig = gv * Iw                                          # dL/dVf per element
    d_vig = np.array([np.sum(t_vig * r2), np.sum(t_vig * r2 ** 2), np.sum(t_vig * r2 ** 3),
                      np.sum(t_vig * dVdr2 * (-2.0 * dx)), np.sum(t_vig * dVdr2 * (-2.0 * dy))])
    d_vig_abs = np.array([np.sum(np.abs(t_vig * r2)), np.sum(np.abs(t_vig * r2 ** 2)),
                          np.sum(np.abs(t_vig * r2 ** 3)), np.sum(np.abs(t_vig * dVdr2 * (-2.0 * dx))),
                          np.sum(np.abs(t_vig * dVdr2 * (-2.0 * dy)))])
    # I_w = I_e * W
    t_w = gw * Ie
    d_white = t_w.sum(axis=(2, 3))
    d_white_abs = np.abs(t_w).sum(axis=(2, 3))
    ge = gw * Wt[:, :, None, None]
    # I_e = I_hdr * 2^-EV:  dI_e/dEV = -ln2 I_e
    t_ev = ge * Ie * -LN2
    d_ev = t_ev.sum(axis=(1, 2, 3))
    d_ev_abs = np.abs(t_ev).sum(axis=(1, 2, 3))
    d_hdr = ge * scale[:, None, None, None]
    return (d_hdr, d_ev, d_white, d_vig, d_crf), (np.abs(d_hdr), d_ev_abs, d_white_abs, d_vig_abs, d_crf_abs)


def gamma_table(K: int, g: float = 0.45) -> np.ndarray:
    """The paper's initial response x^0.45 sampled at k / (K - 1), for all three channels."""
    x = np.arange(K, dtype=np.float64) / (K - 1)
    return np.tile(x ** g, (3, 1))
