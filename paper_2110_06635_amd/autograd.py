"""torch.autograd.Function over the C-ABI rasterizer.

Forward: I_l = Phi_l(C, R, t, x, tau) for l = 0..L-1 (ADOP Eq. render) for V
cameras; returns one tensor [V, C, h_l, w_l] per layer (views of equal size).
Backward: the library's hand-written kernel (approximate spatial gradient of
Eqs. induce/gradp/spatialderiv, feature gradient of Eq. blend) -- there is no
autograd through torch ops.

Pose: every camera has a fixed base pose (R0, t0) and a tangent tensor xi =
(rho, omega) in se(3); the rendered pose is exp(xi) * (R0, t0) (Eq. tangent).
The gradient returned for xi is that of a left perturbation at the rendered
pose, which equals dL/dxi at xi = 0 -- the paper applies xi to the base pose
after every optimizer step and resets it to zero (`Rasterizer.apply_tangent`).
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import adop

INTRINSICS = ("fx", "fy", "cx", "cy", "k1", "k2", "k3", "p1", "p2")


def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(xi: np.ndarray):
    """exp of xi = (rho, omega) in se(3) -> (R, t), float64."""
    rho = np.asarray(xi[:3], dtype=np.float64)
    w = np.asarray(xi[3:], dtype=np.float64)
    th = float(np.linalg.norm(w))
    K = _hat(w)
    if th < 1e-8:
        R = np.eye(3) + K + 0.5 * K @ K
        Vm = np.eye(3) + 0.5 * K + K @ K / 6.0
    else:
        a = math.sin(th) / th
        b = (1.0 - math.cos(th)) / th ** 2
        c = (th - math.sin(th)) / th ** 3
        R = np.eye(3) + a * K + b * K @ K
        Vm = np.eye(3) + b * K + c * K @ K
    return R, Vm @ rho


class Rasterizer:
    """Holds a prepared scene's static state (context, original indices,
    storage type), the cameras' sizes and base poses, and render settings."""

    def __init__(self, ctx: adop.Context, scene: adop.Scene, cams: Sequence, layers: int,
                 alpha: float = 0.01, flags: int = 0, background=None):
        self.ctx = ctx
        self.scene = scene
        self.cams = [c.copy() for c in cams]
        self.base_R = [np.asarray(c.R, dtype=np.float64).copy() for c in cams]
        self.base_t = [np.asarray(c.t, dtype=np.float64).copy() for c in cams]
        self.layers = layers
        self.alpha = alpha
        self.flags = flags
        self.background = background

    def intrinsics(self, dtype=torch.float32, device=None) -> torch.Tensor:
        v = [[float(getattr(c, k)) for k in INTRINSICS] for c in self.cams]
        return torch.tensor(v, dtype=dtype, device=device or self.scene.x.device)

    def cameras(self, intr: torch.Tensor, tangent: torch.Tensor):
        intr = intr.detach().double().cpu().numpy()
        xi = tangent.detach().double().cpu().numpy()
        out = []
        for v, c in enumerate(self.cams):
            c2 = c.copy()
            for j, k in enumerate(INTRINSICS):
                setattr(c2, k, float(intr[v, j]))
            dR, dt = se3_exp(xi[v])
            c2.R = dR @ self.base_R[v]
            c2.t = dR @ self.base_t[v] + dt
            out.append(c2)
        return out

    def apply_tangent(self, tangent: torch.Tensor):
        """(R0, t0) <- exp(xi) * (R0, t0) and xi <- 0 (in place)."""
        xi = tangent.detach().double().cpu().numpy()
        for v in range(len(self.cams)):
            dR, dt = se3_exp(xi[v])
            self.base_R[v] = dR @ self.base_R[v]
            self.base_t[v] = dR @ self.base_t[v] + dt
            self.cams[v].R = self.base_R[v]
            self.cams[v].t = self.base_t[v]
        with torch.no_grad():
            tangent.zero_()

    def __call__(self, x, y, z, feat, intr, tangent):
        return AdopRasterize.apply(x, y, z, feat, intr, tangent, self)


class AdopRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, feat, intr, tangent, rast: Rasterizer):
        scene = adop.Scene(x.detach(), y.detach(), z.detach(), feat.detach(), rast.scene.orig, rast.scene.dtype)
        cams = rast.cameras(intr, tangent)
        frame = adop.render_forward(rast.ctx, scene, cams, rast.layers, alpha=rast.alpha, flags=rast.flags,
                                    background=rast.background)
        ctx.rast = rast
        ctx.scene = scene
        ctx.frame = frame
        ctx.dtypes = (feat.dtype, intr.dtype, tangent.dtype)
        return tuple(frame.layer_images(l) for l in range(rast.layers))

    @staticmethod
    def backward(ctx, *grads):
        rast, scene, frame = ctx.rast, ctx.scene, ctx.frame
        C = scene.channels
        g = torch.zeros(C * frame.pixels, dtype=torch.float32, device=scene.x.device)
        V = len(frame.cams)
        for l, gl in enumerate(grads):
            if gl is None:
                continue
            w, h = frame.cams[0].width >> l, frame.cams[0].height >> l
            o0 = int(frame.offsets[0, l])
            stride_v = C * (int(frame.offsets[1, l]) - o0) if V > 1 else C * w * h
            dst = g.as_strided((V, C, h, w), (stride_v, h * w, w, 1), C * o0)
            dst.copy_(gl.to(torch.float32))
        dfeat, dpos, dpose, dintr = adop.render_backward(rast.ctx, scene, frame, g, alpha=rast.alpha,
                                                         flags=rast.flags, background=rast.background)
        fdt, idt, tdt = ctx.dtypes
        return (dpos[0], dpos[1], dpos[2], dfeat.to(fdt), dintr.to(idt), dpose.to(tdt), None)
