"""torch.autograd.Function over the C-ABI rasterizer.

Forward: I_l = Phi_l(C, R, t, x, tau) for l = 0..L-1 (ADOP Eq. render) for V
cameras; returns one tensor [V, C, h_l, w_l] per layer (views of equal size).
Backward: the library's hand-written kernel (approximate spatial gradient of
Eqs. induce/gradp/spatialderiv, feature gradient of Eq. blend) -- there is no
autograd through torch ops.

Pose: every camera has a fixed base pose (R0, t0) and a tangent tensor xi =
(rho, omega) in se(3); the rendered pose is exp(xi) * (R0, t0) (Eq. tangent),
composed on the device with the intrinsics tensor into the device camera
table the library reads (no camera parameter crosses to the host).
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


def se3_exp_torch(xi: torch.Tensor):
    """Batched exp of xi = (rho, omega) [V, 6] in se(3) -> (R [V,3,3], t [V,3]),
    float64, on xi's device (the same closed form as se3_exp)."""
    xi = xi.to(torch.float64)
    rho, w = xi[:, :3], xi[:, 3:]
    V = xi.shape[0]
    K = torch.zeros((V, 3, 3), dtype=torch.float64, device=xi.device)
    K[:, 0, 1], K[:, 0, 2] = -w[:, 2], w[:, 1]
    K[:, 1, 0], K[:, 1, 2] = w[:, 2], -w[:, 0]
    K[:, 2, 0], K[:, 2, 1] = -w[:, 1], w[:, 0]
    th = torch.linalg.vector_norm(w, dim=1)
    small = th < 1e-8
    ts = torch.where(small, torch.ones_like(th), th)
    a = torch.where(small, torch.ones_like(th), torch.sin(ts) / ts)
    b = torch.where(small, torch.full_like(th, 0.5), (1.0 - torch.cos(ts)) / ts ** 2)
    c = torch.where(small, torch.full_like(th, 1.0 / 6.0), (ts - torch.sin(ts)) / ts ** 3)
    I = torch.eye(3, dtype=torch.float64, device=xi.device).expand(V, 3, 3)
    K2 = K @ K
    R = I + a[:, None, None] * K + b[:, None, None] * K2
    Vm = I + b[:, None, None] * K + c[:, None, None] * K2
    return R, (Vm @ rho[:, :, None])[:, :, 0]


class Rasterizer:
    """Holds a prepared scene's static state (context, original indices,
    storage type), the cameras' sizes, base poses and render settings.  The
    base poses live on the device: the rendered cameras are composed there
    (exp(xi) * (R0, t0) and the intrinsics tensor) into a device camera table
    that the render calls read, so a training step moves no camera parameter
    through the host."""

    def __init__(self, ctx: adop.Context, scene: adop.Scene, cams: Sequence, layers: int,
                 alpha: float = 0.01, flags: int = 0, background=None):
        self.ctx = ctx
        self.scene = scene
        self.cams = [c.copy() for c in cams]
        dev = scene.x.device
        self._R0 = torch.tensor(np.stack([np.asarray(c.R, dtype=np.float64) for c in cams]), device=dev)
        self._t0 = torch.tensor(np.stack([np.asarray(c.t, dtype=np.float64).reshape(3) for c in cams]), device=dev)
        # the static part of the table: sizes, znear, r2_max
        self._table0 = adop.cameras_upload(ctx, self.cams)
        self.layers = layers
        self.alpha = alpha
        self.flags = flags
        self.background = background

    @property
    def base_R(self):
        """Base rotations as numpy (reads the device)."""
        return list(self._R0.cpu().numpy())

    @property
    def base_t(self):
        return list(self._t0.cpu().numpy())

    def intrinsics(self, dtype=torch.float32, device=None) -> torch.Tensor:
        v = [[float(getattr(c, k)) for k in INTRINSICS] for c in self.cams]
        return torch.tensor(v, dtype=dtype, device=device or self.scene.x.device)

    def camera_table(self, intr: torch.Tensor, tangent: torch.Tensor) -> torch.Tensor:
        """Device camera table [V, 25] of the rendered cameras: intrinsics from
        `intr` [V, 9] and pose exp(tangent) * (R0, t0), composed on the device."""
        dR, dt = se3_exp_torch(tangent.detach())
        R = dR @ self._R0
        t = (dR @ self._t0[:, :, None])[:, :, 0] + dt
        tab = self._table0.clone()
        tab[:, 2:11] = intr.detach().to(torch.float32)
        tab[:, 13:22] = R.reshape(-1, 9).to(torch.float32)
        tab[:, 22:25] = t.to(torch.float32)
        return tab

    def cameras(self, intr: torch.Tensor, tangent: torch.Tensor):
        """The rendered cameras as host objects (reads the device; for
        inspection and tests, not used by the render path)."""
        intr = intr.detach().double().cpu().numpy()
        xi = tangent.detach().double().cpu().numpy()
        R0, t0 = self.base_R, self.base_t
        out = []
        for v, c in enumerate(self.cams):
            c2 = c.copy()
            for j, k in enumerate(INTRINSICS):
                setattr(c2, k, float(intr[v, j]))
            dR, dt = se3_exp(xi[v])
            c2.R = dR @ R0[v]
            c2.t = dR @ t0[v] + dt
            out.append(c2)
        return out

    def apply_tangent(self, tangent: torch.Tensor):
        """(R0, t0) <- exp(xi) * (R0, t0) and xi <- 0 (in place, on the device)."""
        with torch.no_grad():
            dR, dt = se3_exp_torch(tangent)
            self._R0 = dR @ self._R0
            self._t0 = (dR @ self._t0[:, :, None])[:, :, 0] + dt
            tangent.zero_()

    def __call__(self, x, y, z, feat, intr, tangent):
        return AdopRasterize.apply(x, y, z, feat, intr, tangent, self)


class AdopRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, feat, intr, tangent, rast: Rasterizer):
        scene = adop.Scene(x.detach(), y.detach(), z.detach(), feat.detach(), rast.scene.orig, rast.scene.dtype)
        table = rast.camera_table(intr, tangent)
        frame = adop.render_forward(rast.ctx, scene, rast.cams, rast.layers, alpha=rast.alpha, flags=rast.flags,
                                    background=rast.background, cams_device=table)
        ctx.rast = rast
        ctx.scene = scene
        ctx.frame = frame
        ctx.table = table
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
                                                         flags=rast.flags, background=rast.background,
                                                         cams_device=ctx.table)
        fdt, idt, tdt = ctx.dtypes
        return (dpos[0], dpos[1], dpos[2], dfeat.to(fdt), dintr.to(idt), dpose.to(tdt), None)
