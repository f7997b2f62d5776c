"""GPU tests of the torch.autograd.Function wrapper: gradients equal the C-ABI
backward, the feature gradient matches finite differences of the forward
(the blend is linear in the features for a fixed selection), and the
approximate pose gradient drives a perturbed camera back toward the true
pose (descent test; the paper's robustness experiment uses real data)."""
import numpy as np
import pytest

from paper_2110_06635_amd import synth
from tests.gpu_parity_lib import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2110_06635_amd import adop
    from paper_2110_06635_amd.autograd import Rasterizer
    ctx = adop.Context(0)
    return torch, adop, ctx, Rasterizer


def _scene(n=60000, w=128, h=96, V=2, C=3, seed=3):
    rng = np.random.default_rng(seed)
    pos, feat = synth.planes(12, n // 12, C, seed, box=1.5, half_lo=0.5, half_hi=1.2)
    cams = synth.orbit_cameras(V, 6.0, seed + 1, width=w, height=h, f=0.9 * w, kmax=0.05)
    return pos, feat, cams


def test_autograd_equals_abi_backward(env):
    torch, adop, ctx, Rasterizer = env
    pos, feat, cams = _scene()
    say("autograd vs ABI backward")
    dev = torch.device("cuda:0")
    scene = adop.Scene.prepare(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(feat).to(dev))
    L = 3
    rast = Rasterizer(ctx, scene, cams, L)
    x = scene.x.clone().requires_grad_()
    y = scene.y.clone().requires_grad_()
    z = scene.z.clone().requires_grad_()
    f = scene.feat.clone().requires_grad_()
    intr = rast.intrinsics(torch.float64).requires_grad_()
    tan = torch.zeros((len(cams), 6), dtype=torch.float64, device=dev, requires_grad=True)
    outs = rast(x, y, z, f, intr, tan)
    gen = torch.Generator(device=dev).manual_seed(5)
    W = [torch.randn(o.shape, device=dev, generator=gen) for o in outs]
    loss = sum((o * w).sum() for o, w in zip(outs, W))
    loss.backward()
    # the same through the binding directly
    frame = adop.render_forward(ctx, scene, cams, L)
    G = torch.zeros(scene.channels * frame.pixels, device=dev)
    for l, w in enumerate(W):
        C = scene.channels
        hl, wl = cams[0].height >> l, cams[0].width >> l
        o0 = int(frame.offsets[0, l])
        sv = C * (int(frame.offsets[1, l]) - o0)
        G.as_strided((len(cams), C, hl, wl), (sv, hl * wl, wl, 1), C * o0).copy_(w)
    dfeat, dpos, dpose, dintr = adop.render_backward(ctx, scene, frame, G)
    torch.cuda.synchronize()
    tol = dict(rtol=1e-4, atol=1e-5)
    torch.testing.assert_close(f.grad, dfeat, **tol)
    torch.testing.assert_close(x.grad, dpos[0], **tol)
    torch.testing.assert_close(y.grad, dpos[1], **tol)
    torch.testing.assert_close(z.grad, dpos[2], **tol)
    torch.testing.assert_close(tan.grad, dpose, rtol=1e-4, atol=1e-3 * float(dpose.abs().max()))
    torch.testing.assert_close(intr.grad, dintr, rtol=1e-4, atol=1e-3 * float(dintr.abs().max()))


def test_feature_gradient_directional_fd(env):
    torch, adop, ctx, Rasterizer = env
    pos, feat, cams = _scene(seed=4)
    say("feature gradient directional FD")
    dev = torch.device("cuda:0")
    scene = adop.Scene.prepare(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(feat).to(dev))
    rast = Rasterizer(ctx, scene, cams, 3)
    intr = rast.intrinsics()
    tan = torch.zeros((len(cams), 6), dtype=torch.float64, device=dev)
    gen = torch.Generator(device=dev).manual_seed(6)
    f = scene.feat.clone().requires_grad_()
    outs = rast(scene.x, scene.y, scene.z, f, intr, tan)
    W = [torch.randn(o.shape, device=dev, generator=gen) for o in outs]
    sum((o * w).sum() for o, w in zip(outs, W)).backward()
    d = torch.randn(f.shape, device=dev, generator=gen)
    h = 1e-2

    def L(ff):
        with torch.no_grad():
            o = rast(scene.x, scene.y, scene.z, ff, intr, tan)
            return sum(float((a.double() * w.double()).sum()) for a, w in zip(o, W))

    fd = (L(f.detach() + h * d) - L(f.detach() - h * d)) / (2 * h)
    an = float((f.grad.double() * d.double()).sum())
    assert abs(fd - an) <= 2e-3 * abs(an) + 1e-3, (fd, an)


def test_pose_descent(env):
    """A camera rotated/shifted away from the pose that rendered the target
    moves back under gradient steps on the L1 loss (tangent-space update)."""
    torch, adop, ctx, Rasterizer = env
    say("pose descent")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(8)
    pos, _ = synth.planes(30, 20000, 3, 9, box=1.5, half_lo=0.4, half_hi=1.0)
    # smooth texture so that every pyramid layer carries structure
    pp = pos.astype(np.float64)
    feat = np.stack([0.5 + 0.5 * np.sin(3.0 * pp[:, 0] + 1.0), 0.5 + 0.5 * np.cos(2.5 * pp[:, 1]),
                     0.5 + 0.5 * np.sin(2.0 * pp[:, 2] + pp[:, 0])], axis=1).astype(np.float32)
    cam = synth.orbit_cameras(1, 5.0, 10, width=160, height=120, f=140.0, kmax=0.0)[0]
    scene = adop.Scene.prepare(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(feat).to(dev))
    L = 4
    truth = Rasterizer(ctx, scene, [cam], L)
    intr = truth.intrinsics()
    zero = torch.zeros((1, 6), dtype=torch.float64, device=dev)
    with torch.no_grad():
        target = [t.clone() for t in truth(scene.x, scene.y, scene.z, scene.feat, intr, zero)]
    off = cam.copy()
    from paper_2110_06635_amd.autograd import se3_exp
    dR, dt = se3_exp(np.array([0.03, -0.02, 0.02, 0.004, -0.006, 0.003]))
    off.R = dR @ np.asarray(cam.R)
    off.t = dR @ np.asarray(cam.t) + dt
    rast = Rasterizer(ctx, scene, [off], L)
    tan = torch.zeros((1, 6), dtype=torch.float64, device=dev, requires_grad=True)

    def pose_err():
        R0 = np.asarray(cam.R)
        R1 = rast.base_R[0]
        ang = np.arccos(np.clip((np.trace(R1 @ R0.T) - 1) / 2, -1, 1))
        c0 = -R0.T @ np.asarray(cam.t)
        c1 = -R1.T @ rast.base_t[0]
        return float(ang), float(np.linalg.norm(c1 - c0))

    e0 = pose_err()
    # sign-descent with decaying steps, separately for translation / rotation
    lr = np.array([4e-3, 4e-3, 4e-3, 8e-4, 8e-4, 8e-4])
    for it in range(120):
        outs = rast(scene.x, scene.y, scene.z, scene.feat, intr, tan)
        loss = sum((o - t).abs().mean() for o, t in zip(outs, target))
        loss.backward()
        with torch.no_grad():
            g = tan.grad.double().cpu().numpy()[0]
            step = -lr * np.sign(g) * (0.97 ** it)
            tan.copy_(torch.from_numpy(step[None]).to(dev))
            tan.grad = None
        rast.apply_tangent(tan)
    e1 = pose_err()
    print("pose error (rad, m):", e0, "->", e1)
    assert e1[0] < 0.5 * e0[0] and e1[1] < 0.5 * e0[1]
