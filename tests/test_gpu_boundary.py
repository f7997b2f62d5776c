"""GPU tests of the boundary calls around the render calls: a device camera
table (adop_cameras_upload, render params' cameras_device) renders and
differentiates exactly like the same cameras given on the host, including a
table whose values differ from the host array's; a scene prepared into one
buffer bound with adop_scene_bind renders like the separate tensors; an
autograd step runs without any host synchronisation."""
import ctypes as ct

import numpy as np
import pytest

from paper_2110_06635_amd import synth
from tests.gpu_parity_lib import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2110_06635_amd import adop
    return torch, adop, adop.Context(0)


def _scene(seed=21, n=40000, V=3, w=200, h=150):
    pos, feat = synth.planes(10, n // 10, 4, seed, box=1.5, half_lo=0.4, half_hi=1.0)
    cams = synth.orbit_cameras(V, 6.0, seed + 1, width=w, height=h, f=0.9 * w, kmax=0.05)
    return pos, feat, cams


def _same_frame(torch, a, b):
    """Keys and counts bit-exact; images within 1e-5 relative (FP32 sums
    whose atomic order differs between launches)."""
    assert torch.equal(a.keys, b.keys) and torch.equal(a.counts, b.counts)
    d = (a.images.double() - b.images.double()).abs()
    assert bool((d <= 1e-5 * a.images.double().abs() + 1e-7).all())


def test_camera_table_equals_host_cameras(env):
    torch, A, ctx = env
    say("camera table vs host cameras")
    pos, feat, cams = _scene()
    dev = torch.device("cuda:0")
    scene = A.Scene.prepare(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(feat).to(dev))
    L = 3
    ref = A.render_forward(ctx, scene, cams, L)
    table = A.cameras_upload(ctx, cams)
    # the host array of the call only gives sizes: feed it wrong intrinsics and poses
    wrong = [c.copy() for c in cams]
    for c in wrong:
        c.fx, c.cx, c.k1 = 3.0 * c.fx, 0.0, 0.3
        c.R = np.eye(3)
        c.t = np.array([5.0, 5.0, 50.0])
    got = A.render_forward(ctx, scene, wrong, L, cams_device=table)
    torch.cuda.synchronize()
    _same_frame(torch, ref, got)
    gen = torch.Generator(device=dev).manual_seed(3)
    G = torch.randn(ref.images.shape, device=dev, generator=gen)
    # the backward of the same frame through both (deterministic: fixed order)
    r = A.render_backward(ctx, scene, ref, G)
    g = A.render_backward(ctx, scene, ref, G, cams_device=table)
    torch.cuda.synchronize()
    for x, y in zip(r, g):
        assert torch.equal(x, y)
    # without the table the wrong cameras render something else
    other = A.render_forward(ctx, scene, wrong, L)
    torch.cuda.synchronize()
    assert not torch.equal(other.keys, ref.keys)


def test_camera_upload_validates(env):
    torch, A, ctx = env
    cams = [synth.Camera(0, 10, 1.0, 1.0, 0.0, 0.0)]
    with pytest.raises(A.AdopError):
        A.cameras_upload(ctx, cams)


def test_scene_in_one_buffer(env):
    torch, A, ctx = env
    say("scene bound in one buffer")
    pos, feat, cams = _scene(seed=31, V=1)
    dev = torch.device("cuda:0")
    n, C = pos.shape[0], feat.shape[1]
    L_ = A.lib()
    nb = L_.adop_scene_bytes(n, C, A.F32)
    mem = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
    base = (mem.data_ptr() + 255) // 256 * 256
    d = A.SceneDesc()
    assert L_.adop_scene_bind(ct.c_void_p(base), n, C, A.F32, ct.byref(d)) == A.OK
    pos_t = torch.from_numpy(pos).to(dev)
    feat_t = torch.from_numpy(feat).to(dev)
    st = L_.adop_scene_prepare(ctx.handle, ct.c_void_p(pos_t.data_ptr()), ct.c_void_p(feat_t.data_ptr()), n, C,
                               A.F32, 0, 1, ct.c_void_p(d.x), ct.c_void_p(d.y), ct.c_void_p(d.z),
                               ct.c_void_p(d.feat), ct.c_void_p(d.orig_index), A._stream(None))
    ctx.check(st, "prepare into bound scene")
    ref_scene = A.Scene.prepare(ctx, pos_t, feat_t)
    ref = A.render_forward(ctx, ref_scene, cams, 3)
    fr = A.Frame(cams, 3, C, dev)
    ws = ctx.workspace(C, 1, fr.pixels)
    p, keep = A._params(3, 0.01, 0, None, C)
    fd = fr.desc()
    st = L_.adop_render_forward(ctx.handle, ct.byref(d), fr.cams, 1, ct.byref(p), ct.byref(fd), A._ptr(ws),
                                ws.numel(), A._stream(None))
    ctx.check(st, "render bound scene")
    torch.cuda.synchronize()
    _same_frame(torch, ref, fr)


def test_autograd_step_without_host_sync(env):
    torch, A, ctx = env
    from paper_2110_06635_amd.autograd import Rasterizer
    say("autograd step without host synchronisation")
    pos, feat, cams = _scene(seed=41)
    dev = torch.device("cuda:0")
    scene = A.Scene.prepare(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(feat).to(dev))
    rast = Rasterizer(ctx, scene, cams, 3)
    intr = rast.intrinsics(torch.float64).requires_grad_()
    tan = torch.full((len(cams), 6), 1e-3, dtype=torch.float64, device=dev, requires_grad=True)
    f = scene.feat.clone().requires_grad_()
    gen = torch.Generator(device=dev).manual_seed(9)
    W = None
    torch.cuda.synchronize()
    # every host read of device data raises during the step (explicitly, and
    # through torch's synchronisation debug mode)
    def forbidden(*a, **k):
        raise AssertionError("host synchronisation inside the training step")
    names = ("cpu", "item", "tolist", "numpy", "__array__")
    saved = {nm: getattr(torch.Tensor, nm) for nm in names}
    saved_sync = torch.cuda.synchronize
    for nm in names:
        setattr(torch.Tensor, nm, forbidden)
    torch.cuda.synchronize = forbidden
    torch.cuda.set_sync_debug_mode("error")
    try:
        outs = rast(scene.x, scene.y, scene.z, f, intr, tan)
        W = [torch.randn(o.shape, device=dev, generator=gen) for o in outs]
        loss = sum((o * w).sum() for o, w in zip(outs, W))
        loss.backward()
        with torch.no_grad():
            tan -= 1e-4 * tan.grad
        rast.apply_tangent(tan)
    finally:
        torch.cuda.set_sync_debug_mode(0)
        for nm, fn in saved.items():
            setattr(torch.Tensor, nm, fn)
        torch.cuda.synchronize = saved_sync
    torch.cuda.synchronize()
    assert torch.isfinite(intr.grad).all() and torch.isfinite(f.grad).all()
    assert bool((tan == 0).all())
    # the device composition equals the host one (float64 on both sides,
    # compared after the float32 rounding the renderer reads)
    rast2 = Rasterizer(ctx, scene, cams, 3)
    xi = torch.full((len(cams), 6), 1e-3, dtype=torch.float64, device=dev)
    host = rast2.cameras(rast2.intrinsics(torch.float64), xi)
    tab = rast2.camera_table(rast2.intrinsics(), xi).cpu().numpy()
    for v, c in enumerate(host):
        np.testing.assert_allclose(tab[v, 13:22], np.asarray(c.R, np.float32).reshape(9), rtol=0, atol=2e-7)
        np.testing.assert_allclose(tab[v, 22:25], np.asarray(c.t, np.float32).reshape(3), rtol=1e-6, atol=1e-6)
        np.testing.assert_array_equal(tab[v, 2:11], np.float32([getattr(c, k) for k in
                                                                 ("fx", "fy", "cx", "cy", "k1", "k2", "k3", "p1", "p2")]))


def test_atomic_probe_results(env):
    """The diagnostic atomics do what they time: each word holds the minimum
    (kind 0) or the count (kind 1) of the ops that targeted it."""
    torch, A, ctx = env
    ops, fp = 1 << 20, 64
    buf = torch.full((fp,), -1, dtype=torch.int64, device="cuda:0")     # all ones: u64 maximum
    ms = A.atomic_probe(ctx, 0, ops, fp, 1, buf)
    torch.cuda.synchronize()
    got = buf.cpu().numpy().view(np.uint64)
    want = np.array([ops - (ops - fp + w) for w in range(fp)], dtype=np.uint64)   # ops - largest i with i % fp == w
    assert ms > 0 and np.array_equal(got, want)
    fbuf = torch.zeros(fp, dtype=torch.float32, device="cuda:0")
    A.atomic_probe(ctx, 1, ops, fp, 1, fbuf)
    torch.cuda.synchronize()
    assert bool((fbuf == ops // fp).all())
    with pytest.raises(A.AdopError):
        A.atomic_probe(ctx, 0, ops, 1 << 20, 1, buf)        # footprint beyond the buffer
