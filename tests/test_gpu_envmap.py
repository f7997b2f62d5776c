"""GPU parity of the environment-map background (Eq. blend's
E(R^T C^-1(u, v)), "Environment Map") against the float64 oracle, through
the C ABI.

The FP32 ray (20 fixed-point steps of the inverse distortion, a rotation,
a normalisation, atan2f and acosf) differs from the float64 one by far less
than delta = 2e-6 S texels for rays away from the poles (the cameras here
look near the horizon), so an empty pixel's value may differ by 2 delta L_E
(L_E: the map's largest difference between adjacent texels).  Bounds:
  hit pixels: 1e-5 relative (as without the map); keys and counts bit-exact;
  empty pixels: 1e-6 |ref| + 2 delta L_E + 1e-7;
  dfeat, dpos, dpose, dintr: the usual 1e-5 S, 1e-4 S, 1e-5 S, 1e-5 S (the
      smooth map keeps the background error far below them);
  dL/dE: 1e-5 of the sum of |terms| plus 4 delta times the sum of |G| over
      the empty pixels that sample the texel (each bilinear weight moves by
      at most 2 delta)."""
import numpy as np
import pytest

from oracle import envmap as EM
from paper_2110_06635_amd import synth
from tests.gpu_parity_lib import say

pytestmark = pytest.mark.gpu


def _views(w=160, h=120):
    k = dict(k1=-0.08, k2=0.01, k3=0.001, p1=5e-4, p2=-5e-4)
    r2 = synth.r2_max_for(k["k1"], k["k2"], k["k3"], k["p1"], k["p2"])
    front = synth.Camera(w, h, 0.9 * w, 0.9 * w, w / 2.0 - 0.3, h / 2.0 + 0.2, r2_max=r2,
                         t=np.array([0.1, -0.05, 6.0]), R=synth.rodrigues([0.03, -0.02, 0.01]), **k)
    # the second view looks along -z: its rays cross the longitude seam
    R = synth.rodrigues([0.0, np.pi, 0.0]) @ synth.rodrigues([0.02, 0.01, 0.0])
    back = synth.Camera(w, h, 0.9 * w, 0.9 * w, w / 2.0, h / 2.0, r2_max=r2,
                        t=np.array([0.0, 0.1, 6.0]), R=R, **k)
    return [front, back]


def _scene(seed, n, C):
    rng = np.random.default_rng(seed)
    # two blobs, one in front of each camera, leaving most pixels empty
    pos = np.concatenate([rng.normal(0, 0.6, (n // 2, 3)) + [0, 0, 0],
                          rng.normal(0, 0.6, (n - n // 2, 3)) + [0, 0, 0]]).astype(np.float32)
    feat = rng.random((n, C)).astype(np.float32)
    return pos, feat


def _smooth_map(C, S, amp=0.1):
    r = (np.arange(S) + 0.5)[:, None] / S
    c = (np.arange(S) + 0.5)[None, :] / S
    return np.stack([0.5 + amp * np.sin(2 * np.pi * c + k) * np.cos(np.pi * r * 1.5 + 0.3 * k)
                     for k in range(C)]).astype(np.float32)


def _lipschitz(Em):
    dx = np.abs(np.diff(Em, axis=2)).max(axis=(1, 2))
    dx = np.maximum(dx, np.abs(Em[:, :, 0] - Em[:, :, -1]).max(axis=1))
    dy = np.abs(np.diff(Em, axis=1)).max(axis=(1, 2))
    return np.maximum(dx, dy)            # [C]


def _image_layout_mask(cams, L, C, counts):
    mask = np.zeros(C * counts.size, bool)
    off = 0
    for cam in cams:
        for l in range(L):
            n = (cam.width >> l) * (cam.height >> l)
            e = counts[off:off + n] == 0
            for ch in range(C):
                mask[C * off + ch * n: C * off + (ch + 1) * n] = e
            off += n
    return mask


def _per_channel(cams, L, C, total, vec):
    out = np.zeros(C * total)
    off = 0
    for cam in cams:
        for l in range(L):
            n = (cam.width >> l) * (cam.height >> l)
            for ch in range(C):
                out[C * off + ch * n: C * off + (ch + 1) * n] = vec[ch]
            off += n
    return out


def test_environment_map_forward_backward(oracle):
    import torch
    from paper_2110_06635_amd import adop as A
    say("environment map: forward + backward, smooth map S=256, two views (one across the seam)")
    ctx = A.Context(0)
    dev = torch.device("cuda:0")
    C, L, S = 4, 3, 256
    cams = _views()
    pos, feat = _scene(1, 6000, C)
    Em = _smooth_map(C, S)
    env = torch.from_numpy(Em).to(dev)
    scene = A.Scene.prepare(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(feat).to(dev))
    fr = A.render_forward(ctx, scene, cams, L, env_map=env)
    torch.cuda.synchronize()
    bg = EM.background_image(cams, L, Em.astype(np.float64))
    ref = oracle.forward(pos, feat, cams, L, bg_image=bg, want64=True)
    keys = fr.keys.cpu().numpy().view(np.uint64)
    counts = fr.counts.cpu().numpy()
    assert np.array_equal(keys, ref["keys"]) and np.array_equal(counts, ref["counts"])
    img = fr.images.cpu().numpy().astype(np.float64)
    empty = _image_layout_mask(cams, L, C, counts)
    assert empty.mean() > 0.5 and (~empty).any()
    delta = 2e-6 * S
    lim_e = 1e-6 * np.abs(ref["images64"]) + 2 * delta * _per_channel(cams, L, C, counts.size, _lipschitz(Em)) + 1e-7
    err = np.abs(img - ref["images64"])
    assert np.all(err[empty] <= lim_e[empty]), float(np.max(err[empty] / lim_e[empty]))
    assert np.all(err[~empty] <= 1e-5 * np.abs(ref["images64"][~empty]) + 1e-7)
    # backward
    G = synth.upstream_grad(img.size, 5).astype(np.float32)
    Gt = torch.from_numpy(G).to(dev)
    dE = torch.empty_like(env)
    dfeat, dpos, dpose, dintr = A.render_backward(ctx, scene, fr, Gt, env_map=env, env_grad=dE)
    torch.cuda.synchronize()
    rb = oracle.backward(pos, feat, cams, L, G, bg_image=bg)
    orig = scene.orig.cpu().numpy()
    got_f = np.empty_like(dfeat.cpu().numpy())
    got_f[orig] = dfeat.cpu().numpy()
    got_p = np.empty_like(dpos.cpu().numpy())
    got_p[:, orig] = dpos.cpu().numpy()
    assert np.all(np.abs(got_f - rb["dfeat"]) <= 1e-5 * rb["dfeat_abs"] + 1e-12)
    assert np.all(np.abs(got_p - rb["dpos"]) <= 1e-4 * rb["dpos_abs"] + 1e-12)
    assert np.all(np.abs(dpose.cpu().numpy() - rb["dpose"]) <= 1e-5 * rb["dpose_abs"] + 1e-12)
    assert np.all(np.abs(dintr.cpu().numpy() - rb["dintr"]) <= 1e-5 * rb["dintr_abs"] + 1e-12)
    _check_map_gradient(EM, cams, L, Em, counts, G, dE.cpu().numpy().astype(np.float64), delta)


def _check_map_gradient(EM_, cams, L, Em, counts, G, got, delta):
    C, S, _ = Em.shape
    want, absw = EM_.map_gradient(cams, L, Em.shape, counts, G.astype(np.float64))
    # sum of |G| over the empty pixels that sample each texel
    gsum = np.zeros((C, S, S))
    off = 0
    for cam in cams:
        for l in range(L):
            wl, hl = cam.width >> l, cam.height >> l
            n = wl * hl
            e = (counts[off:off + n] == 0).reshape(hl, wl)
            g = np.abs(G[C * off: C * (off + n)].astype(np.float64)).reshape(C, hl, wl)
            s, t = EM_.texcoords(EM_.layer_rays(cam, l), S)
            for r, c, w in EM_.bilinear(S, s, t):
                for ch in range(C):
                    np.add.at(gsum[ch], (r[e], c[e]), g[ch][e])
            off += n
    lim = 1e-5 * absw + 4 * delta * gsum + 1e-7
    assert np.all(np.abs(got - want) <= lim), float(np.max(np.abs(got - want) / lim))
    assert np.abs(want).max() > 0


def test_environment_map_gradient_random_texels(oracle):
    import torch
    from paper_2110_06635_amd import adop as A
    say("environment map: gradient of a random map, S=16")
    ctx = A.Context(0)
    dev = torch.device("cuda:0")
    C, L, S = 3, 2, 16
    cams = _views(96, 64)
    pos, feat = _scene(2, 3000, C)
    Em = np.random.default_rng(3).random((C, S, S)).astype(np.float32)
    env = torch.from_numpy(Em).to(dev)
    scene = A.Scene.prepare(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(feat).to(dev))
    fr = A.render_forward(ctx, scene, cams, L, env_map=env)
    G = synth.upstream_grad(C * fr.pixels, 6).astype(np.float32)
    dE = torch.full_like(env, 7.0)          # overwritten
    A.render_backward(ctx, scene, fr, torch.from_numpy(G).to(dev), env_map=env, env_grad=dE)
    torch.cuda.synchronize()
    counts = fr.counts.cpu().numpy()
    _check_map_gradient(EM, cams, L, Em, counts, G, dE.cpu().numpy().astype(np.float64), 2e-6 * S)
    # empty pixels against the oracle's samples of the same random map
    bg = EM.background_image(cams, L, Em.astype(np.float64))
    img = fr.images.cpu().numpy().astype(np.float64)
    empty = _image_layout_mask(cams, L, C, counts)
    lim = 1e-6 * np.abs(bg) + 2 * 2e-6 * S * _per_channel(cams, L, C, counts.size, _lipschitz(Em)) + 1e-7
    assert np.all(np.abs(img - bg)[empty] <= lim[empty])


def test_constant_map_equals_constant_background():
    import torch
    from paper_2110_06635_amd import adop as A
    ctx = A.Context(0)
    dev = torch.device("cuda:0")
    C, L, S = 4, 3, 8
    cams = _views()
    pos, feat = _scene(4, 4000, C)
    const = np.float32([0.25, -1.5, 2.0, 0.0])
    env = torch.from_numpy(np.broadcast_to(const[:, None, None], (C, S, S)).copy()).to(dev)
    scene = A.Scene.prepare(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(feat).to(dev))
    a = A.render_forward(ctx, scene, cams, L, background=const)
    b = A.render_forward(ctx, scene, cams, L, env_map=env)
    torch.cuda.synchronize()
    assert torch.equal(a.keys, b.keys) and torch.equal(a.counts, b.counts)
    d = (a.images.double() - b.images.double()).abs()
    # the four FP32 weights sum to 1 within a few units in the last place
    assert bool((d <= 4e-7 * a.images.double().abs() + 1e-7).all())
