"""GPU parity of the photometric tone mapper (Sec. 3.3) against the float64
oracle, through the C ABI.

R_t has kinks at the table nodes and at 0 and 1; inputs are nudged so that
every response input stays at least 1e-4 table steps away from them, so the
FP32 path and the float64 oracle take the same branch.  Bounds, from the
FP32 arithmetic (about ten roundings from I_hdr to the response input, so a
relative error below 2e-6 of that input):
  forward: |ldr - ref| <= 2e-6 (S_c |x| + |ref|) + 1e-7, S_c the channel's
           largest table slope;
  dL/dI_hdr: 2e-6 of the oracle's value plus 1e-7 of its scale;
  exposure, white point, vignette: 1e-5 of the sum of |terms|;
  table: 1e-5 of the sum of |terms| plus, because the interpolation weight
      f = x (K - 1) - i takes the input's relative error times (K - 1),
      2e-6 (K - 1) times the sum of |g x| over the pixels using the entry."""
import numpy as np
import pytest

from oracle import tonemap as T
from tests.gpu_parity_lib import say

pytestmark = pytest.mark.gpu


def _inputs(seed, V, h, w, K, leak):
    rng = np.random.default_rng(seed)
    hdr = rng.uniform(-0.3, 1.6, (V, 3, h, w))
    ev = rng.uniform(-0.5, 0.5, V).astype(np.float32).astype(np.float64)
    white = rng.uniform(0.8, 1.2, (V, 3))
    white[:, 1] = 1.0
    white = white.astype(np.float32).astype(np.float64)
    vig = np.array([-0.3, 0.1, -0.05, 0.45, 0.55], np.float32).astype(np.float64)
    crf = np.sort(rng.uniform(0, 1, (3, K)), axis=1)
    crf[:, 0], crf[:, -1] = 0.0, 1.0
    crf = crf.astype(np.float32).astype(np.float64)
    # nudge the inputs away from the kinks of R_t (float64 stage values)
    vf = T.vignette_factor(w, h, vig)
    for _ in range(20):
        hdr = hdr.astype(np.float32).astype(np.float64)
        x = hdr * (2.0 ** -ev)[:, None, None, None] * white[:, :, None, None] * vf[None, None]
        pos = np.clip(x, 0, 1) * (K - 1)
        # the FP32 input carries a relative error below 2e-6, i.e. up to
        # 2e-6 (K - 1) |x| table steps: keep ten times that from every node
        near = (x >= 0) & (x <= 1) & (np.abs(pos - np.round(pos)) < 1e-4 + 2e-5 * (K - 1) * np.abs(x))
        near |= np.abs(x) < 1e-4
        near |= np.abs(x - 1.0) < 1e-4
        if not near.any():
            break
        step = rng.uniform(1e-3, 5e-3, hdr.shape)   # random, so no input cycles through nodes
        hdr = np.where(near, hdr + step * np.sign(hdr + 1e-9), hdr)
    else:
        raise AssertionError("could not keep the inputs away from the kinks")
    return hdr, ev, white, vig, crf


def _run(A, ctx, hdr, ev, white, vig, crf, leak, g):
    import torch
    dev = torch.device("cuda:0")
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    tm = A.Tonemapper(f(ev), f(white), f(vig), f(crf), leak)
    ldr = A.tonemap_forward(ctx, f(hdr), tm)
    grads = A.tonemap_backward(ctx, f(hdr), tm, f(g))
    torch.cuda.synchronize()
    return ldr.cpu().numpy().astype(np.float64), [x.cpu().numpy().astype(np.float64) for x in grads]


@pytest.mark.parametrize("V,h,w,K,leak", [(3, 61, 97, 33, 0.01), (2, 40, 23, 2, 0.01), (1, 61, 97, 256, -1.0),
                                          (2, 1080, 1920, 1024, 0.01)])
def test_tonemap_matches_oracle(oracle, V, h, w, K, leak):
    import torch
    from paper_2110_06635_amd import adop as A
    say(f"tone mapper V={V} {w}x{h} K={K} leak={leak}")
    ctx = A.Context(0)
    hdr, ev, white, vig, crf = _inputs(V * 1000 + K, V, h, w, K, leak)
    g = np.random.default_rng(K).normal(size=hdr.shape).astype(np.float32).astype(np.float64)
    ldr, (dh, dev_, dw, dv, dc) = _run(A, ctx, hdr, ev, white, vig, crf, leak, g)
    ref = T.forward(hdr, ev, white, vig, crf, leak)
    x = hdr * (2.0 ** -ev)[:, None, None, None] * white[:, :, None, None] * T.vignette_factor(w, h, vig)[None, None]
    smax = (np.abs(np.diff(crf, axis=1)).max(axis=1) * (K - 1))[None, :, None, None]
    bound = 2e-6 * (smax * np.abs(x) + np.abs(ref)) + 1e-7
    bad = np.abs(ldr - ref) > bound
    assert not bad.any(), f"{int(bad.sum())} ldr values off, worst {np.max(np.abs(ldr - ref)):.3g}"
    (rh, rev, rw, rv, rc), (sh, sev, sw, sv, sc) = T.backward(hdr, ev, white, vig, crf, g, leak)
    scale = np.max(np.abs(rh))
    assert np.all(np.abs(dh - rh) <= 2e-6 * np.abs(rh) + 1e-7 * scale + 1e-12), float(np.max(np.abs(dh - rh)))
    for name, got, want, s in (("ev", dev_, rev, sev), ("white", dw, rw, sw), ("vignette", dv, rv, sv)):
        err = np.abs(got - want)
        assert np.all(err <= 1e-5 * s + 1e-12), (name, float(np.max(err / (s + 1e-30))))
    gx = np.zeros((3, K))
    for c in range(3):
        xc = x[:, c]
        pos = np.clip(xc, 0, 1) * (K - 1)
        i = np.minimum(np.floor(pos).astype(np.int64), K - 2)
        used = np.ones_like(xc, bool) if leak < 0 else (xc >= 0) & (xc <= 1)
        t = np.where(used, np.abs(g[:, c] * xc), 0.0).ravel()
        np.add.at(gx[c], i.ravel(), t)
        np.add.at(gx[c], i.ravel() + 1, t)
    err = np.abs(dc - rc)
    lim = 1e-5 * sc + 2e-6 * (K - 1) * gx + 1e-12
    assert np.all(err <= lim), ("crf", float(np.max(err / lim)))


def test_tonemap_identity_on_device():
    """EV 0, white 1, no vignette, a linear table: the leaky identity, exactly
    representable (closed form of Eq. resonseleak)."""
    import torch
    from paper_2110_06635_amd import adop as A
    ctx = A.Context(0)
    dev = torch.device("cuda:0")
    K = 17
    lin = torch.tensor(np.tile(np.arange(K) / (K - 1), (3, 1)), dtype=torch.float32, device=dev)
    tm = A.Tonemapper(torch.zeros(1, device=dev), torch.ones((1, 3), device=dev),
                      torch.tensor([0, 0, 0, 0.5, 0.5], dtype=torch.float32, device=dev), lin, 0.01)
    vals = torch.tensor([-2.0, -0.5, 0.0, 0.25, 0.5, 1.0, 4.0, 1e30], device=dev)
    hdr = vals.repeat(3).view(1, 3, 1, 8).contiguous()
    out = A.tonemap_forward(ctx, hdr, tm)[0, 0, 0].cpu().numpy()
    want = np.float32([-0.02, -0.005, 0.0, 0.25, 0.5, 1.0, -0.01 / 2.0 + 1.01, 1.01])
    np.testing.assert_allclose(out, want, rtol=2e-7, atol=0)
