"""Pins of the environment-map oracle (Eq. blend's background E(R^T C^-1))
and of the C oracle's per-pixel background: what the geometry and the
sampling fix independently of the code under test.  Planted mistakes must
fail a pin."""
import numpy as np
import pytest

from oracle import envmap as E
from paper_2110_06635_amd import synth


def _cam(seed=0, w=40, h=30, dist=True):
    rng = np.random.default_rng(seed)
    k = dict(k1=-0.08, k2=0.02, k3=0.005, p1=4e-4, p2=-3e-4) if dist else {}
    return synth.Camera(w, h, 0.9 * w, 0.8 * w, w / 2.0 - 0.7, h / 2.0 + 0.4,
                        R=synth.rodrigues(rng.normal(size=3) * 0.4), t=rng.normal(size=3), **k)


def test_undistort_inverts_the_distortion():
    rng = np.random.default_rng(1)
    a = rng.uniform(-0.5, 0.5, 1000)
    b = rng.uniform(-0.5, 0.5, 1000)
    for k in [(-0.1, 0.02, 0.0, 1e-4, 1e-4), (0.1, -0.05, 0.01, -1e-3, 2e-3), (0, 0, 0, 0, 0)]:
        xd, yd = E.distort(a, b, *k)
        a2, b2 = E.undistort(xd, yd, *k)
        np.testing.assert_allclose(a2, a, rtol=0, atol=1e-12)
        np.testing.assert_allclose(b2, b, rtol=0, atol=1e-12)


def test_principal_point_looks_along_the_optical_axis():
    cam = _cam(2)
    d = E.ray(cam, np.float64(np.float32(cam.cx)), np.float64(np.float32(cam.cy)))
    R = np.asarray(cam.R, np.float32).astype(np.float64)      # FP32 rotation: normalise its row
    want = R.T @ np.array([0.0, 0.0, 1.0])
    np.testing.assert_allclose(d, want / np.linalg.norm(want), rtol=0, atol=1e-15)


def test_ray_points_at_the_projected_point():
    """A world point's float64 projection, unprojected, gives the direction
    from the camera centre to the point."""
    cam = _cam(3)
    rng = np.random.default_rng(4)
    R = np.asarray(cam.R, np.float32).astype(np.float64)
    t = np.asarray(cam.t, np.float32).astype(np.float64)
    centre = -R.T @ t
    for _ in range(20):
        xc = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(3, 6)])
        P = R.T @ (xc - t)
        a, b = xc[0] / xc[2], xc[1] / xc[2]
        f = lambda k: float(np.float32(getattr(cam, k)))
        xd, yd = E.distort(a, b, f("k1"), f("k2"), f("k3"), f("p1"), f("p2"))
        u0, v0 = f("fx") * xd + f("cx"), f("fy") * yd + f("cy")
        d = E.ray(cam, np.float64(u0), np.float64(v0))
        want = (P - centre) / np.linalg.norm(P - centre)
        np.testing.assert_allclose(d, want, rtol=0, atol=1e-12)


def test_texcoords_closed_forms():
    S = 64
    s, t = E.texcoords(np.array([0.0, 0.0, 1.0]), S)
    assert s == S / 2 and t == S / 2
    s, t = E.texcoords(np.array([1.0, 0.0, 0.0]), S)
    assert s == 0.75 * S and t == S / 2
    s, t = E.texcoords(np.array([0.0, 1.0, 0.0]), S)
    assert t == 0.0
    s, t = E.texcoords(np.array([0.0, -1.0, 0.0]), S)
    assert t == S


def test_bilinear_reproduces_linear_maps_and_wraps():
    S = 32
    rr, cc = np.meshgrid(np.arange(S) + 0.5, np.arange(S) + 0.5, indexing="ij")
    Emap = (0.3 + 0.02 * cc - 0.01 * rr)[None]          # linear in (s, t) at texel centres
    rng = np.random.default_rng(5)
    s = rng.uniform(1.0, S - 1.0, 200)
    t = rng.uniform(1.0, S - 1.0, 200)
    val = 0.0
    for r, c, w in E.bilinear(S, s, t):
        val = val + Emap[0, r, c] * w
    np.testing.assert_allclose(val, 0.3 + 0.02 * s - 0.01 * t, rtol=0, atol=1e-13)
    # across the longitude seam the weights wrap to the last column
    (r0, c0, w0), (_, c1, w1), _, _ = E.bilinear(S, np.array([0.25]), np.array([5.5]))   # a row centre
    assert c0[0] == S - 1 and c1[0] == 0 and abs(w0[0] - 0.25) < 1e-15 and abs(w1[0] - 0.75) < 1e-15


def test_constant_map_is_the_constant_background(oracle):
    cam = _cam(6)
    rng = np.random.default_rng(7)
    pos = rng.uniform(-1, 1, (300, 3)).astype(np.float32) + np.float32([0, 0, 4])
    feat = rng.random((300, 3)).astype(np.float32)
    L = 3
    const = np.float32([0.25, -1.5, 2.0])
    Emap = np.broadcast_to(const[:, None, None], (3, 16, 16)).astype(np.float64)
    samp = E.background_image([cam], L, Emap)
    # the four bilinear weights sum to 1 up to rounding
    n0 = cam.width * cam.height                           # layer 0 is the first [C][h][w] block
    np.testing.assert_allclose(samp[:3 * n0].reshape(3, n0),
                               np.broadcast_to(const[:, None].astype(np.float64), (3, n0)), rtol=1e-15, atol=0)
    # the per-pixel path of the C oracle with exactly that constant at every
    # pixel (image layout) reproduces the constant background bit for bit
    tot = oracle.total_pixels([cam], L)
    bg = np.empty(3 * tot)
    off = 0
    for l in range(L):
        n = (cam.width >> l) * (cam.height >> l)
        for ch in range(3):
            bg[3 * off + ch * n: 3 * off + (ch + 1) * n] = const[ch]
        off += n
    a = oracle.forward(pos, feat, [cam], L, background=const, want64=True)
    b = oracle.forward(pos, feat, [cam], L, bg_image=bg, want64=True)
    assert np.array_equal(a["images64"], b["images64"])
    G = rng.normal(size=a["images"].size).astype(np.float32)
    ga = oracle.backward(pos, feat, [cam], L, G, background=const)
    gb = oracle.backward(pos, feat, [cam], L, G, bg_image=bg)
    for k in ("dfeat", "dpos", "dpose", "dintr"):
        assert np.array_equal(ga[k], gb[k]), k


def test_empty_pixels_take_the_per_pixel_background(oracle):
    """Eq. blend with a per-pixel background: an empty pixel's value is that
    pixel's background value exactly; hit pixels are the same means as with
    a constant background."""
    cam = _cam(11)
    rng = np.random.default_rng(12)
    pos = rng.uniform(-1, 1, (200, 3)).astype(np.float32) + np.float32([0, 0, 4])
    feat = rng.random((200, 2)).astype(np.float32)
    L = 2
    tot = oracle.total_pixels([cam], L)
    bg = rng.uniform(-3, 3, 2 * tot)
    a = oracle.forward(pos, feat, [cam], L, want64=True)
    b = oracle.forward(pos, feat, [cam], L, bg_image=bg, want64=True)
    mask = np.zeros(2 * tot, bool)
    off = 0
    for l in range(L):
        n = (cam.width >> l) * (cam.height >> l)
        e = a["counts"][off:off + n] == 0
        mask[2 * off: 2 * off + n] = e
        mask[2 * off + n: 2 * off + 2 * n] = e
        off += n
    assert mask.any() and (~mask).any()
    assert np.array_equal(b["images64"][mask], bg[mask])
    assert np.array_equal(b["images64"][~mask], a["images64"][~mask])


def test_empty_neighbour_uses_the_map_value(oracle):
    """One point alone: every neighbour is empty, so its spatial gradient at
    layer 0 is 1/2 (<G(q+), tau - E(q+)> - <G(q-), tau - E(q-)>) (Eq. gradp
    with case 1 of Eq. spatialderiv), with the map's values at q."""
    cam = synth.Camera(9, 7, 8.0, 8.0, 4.0, 3.0)
    pos = np.float32([[0.0, 0.0, 5.0]])          # lands on the centre pixel (4, 3)
    feat = np.float32([[0.7, 0.2]])
    rng = np.random.default_rng(8)
    bg = rng.uniform(-1, 1, 2 * 63).astype(np.float64)
    G = rng.normal(size=2 * 63).astype(np.float32)
    out = oracle.backward(pos, feat, [cam], 1, G, bg_image=bg, want_g=True)
    idx = lambda ch, x, y: ch * 63 + y * 9 + x
    dot = lambda x, y: sum(float(G[idx(ch, x, y)]) * (float(feat[0, ch]) - bg[idx(ch, x, y)]) for ch in range(2))
    gu = 0.5 * (dot(5, 3) - dot(3, 3))
    gv = 0.5 * (dot(4, 4) - dot(4, 2))
    assert abs(out["gu"][0, 0] - gu) < 1e-12 and abs(out["gv"][0, 0] - gv) < 1e-12


def test_map_gradient_is_the_derivative_of_the_blend(oracle):
    """The background is linear in the texels: the gradient equals the change
    of sum(G * image) over the empty pixels when one texel moves."""
    cam = _cam(9, w=24, h=18)
    rng = np.random.default_rng(10)
    pos = rng.uniform(-0.3, 0.3, (50, 3)).astype(np.float32) + np.float32([0, 0, 4])
    feat = rng.random((50, 2)).astype(np.float32)
    L = 2
    S = 8
    Emap = rng.random((2, S, S))
    fw = oracle.forward(pos, feat, [cam], L, bg_image=E.background_image([cam], L, Emap))
    G = rng.normal(size=fw["images"].size)
    dE, aE = E.map_gradient([cam], L, Emap.shape, fw["counts"], G)
    empty = np.repeat((fw["counts"] == 0)[None], 2, axis=0)
    # image layout: per (view, layer) [C][h][w]; build the mask in that layout
    mask = np.zeros(fw["images"].size, bool)
    off = 0
    for l in range(L):
        n = (cam.width >> l) * (cam.height >> l)
        e = fw["counts"][off:off + n] == 0
        mask[2 * off: 2 * off + n] = e
        mask[2 * off + n: 2 * off + 2 * n] = e
        off += n
    for (ch, r, c) in [(0, 3, 4), (1, 0, 0), (1, 7, 2), (0, 5, 7)]:
        E2 = Emap.copy()
        E2[ch, r, c] += 1.0
        diff = E.background_image([cam], L, E2) - E.background_image([cam], L, Emap)
        want = float(np.sum((G * diff)[mask]))
        assert abs(dE[ch, r, c] - want) < 1e-12
        assert aE[ch, r, c] >= abs(dE[ch, r, c]) - 1e-15


# ---- planted mistakes -------------------------------------------------------

def test_mutant_swapped_longitude_is_caught(monkeypatch):
    orig = E.texcoords

    def bad(d, S):
        phi = np.arctan2(d[..., 2], d[..., 0])
        theta = np.arccos(np.clip(d[..., 1], -1.0, 1.0))
        return (phi / (2.0 * np.pi) + 0.5) * S, theta / np.pi * S
    monkeypatch.setattr(E, "texcoords", bad)
    with pytest.raises(AssertionError):
        test_texcoords_closed_forms()


def test_mutant_undistort_sign_is_caught(monkeypatch):
    def bad(xd, yd, k1, k2, k3, p1, p2, iters=E.UNDISTORT_ITERS):
        a, b = np.array(xd, dtype=np.float64), np.array(yd, dtype=np.float64)
        for _ in range(iters):
            r2 = a * a + b * b
            D = 1.0 + k1 * r2 + k2 * r2 ** 2 + k3 * r2 ** 3
            dx = 2.0 * p1 * a * b + p2 * (r2 + 2.0 * a * a)
            dy = 2.0 * p2 * a * b + p1 * (r2 + 2.0 * b * b)
            a, b = (xd + dx) / D, (yd + dy) / D
        return a, b
    monkeypatch.setattr(E, "undistort", bad)
    with pytest.raises(AssertionError):
        test_undistort_inverts_the_distortion()


def test_mutant_bilinear_weights_swapped_is_caught(monkeypatch):
    orig = E.bilinear

    def bad(S, s, t):
        q = orig(S, s, t)
        return [(q[0][0], q[0][1], q[1][2]), (q[1][0], q[1][1], q[0][2]), q[2], q[3]]
    monkeypatch.setattr(E, "bilinear", bad)
    with pytest.raises(AssertionError):
        test_bilinear_reproduces_linear_maps_and_wraps()
