"""Pins of the tone-mapper oracle (Sec. 3.3) against what the paper and the
mathematics fix: closed forms of each stage, the leaky response's
continuity and limit (Eq. resonseleak), the exposure scaling, hand-computed
terms on one pixel, and central finite differences of the forward for every
gradient (the derivatives are written out by hand, the FD uses only the
forward).  Planted mistakes in the oracle must fail a pin."""
import numpy as np
import pytest

from oracle import tonemap as T


def _case(seed=0, V=2, h=4, w=5, K=8, spread=True):
    rng = np.random.default_rng(seed)
    hdr = rng.uniform(-0.3, 1.6, (V, 3, h, w)) if spread else rng.uniform(0.05, 0.95, (V, 3, h, w))
    ev = rng.uniform(-0.5, 0.5, V)
    white = rng.uniform(0.8, 1.2, (V, 3))
    white[:, 1] = 1.0
    vig = np.array([-0.3, 0.1, -0.05, 0.45, 0.55])
    crf = np.sort(rng.uniform(0, 1, (3, K)), axis=1)
    crf[:, 0], crf[:, -1] = 0.0, 1.0
    return hdr, ev, white, vig, crf


def test_identity_settings_are_the_leaky_identity():
    K = 17
    lin = np.tile(np.arange(K) / (K - 1), (3, 1))
    hdr = np.linspace(-2.0, 5.0, 3 * 7 * 11).reshape(1, 3, 7, 11)
    out = T.forward(hdr, np.zeros(1), np.ones((1, 3)), np.array([0, 0, 0, 0.5, 0.5]), lin, leak=0.01)
    want = np.where(hdr < 0, 0.01 * hdr, np.where(hdr > 1, -0.01 / np.sqrt(np.maximum(hdr, 1)) + 1.01, hdr))
    np.testing.assert_allclose(out, want, rtol=1e-15, atol=1e-15)
    clamp = T.forward(hdr, np.zeros(1), np.ones((1, 3)), np.array([0, 0, 0, 0.5, 0.5]), lin, leak=-1.0)
    np.testing.assert_allclose(clamp, np.clip(hdr, 0, 1), rtol=1e-15, atol=1e-15)


def test_leaky_response_continuity_and_limit():
    crf = T.gamma_table(256)
    t = crf[0]
    eps = 1e-12
    for leak in (0.01, 0.2):
        r = lambda x: T.response(np.array([x]), t, leak)[0]
        assert abs(r(0.0)) == 0.0 and abs(r(-eps)) < 1e-12
        assert r(1.0) == 1.0 and abs(r(1.0 + eps) - 1.0) < 1e-11
        assert abs(r(1e24) - (1.0 + leak)) < 1e-11          # R_t(inf) = 1 + leak
        assert r(-3.0) == -3.0 * leak


def test_gamma_table_nodes_and_interpolation():
    K = 33
    crf = T.gamma_table(K)
    xs = np.arange(K) / (K - 1)
    np.testing.assert_allclose(T.response(xs, crf[1], 0.01), xs ** 0.45, rtol=1e-15, atol=1e-15)
    mid = (xs[:-1] + xs[1:]) / 2
    np.testing.assert_allclose(T.response(mid, crf[1], 0.01), (xs[:-1] ** 0.45 + xs[1:] ** 0.45) / 2,
                               rtol=1e-14, atol=1e-15)


def test_exposure_halves_per_stop_and_white_point_scales():
    hdr, ev, white, vig, crf = _case(1)
    a = T.forward(hdr, ev + 1.0, white, vig, crf)
    b = T.forward(hdr / 2.0, ev, white, vig, crf)
    np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-15)
    w2 = white.copy()
    w2[:, 0] *= 2.0
    c = T.forward(hdr, ev, w2, vig, crf)
    h2 = hdr.copy()
    h2[:, 0] *= 2.0
    np.testing.assert_allclose(c, T.forward(h2, ev, white, vig, crf), rtol=1e-14, atol=1e-15)


def test_vignette_closed_form():
    # odd image: the centre pixel sits at (0.5, 0.5), r = 0; a corner pixel at
    # ((0.5/w), (0.5/h)) from a centre at (0.5, 0.5)
    w, h = 5, 3
    vig = np.array([0.4, -0.2, 0.1, 0.5, 0.5])
    f = T.vignette_factor(w, h, vig)
    assert f[1, 2] == 1.0
    r2 = (0.5 / w - 0.5) ** 2 + (0.5 / h - 0.5) ** 2
    assert abs(f[0, 0] - (1 + 0.4 * r2 - 0.2 * r2 ** 2 + 0.1 * r2 ** 3)) < 1e-15


def test_one_pixel_terms_by_hand():
    """A 1x1 image: every gradient is a single term, written out here from
    the chain rule of the four stages."""
    hdr = np.array([0.6, 0.3, 0.2]).reshape(1, 3, 1, 1)
    ev, white = np.array([0.25]), np.array([[1.1, 1.0, 0.9]])
    vig = np.array([0.2, 0.1, 0.05, 0.3, 0.4])
    K = 5
    crf = T.gamma_table(K)
    g = np.array([1.0, -2.0, 0.5]).reshape(1, 3, 1, 1)
    (dh, dev, dw, dv, dc), (ah, aev, aw, av, ac) = T.backward(hdr, ev, white, vig, crf, g)
    r2 = (0.5 - 0.3) ** 2 + (0.5 - 0.4) ** 2
    Vf = 1 + 0.2 * r2 + 0.1 * r2 ** 2 + 0.05 * r2 ** 3
    s = 2.0 ** -0.25
    for c in range(3):
        x = hdr[0, c, 0, 0] * s * white[0, c] * Vf
        i = int(np.floor(x * (K - 1)))
        slope = (crf[c, i + 1] - crf[c, i]) * (K - 1)
        gx = g[0, c, 0, 0] * slope
        assert abs(dh[0, c, 0, 0] - gx * Vf * white[0, c] * s) < 1e-14
        assert abs(dw[0, c] - gx * Vf * hdr[0, c, 0, 0] * s) < 1e-14
    terms = [g[0, c, 0, 0] * (crf[c, int(np.floor(hdr[0, c, 0, 0] * s * white[0, c] * Vf * (K - 1))) + 1]
                              - crf[c, int(np.floor(hdr[0, c, 0, 0] * s * white[0, c] * Vf * (K - 1)))]) * (K - 1)
             * hdr[0, c, 0, 0] * s * white[0, c] * Vf * -np.log(2.0) for c in range(3)]
    assert abs(dev[0] - sum(terms)) < 1e-14
    assert abs(aev[0] - sum(abs(t) for t in terms)) < 1e-14


def _fd(fn, x, h):
    xp, xm = x.copy(), x.copy()
    out = np.empty(x.size)
    for k in range(x.size):
        xp.flat[k] += h
        xm.flat[k] -= h
        out[k] = (fn(xp) - fn(xm)) / (2 * h)
        xp.flat[k] = x.flat[k]
        xm.flat[k] = x.flat[k]
    return out.reshape(x.shape)


@pytest.mark.parametrize("leak", [0.01, -1.0])
def test_gradients_match_finite_differences(leak):
    hdr, ev, white, vig, crf = _case(2)
    g = np.random.default_rng(3).normal(size=hdr.shape)
    L = lambda hd=hdr, e=ev, wt=white, vg=vig, cr=crf: float(np.sum(T.forward(hd, e, wt, vg, cr, leak) * g))
    (dh, dev, dw, dv, dc), absd = T.backward(hdr, ev, white, vig, crf, g, leak)
    h = 1e-6
    np.testing.assert_allclose(dh, _fd(lambda x: L(hd=x), hdr, h), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(dev, _fd(lambda x: L(e=x), ev, h), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(dw, _fd(lambda x: L(wt=x), white, h), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(dv, _fd(lambda x: L(vg=x), vig, h), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(dc, _fd(lambda x: L(cr=x), crf, h), rtol=1e-5, atol=1e-7)
    # the tolerance yardstick bounds every entry (triangle inequality)
    for d, a in zip((dh, dev, dw, dv, dc), absd):
        assert np.all(a >= np.abs(d) - 1e-15)


# ---- planted mistakes: each must make a pin above fail --------------------

def _mutant(monkeypatch, name, fn):
    monkeypatch.setattr(T, name, fn)


def test_mutant_vignette_in_r_not_r2_is_caught(monkeypatch):
    orig = T.vignette_factor

    def bad(w, h, vig):
        a2, a4, a6, cx, cy = vig
        px, py = T._coords(w, h)
        r = np.sqrt((px - cx) ** 2 + (py - cy) ** 2)
        return 1.0 + a2 * r + a4 * r ** 2 + a6 * r ** 3
    _mutant(monkeypatch, "vignette_factor", bad)
    with pytest.raises(AssertionError):
        test_vignette_closed_form()
    monkeypatch.setattr(T, "vignette_factor", orig)


def test_mutant_exposure_multiplies_is_caught(monkeypatch):
    orig = T.forward

    def bad(hdr, ev, white, vig, crf, leak=0.01):
        return orig(hdr, -np.asarray(ev), white, vig, crf, leak)
    _mutant(monkeypatch, "forward", bad)
    with pytest.raises(AssertionError):
        test_exposure_halves_per_stop_and_white_point_scales()


def test_mutant_leak_limit_is_caught(monkeypatch):
    orig = T.response

    def bad(x, table, leak):
        out = orig(x, table, leak)
        return np.where(np.asarray(x) > 1, -leak / np.asarray(x) + leak + 1.0, out)   # 1/x instead of 1/sqrt(x)
    _mutant(monkeypatch, "response", bad)
    with pytest.raises(AssertionError):
        test_identity_settings_are_the_leaky_identity()


def test_mutant_centre_gradient_sign_is_caught(monkeypatch):
    orig = T.backward

    def bad(*a, **k):
        (dh, dev, dw, dv, dc), absd = orig(*a, **k)
        dv = dv.copy()
        dv[3] = -dv[3]
        return (dh, dev, dw, dv, dc), absd
    _mutant(monkeypatch, "backward", bad)
    with pytest.raises(AssertionError):
        test_gradients_match_finite_differences(0.01)
