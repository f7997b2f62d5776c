"""GPU parity of the optional passes against the oracle: normal culling (both
signs), logarithmic descriptors, stochastic discarding, the 4-NN radius
(bit-exact against the brute-force oracle; against a k-d tree at a size the
brute force cannot reach) and all of them together, through the C ABI."""
import numpy as np
import pytest

from paper_2110_06635_amd import synth
from tests.gpu_parity_lib import run_case, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G(oracle):
    import torch
    from paper_2110_06635_amd import adop
    return adop, adop.Context(0), oracle, torch


def _planes_scene(n_planes=30, per_plane=1200, seed=1202, w=320, h=240):
    pos, feat, nrm = synth.planes(n_planes, per_plane, 4, seed, box=3.0, half_lo=0.4, half_hi=1.5,
                                  with_normals=True)
    flip = synth.uniform01(n_planes, seed + 1) < 0.5        # both orientations
    nrm = nrm * np.where(np.repeat(flip, per_plane), -1.0, 1.0)[:, None].astype(np.float32)
    cam = synth.Camera(w, h, 0.8 * w, 0.8 * w, w / 2.0, h / 2.0, **synth.DIST2,
                       r2_max=synth.r2_max_for(**synth.DIST2), t=np.array([0.0, 0.0, 9.0]),
                       R=synth.rodrigues([0.1, -0.2, 0.05]))
    return synth.Scene(pos, feat, [cam], layers=4, name="planes-normals"), nrm.astype(np.float32)


@pytest.mark.parametrize("flag", ["backface", "printed"])
def test_normal_culling(G, flag):
    A, ctx, O, torch = G
    s, nrm = _planes_scene()
    f = A.FLAG_CULL_BACKFACE if flag == "backface" else A.FLAG_CULL_PRINTED
    say(f"normal culling {flag}: {s.n} points on planes, 320x240 L4")
    print(run_case(A, ctx, O, s, flags=f, normals=nrm))


def test_log_features(G):
    A, ctx, O, torch = G
    s, _ = _planes_scene(seed=1203)
    s.feat = (s.feat * 3.0 - 2.0).astype(np.float32)        # log descriptors in [-2, 1]
    say("logarithmic descriptors")
    print(run_case(A, ctx, O, s, flags=A.FLAG_LOG_FEATURES))
    say("logarithmic descriptors, BF16 storage")
    print(run_case(A, ctx, O, s, dtype="bf16", flags=A.FLAG_LOG_FEATURES))


def _discard_inputs(O, s, seed):
    radius = O.knn_radius(s.pos)
    beta = synth.uniform01(s.n, seed)
    return radius, beta


def test_discard(G):
    A, ctx, O, torch = G
    s, _ = _planes_scene(seed=1204)
    radius, beta = _discard_inputs(O, s, 1205)
    say("stochastic discarding, gamma 1.5, oracle radius")
    print(run_case(A, ctx, O, s, flags=A.FLAG_DISCARD, radius=radius, beta=beta, gamma=1.5))
    say("stochastic discarding, gamma 0.7")
    print(run_case(A, ctx, O, s, flags=A.FLAG_DISCARD, radius=radius, beta=beta, gamma=0.7))


def test_everything_together(G):
    A, ctx, O, torch = G
    s, nrm = _planes_scene(seed=1206)
    s.feat = (s.feat * 2.0 - 1.0).astype(np.float32)
    radius, beta = _discard_inputs(O, s, 1207)
    flags = A.FLAG_SPATIAL_ALL | A.FLAG_CULL_BACKFACE | A.FLAG_LOG_FEATURES | A.FLAG_DISCARD
    say("culling + log descriptors + discarding + spatial gradient for all points")
    print(run_case(A, ctx, O, s, flags=flags, normals=nrm, radius=radius, beta=beta))


def _knn_cloud(n, seed):
    """Clusters of very different density, a uniform background and planted
    duplicates."""
    rng = np.random.default_rng(seed)
    k = n // 4
    pos = np.concatenate([rng.normal(0.0, 0.05, (k, 3)), rng.normal(2.0, 0.5, (k, 3)),
                          rng.uniform(-4, 4, (n - 2 * k, 3))]).astype(np.float32)
    pos[10:40] = pos[1000:1030]
    return pos


def test_knn_radius_bit_exact(G):
    A, ctx, O, torch = G
    pos = _knn_cloud(12000, 1208)
    say("4-NN radius: 12k points vs brute-force oracle")
    t = torch.from_numpy(pos).cuda()
    scene = A.Scene.identity(t, torch.zeros((pos.shape[0], 4), device="cuda"))
    got = A.knn_radius(ctx, scene).cpu().numpy()
    ref = O.knn_radius(pos)
    assert np.array_equal(got, ref), int(np.sum(got != ref))


def test_knn_radius_prepared_scene_gather(G):
    """Radius of a Morton-prepared scene equals the caller-order radius
    gathered into the prepared order."""
    A, ctx, O, torch = G
    pos = _knn_cloud(8000, 1209)
    feat = torch.zeros((pos.shape[0], 4), device="cuda")
    scene = A.Scene.prepare(ctx, torch.from_numpy(pos).cuda(), feat)
    got = A.knn_radius(ctx, scene).cpu().numpy()
    ref = scene.gather(ctx, torch.from_numpy(O.knn_radius(pos)).cuda()).cpu().numpy()
    assert np.array_equal(got, ref)


def test_knn_radius_million_points_vs_kdtree(G):
    from scipy.spatial import cKDTree
    A, ctx, O, torch = G
    s = synth.config3(n=1_000_000, seed=1210)
    say("4-NN radius: 1M-point Gaussian mixture vs k-d tree")
    t = torch.from_numpy(s.pos).cuda()
    scene = A.Scene.identity(t, torch.zeros((s.n, 4), device="cuda"))
    got = A.knn_radius(ctx, scene).cpu().numpy().astype(np.float64)
    d, _ = cKDTree(s.pos.astype(np.float64)).query(s.pos.astype(np.float64), k=5, workers=8)
    # binary32 distances against float64 ones: a few units of rounding
    np.testing.assert_allclose(got, d[:, 4], rtol=2e-6, atol=1e-12)
