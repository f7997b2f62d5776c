"""GPU parity of the backward's record paths (Sec. 3.1, "Backward Pass") and
of the feature prefetch for every row width, against the oracle.

* A line of points along the ray through one pixel centre: every working lane
  of every wave sits on one pixel at every layer, so the records come from
  the wave-wide (scalar) loads.
* A tight cluster: waves mix one-pixel layers with layers whose lanes span
  several pixels (the per-lane gathers).
Both run with FP32, BF16 and FP16 features at C = 4 (a 16- or 8-byte row,
loaded as vectors) and C = 3 (12- and 6-byte rows, loaded per element), with
and without the forward's blend-set bits.  Bounds as in the other parity
tests: keys and counts bit-exact, images 1e-5 relative, dfeat 1e-5 S, dpos
1e-4 S, pose and intrinsics 1e-5 S."""
import numpy as np
import pytest

from paper_2110_06635_amd import synth
from tests.gpu_parity_lib import run_case, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G(oracle):
    from paper_2110_06635_amd import adop
    return adop, adop.Context(0), oracle


def _camera():
    return synth.Camera(320, 240, 400.0, 400.0, 160.0, 120.0, t=np.array([0.0, 0.0, 15.0]))


def _line_scene(n, C, seed):
    """Points on the ray through pixel centre (168, 128), which stays an
    integer at layers 0-3 (168, 84, 42, 21; 128, 64, 32, 16): one image
    position, depths spread over 1.5 % (inside and beyond the fuzzy window of
    alpha = 0.01)."""
    rng = np.random.default_rng(seed)
    cam = _camera()
    z = np.sort(rng.uniform(15.0, 15.0 * 1.015, n))          # camera depth
    u, v = 168.0, 128.0
    x = (u - cam.cx) / cam.fx * z
    y = (v - cam.cy) / cam.fy * z
    pos = np.stack([x, y, z - 15.0], axis=1).astype(np.float32)
    pos = pos[rng.permutation(n)]
    feat = rng.random((n, C)).astype(np.float32)
    return synth.Scene(pos, feat, [cam], layers=4, name=f"line-{n}")


def _cluster_scene(n, C, seed):
    rng = np.random.default_rng(seed)
    pos = (rng.normal(0.0, 0.03, (n, 3)) + [0.2, -0.1, 0.0]).astype(np.float32)
    feat = rng.random((n, C)).astype(np.float32)
    return synth.Scene(pos, feat, [_camera()], layers=5, name=f"cluster-{n}")


@pytest.mark.parametrize("shape", ["line", "cluster"])
@pytest.mark.parametrize("C,dtype", [(4, "f32"), (4, "bf16"), (4, "f16"), (3, "f32"), (3, "bf16")])
def test_backward_record_paths(G, shape, C, dtype):
    A, ctx, oracle = G
    say(f"backward record paths: {shape}, C={C}, {dtype}")
    s = (_line_scene if shape == "line" else _cluster_scene)(20_000, C, 11 + C)
    for vis in (True, False):
        rep = run_case(A, ctx, oracle, s, dtype=dtype, visibility=vis)
        assert rep["dfeat"] <= 1e-5 and rep["dpos"] <= 1e-4


def test_line_scene_is_one_pixel_per_layer():
    """The line scene's premise (host arithmetic only): every point projects,
    in float64, within 1e-4 px of the same pixel centre, so each layer's
    pixel is shared by all points."""
    s = _line_scene(20_000, 4, 15)
    cam = s.cams[0]
    X = s.pos.astype(np.float64) + np.asarray(cam.t)
    u = cam.fx * X[:, 0] / X[:, 2] + cam.cx
    v = cam.fy * X[:, 1] / X[:, 2] + cam.cy
    assert np.max(np.abs(u - 168.0)) < 1e-4 and np.max(np.abs(v - 128.0)) < 1e-4
