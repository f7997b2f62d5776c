"""Captured forward graphs (adop_forward_graph_create / _launch) against
direct renders: launches queued back to back on one stream, more of them
than the graph's camera staging slots, each with its own cameras; a copy of
every launch's frame, taken on the same stream, must equal a direct render
of that launch's cameras (keys and counts bit-exact, images within 1e-5
relative, as the FP32 sums may be added in another order)."""
import numpy as np
import pytest

from paper_2110_06635_amd import synth
from tests.gpu_parity_lib import say

pytestmark = pytest.mark.gpu


def _cams(k):
    """Two views of different sizes; view 0 moves with k, view 1 turns."""
    a = synth.Camera(320, 240, 300.0, 300.0, 160.0, 120.0, k1=-0.05, t=np.array([0.04 * k, 0.0, 12.0]))
    b = synth.Camera(200, 150, 220.0, 220.0, 100.0, 75.0, t=np.array([0.0, 0.1, 12.0]),
                     R=synth.rodrigues([0.0, 0.01 * k, 0.0]))
    return [a, b]


@pytest.mark.parametrize("record_visibility", [False, True])
def test_graph_launches_match_direct_renders(record_visibility):
    import torch
    from paper_2110_06635_amd import adop as A
    say(f"forward graph: 7 queued launches, record_visibility={record_visibility}")
    ctx = A.Context(0)
    rng = np.random.default_rng(21)
    pos = (rng.normal(0.0, 1.5, (40_000, 3))).astype(np.float32)
    feat = rng.random((40_000, 4)).astype(np.float32)
    dev = torch.device("cuda:0")
    scene = A.Scene.prepare(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(feat).to(dev))
    L = 3
    g = A.ForwardGraph(ctx, scene, _cams(0), L, record_visibility=record_visibility)
    outs = []
    for k in range(7):
        fr = g.launch(_cams(k))
        outs.append((k, fr.keys.clone(), fr.counts.clone(), fr.images.clone()))
    torch.cuda.synchronize()
    first_keys = outs[0][1]
    assert any(not torch.equal(first_keys, o[1]) for o in outs[1:]), "the cameras must give different frames"
    for k, keys, counts, images in outs:
        ref = A.render_forward(ctx, scene, _cams(k), L)
        torch.cuda.synchronize()
        assert torch.equal(keys, ref.keys), f"launch {k}: keys differ"
        assert torch.equal(counts, ref.counts), f"launch {k}: counts differ"
        d = (images.double() - ref.images.double()).abs()
        assert bool((d <= 1e-5 * ref.images.double().abs() + 1e-7).all()), f"launch {k}: images differ"
    g.close()
