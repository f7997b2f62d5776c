"""Serving on the GPU: mixed-resolution requests batched as they arrive (fused
launches that mix resolution classes) give, for every request, the same image
as that camera rendered alone (floats within
1e-5 relative: both are FP32 sums, in different orders), and a sample matches
the CPU oracle."""
import numpy as np
import pytest

from paper_2110_06635_amd import serve, synth
from tests.gpu_parity_lib import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graphs", [True, False])
def test_served_equals_alone(oracle, graphs):
    import torch
    from paper_2110_06635_amd import adop
    say(f"serving equality graphs={graphs}")
    dev = torch.device("cuda:0")
    ctx = adop.Context(0)
    s = synth.config5_scene(n=1_000_000)
    raw, widened = synth.storage(s.feat, "bf16")
    scene = adop.Scene.prepare(ctx, torch.from_numpy(s.pos).to(dev),
                               torch.from_numpy(raw.view(np.int16)).to(dev).view(torch.bfloat16), adop.BF16)
    be = serve.GpuBackend(ctx, scene, layers=4, use_graphs=graphs)
    srv = serve.Server(be, 24 << 30, max_batch=4, max_inflight=3)
    # a burst queued before the scheduler starts: batches of several views
    # are formed and several batches are on the GPU at once
    burst = [srv.submit(cam) for _, cam in synth.config5_requests(24, seed=78)]
    srv.start()
    for r in burst:
        assert r.done.wait(120)
    st = srv.stats()
    print("burst", st)
    assert st["completed"] == len(burst) and st["failed"] == 0
    assert st["max_batch"] > 1, "no batch held more than one view"
    assert st["peak_inflight"] > 1, "batches never overlapped on the GPU"
    assert st["mixed_batches"] > 0, "no batch mixed resolution classes"
    mixed = [r for r in burst if sum(q.batch_id == r.batch_id for q in burst) > 1]
    assert len(mixed) >= 4
    # then a Poisson trace while the server runs
    tr = synth.config5_requests(48, rate=400.0, seed=77)
    reqs = burst + serve.replay(srv, tr)
    srv.close()
    st = srv.stats()
    print(st)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    worst = 0.0
    for r in reqs:
        fr = adop.render_forward(ctx, scene, [r.camera], 4)
        alone = fr.images
        torch.cuda.synchronize()
        got = r.result
        assert got.shape == alone.shape
        err = (got.double() - alone.double()).abs()
        lim = 1e-5 * alone.double().abs() + 1e-7
        assert bool((err <= lim).all()), float((err / (alone.double().abs() + 1e-7)).max())
        worst = max(worst, float((err / (alone.double().abs() + 1e-7)).max()))
    print("worst relative difference served vs alone", worst)
    # a sample against the oracle (bf16 features widened exactly)
    for r in reqs[:4]:
        ref = oracle.forward(s.pos, widened, [r.camera], 4, want64=True)
        got = r.result.cpu().numpy().astype(np.float64)
        err = np.abs(got - ref["images64"])
        assert np.all(err <= 1e-5 * np.abs(ref["images64"]) + 1e-7)
