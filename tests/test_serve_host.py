"""Scheduling policies of the render server, on the CPU with a fake backend
whose launches take a known time and whose allocations are tracked:
admission and eviction by memory (slots included), mixed-class and
class-homogeneous batches, overlap of in-flight batches, failure isolation,
reproducible traces."""
import threading
import time

import numpy as np
import pytest

from paper_2110_06635_amd import serve, synth


class FakeBackend(serve.Backend):
    """Launches take a known time; every slot and every in-flight output is
    an allocation whose live total is tracked."""

    def __init__(self, per_view_s=0.004, fixed_s=0.002, fail_launch=None):
        self.per_view_s = per_view_s
        self.fixed_s = fixed_s
        self.launches = []
        self.live = 0
        self.max_live = 0
        self.live_bytes = 0
        self.max_live_bytes = 0
        self.slots_alive = 0
        self.lock = threading.Lock()
        self.fail_launch = fail_launch

    def _alloc(self, nb):
        with self.lock:
            self.live_bytes += nb
            self.max_live_bytes = max(self.max_live_bytes, self.live_bytes)

    def out_bytes(self, klass):
        return klass[0] * klass[1] * 16

    def slot_bytes(self, combo):
        return sum(w * h * 12 for w, h in combo)

    def create_slot(self, combo):
        nb = self.slot_bytes(combo)
        self._alloc(nb)
        self.slots_alive += 1
        return {"combo": tuple(combo), "bytes": nb, "alive": True}

    def destroy_slot(self, slot):
        assert slot["alive"]
        slot["alive"] = False
        self.slots_alive -= 1
        self._alloc(-slot["bytes"])

    def launch(self, slot, cams, lane):
        assert slot["alive"]
        assert tuple((c.width, c.height) for c in cams) == slot["combo"]
        if self.fail_launch is not None and self.fail_launch(len(self.launches)):
            self.launches.append(None)
            raise RuntimeError("backend error")
        t = time.perf_counter()
        ob = sum(self.out_bytes((c.width, c.height)) for c in cams)
        self._alloc(ob)
        h = {"start": t, "end": t + self.fixed_s + self.per_view_s * len(cams), "cams": list(cams),
             "lane": lane, "out": ob}
        with self.lock:
            self.launches.append(h)
            self.live += 1
            self.max_live = max(self.max_live, self.live)
        return h

    def poll(self, h):
        return time.perf_counter() >= h["end"]

    def finish(self, h):
        with self.lock:
            self.live -= 1
        return [("img", c.width, c.height, id(c)) for c in h["cams"]]

    def release(self, h):
        self._alloc(-h["out"])   # the outputs leave the server with the completion


def trace(n, rate=400.0, seed=2005):
    return synth.config5_requests(n, rate=rate, seed=seed)


def test_trace_reproducible():
    a = trace(50)
    b = trace(50)
    assert [t for t, _ in a] == [t for t, _ in b]
    assert [(c.width, np.asarray(c.R).tobytes()) for _, c in a] == [(c.width, np.asarray(c.R).tobytes()) for _, c in b]
    counts = {}
    for _, c in trace(4000):
        counts[c.width] = counts.get(c.width, 0) + 1
    frac = np.array([counts[w] for w, _ in synth.SERVE_CLASSES]) / 4000
    np.testing.assert_allclose(frac, [0.4, 0.3, 0.2, 0.1], atol=0.03)
    gaps = np.diff([t for t, _ in trace(4000)])
    assert abs(gaps.mean() - 1 / 400.0) < 0.1 / 400.0


@pytest.mark.parametrize("mix", [True, False])
def test_batches_and_admission_by_memory(mix):
    fb = FakeBackend()
    budget = 3840 * 2160 * 28 * 3          # about three 4K views of outputs + slots
    srv = serve.Server(fb, budget, max_batch=6, max_inflight=3, mix_classes=mix)
    srv.start()
    reqs = serve.replay(srv, trace(300))
    srv.stop()
    st = srv.stats()
    assert st["completed"] == 300 and st["failed"] == 0
    assert srv._peak <= budget
    assert fb.max_live_bytes <= budget    # real allocations, slots included
    for h in fb.launches:
        assert 1 <= len(h["cams"]) <= 6
        if not mix:
            assert len({(c.width, c.height) for c in h["cams"]}) == 1     # one class per batch
    if mix:
        assert st["mixed_batches"] > 0
    assert st["mean_batch"] > 1.0          # requests arriving during a batch get batched
    assert fb.max_live >= 2                # batches overlapped on the device
    for r in reqs:
        assert r.result[1:3] == (r.camera.width, r.camera.height)
        assert r.result[3] == id(r.camera)


def test_cached_slots_count_against_the_budget():
    """A budget that holds only a few slots: idle slots are evicted to make
    room, live allocations (slots + in-flight outputs) never exceed it, and
    every request still completes."""
    fb = FakeBackend(per_view_s=0.001, fixed_s=0.0005)
    budget = 3840 * 2160 * 28 * 2 + 1920 * 1080 * 28 * 2
    srv = serve.Server(fb, budget, max_batch=4, max_inflight=3)
    srv.start()
    reqs = serve.replay(srv, trace(400, rate=2000.0))
    srv.stop()
    st = srv.stats()
    assert st["completed"] == 400 and st["failed"] == 0 and st["rejected"] == 0
    assert fb.max_live_bytes <= budget
    assert st["peak_mem_bytes"] <= budget
    assert st["evictions"] > 0 and st["slots_created"] > st["evictions"]
    assert fb.slots_alive == len(srv._slots)
    srv.close()
    assert fb.slots_alive == 0 and fb.live_bytes == 0
    assert all(r.result[1:3] == (r.camera.width, r.camera.height) for r in reqs)


def test_slot_reused_when_idle():
    fb = FakeBackend(per_view_s=0.0005, fixed_s=0.0002)
    srv = serve.Server(fb, 10 ** 10, max_batch=1, max_inflight=1)
    srv.start()
    cam = synth.Camera(640, 480, 500.0, 500.0, 320.0, 240.0)
    for _ in range(5):
        srv.wait(srv.submit(cam), 5)
    srv.stop()
    assert srv.stats()["slots_created"] == 1 and len(fb.launches) == 5


def test_oversized_request_rejected():
    fb = FakeBackend()
    srv = serve.Server(fb, budget_bytes := 640 * 480 * 28 * 2, max_batch=4)
    srv.start()
    big = synth.Camera(3840, 2160, 1000.0, 1000.0, 1920.0, 1080.0)
    small = synth.Camera(640, 480, 500.0, 500.0, 320.0, 240.0)
    r1 = srv.submit(big)
    r2 = srv.submit(small)
    with pytest.raises(RuntimeError):
        srv.wait(r1, 5)
    assert srv.wait(r2, 5)[1] == 640
    srv.stop()
    assert srv.stats()["rejected"] == 1


def test_failure_isolated_to_its_batch():
    fb = FakeBackend()
    srv = serve.Server(fb, 10 ** 10, max_batch=4, max_inflight=2)
    srv.fail_hook = lambda bid: bid == 3
    srv.start()
    reqs = serve.replay(srv, trace(120))
    srv.stop()
    bad = [r for r in reqs if r.error]
    assert bad and all(r.batch_id == 3 for r in bad)
    assert srv.stats()["errors"] == {"render failed: injected failure": len(bad)}
    good = [r for r in reqs if not r.error]
    assert len(good) + len(bad) == 120 and len(good) > 100
    assert all(r.result is not None for r in good)


def test_backend_exception_isolated():
    fb = FakeBackend(fail_launch=lambda k: k == 5)
    srv = serve.Server(fb, 10 ** 10, max_batch=4, max_inflight=2)
    srv.start()
    reqs = serve.replay(srv, trace(100))
    srv.stop()
    bad = {r.batch_id for r in reqs if r.error}
    assert len(bad) == 1
    assert sum(1 for r in reqs if not r.error) >= 90


def test_unbatched_baseline_is_fifo():
    fb = FakeBackend(per_view_s=0.001, fixed_s=0.0005)
    srv = serve.Server(fb, 10 ** 10, max_batch=1, max_inflight=1)
    srv.start()
    reqs = serve.replay(srv, trace(80))
    srv.stop()
    order = [h["cams"][0] for h in fb.launches]
    assert order == [r.camera for r in sorted(reqs, key=lambda r: r.rid)]
    assert fb.max_live == 1


def test_results_released_when_not_kept():
    """keep_results=False: completions and latencies are recorded, the
    images are not held by the requests."""
    fb = FakeBackend(per_view_s=0.001, fixed_s=0.0005)
    srv = serve.Server(fb, 10 ** 10, max_batch=4, max_inflight=2, keep_results=False)
    srv.start()
    reqs = serve.replay(srv, trace(100))
    srv.stop()
    st = srv.stats()
    assert st["completed"] == 100 and st["failed"] == 0 and st["errors"] == {}
    assert all(r.result is None and r.error is None and r.latency > 0 for r in reqs)
