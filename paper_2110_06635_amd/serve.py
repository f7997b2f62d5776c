"""Continuous-batching render server for novel views of a resident scene.

One scheduler thread owns the GPU work:
  * requests (a camera each) wait in a FIFO queue, stamped with their
    scheduled arrival time;
  * a batch is formed from the oldest request and the following requests of
    the same resolution class (up to `max_batch`) whose output memory fits in
    the free part of the memory budget; it is launched as ONE fused
    multi-view forward (every point is read once and projected into all the
    batch's views) by replaying a HIP graph captured for (class, batch size);
  * up to `max_inflight` batches run at once, each on its own stream, so a
    batch is admitted while others are still on the GPU; a finished batch's
    images are copied to per-request tensors and its graph buffers are
    reused;
  * a render call that fails fails only the requests of its batch;
  * with keep_results=False a request's images are released as soon as its
    completion is recorded (a client that consumes each frame as it
    arrives), so a long trace does not accumulate output memory.
Latency is measured from the scheduled arrival to the moment the host sees
the batch's completion event.

The GPU specifics live in `GpuBackend`; `Server` only schedules, so its
policies (admission by memory, batching, failure isolation) are testable on
the CPU with a fake backend.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Any, Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    camera: Any
    klass: Tuple[int, int]
    arrival: float                 # scheduled arrival (time.perf_counter base)
    out_bytes: int = 0
    done: threading.Event = dataclasses.field(default_factory=threading.Event)
    result: Any = None
    error: Optional[str] = None
    t_done: float = 0.0
    batch_id: int = -1

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Backend:
    """Interface the scheduler drives."""

    def out_bytes(self, klass) -> int:
        raise NotImplementedError

    def slot_bytes(self, klass, batch: int) -> int:
        """Device memory of one reusable batch slot (frame + workspace)."""
        raise NotImplementedError

    def launch(self, klass, cams: Sequence, lane: int) -> Any:
        """Enqueue a fused forward of `cams` on execution lane `lane`; return
        a handle for poll()/finish()."""
        raise NotImplementedError

    def poll(self, handle) -> bool:
        raise NotImplementedError

    def finish(self, handle) -> List[Any]:
        """Per-view results of a completed launch."""
        raise NotImplementedError

    def release(self, handle) -> None:
        pass


class Server:
    def __init__(self, backend: Backend, mem_budget_bytes: int, max_batch: int = 8,
                 max_inflight: int = 3, idle_sleep: float = 50e-6, keep_results: bool = True):
        self.backend = backend
        self.keep_results = keep_results
        self.budget = int(mem_budget_bytes)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.idle_sleep = idle_sleep
        self._q: "collections.deque[Request]" = collections.deque()
        self._lock = threading.Lock()
        self._inflight: List[Tuple[int, Any, List[Request], int]] = []
        self._used = 0
        self._peak = 0
        self._next_id = 0
        self._next_batch = 0
        self._stop = False
        self._thread: Optional[threading.Thread] = None
        self.completed: List[Request] = []
        self.rejected = 0
        self.batches = 0
        self.batch_sizes: List[int] = []
        self.peak_inflight = 0          # most batches on the GPU at once
        self.fail_hook: Optional[Callable[[int], bool]] = None   # test hook: batch id -> fail?

    # ---------------------------------------------------------------- client
    def submit(self, camera, arrival: Optional[float] = None) -> Request:
        klass = (int(camera.width), int(camera.height))
        ob = self.backend.out_bytes(klass)
        with self._lock:
            rid = self._next_id
            self._next_id += 1
        r = Request(rid, camera, klass, time.perf_counter() if arrival is None else arrival, ob)
        if ob + self.backend.slot_bytes(klass, 1) > self.budget:
            r.error = "request larger than the memory budget"
            r.t_done = time.perf_counter()
            r.done.set()
            with self._lock:
                self.rejected += 1
            return r
        with self._lock:
            self._q.append(r)
        return r

    def wait(self, r: Request, timeout: Optional[float] = None):
        if not r.done.wait(timeout):
            raise TimeoutError(f"request {r.rid} not done")
        if r.error:
            raise RuntimeError(r.error)
        return r.result

    # ------------------------------------------------------------- scheduler
    def start(self):
        self._stop = False
        self._thread = threading.Thread(target=self._loop, name="adop-serve", daemon=True)
        self._thread.start()

    def stop(self, drain: bool = True, timeout: float = 120.0):
        t0 = time.perf_counter()
        if drain:
            while True:
                with self._lock:
                    busy = bool(self._q) or bool(self._inflight)
                if not busy or time.perf_counter() - t0 > timeout:
                    break
                time.sleep(1e-3)
        self._stop = True
        if self._thread:
            self._thread.join(timeout)

    def _free(self) -> int:
        return self.budget - self._used

    def _form_batch(self) -> Optional[List[Request]]:
        with self._lock:
            if not self._q:
                return None
            head = self._q[0]
            klass = head.klass
            batch = []
            for r in list(self._q):
                if r.klass != klass:
                    continue
                if len(batch) >= self.max_batch:
                    break
                need = sum(x.out_bytes for x in batch) + r.out_bytes + \
                    self.backend.slot_bytes(klass, len(batch) + 1)
                if need > self._free():
                    break
                batch.append(r)
            if not batch:
                return None
            for r in batch:
                self._q.remove(r)
            return batch

    def _loop(self):
        lanes = list(range(self.max_inflight))
        while not self._stop:
            progressed = False
            # completions
            for item in list(self._inflight):
                bid, h, batch, lane = item
                if self.backend.poll(h):
                    try:
                        outs = self.backend.finish(h)
                        err = None
                    except Exception as e:   # a failed launch fails its batch only
                        outs, err = [None] * len(batch), f"render failed: {e}"
                    now = time.perf_counter()
                    for r, o in zip(batch, outs):
                        r.result, r.error, r.t_done = (o if self.keep_results else None), err, now
                        r.done.set()
                    outs = None
                    self.backend.release(h)
                    with self._lock:
                        self._inflight.remove(item)
                        self._used -= sum(r.out_bytes for r in batch) + \
                            self.backend.slot_bytes(batch[0].klass, len(batch))
                        self.completed.extend(batch)
                    lanes.append(lane)
                    progressed = True
            # admissions
            while lanes:
                batch = self._form_batch()
                if batch is None:
                    break
                klass = batch[0].klass
                bid = self._next_batch
                self._next_batch += 1
                mem = sum(r.out_bytes for r in batch) + self.backend.slot_bytes(klass, len(batch))
                lane = lanes.pop(0)
                try:
                    if self.fail_hook is not None and self.fail_hook(bid):
                        raise RuntimeError("injected failure")
                    h = self.backend.launch(klass, [r.camera for r in batch], lane)
                except Exception as e:
                    now = time.perf_counter()
                    for r in batch:
                        r.error, r.t_done, r.batch_id = f"render failed: {e}", now, bid
                        r.done.set()
                    with self._lock:
                        self.completed.extend(batch)
                    lanes.append(lane)
                    continue
                for r in batch:
                    r.batch_id = bid
                with self._lock:
                    self._used += mem
                    self._peak = max(self._peak, self._used)
                    self._inflight.append((bid, h, batch, lane))
                    self.peak_inflight = max(self.peak_inflight, len(self._inflight))
                self.batches += 1
                self.batch_sizes.append(len(batch))
                progressed = True
            if not progressed:
                time.sleep(self.idle_sleep)

    # ----------------------------------------------------------------- stats
    def stats(self) -> Dict[str, Any]:
        ok = [r for r in self.completed if r.error is None]
        lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
        per_class = {}
        for k in sorted({r.klass for r in ok}):
            lk = np.array([r.latency for r in ok if r.klass == k])
            per_class[f"{k[0]}x{k[1]}"] = {"n": int(lk.size), "p50_ms": float(np.percentile(lk, 50) * 1e3),
                                           "p99_ms": float(np.percentile(lk, 99) * 1e3)}
        span = (max(r.t_done for r in ok) - min(r.arrival for r in ok)) if ok else 0.0
        errors = collections.Counter(r.error for r in self.completed if r.error is not None)
        return {"completed": len(ok), "failed": len(self.completed) - len(ok), "rejected": self.rejected,
                "errors": dict(errors.most_common(3)),
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "renders_per_s": len(ok) / span if span > 0 else 0.0,
                "batches": self.batches,
                "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
                "max_batch": int(max(self.batch_sizes)) if self.batch_sizes else 0,
                "peak_inflight": int(self.peak_inflight),
                "peak_mem_bytes": int(self._peak), "per_class": per_class}


def replay(server: Server, trace: Sequence[Tuple[float, Any]], warmup: int = 0):
    """Submit a trace of (arrival offset s, camera) at its scheduled times;
    returns the measured requests (after `warmup`)."""
    t0 = time.perf_counter() + 0.05
    reqs = []
    for k, (ta, cam) in enumerate(trace):
        target = t0 + ta
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            time.sleep(min(target - now, 1e-3))
        reqs.append(server.submit(cam, arrival=target))
    for r in reqs:
        r.done.wait(300)
    return reqs[warmup:]


# ---------------------------------------------------------------------------
# GPU backend
# ---------------------------------------------------------------------------

class GpuBackend(Backend):
    """Fused multi-view forward of a batch of same-size views, replayed from a
    HIP graph captured per (class, batch size, lane)."""

    def __init__(self, ctx, scene, layers: int = 4, alpha: float = 0.01, use_graphs: bool = True):
        import torch
        from . import adop
        self.torch = torch
        self.adop = adop
        self.ctx = ctx
        self.scene = scene
        self.layers = layers
        self.alpha = alpha
        self.use_graphs = use_graphs
        self.C = scene.channels
        self.dev = scene.x.device
        self.streams = {}
        self.slots: Dict[Tuple[Tuple[int, int], int, int], Any] = {}

    def _pixels(self, klass, b=1):
        w, h = klass
        return b * sum((w >> l) * (h >> l) for l in range(self.layers))

    def out_bytes(self, klass) -> int:
        return self._pixels(klass) * self.C * 4

    def slot_bytes(self, klass, batch: int) -> int:
        px = self._pixels(klass, batch)
        return px * (self.C * 4 + 8 + 4) + self.ctx.workspace_bytes(self.C, batch, px)

    def _stream(self, lane):
        if lane not in self.streams:
            self.streams[lane] = self.torch.cuda.Stream(device=self.dev)
        return self.streams[lane]

    def _slot(self, klass, cams, lane):
        key = (klass, len(cams), lane)
        s = self.slots.get(key)
        if s is None:
            if self.use_graphs:
                s = self.adop.ForwardGraph(self.ctx, self.scene, cams, self.layers, alpha=self.alpha)
            else:
                fr = self.adop.Frame(cams, self.layers, self.C, self.dev)
                ws = self.torch.empty(self.ctx.workspace_bytes(self.C, len(cams), fr.pixels),
                                      dtype=self.torch.uint8, device=self.dev)
                s = (fr, ws)
            self.slots[key] = s
        return s

    def launch(self, klass, cams, lane):
        torch = self.torch
        st = self._stream(lane)
        slot = self._slot(klass, cams, lane)
        if self.use_graphs:
            frame = slot.launch(cams, stream=st)
        else:
            fr, ws = slot
            frame = self.adop.render_forward(self.ctx, self.scene, cams, self.layers, alpha=self.alpha,
                                             frame=fr, workspace=ws, stream=st, record_visibility=False)
        with torch.cuda.stream(st):
            outs = [frame.images[self.C * int(frame.offsets[v, 0]):
                                 self.C * (int(frame.offsets[v, 0]) + self._pixels(klass))].clone()
                    for v in range(len(cams))]
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, outs)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle):
        return handle[1]


class PlainBackend(GpuBackend):
    """The unbatched baseline: FP32 scene, eager launches, one view at a time."""

    def __init__(self, ctx, scene, layers: int = 4, alpha: float = 0.01):
        super().__init__(ctx, scene, layers, alpha, use_graphs=False)
