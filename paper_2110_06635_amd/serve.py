"""Continuous-batching render server for novel views of a resident scene.

One scheduler thread owns the GPU work:
  * requests (a camera each) wait in a FIFO queue, stamped with their
    scheduled arrival time;
  * a batch is formed from the oldest request and the requests after it (of
    any resolution class, or of the head's class only with
    mix_classes=False), up to `max_batch`, as long as its memory fits the
    budget; it is launched as ONE fused multi-view forward (every point is
    read once per pass and projected into all the batch's views) on a batch
    slot: a HIP graph captured for the batch's multiset of classes, with its
    frame and workspace;
  * up to `max_inflight` batches run at once, each on its own stream, so a
    batch is admitted while others are still on the GPU;
  * a render call that fails fails only the requests of its batch;
  * with keep_results=False a request's images are released as soon as its
    completion is recorded (a client that consumes each frame as it
    arrives).

Memory.  The budget bounds everything the server holds on the device:
  * every cached batch slot, idle or busy, from its creation until it is
    evicted (idle slots are kept for reuse and evicted least recently used
    first when a new slot would not fit);
  * the output images of every request from its launch until its completion
    is recorded (with keep_results=True the client owns them afterwards).
A batch is admitted only if its outputs and, when no idle slot of its class
multiset exists, a new slot fit after evicting idle slots.  A single request
that cannot fit even in an empty server is rejected.

Latency is measured from the scheduled arrival to the moment the host sees
the batch's completion event.  The GPU specifics live in `GpuBackend`;
`Server` only schedules, so its policies (admission and eviction by memory,
batching, failure isolation) are testable on the CPU with a fake backend.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Any, Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

Klass = Tuple[int, int]
Combo = Tuple[Klass, ...]


@dataclasses.dataclass
class Request:
    rid: int
    camera: Any
    klass: Klass
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


@dataclasses.dataclass
class _Slot:
    combo: Combo
    handle: Any
    nbytes: int
    busy: bool = False
    last_use: int = 0


class Backend:
    """Interface the scheduler drives.  A slot holds the device buffers of a
    fused render of one multiset of classes (`combo`, sorted); views are
    always passed in the order of their sorted classes."""

    def out_bytes(self, klass: Klass) -> int:
        raise NotImplementedError

    def slot_bytes(self, combo: Combo) -> int:
        """Device memory of one batch slot for `combo` (frame + workspace)."""
        raise NotImplementedError

    def create_slot(self, combo: Combo) -> Any:
        raise NotImplementedError

    def destroy_slot(self, slot: Any) -> None:
        pass

    def launch(self, slot: Any, cams: Sequence, lane: int) -> Any:
        """Enqueue a fused forward of `cams` (sorted by class, matching the
        slot) on execution lane `lane`; return a handle for poll()/finish()."""
        raise NotImplementedError

    def poll(self, handle) -> bool:
        raise NotImplementedError

    def finish(self, handle) -> List[Any]:
        """Per-view results of a completed launch, in launch order."""
        raise NotImplementedError

    def release(self, handle) -> None:
        pass


class Server:
    def __init__(self, backend: Backend, mem_budget_bytes: int, max_batch: int = 8,
                 max_inflight: int = 3, idle_sleep: float = 50e-6, keep_results: bool = True,
                 mix_classes: bool = True):
        self.backend = backend
        self.keep_results = keep_results
        self.mix_classes = mix_classes
        self.budget = int(mem_budget_bytes)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.idle_sleep = idle_sleep
        self._q: "collections.deque[Request]" = collections.deque()
        self._lock = threading.Lock()
        self._inflight: List[Tuple[int, Any, List[Request], int, _Slot]] = []
        self._slots: List[_Slot] = []
        self._slot_mem = 0              # bytes of every cached slot
        self._out_mem = 0               # bytes of outputs not yet handed over
        self._peak = 0
        self._tick = 0
        self._next_id = 0
        self._next_batch = 0
        self._stop = False
        self._thread: Optional[threading.Thread] = None
        self.completed: List[Request] = []
        self.rejected = 0
        self.batches = 0
        self.batch_sizes: List[int] = []
        self.mixed_batches = 0          # batches holding more than one class
        self.evictions = 0
        self.slots_created = 0
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
        if ob + self.backend.slot_bytes((klass,)) > self.budget:
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

    def prewarm(self, combo: Sequence[Klass]) -> bool:
        """Create an idle slot for a class multiset before serving (e.g. to
        capture its graph outside the measured trace), if it fits the budget
        after evicting idle slots; returns whether it was created."""
        combo = tuple(sorted(tuple(k) for k in combo))
        with self._lock:
            if not self._fits(combo, 0) or self._idle(combo):
                return False
            s = self._acquire(combo, 0)
            s.busy = False
        return True

    def close(self):
        """Stop and destroy every cached slot."""
        self.stop()
        for s in list(self._slots):
            self._drop(s)

    @property
    def used_bytes(self) -> int:
        return self._slot_mem + self._out_mem

    def _idle(self, combo: Optional[Combo] = None) -> List[_Slot]:
        return [s for s in self._slots if not s.busy and (combo is None or s.combo == combo)]

    def _cost(self, combo: Combo, outs: int) -> int:
        """Memory the batch would add: its outputs, plus a new slot unless an
        idle one of the same multiset exists."""
        return outs + (0 if self._idle(combo) else self.backend.slot_bytes(combo))

    def _fits(self, combo: Combo, outs: int) -> bool:
        reuse = bool(self._idle(combo))
        evictable = sum(s.nbytes for s in self._idle() if not (reuse and s.combo == combo))
        return self.used_bytes - evictable + self._cost(combo, outs) <= self.budget

    def _form_batch(self) -> Optional[Tuple[List[Request], Combo]]:
        with self._lock:
            if not self._q:
                return None
            head = self._q[0]
            batch: List[Request] = []
            for r in list(self._q):
                if len(batch) >= self.max_batch:
                    break
                if not self.mix_classes and r.klass != head.klass:
                    continue
                cand = batch + [r]
                combo = tuple(sorted(q.klass for q in cand))
                if not self._fits(combo, sum(q.out_bytes for q in cand)):
                    break
                batch = cand
            if not batch:
                return None
            for r in batch:
                self._q.remove(r)
            batch.sort(key=lambda q: (q.klass, q.rid))
            return batch, tuple(q.klass for q in batch)

    def _drop(self, s: _Slot):
        self.backend.destroy_slot(s.handle)
        self._slots.remove(s)
        self._slot_mem -= s.nbytes

    def _acquire(self, combo: Combo, outs: int) -> _Slot:
        """An idle slot of `combo` (or a new one), after evicting other idle
        slots, least recently used first, until the batch's outputs and the
        new slot fit."""
        self._tick += 1
        idle = self._idle(combo)
        keep = max(idle, key=lambda x: x.last_use) if idle else None
        need = 0 if keep is not None else self.backend.slot_bytes(combo)
        for victim in sorted(self._idle(), key=lambda x: x.last_use):
            if self.used_bytes + need + outs <= self.budget:
                break
            if victim is keep:
                continue
            self._drop(victim)
            self.evictions += 1
        if keep is not None:
            s = keep
        else:
            s = _Slot(combo, self.backend.create_slot(combo), need)
            self._slots.append(s)
            self._slot_mem += need
            self.slots_created += 1
        s.busy = True
        s.last_use = self._tick
        return s

    def _loop(self):
        lanes = list(range(self.max_inflight))
        while not self._stop:
            progressed = False
            # completions
            for item in list(self._inflight):
                bid, h, batch, lane, slot = item
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
                        self._out_mem -= sum(r.out_bytes for r in batch)
                        slot.busy = False
                        self.completed.extend(batch)
                    lanes.append(lane)
                    progressed = True
            # admissions
            while lanes:
                formed = self._form_batch()
                if formed is None:
                    break
                batch, combo = formed
                bid = self._next_batch
                self._next_batch += 1
                outs = sum(r.out_bytes for r in batch)
                lane = lanes.pop(0)
                slot = None
                try:
                    if self.fail_hook is not None and self.fail_hook(bid):
                        raise RuntimeError("injected failure")
                    with self._lock:
                        slot = self._acquire(combo, outs)
                    h = self.backend.launch(slot.handle, [r.camera for r in batch], lane)
                except Exception as e:
                    now = time.perf_counter()
                    for r in batch:
                        r.error, r.t_done, r.batch_id = f"render failed: {e}", now, bid
                        r.done.set()
                    with self._lock:
                        if slot is not None:
                            slot.busy = False
                        self.completed.extend(batch)
                    lanes.append(lane)
                    continue
                for r in batch:
                    r.batch_id = bid
                with self._lock:
                    self._out_mem += outs
                    self._peak = max(self._peak, self.used_bytes)
                    self._inflight.append((bid, h, batch, lane, slot))
                    self.peak_inflight = max(self.peak_inflight, len(self._inflight))
                self.batches += 1
                self.batch_sizes.append(len(batch))
                if len(set(combo)) > 1:
                    self.mixed_batches += 1
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
                "mixed_batches": self.mixed_batches,
                "peak_inflight": int(self.peak_inflight),
                "slots_created": self.slots_created, "evictions": self.evictions,
                "peak_mem_bytes": int(self._peak), "budget_bytes": self.budget,
                "per_class": per_class}


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
    """Fused multi-view forward of a batch, replayed from a HIP graph captured
    for the batch's multiset of classes (or launched eagerly with
    use_graphs=False)."""

    def __init__(self, ctx, scene, layers: int = 4, alpha: float = 0.01, use_graphs: bool = True,
                 candidates: bool = True):
        """candidates: every slot holds a [V, n] byte buffer for the depth
        pass's candidate layers, so the accumulation skips the points that
        cannot blend (n bytes per view of slot memory)."""
        import torch
        from . import adop
        self.torch = torch
        self.adop = adop
        self.ctx = ctx
        self.scene = scene
        self.layers = layers
        self.alpha = alpha
        self.use_graphs = use_graphs
        self.candidates = candidates
        self.C = scene.channels
        self.dev = scene.x.device
        self.streams = {}

    def _pixels(self, klass):
        w, h = klass
        return sum((w >> l) * (h >> l) for l in range(self.layers))

    def out_bytes(self, klass) -> int:
        return self._pixels(klass) * self.C * 4

    def slot_bytes(self, combo) -> int:
        px = sum(self._pixels(k) for k in combo)
        cand = len(combo) * self.scene.n if self.candidates else 0
        return px * (self.C * 4 + 8 + 4) + self.ctx.workspace_bytes(self.C, len(combo), px) + cand

    def _stream(self, lane):
        if lane not in self.streams:
            self.streams[lane] = self.torch.cuda.Stream(device=self.dev)
        return self.streams[lane]

    def _dummy(self, combo):
        from . import synth
        return [synth.Camera(w, h, 0.8 * w, 0.8 * w, w / 2.0, h / 2.0) for (w, h) in combo]

    def create_slot(self, combo):
        cams = self._dummy(combo)
        if self.use_graphs:
            return self.adop.ForwardGraph(self.ctx, self.scene, cams, self.layers, alpha=self.alpha,
                                          record_visibility=self.candidates)
        fr = self.adop.Frame(cams, self.layers, self.C, self.dev)
        if self.candidates:
            fr.visible = self.torch.empty((len(cams), self.scene.n), dtype=self.torch.uint8, device=self.dev)
        ws = self.torch.empty(self.ctx.workspace_bytes(self.C, len(cams), fr.pixels),
                              dtype=self.torch.uint8, device=self.dev)
        return (fr, ws)

    def destroy_slot(self, slot):
        if self.use_graphs:
            slot.close()

    def launch(self, slot, cams, lane):
        torch = self.torch
        st = self._stream(lane)
        if self.use_graphs:
            frame = slot.launch(cams, stream=st)
        else:
            fr, ws = slot
            frame = self.adop.render_forward(self.ctx, self.scene, cams, self.layers, alpha=self.alpha,
                                             frame=fr, workspace=ws, stream=st,
                                             record_visibility=self.candidates)
        with torch.cuda.stream(st):
            outs = []
            for v, c in enumerate(cams):
                o = int(frame.offsets[v, 0])
                outs.append(frame.images[self.C * o: self.C * (o + self._pixels((c.width, c.height)))].clone())
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, outs)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle):
        return handle[1]


class PlainBackend(GpuBackend):
    """The unbatched baseline: FP32 scene, eager launches of the plain
    forward (no candidate buffer), one view at a time."""

    def __init__(self, ctx, scene, layers: int = 4, alpha: float = 0.01):
        super().__init__(ctx, scene, layers, alpha, use_graphs=False, candidates=False)
