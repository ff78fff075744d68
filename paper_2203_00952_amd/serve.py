"""Continuous-batching service for SRT3D frames on one GPU.

A request is one frame whose photon stamps are already in device memory; serving it means the
photon sketch (eq. 3) followed by the SRT3D reconstruction (Section 3) with its own iteration
count.  Requests arrive over time.  The scheduler admits a request once it has arrived, an
execution slot (a HIP stream) is free and its device working memory fits the HBM budget; an
admitted request's kernels are enqueued on its slot's stream at once, so requests that arrive
while others are running start as soon as a slot and memory free up and their kernels overlap
on the device.  Admission is first-come first-served: a request that does not fit blocks later
ones, so none starves.

Every request works on its own buffers and every reduction is per frame, so a request's result
does not depend on what runs beside it.

The scheduler itself (`Scheduler`) knows nothing about GPUs: it drives an executor through
`start / done / finish_time`, which lets the admission logic be tested with a simulated one.
When nothing can be admitted it does not spin: an executor with `token / wait` (the GPU one)
blocks it until a running job completes or the next request arrives; otherwise `idle(dt)` is
called.
"""
from __future__ import annotations

import ctypes
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable


@dataclass
class Job:
    rid: int
    arrival: float          # seconds on the service clock
    nbytes: int             # device working memory while the job runs
    payload: Any = None


@dataclass
class Record:
    rid: int
    arrival: float
    admitted: float
    finished: float
    slot: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Scheduler:
    executor: Any
    slots: int
    budget_bytes: int
    clock: Callable[[], float] = time.perf_counter
    idle: Callable[[float], None] | None = None    # called when nothing can progress (no `wait`)
    peak_bytes: int = field(default=0, init=False)

    def run(self, jobs: list[Job]) -> list[Record]:
        for j in jobs:
            if j.nbytes > self.budget_bytes:
                raise ValueError(f"request {j.rid} needs {j.nbytes} B, more than the whole budget")
        pending = sorted(jobs, key=lambda j: (j.arrival, j.rid))
        t0 = self.clock()
        free = list(range(self.slots))
        running: dict[int, tuple[Job, Any, float]] = {}
        in_use = 0
        out: list[Record] = []
        waits = self.idle is None and hasattr(self.executor, "wait")
        while pending or running:
            token = self.executor.token() if waits else None
            now = self.clock() - t0
            for slot in list(running):
                job, handle, admitted = running[slot]
                if self.executor.done(handle):
                    fin = self.executor.finish_time(handle, t0)
                    out.append(Record(job.rid, job.arrival, admitted, fin, slot))
                    in_use -= job.nbytes
                    free.append(slot)
                    del running[slot]
            progressed = False
            while pending and free and pending[0].arrival <= now and in_use + pending[0].nbytes <= self.budget_bytes:
                job = pending.pop(0)
                slot = free.pop(0)
                in_use += job.nbytes
                self.peak_bytes = max(self.peak_bytes, in_use)
                admitted = self.clock() - t0
                running[slot] = (job, self.executor.start(job, slot), admitted)
                progressed = True
            if not progressed and (pending or running):
                if waits:
                    # sleep until a running job completes (the token moves) or the next arrival
                    nxt = pending[0].arrival - (self.clock() - t0) if pending and pending[0].arrival > now else None
                    if running or nxt is not None:
                        self.executor.wait(token, None if nxt is None else max(nxt, 0.0))
                elif self.idle is not None:
                    nxt = pending[0].arrival - now if pending and not running else 0.0
                    self.idle(max(nxt, 0.0))
        return sorted(out, key=lambda r: r.rid)


def percentile(values, q):
    v = sorted(values)
    if not v:
        return float("nan")
    k = (len(v) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


# ----------------------------------------------------------------------------- GPU executor
class Request:
    """One frame to serve: device stamps and offsets, the impulse response and its parameters.
    `sketch` picks the sketch route (default "auto": binned for m <= 32 and at least 0.04 T
    photons per pixel, else the photon pass)."""

    def __init__(self, rid, stamps, offsets, irf, irf_origin, params, arrival=0.0, sketch=None):
        self.rid = rid
        self.stamps, self.offsets = stamps, offsets
        self.irf, self.irf_origin = irf, irf_origin
        self.params = params
        self.arrival = arrival
        self.sketch = sketch or "auto"

    def working_bytes(self) -> int:
        """Device memory the request holds while it runs: its photon stamps and offsets, the
        sketch and counts, two state halves, the outputs and scratch."""
        p = self.params
        P, K = p.P, p.K_max
        frame = 4 * self.stamps.numel() + 8 * self.offsets.numel()
        return int(frame + 8 * p.m * P + 4 * P + 2 * 9 * P * K + 9 * P * K + 4 * P + 8 * p.m + 32 + (1 << 14))

    def job(self) -> Job:
        return Job(self.rid, self.arrival, self.working_bytes(), self)


class _Running:
    """A started request: its completion event, the buffers that must outlive it, and the host
    time at which a watcher saw it complete (None until then)."""

    def __init__(self, event, keep):
        self.event, self.keep = event, keep
        self.finished = None


class GpuExecutor:
    """Runs each admitted request on its slot's stream: sketch, then reconstruct.  One watcher
    thread per slot blocks on the slot's completion events (blocking-sync events, so the thread
    sleeps in the driver) and wakes the scheduler through a condition variable."""

    def __init__(self, slots: int, device="cuda:0"):
        import torch

        from . import _lib as L

        self.torch, self.L = torch, L
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.results: dict[int, dict] = {}
        self._event_sync = L._lib().hipEventSynchronize
        self._event_sync.restype = ctypes.c_int
        self._event_sync.argtypes = [ctypes.c_void_p]
        self._cv = threading.Condition()
        self._completions = 0
        self._queues = [queue.SimpleQueue() for _ in range(slots)]
        self._watchers = [threading.Thread(target=self._watch, args=(q,), daemon=True) for q in self._queues]
        for t in self._watchers:
            t.start()

    def _watch(self, q):
        while True:
            h = q.get()
            if h is None:
                return
            # hipEventSynchronize through ctypes, which releases the interpreter lock while the
            # thread sleeps (the symbol resolves through libsrt3d's own HIP runtime dependency,
            # the runtime that created the event)
            self._event_sync(h.event._as_parameter_)
            with self._cv:
                h.finished = time.perf_counter()
                self._completions += 1
                self._cv.notify_all()

    def start(self, job: Job, slot: int):
        torch, L = self.torch, self.L
        req: Request = job.payload
        s = self.streams[slot]
        table = L.cached_phase_table(req.params.T, self.device)
        with torch.cuda.stream(s):
            z, n = L.sketch(req.stamps, req.offsets, req.params.T, req.params.m, table=table, method=req.sketch)
            rec = L.Reconstructor(req.params, self.device)
            out = rec.reconstruct(z, n, req.irf, req.irf_origin)
            ev = torch.cuda.Event(blocking=True)
            ev.record(s)
        self.results[req.rid] = out
        h = _Running(ev, (rec, z, n))
        self._queues[slot].put(h)
        return h

    def done(self, handle) -> bool:
        with self._cv:
            return handle.finished is not None

    def finish_time(self, handle, t0: float) -> float:
        return handle.finished - t0

    def token(self) -> int:
        with self._cv:
            return self._completions

    def wait(self, token: int, timeout):
        """Block until a completion after `token` was observed, or `timeout` seconds (None: no
        limit) have passed."""
        with self._cv:
            self._cv.wait_for(lambda: self._completions != token, timeout)

    def close(self):
        for q in self._queues:
            q.put(None)
        for t in self._watchers:
            t.join()


def serve(requests: list[Request], slots: int = 4, budget_bytes: int = 16 << 30, device="cuda:0"):
    """Serve `requests` (arrival times in seconds from now); returns (records, results by rid)."""
    ex = GpuExecutor(slots, device)
    try:
        sch = Scheduler(ex, slots, budget_bytes)
        recs = sch.run([r.job() for r in requests])
        ex.torch.cuda.synchronize()
    finally:
        ex.close()
    return recs, ex.results, sch.peak_bytes
