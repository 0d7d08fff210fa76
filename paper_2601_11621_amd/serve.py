"""Request loop for exact C(n) on one GPU (continuous admission).

Requests of mixed n arrive over time.  A request is admitted as soon as a
slot is free and its HBM footprint (the library's workspace bound for n plus
the result buffer) fits in the budget next to the requests already running;
admission is FIFO, so a large request at the head waits for memory rather than
being overtaken.  Each slot owns a HIP stream; an admitted request runs as
library tickets on its slot's stream — Phase 1 queued at admission, Phase 2
queued once Phase 1 has finished — so the work of all admitted requests
overlaps on the device, and everything a request builds (primes, groups,
partial product trees) stays resident in its workspace until it finishes.
The host loop only polls events; it never waits on the GPU.

`Server` is independent of the device: it drives an executor with
`footprint / begin / ready / advance / finish`.  `GpuExecutor` binds that to
the C ABI; `FakeExecutor` (used by the CPU tests) simulates durations.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, List, Optional


QUEUED, PHASE1, PHASE2, DONE, FAILED = "queued", "phase1", "phase2", "done", "failed"


@dataclass
class Request:
    rid: int
    n: int
    arrival: float
    footprint: int = 0
    state: str = QUEUED
    admitted: float = 0.0
    finished: float = 0.0
    slot: int = -1
    n_limbs: int = 0
    error: Optional[str] = None
    handle: object = None          # executor's per-request state
    result: object = None          # executor's result (device tensor for the GPU executor)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    def __init__(self, executor, budget_bytes: int, max_slots: int = 8,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.clock = clock
        self.queue: Deque[Request] = collections.deque()
        self.active: List[Request] = []
        self.done: List[Request] = []
        self.free_slots = list(range(self.max_slots - 1, -1, -1))
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0
        self._next = 0

    # -------------------------------------------------------------- intake
    def submit(self, n: int, arrival: Optional[float] = None) -> Request:
        r = Request(self._next, int(n), self.clock() if arrival is None else float(arrival))
        self._next += 1
        r.footprint = self.ex.footprint(r.n)
        self.queue.append(r)
        return r

    # -------------------------------------------------------------- loop
    def _admit(self, now: float) -> bool:
        moved = False
        while self.queue and self.free_slots and self.queue[0].arrival <= now:
            r = self.queue[0]
            if r.footprint > self.budget:
                self.queue.popleft()
                r.state, r.error, r.finished = FAILED, "footprint exceeds the budget", now
                self.done.append(r)
                moved = True
                continue
            if self.used + r.footprint > self.budget:
                break                      # FIFO: wait for memory
            self.queue.popleft()
            r.slot = self.free_slots.pop()
            self.used += r.footprint
            self.peak_used = max(self.peak_used, self.used)
            r.admitted = now
            try:
                self.ex.begin(r)
                r.state = PHASE1
            except Exception as e:  # noqa: BLE001 - reported on the request
                self._retire(r, now, str(e))
            else:
                self.active.append(r)
                self.peak_active = max(self.peak_active, len(self.active))
            moved = True
        return moved

    def _retire(self, r: Request, now: float, error: Optional[str] = None):
        r.finished = now
        r.state = FAILED if error else DONE
        r.error = error
        self.used -= r.footprint
        self.free_slots.append(r.slot)
        self.done.append(r)

    def step(self) -> bool:
        """One pass: poll running requests, then admit.  True if anything moved."""
        moved = False
        now = self.clock()
        still = []
        for r in self.active:
            try:
                if not self.ex.ready(r):
                    still.append(r)
                    continue
                if r.state == PHASE1:
                    self.ex.advance(r)
                    r.state = PHASE2
                    still.append(r)
                else:
                    r.n_limbs = self.ex.finish(r)
                    self._retire(r, self.clock())
            except Exception as e:  # noqa: BLE001
                self.ex.abort(r)
                self._retire(r, self.clock(), str(e))
            moved = True
        self.active = still
        if self._admit(self.clock()):
            moved = True
        return moved

    def idle(self) -> bool:
        return not self.queue and not self.active

    def run(self, poll_sleep: float = 0.0):
        """Run until every submitted request has finished."""
        while not self.idle():
            if not self.step():
                if self.active or (self.queue and self.queue[0].arrival <= self.clock()):
                    if poll_sleep:
                        time.sleep(poll_sleep)
                else:
                    self.ex.wait_until(self.queue[0].arrival)

    # -------------------------------------------------------------- stats
    def stats(self, skip: int = 0) -> dict:
        rs = [r for r in self.done if r.rid >= skip and r.state == DONE]
        lat = sorted(r.latency for r in rs)
        if not lat:
            return {"completed": 0}

        def pct(q):
            return lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]

        t0 = min(r.arrival for r in rs)
        t1 = max(r.finished for r in rs)
        return {"completed": len(rs), "failed": sum(1 for r in self.done if r.state == FAILED),
                "p50_ms": pct(0.5) * 1e3, "p99_ms": pct(0.99) * 1e3, "mean_ms": sum(lat) / len(lat) * 1e3,
                "req_per_s": len(rs) / (t1 - t0) if t1 > t0 else float("inf"),
                "peak_active": self.peak_active, "peak_bytes": self.peak_used}


# ---------------------------------------------------------------------------
class GpuExecutor:
    """Executor on the library's ticket API; one HIP stream per slot."""

    def __init__(self, max_slots: int, device: int = 0):
        import torch

        from . import _check, _ptr, init, load, sizes

        self._torch = torch
        self._check, self._ptr, self._sizes = _check, _ptr, sizes
        init(device)
        self.lib = load()
        # default-priority streams, one per slot
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max_slots)]
        self._pool = collections.defaultdict(list)     # size class -> free workspace tensors

    @staticmethod
    def _cls(nbytes: int) -> int:
        c = 1 << 20
        while c < nbytes:
            c <<= 1
        return c

    def footprint(self, n: int) -> int:
        _, max_limbs, wbytes = self._sizes(n)
        return self._cls(wbytes) + 4 * max_limbs

    def begin(self, r: Request):
        torch = self._torch
        _, max_limbs, wbytes = self._sizes(r.n)
        cls = self._cls(wbytes)
        free = self._pool[cls]
        w = free.pop() if free else torch.empty(cls, dtype=torch.uint8, device="cuda")
        out = torch.empty(max_limbs, dtype=torch.int32, device="cuda")
        st = self.streams[r.slot]
        t = ctypes.c_void_p()
        self._check(self.lib.catalan_begin(r.n, self._ptr(w), w.numel(), ctypes.c_void_p(st.cuda_stream),
                                           ctypes.byref(t)), "catalan_begin")
        r.handle = (t, w, out, cls)

    def ready(self, r: Request) -> bool:
        s = self.lib.cat_ticket_query(r.handle[0])
        if s == -6:
            return False
        self._check(s, "cat_ticket_query")
        return True

    def advance(self, r: Request):
        t, w, out, cls = r.handle
        self._check(self.lib.catalan_continue(t, self._ptr(out), out.numel()), "catalan_continue")

    def finish(self, r: Request) -> int:
        t, w, out, cls = r.handle
        nl = ctypes.c_size_t()
        self._check(self.lib.catalan_end(t, ctypes.byref(nl)), "catalan_end")
        r.result = out[: nl.value]
        self._pool[cls].append(w)
        r.handle = None
        return nl.value

    def abort(self, r: Request):
        if r.handle is not None:
            t, w, out, cls = r.handle
            self.lib.cat_ticket_release(t)
            self._pool[cls].append(w)
            r.handle = None

    def wait_until(self, t: float):
        while time.perf_counter() < t:
            pass


class FakeExecutor:
    """Simulated executor for CPU tests: Phase 1 and Phase 2 take given times on
    a fake clock; footprints are n bytes."""

    def __init__(self, phase1: Callable[[int], float], phase2: Callable[[int], float]):
        self.now = 0.0
        self.p1, self.p2 = phase1, phase2
        self.log = []

    def clock(self) -> float:
        return self.now

    def footprint(self, n: int) -> int:
        return n

    def begin(self, r: Request):
        r.handle = self.now + self.p1(r.n)
        self.log.append(("begin", r.rid, self.now))

    def ready(self, r: Request) -> bool:
        return self.now >= r.handle

    def advance(self, r: Request):
        r.handle = self.now + self.p2(r.n)
        self.log.append(("advance", r.rid, self.now))

    def finish(self, r: Request) -> int:
        self.log.append(("finish", r.rid, self.now))
        return r.n

    def abort(self, r: Request):
        pass

    def wait_until(self, t: float):
        self.now = max(self.now, t)

    def tick(self, dt: float):
        self.now += dt
