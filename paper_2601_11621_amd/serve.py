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
The host loop only polls events; it never waits on the GPU.  A request can be
cancelled at any point: a queued one leaves the queue, a running one has its
device work drained and its slot and memory freed.

`Server` is independent of the device: it drives an executor with
`footprint / begin / ready / advance / finish` (and `flush` after each
admission step, for executors that batch).  `GpuExecutor` binds that to the
C ABI with one ticket per request; `BatchExecutor` runs the requests admitted
in one step as one library batch (continuous batching: each tree level of all
of them, and each step of their powers and outer products, is one launch per
kernel stage, while the requests of earlier steps keep running on other
streams); `FakeExecutor` (used by the CPU tests) simulates durations.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, List, Optional


QUEUED, PHASE1, PHASE2, DONE, FAILED, CANCELLED = "queued", "phase1", "phase2", "done", "failed", "cancelled"


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
    """`on_done(request)`, if given, is called once per request as it leaves
    the server (done, failed or cancelled), e.g. to consume and drop results."""

    def __init__(self, executor, budget_bytes: int, max_slots: int = 8,
                 clock: Callable[[], float] = time.perf_counter, on_done: Optional[Callable] = None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.on_done = on_done
        # the executor keeps freed workspaces for reuse only within the budget
        attach = getattr(executor, "attach", None)
        if attach is not None:
            attach(self.budget)
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
                self._finished(r)
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
                self.ex.abort(r)
                self._retire(r, now, str(e))
            else:
                self.active.append(r)
                self.peak_active = max(self.peak_active, len(self.active))
            moved = True
        # a batching executor launches what this step admitted as one batch
        flush = getattr(self.ex, "flush", None)
        if moved and flush is not None:
            for r, err in flush() or []:
                if r in self.active:
                    self.active.remove(r)
                    self.ex.abort(r)
                    self._retire(r, now, err)
        return moved

    def _finished(self, r: Request):
        self.done.append(r)
        if self.on_done is not None:
            self.on_done(r)

    def _retire(self, r: Request, now: float, error: Optional[str] = None, state: Optional[str] = None):
        r.finished = now
        r.state = state or (FAILED if error else DONE)
        r.error = error
        self.used -= r.footprint
        self.free_slots.append(r.slot)
        self._finished(r)

    def cancel(self, r: Request) -> bool:
        """Withdraw a request.  A queued one leaves the queue; a running one has
        its queued device work drained by the executor, then its slot and its
        memory are freed.  False if it had already left the server."""
        now = self.clock()
        if r.state == QUEUED:
            try:
                self.queue.remove(r)
            except ValueError:
                return False
            r.state, r.error, r.finished = CANCELLED, "cancelled", now
            self._finished(r)
            return True
        if r in self.active:
            self.active.remove(r)
            self.ex.abort(r)
            self._retire(r, now, "cancelled", CANCELLED)
            return True
        return False

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
                "cancelled": sum(1 for r in self.done if r.state == CANCELLED),
                "p50_ms": pct(0.5) * 1e3, "p99_ms": pct(0.99) * 1e3, "mean_ms": sum(lat) / len(lat) * 1e3,
                "req_per_s": len(rs) / (t1 - t0) if t1 > t0 else float("inf"),
                "peak_active": self.peak_active, "peak_bytes": self.peak_used}


# ---------------------------------------------------------------------------
class GpuExecutor:
    """Executor on the library's ticket API.

    Slots share at most `max_streams` HIP streams (default 4: the hardware
    queues a process gets by default; more streams would only be multiplexed
    onto them).  Workspaces of finished requests are kept for reuse by size
    class, but only while the active requests plus the kept buffers stay
    within the budget the server attaches; beyond it they are released."""

    def __init__(self, max_slots: int, device: int = 0, max_streams: int = 4):
        import torch

        from . import _check, _ptr, init, load, sizes

        self._torch = torch
        self._check, self._ptr, self._sizes = _check, _ptr, sizes
        init(device)
        self.lib = load()
        # default-priority streams shared round-robin by the slots
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, min(max_slots, max_streams)))]
        self._pool = collections.defaultdict(list)     # size class -> free workspace tensors
        self.pooled = 0                                 # bytes held by the pool
        self.active_bytes = 0                           # bytes held by running requests
        self.budget: Optional[int] = None

    def attach(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self._trim(0)

    @staticmethod
    def _cls(nbytes: int) -> int:
        c = 1 << 20
        while c < nbytes:
            c <<= 1
        return c

    def _trim(self, need: int):
        """Release pooled workspaces (largest first) until active + pooled +
        need fits the budget."""
        if self.budget is None:
            return
        for cls in sorted(self._pool, reverse=True):
            free = self._pool[cls]
            while free and self.active_bytes + self.pooled + need > self.budget:
                free.pop()
                self.pooled -= cls

    def _release(self, cls: int, w):
        self._pool[cls].append(w)
        self.pooled += cls
        self._trim(0)

    def footprint(self, n: int) -> int:
        _, max_limbs, wbytes = self._sizes(n)
        return self._cls(wbytes) + 4 * max_limbs

    def begin(self, r: Request):
        torch = self._torch
        _, max_limbs, wbytes = self._sizes(r.n)
        cls = self._cls(wbytes)
        free = self._pool[cls]
        if free:
            w = free.pop()
            self.pooled -= cls
        else:
            self._trim(cls + 4 * max_limbs)
            w = torch.empty(cls, dtype=torch.uint8, device="cuda")
        held = cls + 4 * max_limbs
        self.active_bytes += held
        out = torch.empty(max_limbs, dtype=torch.int32, device="cuda")
        st = self.streams[r.slot % len(self.streams)]
        t = ctypes.c_void_p()
        r.handle = (None, w, out, cls, held)
        self._check(self.lib.catalan_begin(r.n, self._ptr(w), w.numel(), ctypes.c_void_p(st.cuda_stream),
                                           ctypes.byref(t)), "catalan_begin")
        r.handle = (t, w, out, cls, held)

    def ready(self, r: Request) -> bool:
        s = self.lib.cat_ticket_query(r.handle[0])
        if s == -6:
            return False
        self._check(s, "cat_ticket_query")
        return True

    def advance(self, r: Request):
        t, w, out = r.handle[:3]
        self._check(self.lib.catalan_continue(t, self._ptr(out), out.numel()), "catalan_continue")

    def _done_with(self, r: Request):
        t, w, out, cls, held = r.handle
        r.handle = None
        self.active_bytes -= held
        self._release(cls, w)
        return out

    def finish(self, r: Request) -> int:
        t = r.handle[0]
        nl = ctypes.c_size_t()
        # catalan_end waits for the ticket's work and releases the ticket on
        # every path, so the handle is dropped before its status is checked
        st = self.lib.catalan_end(t, ctypes.byref(nl))
        out = self._done_with(r)
        self._check(st, "catalan_end")
        r.result = out[: nl.value]
        return nl.value

    def abort(self, r: Request):
        if r.handle is None:
            return
        t = r.handle[0]
        if t is not None and t.value:
            # waits until everything queued on the ticket's stream has finished
            self.lib.cat_ticket_release(t)
        self._done_with(r)

    def wait_until(self, t: float):
        while time.perf_counter() < t:
            pass


class BatchExecutor:
    """Executor on the library's batch API (catalan_batch_*): the requests the
    server admits in one step (at most `max_batch`) share one batch ticket,
    one workspace and one set of Phase-2 launches; successive batches run on
    up to `max_streams` streams, so a new batch's Phase 1 overlaps the running
    ones.  A request's footprint counts twice its own workspace (the batch's
    combined scratch rounds up over the requests) plus its output."""

    def __init__(self, max_slots: int, device: int = 0, max_streams: int = 4, max_batch: int = 16):
        import torch

        from . import BATCH_MAX, _check, _ptr, init, load, sizes

        self._torch = torch
        self._check, self._ptr, self._sizes = _check, _ptr, sizes
        init(device)
        self.lib = load()
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, max_streams))]
        self._next_stream = 0
        self.max_batch = max(1, min(int(max_batch), BATCH_MAX))
        self.forming: List[Request] = []
        self._pool = collections.defaultdict(list)
        self.pooled = 0
        self.active_bytes = 0
        self.budget: Optional[int] = None
        self.batches = 0
        self.batched_requests = 0

    attach = GpuExecutor.attach
    _cls = staticmethod(GpuExecutor._cls)
    _trim = GpuExecutor._trim
    _release = GpuExecutor._release

    def footprint(self, n: int) -> int:
        _, max_limbs, wbytes = self._sizes(n)
        return 2 * self._cls(wbytes) + 4 * max_limbs

    def begin(self, r: Request):
        _, max_limbs, _ = self._sizes(r.n)
        r.handle = None
        out = self._torch.empty(max_limbs, dtype=self._torch.int32, device="cuda")
        r.handle = {"batch": None, "out": out}
        self.forming.append(r)

    def flush(self):
        """Launch the forming requests as batches of at most max_batch;
        returns the (request, error) pairs of batches that failed to start."""
        import ctypes

        failed = []
        while self.forming:
            reqs, self.forming = self.forming[: self.max_batch], self.forming[self.max_batch:]
            torch = self._torch
            import numpy as np

            ns = np.ascontiguousarray(np.array([r.n for r in reqs], dtype=np.uint64))
            p64 = ns.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
            wb = ctypes.c_size_t()
            st = self.lib.catalan_batch_sizes(len(reqs), p64, ctypes.byref(wb))
            if st != 0:
                failed += [(r, "catalan_batch_sizes failed (%d)" % st) for r in reqs]
                continue
            cls = self._cls(wb.value)
            free = self._pool[cls]
            if free:
                w = free.pop()
                self.pooled -= cls
            else:
                self._trim(cls)
                w = torch.empty(cls, dtype=torch.uint8, device="cuda")
            self.active_bytes += cls
            stream = self.streams[self._next_stream % len(self.streams)]
            self._next_stream += 1
            t = ctypes.c_void_p()
            st = self.lib.catalan_batch_begin(len(reqs), p64, self._ptr(w), w.numel(),
                                              ctypes.c_void_p(stream.cuda_stream), ctypes.byref(t))
            if st != 0:
                self.active_bytes -= cls
                self._release(cls, w)
                failed += [(r, "catalan_batch_begin failed (%d)" % st) for r in reqs]
                continue
            b = {"ticket": t, "reqs": reqs, "w": w, "cls": cls, "state": 1, "left": len(reqs),
                 "n_limbs": None, "status": None}
            for r in reqs:
                r.handle["batch"] = b
            self.batches += 1
            self.batched_requests += len(reqs)
        return failed

    def ready(self, r: Request) -> bool:
        b = r.handle["batch"]
        if b["state"] == 3:
            return True
        s = self.lib.cat_ticket_query(b["ticket"])
        if s == -6:
            return False
        self._check(s, "cat_ticket_query")
        return True

    def advance(self, r: Request):
        import ctypes

        b = r.handle["batch"]
        if b["state"] != 1:
            return
        reqs = b["reqs"]
        k = len(reqs)
        outs = [q.handle["out"] for q in reqs]
        ptrs = (ctypes.c_void_p * k)(*[o.data_ptr() for o in outs])
        caps = (ctypes.c_size_t * k)(*[o.numel() for o in outs])
        b["keep"] = (ptrs, caps)
        self._check(self.lib.catalan_batch_continue(b["ticket"], ptrs, caps), "catalan_batch_continue")
        b["state"] = 2

    def _end(self, b):
        import ctypes

        k = len(b["reqs"])
        nl = (ctypes.c_size_t * k)()
        rs = (ctypes.c_int32 * k)()
        self.lib.catalan_batch_end(b["ticket"], nl, rs)     # releases the ticket; statuses per request
        b["n_limbs"], b["status"] = list(nl), list(rs)
        b["state"] = 3
        self.active_bytes -= b["cls"]
        self._release(b["cls"], b["w"])
        b["w"] = None

    def finish(self, r: Request) -> int:
        b = r.handle["batch"]
        if b["state"] == 2:
            self._end(b)
        b["left"] -= 1
        i = b["reqs"].index(r)
        out = r.handle["out"]
        r.handle = None
        self._check(b["status"][i], "catalan_batch_end")
        r.result = out[: b["n_limbs"][i]]
        return b["n_limbs"][i]

    def abort(self, r: Request):
        if r.handle is None:
            return
        b = r.handle["batch"]
        r.handle = None
        if b is None:
            if r in self.forming:
                self.forming.remove(r)
            return
        b["left"] -= 1
        if b["left"] == 0 and b["state"] in (1, 2):
            # nobody waits for this batch any more: drain it and free its workspace
            self.lib.cat_ticket_release(b["ticket"])
            b["state"] = 3
            self.active_bytes -= b["cls"]
            self._release(b["cls"], b["w"])
            b["w"] = None

    def wait_until(self, t: float):
        while time.perf_counter() < t:
            pass


class FakeExecutor:
    """Simulated executor for CPU tests: Phase 1 and Phase 2 take given times on
    a fake clock; footprints are n bytes."""

    def __init__(self, phase1: Callable[[int], float], phase2: Callable[[int], float],
                 fail_finish: Callable[[int], bool] = lambda n: False):
        self.now = 0.0
        self.p1, self.p2 = phase1, phase2
        self.fail_finish = fail_finish
        self.log = []
        self.open = set()     # requests with device work the executor holds

    def clock(self) -> float:
        return self.now

    def footprint(self, n: int) -> int:
        return n

    def begin(self, r: Request):
        r.handle = self.now + self.p1(r.n)
        self.open.add(r.rid)
        self.log.append(("begin", r.rid, self.now))

    def ready(self, r: Request) -> bool:
        return self.now >= r.handle

    def advance(self, r: Request):
        r.handle = self.now + self.p2(r.n)
        self.log.append(("advance", r.rid, self.now))

    def finish(self, r: Request) -> int:
        self.log.append(("finish", r.rid, self.now))
        self.open.discard(r.rid)
        r.handle = None
        if self.fail_finish(r.n):
            raise RuntimeError("finish failed")
        return r.n

    def abort(self, r: Request):
        self.log.append(("abort", r.rid, self.now))
        if r.handle is not None:
            self.open.discard(r.rid)
            r.handle = None

    def wait_until(self, t: float):
        self.now = max(self.now, t)

    def tick(self, dt: float):
        self.now += dt
