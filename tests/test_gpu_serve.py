"""Serving on the GPU: requests of mixed n admitted while others run, their
work overlapping on several streams; every result must equal the same n
computed alone (bit for bit) and, where cheap, the CPU oracle."""
import numpy as np
import pytest

import oracle
from tests import batch_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cat():
    import torch

    import paper_2601_11621_amd as c

    torch.cuda.set_device(0)
    c.init(0)
    return c


def _solo(cat, ns):
    out = {}
    for n in sorted(set(ns)):
        out[n] = cat.to_numpy(cat.exact(n, mode="batched"))
    return out


def test_mix_equals_solo_closed_loop(cat):
    from paper_2601_11621_amd.serve import DONE, GpuExecutor, Server

    ns, _ = batch_inputs.serving_requests(seed=11621, count=60)
    ns = [int(x) for x in ns] + [0, 1, 2, 13, 1000, 1000, int(ns[3]), 10**7]
    srv = Server(GpuExecutor(max_slots=8), budget_bytes=8 << 30, max_slots=8)
    reqs = [srv.submit(n, arrival=0.0) for n in ns]
    srv.run()
    assert srv.peak_active > 1                        # work really overlapped
    solo = _solo(cat, ns)
    for r in reqs:
        assert r.state == DONE, (r.n, r.error)
        got = cat.to_numpy(r.result)
        assert np.array_equal(got, solo[r.n]), r.n
        if r.n <= 20000:
            assert np.array_equal(got, oracle.catalan(r.n)), r.n


def test_mix_equals_solo_poisson_arrivals(cat):
    import time

    from paper_2601_11621_amd.serve import DONE, GpuExecutor, Server

    ns, gaps = batch_inputs.serving_requests(seed=7, count=80, lo_exp=3.0, hi_exp=6.0)
    srv = Server(GpuExecutor(max_slots=6), budget_bytes=1 << 30, max_slots=6)
    t0 = time.perf_counter() + 0.01
    arr = t0 + np.cumsum(gaps) * 0.0005                # about 2000 requests/s offered
    reqs = [srv.submit(int(n), arrival=float(a)) for n, a in zip(ns, arr)]
    srv.run()
    solo = _solo(cat, [int(n) for n in ns])
    for r in reqs:
        assert r.state == DONE, (r.n, r.error)
        assert np.array_equal(cat.to_numpy(r.result), solo[r.n]), r.n
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0


def test_budget_smaller_than_one_request_fails_cleanly(cat):
    from paper_2601_11621_amd.serve import DONE, FAILED, GpuExecutor, Server

    ex = GpuExecutor(max_slots=2)
    srv = Server(ex, budget_bytes=ex.footprint(10**5) + 1, max_slots=2)
    a = srv.submit(10**7, arrival=0.0)
    b = srv.submit(10**5, arrival=0.0)
    srv.run()
    assert a.state == FAILED and b.state == DONE
    assert np.array_equal(cat.to_numpy(b.result), oracle.catalan(10**5))
