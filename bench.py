"""Benchmark: exact C(n) on one MI355X (default n = 2,050,572,903, the paper's
Table 1 run).

One step = one whole pass of the hot path: catalan_exact(n) — the device
sieve with Legendre exponents (Phase 1) and the batched product tree with
multi-prime NTT products (Phase 2) — launched as one cached HIP graph.  The
result is verified before and after the timed steps: at n = 2,050,572,903
against Table 1 (bit length, file size, digit count) and residue pins (the
2-adic low limbs and C mod 2^32 - 5 from the oracle's definition-based
routines, C mod 2^32 + 1 by Lucas' theorem, the top 64 bits from log-gamma);
at smaller n bit for bit against the oracle's digest.

Prints ONE JSON line.  `value` is the whole-step throughput in product limbs
per second: the sum over every product of the tree (Q_e trees, powers, outer
product) of la + lb, divided by the step time.  The same line carries the
batched-vs-plain comparisons (C(10^7), C(10^8), the 4,096-product level
batch), serving, the dominant kernel's roofline (timed live with HIP events)
and the CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_catalan.json")
PROFILES = os.path.join(ROOT, "profiles")
METRIC = "C(n) exact-reconstruction time; batched bigint-mul limbs/s vs plain, bit-exact"
HEADLINE_N = 2050572903

# MI355X figures: 256 CUs x 64 lanes x 2.4 GHz = 39.3 T 32-bit VALU lane
# operations per second.  A radix-2 NTT butterfly with a precomputed-quotient
# twiddle costs about 9 lane operations as an algorithm (3 multiplies plus
# about 6 additions, subtractions and selects): that prices the butterfly
# peak.  This library's own butterfly issues 14 instructions (the primes
# exceed 2^31, which leaves no room for lazy reduction); the fraction against
# that count is reported as a labelled secondary figure.
CLOCK_HZ = 2.4e9
VALU_LANE_OPS = 256 * 64 * CLOCK_HZ
BFLY_OPS = 9.0
BFLY_OPS_CODE = 14.0
PEAK_BFLY = VALU_LANE_OPS / BFLY_OPS
PEAK_BFLY_CODE = VALU_LANE_OPS / BFLY_OPS_CODE
HBM_PEAK_GBS = 8000.0

CANDIDATES = ["k_row", "k_pass_fwd", "k_pass_inv", "k_ntt_lds", "k_tree_fused", "k_crt", "k_school", "k_leaf"]
NTT_KERNELS = {"k_row", "k_pass_fwd", "k_pass_inv", "k_ntt_lds", "k_tree_fused"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


_PINS = {}


def largest_pins(n):
    """Pins of C(n) where the oracle cannot multiply it out: Table 1 and the
    stored residues (the oracle's definition-based routines), plus C mod
    2^32 + 1 by Lucas' theorem and the bit length, digit count and top 64 bits
    from log-gamma (computed here, once)."""
    if n in _PINS:
        return _PINS[n]
    pz = os.path.join(ROOT, "tests", "golden", "pins_n%d.json" % n)
    t1 = os.path.join(ROOT, "tests", "golden", "table1_n%d.json" % n)
    if not (os.path.exists(pz) and os.path.exists(t1)):
        _PINS[n] = None
        return None
    from tests import pins

    with open(pz) as f:
        pz = json.load(f)
    with open(t1) as f:
        t1 = json.load(f)
    b2, digits, top64, _ = pins.log_pins(n, dps=80)
    if b2 != t1["bit_length"] or digits != t1["decimal_digits"]:
        raise SystemExit("bench: log-gamma pins disagree with Table 1")
    _PINS[n] = {"bits": t1["bit_length"], "bytes": t1["result_file_bytes"], "digits": t1["decimal_digits"],
                "limb0": pz["limb0"], "limb1": pz["limb1"], "mod_2p32_minus_5": pz["mod_2p32_minus_5"],
                "mod_2p32_plus_1": pins.catalan_mod_composite(n, [641, 6700417]), "top64": top64}
    return _PINS[n]


def check_output(cat, t, n, gold):
    """Bit-exact check of a device result against the oracle digest, or, for
    the largest n (no oracle product), against Table 1 and the residue pins.
    Returns the list of what was checked; raises SystemExit on a mismatch."""
    if gold is None:
        pz = largest_pins(n)
        if pz is None:
            return None
        L = t.numel()
        top = int(t[-1].item()) & 0xFFFFFFFF
        bits = 32 * (L - 1) + top.bit_length()
        low = cat.to_numpy(t[:2])
        hi = cat.to_numpy(t[L - 2:])
        r = cat.residues(t)
        ok = (bits == pz["bits"] and (bits + 7) // 8 == pz["bytes"] and int(low[0]) == pz["limb0"]
              and int(low[1]) == pz["limb1"] and r[0] == pz["mod_2p32_minus_5"] and r[1] == pz["mod_2p32_plus_1"]
              and (int(hi[1]) << 32 | int(hi[0])) == pz["top64"])
        if not ok:
            raise SystemExit("bench: C(%d) does NOT match Table 1 / residue pins" % n)
        return ["table1_bit_length", "table1_file_bytes", "limb0", "limb1", "mod_2^32-5", "mod_2^32+1",
                "top64_log_gamma"]
    got = cat.to_numpy(t)
    h = hashlib.sha256(got.astype("<u4").tobytes()).hexdigest()
    ok = (len(got) == gold["n_limbs"] and h == gold["sha256_le_limbs"])
    if not ok:
        raise SystemExit("bench: C(%d) does NOT match the oracle digest" % n)
    return ["oracle_sha256_all_limbs"]


def time_steps(cat, n, mode, steps, out):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cat.exact(n, mode=mode, out=out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def kernel_times(cat, n, out):
    """Per-kernel summed time of one batched (non-graph) step, via the library's event timer."""
    res = {}
    for k in CANDIDATES:
        cat.timer_set(k)
        cat.exact(n, mode="batched", out=out)
        ms, launches, work = cat.timer_get()
        res[k] = (ms, launches, work)
    cat.timer_set(None)
    return res


def source_sha1(files=None):
    """SHA-1 over the library sources `files` (names under csrc/; all of them
    when None)."""
    import glob

    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2601_11621_amd", "csrc")
    paths = sorted(glob.glob(os.path.join(csrc, "*"))) if files is None else [os.path.join(csrc, f) for f in files]
    for f in paths:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_traffic(kernel, n):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the sources that define the kernel changed after the counters
    were taken."""
    path = os.path.join(PROFILES, "traffic_%s_n%d.json" % (kernel, n))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha1") != source_sha1(t.get("sources")):
        return None
    return t


def _time_plan(plan, da, db, c, reps):
    import torch

    plan(da, db, c)
    plan.check()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        plan(da, db, c)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    plan.check()
    return sorted(ts)[len(ts) // 2] * 1e3


def batch_buckets(cat, a, a_off, b, b_off, reps=5):
    """The batch split by transform size (N = 2^ceil(log2(la + lb - 1)), at
    least 2^6): each bucket alone as one graph replay, median of `reps`."""
    import torch

    la = (a_off[1:] - a_off[:-1]).astype(np.int64)
    lb = (b_off[1:] - b_off[:-1]).astype(np.int64)
    logn = np.maximum(6, np.ceil(np.log2(np.maximum(la + lb - 1, 1))).astype(np.int64))
    out = {}
    for k in sorted(set(logn.tolist())):
        idx = np.nonzero(logn == k)[0]
        sa = np.concatenate([a[int(a_off[i]):int(a_off[i + 1])] for i in idx])
        sb = np.concatenate([b[int(b_off[i]):int(b_off[i + 1])] for i in idx])
        oa = np.concatenate([[0], np.cumsum(la[idx])]).astype(np.uint64)
        ob = np.concatenate([[0], np.cumsum(lb[idx])]).astype(np.uint64)
        limbs = int((la[idx] + lb[idx]).sum())
        da, db = cat.from_numpy(sa), cat.from_numpy(sb)
        c = torch.empty(limbs, dtype=torch.int32, device="cuda")
        g = cat.MulPlan(oa, ob, mode="graph")
        ms = _time_plan(g, da, db, c, reps)
        g.close()
        out["2^%d" % k] = {"products": int(len(idx)), "product_limbs": limbs, "ms": round(ms, 4),
                           "limbs_per_s": limbs / (ms / 1e3)}
    return out


def batch_bench(cat, steps):
    """The synthetic level-batch: 4,096 products, operand lengths log-uniform in
    [64, 65536] limbs (uneven), one graph replay vs one product per launch;
    then the same lengths with lb = la (balanced), and the uneven batch split
    by transform size."""
    import torch

    from tests import batch_inputs

    a, a_off, b, b_off = batch_inputs.level_batch(seed=0)
    la = a_off[1:] - a_off[:-1]
    lb = b_off[1:] - b_off[:-1]
    limbs = int((la + lb).sum())
    da, db = cat.from_numpy(a), cat.from_numpy(b)
    c = torch.empty(limbs, dtype=torch.int32, device="cuda")
    c2 = torch.empty_like(c)
    g = cat.MulPlan(a_off, b_off, mode="graph")
    p = cat.MulPlan(a_off, b_off, mode="plain")
    g(da, db, c)
    g.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g(da, db, c)
    torch.cuda.synchronize()
    ms_g = (time.perf_counter() - t0) * 1e3 / steps
    g.check()
    oracle_ok = None
    gpath = os.path.join(ROOT, "tests", "golden", "batch4096_digests.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            want = json.load(f)["uneven"]["sha256_128"]
        got = cat.to_numpy(c)
        d = [hashlib.sha256(got[int(g.c_off[i]):int(g.c_off[i + 1])].astype("<u4").tobytes()).hexdigest()[:32]
             for i in range(len(want))]
        oracle_ok = d == want
        if not oracle_ok:
            raise SystemExit("bench: level-batch products differ from the oracle's digests")
    p(da, db, c2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p(da, db, c2)
    torch.cuda.synchronize()
    ms_p = (time.perf_counter() - t0) * 1e3
    p.check()
    same = bool(torch.equal(c, c2))
    if not same:
        raise SystemExit("bench: batched and plain level-batch products differ")
    g.close()
    p.close()
    buckets = batch_buckets(cat, a, a_off, b, b_off)
    # balanced variant: lb = la
    a2, a2_off, b2, b2_off = batch_inputs.level_batch(seed=0, balanced=True)
    limbs2 = int((a2_off[1:] - a2_off[:-1]).sum() * 2)
    da2, db2 = cat.from_numpy(a2), cat.from_numpy(b2)
    c3 = torch.empty(limbs2, dtype=torch.int32, device="cuda")
    c4 = torch.empty_like(c3)
    g2 = cat.MulPlan(a2_off, b2_off, mode="graph")
    ms_b = _time_plan(g2, da2, db2, c3, steps)
    p2 = cat.MulPlan(a2_off, b2_off, mode="plain")
    p2(da2, db2, c4)
    p2.check()
    torch.cuda.synchronize()
    if not torch.equal(c3, c4):
        raise SystemExit("bench: batched and plain balanced products differ")
    g2.close()
    p2.close()
    balanced = {"products": 4096, "product_limbs": limbs2, "batched_graph_ms": round(ms_b, 3),
                "batched_limbs_per_s": limbs2 / (ms_b / 1e3), "batched_equals_plain": True,
                "inputs": "numpy default_rng(0): la = rint(2**U(6,16)) x 4096, lb = la, limbs U[0,2^32)"}
    return {"products": 4096, "product_limbs": limbs, "batched_graph_ms": round(ms_g, 3),
            "batched_limbs_per_s": limbs / (ms_g / 1e3), "plain_ms": round(ms_p, 3),
            "plain_limbs_per_s": limbs / (ms_p / 1e3), "speedup": round(ms_p / ms_g, 2),
            "batched_equals_plain": same, "every_product_equals_oracle_digest": oracle_ok,
            "inputs": "numpy default_rng(0): la, lb = rint(2**U(6,16)) x 4096 each, limbs U[0,2^32)",
            "by_transform_size": buckets, "balanced": balanced}


def phase_times(cat, n, reps=9):
    """Phase 1 (catalan_factor: sieve, exponents, groups, back to the host) and
    Phase 2 from that factorisation (prime_power_product, batched launches)
    as separate calls, medians of wall time around each synchronised call.
    The fused catalan_exact call avoids the host round trip between them."""
    import torch

    exps, off, primes = cat.factor(n)
    t = cat.product(exps, off, primes)
    torch.cuda.synchronize()
    t1, t2 = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        exps, off, primes = cat.factor(n)
        torch.cuda.synchronize()
        t1.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        t = cat.product(exps, off, primes)
        torch.cuda.synchronize()
        t2.append(time.perf_counter() - t0)
    return t, {"phase1_ms": round(sorted(t1)[reps // 2] * 1e3, 4), "phase2_ms": round(sorted(t2)[reps // 2] * 1e3, 4),
               "note": "separate synchronised calls (factorisation to the host, then its product); "
                       "the headline value is the fused call"}


def _prod_mod(lo: int, hi: int, q: int) -> int:
    """prod_{k=lo}^{hi} k mod q (q < 2^32), by a vectorised pairwise reduction."""
    import numpy as np

    if hi < lo:
        return 1 % q
    v = (np.arange(lo, hi + 1, dtype=np.uint64) % np.uint64(q))
    while len(v) > 1:
        if len(v) & 1:
            v = np.append(v, np.uint64(1))
        v = (v[0::2] * v[1::2]) % np.uint64(q)
    return int(v[0])


def ratio_bench(cat, reps=5):
    """Factorial ratios (the reconstruction engine on other exponent sources):
    the central binomial C(2*10^7, 10^7) and 10^6!, batched, checked by their
    residue mod the prime 2^32 - 5 from the product formula."""
    import numpy as np
    import torch

    q = 2**32 - 5
    out = {}
    for name, num, den in [("binomial_2e7_1e7", [2 * 10**7], [10**7, 10**7]), ("factorial_1e6", [10**6], [])]:
        want = _prod_mod(1, num[0], q)
        for d in den:
            want = want * pow(_prod_mod(1, d, q), q - 2, q) % q
        t = cat.ratio_exact(num, den)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            t = cat.ratio_exact(num, den)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        st = cat.stats()
        ms = float(np.median(ts)) * 1e3
        out[name] = {"num": num, "den": den, "ms": round(ms, 3), "result_limbs": int(t.numel()),
                     "product_limbs": st["product_limbs"], "limbs_per_s": st["product_limbs"] / (ms / 1e3),
                     "verified_mod_2p32_minus_5": cat.residues(t)[0] == want}
    return out


def decimal_bench(cat, reps=5):
    """Decimal text of C(10^7) and C(10^8) (radix-10^9 conversion on the GPU),
    checked by its nine-digit groups against the limbs modulo 10^9 +- 1."""
    import numpy as np
    import torch

    from tests import pins

    out = {}
    for n in (10**7, 10**8):
        t = cat.exact(n)
        text = cat.to_decimal_device(t)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            text = cat.to_decimal_device(t)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        st = cat.stats()
        s1, s2, _ = pins.decimal_group_residues(text)
        ok = s1 == pins.limbs_mod_torch(t, 10**9 - 1) and s2 == pins.limbs_mod_torch(t, 10**9 + 1)
        ms = float(np.median(ts)) * 1e3
        out["catalan_%s" % ("1e7" if n == 10**7 else "1e8")] = {
            "digits": int(text.numel()), "ms": round(ms, 3), "digits_per_s": text.numel() / (ms / 1e3),
            "levels": st["levels"], "products": st["products"], "verified_mod_1e9_pm_1": bool(ok)}
    return out


def _serve_once(cat, ex_kind, ns, gaps, lam, slots, budget, warm):
    """One run of the request stream: closed loop (everything queued at once)
    when lam is None, else Poisson arrivals at rate lam.  Returns the server
    and its requests."""
    from paper_2601_11621_amd.serve import BatchExecutor, GpuExecutor, Server

    ex = _serve_once.ex.get(ex_kind)
    if ex is None:
        ex = GpuExecutor(max_slots=slots) if ex_kind == "tickets" else BatchExecutor(max_slots=slots, max_batch=16)
        _serve_once.ex[ex_kind] = ex
    srv = Server(ex, budget_bytes=budget, max_slots=slots)
    if lam is None:
        reqs = [srv.submit(n, arrival=0.0) for n in ns]
    else:
        start = time.perf_counter() + 0.05
        arr = start + np.cumsum(gaps) / lam
        reqs = [srv.submit(n, arrival=float(a)) for n, a in zip(ns, arr)]
    t0 = time.perf_counter()
    srv.run()
    return srv, reqs, time.perf_counter() - t0


_serve_once.ex = {}


def serving_bench(cat, count=1100, warm=100, slots=None, budget=16 << 30, frac=0.7):
    """Request stream of catalan_exact(n), n = floor(10^(3 + 4u)) from
    default_rng(11621), served two ways: one ticket per request on its own
    stream (work overlapping across up to 4 streams), and continuous batching
    (the requests admitted in one step share one batch: one launch per tree
    level for all of them).  For each: closed-loop saturated throughput, then
    Poisson arrivals at `frac` of the ticket form's saturated rate (the same
    offered load for both), p50/p99 latency (arrival -> result on the device)
    and requests/s over the requests after the first `warm`; every output
    compared bit for bit with the same n computed alone and with the oracle's
    digest."""
    from paper_2601_11621_amd.serve import DONE
    from tests import batch_inputs

    ns, gaps = batch_inputs.serving_requests(seed=11621, count=count)
    ns = [int(x) for x in ns]
    gold = {}
    gpath = os.path.join(ROOT, "tests", "golden", "serving_digests.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            gold = json.load(f)["digests"]
    solo = {}
    # slots of each form: tickets beyond 16 gain nothing (4 streams); batches
    # need room for several batches in flight
    slots = slots or {"tickets": 16, "batched": 64}
    out = {"requests": count, "warmup_requests": warm, "slots": slots, "budget_bytes": budget,
           "inputs": "n = floor(10^(3+4u)), Poisson arrivals, numpy default_rng(11621)"}
    lam = None
    for kind in ("tickets", "batched"):
        _serve_once(cat, kind, ns, gaps, None, slots[kind], budget, warm)        # warm pools and plans
        srv, reqs, dt = _serve_once(cat, kind, ns, gaps, None, slots[kind], budget, warm)
        sat = len(ns) / dt
        if lam is None:
            lam = frac * sat
        def verify(reqs):
            bad = checked = 0
            for r in reqs:
                if r.state != DONE:
                    bad += 1
                    continue
                if r.n not in solo:
                    solo[r.n] = cat.to_numpy(cat.exact(r.n, mode="batched"))
                got = cat.to_numpy(r.result)
                if not np.array_equal(got, solo[r.n]):
                    bad += 1
                if str(r.n) in gold:
                    L, h = gold[str(r.n)]
                    checked += 1
                    if len(got) != L or hashlib.sha256(got.astype("<u4").tobytes()).hexdigest() != h:
                        bad += 1
                r.result = None
            if bad:
                raise SystemExit("bench: %d %s serving outputs differ from the same n alone or the oracle" % (bad, kind))
            return checked

        srv, reqs, _ = _serve_once(cat, kind, ns, gaps, lam, slots[kind], budget, warm)
        st = srv.stats(skip=warm)
        checked = verify(reqs)
        ex = _serve_once.ex[kind]
        out[kind] = {"saturated_req_per_s": round(sat, 1), "offered_req_per_s": round(lam, 1),
                     "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                     "mean_ms": round(st["mean_ms"], 3), "req_per_s": round(st["req_per_s"], 1),
                     "peak_active": st["peak_active"], "all_outputs_equal_solo": True,
                     "outputs_checked_against_oracle_digests": checked}
        if kind == "batched":
            out[kind]["batches"] = ex.batches
            out[kind]["requests_per_batch"] = round(ex.batched_requests / max(ex.batches, 1), 2)
            # at frac of its own saturated rate (beyond what the ticket form sustains)
            lam2 = frac * sat
            srv, reqs, _ = _serve_once(cat, kind, ns, gaps, lam2, slots[kind], budget, warm)
            st2 = srv.stats(skip=warm)
            verify(reqs)
            out[kind]["at_own_saturation"] = {"offered_req_per_s": round(lam2, 1), "p50_ms": round(st2["p50_ms"], 3),
                                              "p99_ms": round(st2["p99_ms"], 3),
                                              "req_per_s": round(st2["req_per_s"], 1)}
    # the headline keys keep their meaning: the batched form
    for key in ("p50_ms", "p99_ms", "req_per_s"):
        out[key] = out["batched"][key]
    return out


def steady_state(cat, kernel="k_ntt_lds", half=2048, count=1024, reps=10):
    """The transform kernel fed enough work to fill the GPU: one launch over
    `count` products of half x half limbs (N = 2 * half), timed per launch with
    the library's event timer; butterflies per second against the peak."""
    import torch

    rng = np.random.default_rng(1)
    off = np.arange(count + 1, dtype=np.uint64) * np.uint64(half)
    a = cat.from_numpy(rng.integers(0, 2**32, size=count * half, dtype=np.uint64).astype(np.uint32))
    plan = cat.MulPlan(off, off, mode="batched")
    c = torch.empty(2 * count * half, dtype=torch.int32, device="cuda")
    plan(a, a, c)
    plan.check()
    cat.timer_set(kernel)
    for _ in range(reps):
        plan(a, a, c)
    torch.cuda.synchronize()
    kms, launches, work = cat.timer_get()
    cat.timer_set(None)
    plan.check()
    plan.close()
    achieved = work / (kms / 1e3)
    return {"kernel": kernel, "workload": "%d products of %d x %d limbs (N = %d), one launch" % (count, half, half,
                                                                                              2 * half),
            "avg_launch_ms": round(kms / launches, 5), "achieved_Tbfly_s": round(achieved / 1e12, 4),
            "frac": round(achieved / PEAK_BFLY, 4), "frac_code_14_ops": round(achieved / PEAK_BFLY_CODE, 4)}


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True,
                             timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:  # noqa: BLE001 - informational only
        pass
    return platform.processor() or "unknown"


def cpu_baseline(n_sample, limbs, gpu_limbs_per_s):
    """The CPU oracle on a bounded sample of the workload: one full C(n_sample)
    with every host thread and again with one thread.  `value` is product
    limbs per second: `limbs` is the sum of la + lb over the product tree of
    C(n_sample) (the GPU's count at that n; the oracle multiplies the same
    factors in a tree of the same shape)."""
    import oracle

    res = {}
    for threads in (oracle.num_threads(), 1):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        c = oracle.catalan(n_sample)
        dt = time.perf_counter() - t0
        res[threads] = (dt, len(c))
    oracle.set_threads(0)
    nt = max(res)
    dt_all, L = res[nt]
    return {
        "value": limbs / dt_all,
        "unit": "limbs/s",
        "cores": nt,
        "kind": "oracle",
        "sample": "one full C(%d) by the CPU oracle (trial-division primes, Legendre exponents, Karatsuba product "
                  "tree, OpenMP over the nodes of a level) on %d threads: %.2f s for %d product limbs (%d result "
                  "limbs); one thread: %.2f s.  The oracle's cost per limb grows with n (Karatsuba), so its rate "
                  "at n = 2,050,572,903 is lower than this sample's" % (n_sample, nt, dt_all, limbs, L, res[1][0]),
        "n": n_sample,
        "seconds_all_threads": round(dt_all, 3),
        "seconds_one_thread": round(res[1][0], 3),
        "one_thread_limbs_per_s": limbs / res[1][0],
        "cpu_model": cpu_model(),
        "gpu_over_cpu": round(gpu_limbs_per_s / (limbs / dt_all), 1),
    }


def catalan_mode_times(cat, n, steps, plain_steps, out_bytes_limit=None):
    """C(n) batched (one graph replay per call, and plain launches without a
    graph) against the plain form (one product per launch), on the same GPU,
    every output checked against the oracle's digest."""
    import torch

    with open(GOLDEN) as f:
        gold = json.load(f).get(str(n))
    _, max_limbs, _ = cat.sizes(n)
    out = torch.empty(max_limbs, dtype=torch.int32, device="cuda")
    for _ in range(2):
        t = cat.exact(n, mode="graph", out=out)
    checks = check_output(cat, t, n, gold)
    st = cat.stats()
    ms_g = time_steps(cat, n, "graph", steps, out)
    t = cat.exact(n, mode="graph", out=out)
    check_output(cat, t, n, gold)
    ms_b = time_steps(cat, n, "batched", max(1, steps // 2), out)
    r = {"n": n, "graph_ms": round(ms_g, 4), "batched_no_graph_ms": round(ms_b, 4),
         "products": st["products"], "product_limbs": st["product_limbs"],
         "graph_limbs_per_s": st["product_limbs"] / (ms_g / 1e3), "verified": checks}
    if plain_steps > 0:
        cat.exact(n, mode="plain", out=out)
        ms_p = time_steps(cat, n, "plain", plain_steps, out)
        t = cat.exact(n, mode="plain", out=out)
        check_output(cat, t, n, gold)
        sp = cat.stats()
        r.update({"plain_ms": round(ms_p, 3), "plain_launches": sp["launches"],
                  "plain_limbs_per_s": st["product_limbs"] / (ms_p / 1e3),
                  "speedup_graph_vs_plain": round(ms_p / ms_g, 1)})
    del out
    torch.cuda.empty_cache()
    return r


def roofline(cat, n, out, steps, st, ms):
    """The dominant kernel of a step (most summed time, library event timer on
    batched launches), timed live over `steps` further steps: algorithmic
    butterflies per second against the 9-lane-op butterfly peak; the HBM
    counters of that kernel from the committed rocprofv3 summary when it was
    taken on the current sources; and the step's algorithmic HBM traffic
    (8 bytes per product limb) and overall butterfly rate."""
    kt = kernel_times(cat, n, out)
    dom = max(kt, key=lambda k: kt[k][0])
    cat.timer_set(dom)
    for _ in range(steps):
        cat.exact(n, mode="batched", out=out)
    kms, klaunch, kwork = cat.timer_get()
    cat.timer_set(None)
    avg_ms = kms / max(klaunch, 1)
    tr = load_traffic(dom, n)
    if dom in NTT_KERNELS:
        achieved = kwork / (kms / 1e3)
        roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved / 1e12, 4),
                "peak": round(PEAK_BFLY / 1e12, 4), "unit": "Tbfly/s", "frac": round(achieved / PEAK_BFLY, 4),
                "basis": "radix-2 butterflies: 3 primes x (2 forward + 1 inverse) x (M/2) log2 M per row of M "
                         "points (the row stages of each product's 9 (N/2) log2 N); peak = 256 CU x 64 lanes x "
                         "2.4 GHz / 9 lane-ops per butterfly",
                "frac_code_14_ops": round(achieved / PEAK_BFLY_CODE, 4)}
    else:
        per_limb = 16.0 if dom == "k_crt" else 8.0
        achieved = kwork * per_limb / (kms / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}
    roof["avg_launch_ms"] = round(avg_ms, 5)
    roof["launches"] = klaunch
    roof["work_per_launch"] = kwork / max(klaunch, 1)
    roof["traffic"] = tr.get("bytes_per_launch") if tr else None
    if tr:
        roof["traffic_GBps"] = round(tr["bytes_per_launch"] / (avg_ms / 1e3) / 1e9, 1)
        roof["traffic_hbm_frac"] = round(tr["bytes_per_launch"] / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    # the whole step: every NTT product's butterflies (the four transform
    # kernels' algorithmic counts) and the operands-in + product-out bytes
    bfly = sum(kt[k][2] for k in NTT_KERNELS if k in kt)
    step_s = ms / 1e3
    step = {"butterflies_per_step": bfly, "achieved_Tbfly_s": round(bfly / step_s / 1e12, 4),
            "frac": round(bfly / step_s / PEAK_BFLY, 4),
            "algorithmic_bytes_per_step": 8 * st["product_limbs"],
            "algorithmic_GBps": round(8 * st["product_limbs"] / step_s / 1e9, 1),
            "hbm_frac": round(8 * st["product_limbs"] / step_s / 1e9 / HBM_PEAK_GBS, 4)}
    kms_step = {k: round(v[0], 4) for k, v in kt.items()}
    return roof, step, kms_step, dom


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=HEADLINE_N)
    ap.add_argument("--plain-steps", type=int, default=1, help="plain-form steps of C(10^7) and C(10^8)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=10_000_000, help="n of the CPU oracle's sample")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the C(10^7) and C(10^8) comparisons")
    ap.add_argument("--no-batch", action="store_true", help="skip the 4,096-product level-batch measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream measurement")
    ap.add_argument("--no-ratio", action="store_true", help="skip the factorial-ratio measurement")
    ap.add_argument("--no-decimal", action="store_true", help="skip the decimal-text measurement")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--only-kernel", default="", help="profiling aid: run graph steps only")
    ap.add_argument("--valu-rates", action="store_true",
                    help="only measure the issue rate of the VALU instruction forms the butterflies use")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU (one MI355X); --gpus %d is not supported" % max(args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2601_11621_amd as cat

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "reps": 5}))
        return

    if args.valu_rates:
        cat.init(0)
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        lane_rate = cus * 64 * CLOCK_HZ          # one lane-op per lane per clock
        rates = {}
        for op in cat.VALU_OPS:
            r, ms = cat.valu_rate(op, 4096)
            r, ms = cat.valu_rate(op, max(64, int(4096 * 40.0 / max(ms, 1e-3))))   # about 40 ms per launch
            rates[op] = {"lane_ops_per_s": r, "ms": round(ms, 3), "of_full_rate": round(r / lane_rate, 4),
                         "cycles_per_wave64_instr": round(4.0 * lane_rate / r, 2)}
            log("bench: %-14s %.3e lane-ops/s = %.3f of %d CU x 64 lanes x %.1f GHz" %
                (op, r, r / lane_rate, cus, CLOCK_HZ / 1e9))
        print(json.dumps({"valu_rates": rates, "compute_units": cus, "clock_hz": CLOCK_HZ}))
        return

    cat.init(0)
    n = args.n
    gold = None
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            gold = json.load(f).get(str(n))
    _, max_limbs, wbytes = cat.sizes(n)
    out = torch.empty(max_limbs, dtype=torch.int32, device="cuda")

    log("bench: n=%d warmup=%d steps=%d workspace %.2f GB" % (n, args.warmup, args.steps, wbytes / 1e9))
    t0 = time.perf_counter()
    t = cat.exact(n, mode="graph", out=out)
    first_s = time.perf_counter() - t0
    for _ in range(max(args.warmup - 1, 0)):
        t = cat.exact(n, mode="graph", out=out)
    verified = check_output(cat, t, n, gold)
    st = cat.stats()
    ms = time_steps(cat, n, "graph", args.steps, out)
    t = cat.exact(n, mode="graph", out=out)
    check_output(cat, t, n, gold)
    if args.only_kernel:
        print(json.dumps({"ms_per_step": ms}))
        return
    product_limbs = st["product_limbs"]
    value = product_limbs / (ms / 1e3)
    log("bench: graph %.3f ms/step, %d products, %d product limbs" % (ms, st["products"], product_limbs))

    ms_batched = time_steps(cat, n, "batched", max(1, args.steps // 4), out)
    t2, phases = phase_times(cat, n, reps=5)
    phases["phase2_output_verified"] = bool(check_output(cat, t2, n, gold))
    del t2
    log("bench: phase 1 %.3f ms, phase 2 %.3f ms (separate calls)" % (phases["phase1_ms"], phases["phase2_ms"]))

    roof = step_roof = kms_step = None
    if not args.no_roofline:
        roof, step_roof, kms_step, dom = roofline(cat, n, out, args.steps, st, ms)
        # Phase 2 alone: the step less the separately timed Phase 1 (which runs
        # first in the same graph), and the separate Phase 2 call
        p2 = ms - phases["phase1_ms"]
        bf = step_roof["butterflies_per_step"]
        step_roof["phase2_ms_in_step"] = round(p2, 4)
        step_roof["phase2_frac"] = round(bf / (p2 / 1e3) / PEAK_BFLY, 4)
        step_roof["phase2_separate_call_frac"] = round(bf / (phases["phase2_ms"] / 1e3) / PEAK_BFLY, 4)
        if dom == "k_ntt_lds":
            roof["steady_state"] = steady_state(cat)
        log("bench: dominant kernel %s: %.4f ms avg over %d launches, frac %.3f" % (
            dom, roof["avg_launch_ms"], roof["launches"], roof["frac"]))
    # the fingerprint kernel on the result (the residues every check reads):
    # 4 B per limb read, against 8 TB/s
    fp = None
    if t.numel() >= (1 << 20):
        cat.residues(t)
        cat.timer_set("k_residues")
        for _ in range(5):
            cat.residues(t)
        rms, rl, rw = cat.timer_get()
        cat.timer_set(None)
        gbs = 4.0 * rw / (rms / 1e3) / 1e9
        fp = {"kernel": "k_residues", "limbs": int(t.numel()), "avg_launch_ms": round(rms / max(rl, 1), 4),
              "achieved_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        ftr = load_traffic("k_residues", args.n)
        fp["traffic"] = ftr.get("bytes_per_launch") if ftr else None
        log("bench: fingerprints %s" % fp)
    del out
    cat.release_workspaces()
    torch.cuda.empty_cache()

    secondary = None
    if not args.no_secondary:
        secondary = {}
        for n2 in (10**7, 10**8):
            if n2 == n:
                continue
            secondary["catalan_%s" % ("1e7" if n2 == 10**7 else "1e8")] = catalan_mode_times(
                cat, n2, max(3, args.steps // 2), 0 if args.no_plain else args.plain_steps)
            log("bench: C(%d) %s" % (n2, secondary["catalan_%s" % ("1e7" if n2 == 10**7 else "1e8")]))

    batch = None if args.no_batch else batch_bench(cat, max(3, args.steps // 4))
    if batch:
        log("bench: level-batch 4096: graph %.2f ms, plain %.1f ms" % (batch["batched_graph_ms"], batch["plain_ms"]))
    serving = None if args.no_serving else serving_bench(cat)
    if serving:
        log("bench: serving tickets %s" % serving["tickets"])
        log("bench: serving batched %s" % serving["batched"])
    ratios = None if args.no_ratio else ratio_bench(cat)
    if ratios:
        log("bench: ratios %s" % {k: v["ms"] for k, v in ratios.items()})
    decimal = None if args.no_decimal else decimal_bench(cat)
    if decimal:
        log("bench: decimal %s" % {k: v["ms"] for k, v in decimal.items()})
    cpu = None
    if not args.no_cpu:
        if secondary and "catalan_1e7" in secondary and args.cpu_n == 10**7:
            cpu_limbs = secondary["catalan_1e7"]["product_limbs"]
        else:
            cat.exact(args.cpu_n, mode="batched")
            cpu_limbs = cat.stats()["product_limbs"]
        cpu = cpu_baseline(args.cpu_n, cpu_limbs, value)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "limbs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "catalan_exact n=%d (Phase 1 device sieve + Phase 2 batched product tree; "
                               "the paper's Table 1 run)" % n if n == HEADLINE_N else
                               "catalan_exact n=%d (Phase 1 device sieve + Phase 2 batched product tree)" % n,
                   "n": n, "mode": "batched, one HIP graph per call", "products_per_step": st["products"],
                   "product_limbs_per_step": product_limbs, "result_limbs": int(t.numel()),
                   "primes": st["n_primes"], "tree_levels": st["levels"], "verified_bit_exact": bool(verified),
                   "checks": verified},
        "reconstruction_s": round(ms / 1e3, 6),
        "first_call_s": round(first_s, 3),
        "batched_no_graph_ms_per_step": round(ms_batched, 3),
        "phases": phases,
        "roofline": roof,
        "phase2_roofline": step_roof,
        "fingerprint_kernel": fp,
        "cpu_baseline": cpu,
        "batched_vs_plain": secondary,
        "level_batch_4096": batch,
        "serving": serving,
        "factorial_ratios": ratios,
        "decimal_text": decimal,
        "kernel_ms_per_step": kms_step,
        "paper_context": {"phase2_s": 1369.77, "total_s": 1549.14, "phase1_s": 179.37,
                          "n": 2050572903, "hardware": "AMD Ryzen 9 4900HS laptop, 16 GB, Python 3.11 + gmpy2 "
                                                      "(Sec. 5, Table 1)",
                          "table2_proposed_s": {"1e6": 2.923, "1e7": 6.817, "1e8": 62.835}},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
