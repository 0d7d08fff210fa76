"""Benchmark: exact C(n) on one MI355X (default n = 10,000,000).

One step = one whole pass of the hot path: catalan_exact(n) — the device
sieve with Legendre exponents (Phase 1) and the batched product tree with
multi-prime NTT products (Phase 2) — launched as cached HIP graphs, with the
result verified bit-exact against the oracle's digest before a time is kept.

Prints ONE JSON line.  `value` is the whole-step throughput in product limbs
per second: the sum over every product of the tree (Q_e trees, powers, outer
product) of la + lb, divided by the step time.  The unbatched form (one
product per launch) is timed on the same GPU for the "vs plain" comparison,
the dominant kernel is timed live with HIP events for the roofline, and the
CPU oracle is timed on the host for the baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_catalan.json")
PROFILES = os.path.join(ROOT, "profiles")
METRIC = "C(n) exact-reconstruction time; batched bigint-mul limbs/s vs plain, bit-exact"

# MI355X figures: 256 CUs x 64 lanes x 2.4 GHz of 32-bit VALU issue; one modular
# radix-2 butterfly of this library issues 14 VALU instructions (Montgomery
# twiddle product: 3 multiplies + 4 other; modular add: 4; modular subtract: 3).
VALU_LANE_OPS = 256 * 64 * 2.4e9
BFLY_OPS = 14.0
PEAK_BFLY = VALU_LANE_OPS / BFLY_OPS
HBM_PEAK_GBS = 8000.0

CANDIDATES = ["k_row", "k_pass_fwd", "k_pass_inv", "k_ntt_lds", "k_crt", "k_school", "k_leaf"]
NTT_KERNELS = {"k_row", "k_pass_fwd", "k_pass_inv", "k_ntt_lds"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def check_output(cat, t, n, gold):
    """Bit-exact check of a device result against the oracle digest, or, for
    n = 2,050,572,903 (no oracle product), against Table 1's bit length and the
    oracle's definition-based residues."""
    if gold is None:
        pz = os.path.join(ROOT, "tests", "golden", "pins_n%d.json" % n)
        t1 = os.path.join(ROOT, "tests", "golden", "table1_n%d.json" % n)
        if not (os.path.exists(pz) and os.path.exists(t1)):
            return None
        with open(pz) as f:
            pz = json.load(f)
        with open(t1) as f:
            t1 = json.load(f)
        top = int(t[-1].item()) & 0xFFFFFFFF
        bits = 32 * (t.numel() - 1) + top.bit_length()
        low = cat.to_numpy(t[:2])
        r = cat.residues(t)
        ok = (bits == t1["bit_length"] and int(low[0]) == pz["limb0"] and int(low[1]) == pz["limb1"]
              and r[0] == pz["mod_2p32_minus_5"])
        if not ok:
            raise SystemExit("bench: C(%d) does NOT match Table 1 / residue pins" % n)
        return True
    got = cat.to_numpy(t)
    h = hashlib.sha256(got.astype("<u4").tobytes()).hexdigest()
    ok = (len(got) == gold["n_limbs"] and h == gold["sha256_le_limbs"])
    if not ok:
        raise SystemExit("bench: C(%d) does NOT match the oracle digest" % n)
    return True


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


def source_sha1():
    import glob

    h = hashlib.sha1()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2601_11621_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_traffic(kernel, n):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernels changed after the counters were taken."""
    path = os.path.join(PROFILES, "traffic_%s_n%d.json" % (kernel, n))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha1") != source_sha1():
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
            "batched_equals_plain": same,
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


def serving_bench(cat, count=1100, warm=100, slots=8, budget=16 << 30, frac=0.7):
    """Request stream of catalan_exact(n), n = floor(10^(3 + 4u)) from
    default_rng(11621): closed-loop saturation first, then Poisson arrivals at
    `frac` of that rate; p50/p99 latency (arrival -> result on the device) and
    requests/s over the requests after the first `warm`; every output compared
    bit for bit with the same n computed alone."""
    import numpy as np

    from paper_2601_11621_amd.serve import DONE, GpuExecutor, Server
    from tests import batch_inputs

    ns, gaps = batch_inputs.serving_requests(seed=11621, count=count)
    ns = [int(x) for x in ns]
    ex = GpuExecutor(max_slots=slots)
    # closed loop: everything queued at once
    srv = Server(ex, budget_bytes=budget, max_slots=slots)
    for n in ns:
        srv.submit(n, arrival=0.0)
    t0 = time.perf_counter()
    srv.run()
    sat = len(ns) / (time.perf_counter() - t0)
    # open loop at frac * saturation
    lam = frac * sat
    srv = Server(ex, budget_bytes=budget, max_slots=slots)
    start = time.perf_counter() + 0.05
    arr = start + np.cumsum(gaps) / lam
    reqs = [srv.submit(n, arrival=float(a)) for n, a in zip(ns, arr)]
    srv.run()
    st = srv.stats(skip=warm)
    bad = 0
    solo = {}
    for r in reqs:
        if r.state != DONE:
            bad += 1
            continue
        if r.n not in solo:
            solo[r.n] = cat.to_numpy(cat.exact(r.n, mode="batched"))
        if not np.array_equal(cat.to_numpy(r.result), solo[r.n]):
            bad += 1
    if bad:
        raise SystemExit("bench: %d serving outputs differ from the same n alone" % bad)
    return {"requests": count, "warmup_requests": warm, "slots": slots, "budget_bytes": budget,
            "saturated_req_per_s": round(sat, 1), "offered_req_per_s": round(lam, 1),
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3), "mean_ms": round(st["mean_ms"], 3),
            "req_per_s": round(st["req_per_s"], 1), "peak_active": st["peak_active"],
            "all_outputs_equal_solo": True,
            "inputs": "n = floor(10^(3+4u)), Poisson arrivals, numpy default_rng(11621)"}


def steady_state(cat, kernel="k_ntt_lds", half=2048, count=1024, reps=10):
    """The transform kernel fed enough work to fill the GPU: one launch over
    `count` products of half x half limbs (N = 2 * half), timed per launch with
    the library's event timer; butterflies per second against the VALU peak."""
    import numpy as np
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
            "avg_launch_ms": round(kms / launches, 5), "achieved": round(achieved / 1e12, 4),
            "frac": round(achieved / PEAK_BFLY, 4)}


def cpu_baseline(n, product_limbs):
    import oracle

    t0 = time.perf_counter()
    c = oracle.catalan(n)
    dt = time.perf_counter() - t0
    return {
        "value": product_limbs / dt,
        "unit": "limbs/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "one full C(%d) by the CPU oracle (trial-division primes, Legendre exponents, "
                  "Karatsuba product tree, OpenMP over tree nodes): %.2f s; value = the GPU step's "
                  "product limbs / that time" % (n, dt),
        "seconds": round(dt, 3),
        "limbs": int(len(c)),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 4,096-product level-batch measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream measurement")
    ap.add_argument("--no-ratio", action="store_true", help="skip the factorial-ratio measurement")
    ap.add_argument("--no-decimal", action="store_true", help="skip the decimal-text measurement")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--only-kernel", default="", help="profiling aid: run graph steps only")
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

    cat.init(0)
    n = args.n
    gold = None
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            gold = json.load(f).get(str(n))
    _, max_limbs, _ = cat.sizes(n)
    out = torch.empty(max_limbs, dtype=torch.int32, device="cuda")

    log("bench: n=%d warmup=%d steps=%d" % (n, args.warmup, args.steps))
    for _ in range(max(args.warmup, 1)):
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

    # batched without graph (launch overhead visible) and the plain form
    ms_batched = time_steps(cat, n, "batched", max(1, args.steps // 4), out)
    t2, phases = phase_times(cat, n)
    phases["phase2_output_verified"] = bool(check_output(cat, t2, n, gold))
    log("bench: phase 1 %.3f ms, phase 2 %.3f ms (separate calls)" % (phases["phase1_ms"], phases["phase2_ms"]))
    plain = None
    if not args.no_plain and args.plain_steps > 0:
        cat.exact(n, mode="plain", out=out)   # plan + warm
        ms_plain = time_steps(cat, n, "plain", args.plain_steps, out)
        t = cat.exact(n, mode="plain", out=out)
        check_output(cat, t, n, gold)
        sp = cat.stats()
        plain = {"ms_per_step": round(ms_plain, 3), "limbs_per_s": product_limbs / (ms_plain / 1e3),
                 "launches_per_step": sp["launches"], "speedup_batched_graph_vs_plain": round(ms_plain / ms, 2)}
        log("bench: plain %.1f ms/step (%d launches)" % (ms_plain, sp["launches"]))

    roof = None
    kt = None
    if not args.no_roofline:
        kt = kernel_times(cat, n, out)
        dom = max(kt, key=lambda k: kt[k][0])
        # live measurement of the dominant kernel over the timed steps (batched launches)
        cat.timer_set(dom)
        for _ in range(args.steps):
            cat.exact(n, mode="batched", out=out)
        kms, klaunch, kwork = cat.timer_get()
        cat.timer_set(None)
        avg_ms = kms / max(klaunch, 1)
        if dom in NTT_KERNELS:
            achieved = kwork / (kms / 1e3) / 1e12
            roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 4), "peak": round(PEAK_BFLY / 1e12, 4),
                    "unit": "Tbfly/s", "frac": round(achieved * 1e12 / PEAK_BFLY, 4),
                    "avg_launch_ms": round(avg_ms, 5), "launches": klaunch}
        else:
            # HBM-bound kernels: algorithmic bytes (12 B per limb read as residues + 4 B written for k_crt)
            per_limb = 16.0 if dom == "k_crt" else 8.0
            achieved = kwork * per_limb / (kms / 1e3) / 1e9
            roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "avg_launch_ms": round(avg_ms, 5), "launches": klaunch}
        tr = load_traffic(dom, n)
        roof["traffic"] = tr.get("bytes_per_launch") if tr else None
        if dom == "k_ntt_lds":
            roof["steady_state"] = steady_state(cat)
        log("bench: dominant kernel %s: %.4f ms avg over %d launches" % (dom, avg_ms, klaunch))

    batch = None if args.no_batch else batch_bench(cat, max(3, args.steps // 4))
    if batch:
        log("bench: level-batch 4096: graph %.2f ms, plain %.1f ms" % (batch["batched_graph_ms"], batch["plain_ms"]))
    serving = None if args.no_serving else serving_bench(cat)
    if serving:
        log("bench: serving p50 %.2f ms p99 %.2f ms %.0f req/s" % (serving["p50_ms"], serving["p99_ms"],
                                                                  serving["req_per_s"]))
    ratios = None if args.no_ratio else ratio_bench(cat)
    if ratios:
        log("bench: ratios %s" % {k: v["ms"] for k, v in ratios.items()})
    decimal = None if args.no_decimal else decimal_bench(cat)
    if decimal:
        log("bench: decimal %s" % {k: v["ms"] for k, v in decimal.items()})
    cpu = None if args.no_cpu else cpu_baseline(n, product_limbs)

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
        "config": {"workload": "catalan_exact n=%d (Phase 1 sieve + Phase 2 product tree)" % n, "n": n,
                   "mode": "batched, one HIP graph per call", "products_per_step": st["products"],
                   "product_limbs_per_step": product_limbs, "result_limbs": int(t.numel()),
                   "primes": st["n_primes"], "tree_levels": st["levels"], "verified_bit_exact": bool(verified)},
        "reconstruction_s": round(ms / 1e3, 6),
        "batched_no_graph_ms_per_step": round(ms_batched, 3),
        "phases": phases,
        "plain": plain,
        "roofline": roof,
        "cpu_baseline": cpu,
        "level_batch_4096": batch,
        "serving": serving,
        "factorial_ratios": ratios,
        "decimal_text": decimal,
        "kernel_ms_per_step": {k: round(v[0], 4) for k, v in kt.items()} if kt else None,
        "paper_context": {"wall_s_n1e7": 6.817, "hardware": "AMD Ryzen 9 4900HS laptop, Python 3.11 + gmpy2 "
                                                            "(Table 2, proposed algorithm)"},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
