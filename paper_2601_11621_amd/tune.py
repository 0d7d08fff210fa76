"""Autotuner of the product schedule (per transform-length bucket).

For every bucket 2^k it times the valid schedules on a synthetic level of
balanced products (la = lb = 2^(k-1) limbs, about 2^22 coefficients in all, as
in a tree level) and keeps the fastest:

  * k <= 8:  schoolbook kernel vs the one-workgroup transform (this sets the
             schoolbook threshold on operand length);
  * k <= 14: one-workgroup transform with tiles of 2^12, 2^13 or 2^14 slots
             (products per workgroup and workgroup size: 2^(t-k) and 2^t / 16
             threads) vs the four-step transform with rows of 2^8 .. 2^(k-1);
  * k > 14:  four-step transform, rows of 2^10 .. 2^14, column passes of at
             most 2^6 / 2^8 / 2^10 points.

Every candidate's output is compared bit for bit with the default schedule's;
a candidate that differs is an error (schedules change speed, never bits).

    python -m paper_2601_11621_amd.tune --max-k 24 --out paper_2601_11621_amd/tuning/gfx950.json
    python -m paper_2601_11621_amd.tune --min-k 25 --max-k 27 \
        --merge paper_2601_11621_amd/tuning/gfx950.json --out paper_2601_11621_amd/tuning/gfx950.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np


def _time_plan(cat, a_off, b_off, da, db, c, reps):
    import torch

    plan = cat.MulPlan(a_off, b_off, mode="graph")
    plan(da, db, c)
    plan.check()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan(da, db, c)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    plan.close()
    return float(np.median(ts)) * 1e3


def autotune(max_k: int = 24, reps: int = 5, total_log2: int = 22, verbose: bool = True, min_k: int = 7,
             start: dict | None = None) -> dict:
    """Tune buckets min_k..max_k.  `start` (a previous result) supplies the
    table and measurements of the other buckets; the schoolbook threshold is
    only re-decided when min_k <= 8."""
    import torch

    import paper_2601_11621_amd as cat

    cat.init(0, tuned=False)
    cat.set_tuning(None)
    base = cat.get_tuning()
    table = json.loads(json.dumps(start["table"] if start else base))
    meas = {int(k): v for k, v in (start or {}).get("ms", {}).items()}
    rng = np.random.default_rng(2024)
    school_max = 0 if min_k <= 8 else table["school_max"]
    for k in range(min_k, max_k + 1):
        half = 1 << (k - 1)
        count = max(1, 1 << max(0, total_log2 - k))
        la = np.full(count, half, dtype=np.int64)
        a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
        b_off = a_off.copy()
        a = rng.integers(0, 2**32, size=int(a_off[-1]), dtype=np.uint64).astype(np.uint32)
        b = rng.integers(0, 2**32, size=int(b_off[-1]), dtype=np.uint64).astype(np.uint32)
        da, db = cat.from_numpy(a), cat.from_numpy(b)
        c = torch.empty(int(2 * a_off[-1]), dtype=torch.int32, device="cuda")
        # reference bits: the default schedule
        cat.set_tuning(base)
        ref_plan = cat.MulPlan(a_off, b_off, mode="batched")
        ref = torch.empty_like(c)
        ref_plan(da, db, ref)
        ref_plan.check()
        ref_plan.close()
        cands = []
        if half <= 128:
            cands.append(("school", {"school_max": 128}))
        if k <= 14:
            seen = set()
            for lt in (12, 13, 14):
                # the tile the library uses: at least the transform, at most 64 products
                eff = max(k, min(lt, k + 6, 14))
                if eff in seen:
                    continue
                seen.add(eff)
                cands.append(("lds_t%d" % eff, {"school_max": min(half - 1, 128) if half <= 128 else 128, "cls": 1,
                                                "log_row": lt}))
            for lr in range(8, k):
                cands.append(("rows%d" % lr, {"school_max": min(half - 1, 128) if half <= 128 else 128, "cls": 2,
                                              "log_row": lr, "log_pass": 10}))
        else:
            for lr in (10, 11, 12, 13, 14):
                for lp in (6, 8, 10):
                    if k - lr > 0:
                        cands.append(("rows%d_pass%d" % (lr, lp),
                                      {"school_max": 128, "cls": 2, "log_row": lr, "log_pass": lp}))
        res = {}
        for name, cfg in cands:
            t = json.loads(json.dumps(table))
            t["school_max"] = cfg["school_max"]
            if "cls" in cfg:
                t["cls"][k] = cfg["cls"]
                t["log_row"][k] = cfg["log_row"]
                if cfg["cls"] == 2:
                    t["log_pass"][k] = cfg["log_pass"]
            try:
                cat.set_tuning(t)
            except Exception:
                continue
            ms = _time_plan(cat, a_off, b_off, da, db, c, reps)
            if not torch.equal(c, ref):
                raise RuntimeError("schedule %s of bucket 2^%d changed the product bits" % (name, k))
            res[name] = (ms, cfg)
        best = min(res, key=lambda x: res[x][0])
        cfg = res[best][1]
        if best == "school":
            school_max = half
        else:
            if "cls" in cfg:
                table["cls"][k] = cfg["cls"]
                table["log_row"][k] = cfg["log_row"]
                if cfg["cls"] == 2:
                    table["log_pass"][k] = cfg["log_pass"]
        meas[k] = {n: round(v[0], 4) for n, v in res.items()}
        meas = dict(sorted(meas.items()))
        if verbose:
            print("bucket 2^%d (%d products of %d limbs): best %s  %s" % (k, count, half, best, meas[k]),
                  flush=True)
        del da, db, c, ref
        torch.cuda.empty_cache()
    table["school_max"] = max(school_max, 1)
    cat.set_tuning(table)
    props = torch.cuda.get_device_properties(0)
    return {"arch": getattr(props, "gcnArchName", "gfx950"),
            "device": "%s, %d compute units" % (props.name, props.multi_processor_count), "reps": reps,
            "workload": "per bucket 2^k: 2^max(0,%d-k) products of 2^(k-1) x 2^(k-1) limbs" % total_log2,
            "table": table, "ms": meas}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--min-k", type=int, default=7)
    ap.add_argument("--max-k", type=int, default=24)
    ap.add_argument("--merge", default=None, help="previous result: keep its other buckets")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--total-log2", type=int, default=22, help="coefficient slots per bucket (log2)")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning",
                                                  "gfx950.json"))
    args = ap.parse_args()
    start = None
    if args.merge:
        with open(args.merge) as f:
            start = json.load(f)
    res = autotune(args.max_k, args.reps, total_log2=args.total_log2, min_k=args.min_k, start=start)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
