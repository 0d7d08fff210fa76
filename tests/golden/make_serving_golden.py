"""Write tests/golden/serving_digests.json: for every distinct n of the seeded
serving request streams (the GPU serving tests' streams and the benchmark's
1,100-request stream), the limb count and SHA-256 of the CPU oracle's C(n).

Calls only ``oracle/`` for arithmetic; ``tests/batch_inputs.py`` supplies the
seeded request streams and holds no arithmetic of the method.

Usage:  python tests/golden/make_serving_golden.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from tests import batch_inputs  # noqa: E402

OUT = os.path.join(HERE, "serving_digests.json")

# the streams of tests/test_gpu_serve.py and of bench.py's serving run
STREAMS = [dict(seed=11621, count=60), dict(seed=7, count=80, lo_exp=3.0, hi_exp=6.0),
           dict(seed=5, count=60, lo_exp=3.0, hi_exp=6.3), dict(seed=11621, count=1100)]
EXTRA = [0, 1, 2, 13, 777, 1000, 1234, 3000, 5000, 20000, 10**4, 2 * 10**4, 3 * 10**4, 10**7]


def _save(data, digests):
    data["digests"] = digests
    data["streams"] = STREAMS
    with open(OUT + ".tmp", "w") as f:
        json.dump(data, f, indent=0, sort_keys=True)
    os.replace(OUT + ".tmp", OUT)


def main():
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_about"] = ("Limb count and SHA-256 (little-endian uint32 limbs) of the CPU oracle's C(n) for every "
                      "distinct n of the seeded serving streams; written by tests/golden/make_serving_golden.py, "
                      "which calls only oracle/ for arithmetic.")
    digests = data.get("digests", {})
    t0 = time.time()
    last = t0
    # stream by stream (the tests' streams first), saving as it goes
    for kw in [None] + STREAMS:
        ns = set(EXTRA) if kw is None else set(int(x) for x in batch_inputs.serving_requests(**kw)[0])
        for n in sorted(ns):
            if str(n) in digests:
                continue
            c = oracle.catalan(n)
            digests[str(n)] = [int(len(c)), hashlib.sha256(c.astype("<u4").tobytes()).hexdigest()]
            if time.time() - last > 30:
                _save(data, digests)
                last = time.time()
        _save(data, digests)
        print("stream", kw, len(digests), "digests", "%.1f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
