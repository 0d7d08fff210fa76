"""Write tests/golden/batch4096_digests.json: the SHA-256 of every product of
the seeded 4,096-product level batch (and of its balanced variant), each
computed by the CPU oracle's multiplication (schoolbook / Karatsuba).

Calls only ``oracle/`` for arithmetic; ``tests/batch_inputs.py`` supplies the
seeded operands and holds no arithmetic of the method.  The digest of a
product is over its la + lb little-endian uint32 limbs (not normalised), the
layout bigint_mul_batched writes.

Usage:  python tests/golden/make_batch_golden.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from tests import batch_inputs  # noqa: E402

OUT = os.path.join(HERE, "batch4096_digests.json")


def digests(balanced):
    a, a_off, b, b_off = batch_inputs.level_batch(seed=0, balanced=balanced)
    t0 = time.time()
    c, c_off = oracle.mul_batched(a, a_off, b, b_off)
    dt = time.time() - t0
    out = []
    for i in range(len(a_off) - 1):
        ci = c[int(c_off[i]):int(c_off[i + 1])]
        out.append(hashlib.sha256(ci.astype("<u4").tobytes()).hexdigest()[:32])
    return out, dt, int(c_off[-1])


def main():
    data = {"_about": "First 128 bits of the SHA-256 of every product (la + lb little-endian uint32 limbs) of "
                      "the seed-0 4,096-product level batch, by the CPU oracle's multiplication; written by "
                      "tests/golden/make_batch_golden.py, which calls only oracle/ for arithmetic."}
    for name, bal in (("uneven", False), ("balanced", True)):
        d, dt, limbs = digests(bal)
        data[name] = {"products": len(d), "product_limbs": limbs, "oracle_seconds": round(dt, 1),
                      "oracle_threads": oracle.num_threads(), "sha256_128": d}
        print(name, len(d), "products", limbs, "limbs", "%.1f s" % dt, flush=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=0)


if __name__ == "__main__":
    main()
