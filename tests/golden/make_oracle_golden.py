"""Write tests/golden/oracle_catalan.json: digests of the CPU oracle's C(n).

Calls only the oracle (``oracle/``).  For each n it stores the limb count, the
SHA-256 of the little-endian limb bytes, the two lowest and two highest limbs
and the residue modulo 2^32 - 5, so the device result at the full benchmark
sizes can be compared without storing megabytes of limbs.

Usage:  python tests/golden/make_oracle_golden.py 100000 1000000 10000000 [...]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

OUT = os.path.join(HERE, "oracle_catalan.json")


def digest(n):
    t0 = time.time()
    c = oracle.catalan(n)
    dt = time.time() - t0
    q = 2**32 - 5
    r = 0
    for x in c[::-1].tolist():
        r = (r * (1 << 32) + x) % q
    return {
        "n_limbs": int(len(c)),
        "sha256_le_limbs": hashlib.sha256(c.astype("<u4").tobytes()).hexdigest(),
        "limb0": int(c[0]), "limb1": int(c[1]) if len(c) > 1 else 0,
        "limb_top": int(c[-1]), "limb_top_minus_1": int(c[-2]) if len(c) > 1 else 0,
        "mod_2p32_minus_5": r,
        "oracle_seconds": round(dt, 3), "oracle_threads": oracle.num_threads(),
    }


def main(ns):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_about"] = ("Digests of the CPU oracle's C(n) (LE uint32 limbs), written by "
                      "tests/golden/make_oracle_golden.py, which calls only oracle/.")
    for n in ns:
        data[str(n)] = digest(n)
        print(n, data[str(n)], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main([int(x) for x in sys.argv[1:]] or [100000, 1000000, 10000000])
