"""Write tests/golden/pins_n2050572903.json: residues of C(2,050,572,903)
computed by the CPU oracle from the factorial definition in O(n) time
(C(n) mod 2^32-5 and C(n) mod 2^64).  Calls only oracle/."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

N = 2050572903


def main():
    t0 = time.time()
    r = oracle.catalan_mod_prime(N, 2**32 - 5)
    low = oracle.catalan_low64(N)
    out = {
        "_about": "Residues of C(2,050,572,903) from the CPU oracle's O(n) definition-based routines "
                  "(tests/golden/make_largest_pins.py calls only oracle/).",
        "n": N,
        "mod_2p32_minus_5": r,
        "low64": low,
        "limb0": low & 0xFFFFFFFF,
        "limb1": low >> 32,
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "pins_n2050572903.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
