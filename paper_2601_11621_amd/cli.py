"""Command line for the two-phase workflow of the method (Sec. 3.1 and
Sec. 3.2, Alg. 1 and Alg. 2), every step on the GPU:

    python -m paper_2601_11621_amd.cli factor N --out catalan_N_factorization.txt
        Phase 1: the factorisation of C(N) as the grouped text file.
    python -m paper_2601_11621_amd.cli rebuild FILE --bin OUT.bin [--txt OUT.txt]
        Phase 2 from a factorisation file: the integer as ceil(B/8) bytes
        with its SHA-256, and optionally the decimal text.
    python -m paper_2601_11621_amd.cli exact N [--bin OUT.bin] [--txt OUT.txt] [--decimal]
        Both phases; prints the time, bit length and digit count.

Options: --byteorder little|big for the binary file (the paper does not state
one), --reps R to time R calls (and R decimal conversions) after a warm-up one.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def _parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser(prog="python -m paper_2601_11621_amd.cli", description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    f = sub.add_parser("factor", help="Phase 1: write the factorisation text file")
    f.add_argument("n", type=int)
    f.add_argument("--out", required=True)
    r = sub.add_parser("rebuild", help="Phase 2 from a factorisation text file")
    r.add_argument("file")
    r.add_argument("--bin")
    r.add_argument("--txt")
    r.add_argument("--byteorder", choices=["little", "big"], default="little")
    e = sub.add_parser("exact", help="C(n) by both phases")
    e.add_argument("n", type=int)
    e.add_argument("--bin")
    e.add_argument("--txt")
    e.add_argument("--decimal", action="store_true", help="convert to decimal text on the GPU (timed)")
    e.add_argument("--byteorder", choices=["little", "big"], default="little")
    e.add_argument("--reps", type=int, default=0)
    return ap


def _finish(cat, t, args, info: dict) -> dict:
    import torch

    from . import factorfile

    L = int(t.numel())
    top = int(t[-1].item()) & 0xFFFFFFFF
    info["limbs"] = L
    info["bits"] = 32 * (L - 1) + top.bit_length()
    if args.bin:
        info["bin"] = args.bin
        info["sha256"] = factorfile.write_bin(args.bin, cat.to_numpy(t), args.byteorder)
    if args.txt or getattr(args, "decimal", False):
        ts = []
        for _ in range(max(1, getattr(args, "reps", 0))):
            t0 = time.perf_counter()
            text = cat.to_decimal_device(t)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        info["decimal_s"] = round(sorted(ts)[len(ts) // 2], 6)
        info["digits"] = int(text.numel())
        if args.txt:
            with open(args.txt, "wb") as fh:
                for s in range(0, text.numel(), 1 << 28):
                    fh.write(text[s:s + (1 << 28)].cpu().numpy().tobytes())
            info["txt"] = args.txt
    return info


def main(argv=None) -> int:
    args = _parser().parse_args(argv)
    import torch

    import paper_2601_11621_amd as cat
    from . import factorfile

    torch.cuda.set_device(0)
    cat.init(0)
    if args.cmd == "factor":
        t0 = time.perf_counter()
        factorfile.factorize_to_file(cat, args.n, args.out)
        print(json.dumps({"n": args.n, "factorization": args.out, "seconds": round(time.perf_counter() - t0, 6)}))
        return 0
    if args.cmd == "rebuild":
        t0 = time.perf_counter()
        t = factorfile.reconstruct_from_file(cat, args.file)
        torch.cuda.synchronize()
        info = {"file": args.file, "seconds": round(time.perf_counter() - t0, 6)}
        print(json.dumps(_finish(cat, t, args, info)))
        return 0
    t = cat.exact(args.n)
    torch.cuda.synchronize()
    ts = []
    for _ in range(max(0, args.reps)):
        t0 = time.perf_counter()
        t = cat.exact(args.n)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    info = {"n": args.n}
    if ts:
        info["seconds_median"] = round(sorted(ts)[len(ts) // 2], 6)
    print(json.dumps(_finish(cat, t, args, info)))
    return 0


if __name__ == "__main__":
    sys.exit(main())
