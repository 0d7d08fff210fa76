"""The two-phase file interface of the method (Sec. 3.1 and Sec. 3.2, Alg. 1
and Alg. 2): Phase 1 writes the factorisation as text grouped by exponent,
Phase 2 reads it back, rebuilds the integer and writes it as binary.

Text format (Sec. 3.1): a title line, then one block per exponent E, each a
header line "# exponent=E count=K" followed by the K primes of G_E in
ascending order, separated by blanks (written here in lines of at most
100,000 primes; any whitespace is accepted when reading).

Binary result: the magnitude of the integer as ceil(B/8) bytes (B its bit
length, as the size in Table 1), little-endian by default; the paper does not
state the byte order, so both orders can be written and hashed.
"""
from __future__ import annotations

import hashlib
from typing import Iterable, Tuple

import numpy as np

LINE_PRIMES = 100_000


def write_factorization(path: str, exps: Iterable[int], off: Iterable[int], primes, title: str) -> None:
    """Write groups (exps[g], primes[off[g]:off[g+1]]) as the paper's text file."""
    exps = [int(e) for e in exps]
    off = [int(o) for o in off]
    primes = np.asarray(primes, dtype=np.uint64)
    with open(path, "w") as f:
        f.write("# Prime factorization of %s\n" % title)
        for g, e in enumerate(exps):
            grp = primes[off[g]:off[g + 1]]
            f.write("# exponent=%d count=%d\n" % (e, len(grp)))
            for s in range(0, len(grp), LINE_PRIMES):
                f.write(" ".join(map(str, grp[s:s + LINE_PRIMES].tolist())))
                f.write("\n")


def read_factorization(path: str) -> Tuple[str, np.ndarray, np.ndarray, np.ndarray]:
    """(title, exps uint32[g], off uint64[g+1], primes uint32[]) from a text file
    of the paper's format; the counts in the headers are checked."""
    title = ""
    exps, counts, chunks = [], [], []
    cur = None
    with open(path) as f:
        for line in f:
            s = line.strip()
            if not s:
                continue
            if s.startswith("#"):
                body = s[1:].strip()
                if body.startswith("exponent="):
                    kv = dict(part.split("=", 1) for part in body.split())
                    exps.append(int(kv["exponent"]))
                    counts.append(int(kv["count"]))
                    cur = []
                    chunks.append(cur)
                elif body.startswith("Prime factorization of"):
                    title = body[len("Prime factorization of"):].strip()
                continue
            if cur is None:
                raise ValueError("primes before the first exponent header")
            cur.append(np.array(s.split(), dtype=np.uint64))
    groups = [np.concatenate(c) if c else np.zeros(0, dtype=np.uint64) for c in chunks]
    for e, k, grp in zip(exps, counts, groups):
        if len(grp) != k:
            raise ValueError("exponent %d: header count %d, %d primes listed" % (e, k, len(grp)))
        if grp.size and (grp.max() >= 2**32):
            raise ValueError("entries must be below 2^32")
    off = np.zeros(len(exps) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(g) for g in groups]) if groups else []
    primes = np.concatenate(groups).astype(np.uint32) if groups else np.zeros(0, dtype=np.uint32)
    return title, np.asarray(exps, dtype=np.uint32), off, primes


def limbs_to_bytes(limbs, byteorder: str = "little") -> bytes:
    """ceil(B/8) bytes of the magnitude held in little-endian uint32 limbs."""
    x = np.ascontiguousarray(np.asarray(limbs, dtype=np.uint32))
    n = len(x)
    while n > 0 and x[n - 1] == 0:
        n -= 1
    if n == 0:
        return b""
    bits = 32 * (n - 1) + int(x[n - 1]).bit_length()
    raw = x[:n].astype("<u4").tobytes()[: (bits + 7) // 8]
    return raw if byteorder == "little" else raw[::-1]


def write_bin(path: str, limbs, byteorder: str = "little") -> str:
    """Write the integer as ceil(B/8) bytes; returns the SHA-256 of the file."""
    data = limbs_to_bytes(limbs, byteorder)
    with open(path, "wb") as f:
        f.write(data)
    return hashlib.sha256(data).hexdigest()


def read_bin(path: str, byteorder: str = "little") -> np.ndarray:
    """The integer of a .bin file as normalised little-endian uint32 limbs."""
    with open(path, "rb") as f:
        data = f.read()
    if byteorder != "little":
        data = data[::-1]
    pad = (-len(data)) % 4
    x = np.frombuffer(data + b"\0" * pad, dtype="<u4").astype(np.uint32)
    n = len(x)
    while n > 1 and x[n - 1] == 0:
        n -= 1
    return x[:n] if n else np.ones(1, dtype=np.uint32)


def factorize_to_file(cat, n: int, path: str) -> None:
    """Phase 1 of C(n) on the GPU, written as the paper's text file."""
    exps, off, primes = cat.factor(n)
    write_factorization(path, exps, off, cat.to_numpy(primes), "Catalan(%d)" % n)


def reconstruct_from_file(cat, path: str, mode: str = "batched"):
    """Phase 2 from a factorisation file on the GPU: the integer as a device tensor."""
    _, exps, off, primes = read_factorization(path)
    bits = int(primes.max()).bit_length() if primes.size else 1
    return cat.product(exps, off, primes, max_entry_bits=max(1, bits), mode=mode)


def write_decimal(cat, x, path: str, chunk: int = 1 << 28) -> int:
    """The decimal text of the limb tensor x (converted on the GPU) written to
    `path` without a line break (the optional decimal output of Sec. 3.2);
    returns the digit count."""
    text = cat.to_decimal_device(x)
    with open(path, "wb") as f:
        for s in range(0, text.numel(), chunk):
            f.write(text[s:s + chunk].cpu().numpy().tobytes())
    return int(text.numel())
