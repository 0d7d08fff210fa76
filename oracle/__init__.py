"""CPU oracle for the exact Catalan-number method (arXiv 2601.11621).

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The product path (the HIP
library and its binding) never imports this package, and this package never
imports the product path; the two share no code.

The arithmetic lives in ``catalan_oracle.c`` (plain C, gcc), which follows the
paper step by step: primes by trial division, Legendre exponents (Sec. 2),
groups G_e (Sec. 3.1, Alg. 1), Q_e by balanced product tree, P_e = Q_e^e by
square-and-multiply and C(n) = prod_e P_e (Sec. 3.2, Alg. 2).  This module
only builds the shared object and marshals arguments with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "catalan_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_OK, ORC_EINVAL, ORC_ERANGE, ORC_ENOMEM, ORC_EINTERNAL = 0, -1, -2, -3, -5

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    szp = ctypes.POINTER(ctypes.c_size_t)
    lib.orc_primes.argtypes = [ctypes.c_uint64, u32p, ctypes.c_size_t]
    lib.orc_primes.restype = ctypes.c_size_t
    lib.orc_pi_bound.argtypes = [ctypes.c_uint64]
    lib.orc_pi_bound.restype = ctypes.c_size_t
    lib.orc_legendre.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.orc_legendre.restype = ctypes.c_uint64
    lib.orc_exponents.argtypes = [ctypes.c_uint64, u32p, ctypes.c_size_t, i32p]
    lib.orc_exponents.restype = ctypes.c_int
    lib.orc_factor.argtypes = [ctypes.c_uint64, u32p, ctypes.c_size_t, u32p, u64p,
                               u32p, szp]
    lib.orc_factor.restype = ctypes.c_int
    lib.orc_mul.argtypes = [u32p, ctypes.c_size_t, u32p, ctypes.c_size_t, u32p]
    lib.orc_mul.restype = None
    lib.orc_mul_batched.argtypes = [ctypes.c_size_t, u32p, u64p, u32p, u64p, u32p, u64p]
    lib.orc_mul_batched.restype = None
    lib.orc_catalan.argtypes = [ctypes.c_uint64, u32p, ctypes.c_size_t, szp]
    lib.orc_catalan.restype = ctypes.c_int
    lib.orc_catalan_limbs_bound.argtypes = [ctypes.c_uint64]
    lib.orc_catalan_limbs_bound.restype = ctypes.c_size_t
    lib.orc_product.argtypes = [u32p, u64p, ctypes.c_size_t, u32p, ctypes.c_size_t, szp]
    lib.orc_product.restype = ctypes.c_int
    lib.orc_set_fault.argtypes = [ctypes.c_int]
    lib.orc_set_fault.restype = None
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads.restype = None
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_catalan_mod_prime.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.orc_catalan_mod_prime.restype = ctypes.c_uint64
    lib.orc_catalan_low64.argtypes = [ctypes.c_uint64]
    lib.orc_ratio_factor.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_size_t, u32p, u64p, ctypes.c_size_t, szp]
    lib.orc_ratio_factor.restype = ctypes.c_int
    lib.orc_ratio.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_size_t, u32p, ctypes.c_size_t, szp]
    lib.orc_ratio.restype = ctypes.c_int
    lib.orc_catalan_low64.restype = ctypes.c_uint64
    lib.orc_to_decimal.argtypes = [u32p, ctypes.c_size_t, ctypes.c_char_p, ctypes.c_size_t]
    lib.orc_to_decimal.restype = ctypes.c_size_t
    _lib = lib
    return lib


def _p(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def set_fault(code: int) -> None:
    """Plant a known mistake in the oracle (0 = none).  Tests use it to show
    that the pins reject a wrong oracle."""
    _load().orc_set_fault(int(code))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(t: int) -> None:
    """Threads of the oracle's parallel loops (t <= 0: the runtime's default)."""
    _load().orc_set_threads(int(t))


def primes(limit: int) -> np.ndarray:
    """All primes <= limit, ascending, by trial division."""
    lib = _load()
    cap = lib.orc_pi_bound(limit)
    out = np.zeros(max(cap, 1), dtype=np.uint32)
    cnt = lib.orc_primes(limit, _p(out, ctypes.c_uint32), cap)
    if cnt == ctypes.c_size_t(-1).value:
        raise RuntimeError("prime bound too small")
    return out[:cnt].copy()


def legendre(m: int, p: int) -> int:
    """v_p(m!) by Legendre's formula."""
    return int(_load().orc_legendre(m, p))


def exponents(n: int, prime_list: np.ndarray) -> np.ndarray:
    """e_p = v_p((2n)!) - 2 v_p(n!) - v_p(n+1) for each prime of the list."""
    lib = _load()
    pr = np.ascontiguousarray(prime_list, dtype=np.uint32)
    out = np.zeros(max(len(pr), 1), dtype=np.int32)
    st = lib.orc_exponents(n, _p(pr, ctypes.c_uint32), len(pr), _p(out, ctypes.c_int32))
    if st != ORC_OK:
        raise RuntimeError("orc_exponents failed: %d" % st)
    return out[: len(pr)].copy()


def factor(n: int):
    """Groups G_e of C(n): returns (exps uint32[g], off uint64[g+1], primes uint32[...])."""
    lib = _load()
    cap = lib.orc_pi_bound(2 * n)
    pr = np.zeros(max(cap, 1), dtype=np.uint32)
    exps = np.zeros(64, dtype=np.uint32)
    off = np.zeros(65, dtype=np.uint64)
    ng = ctypes.c_uint32(0)
    npr = ctypes.c_size_t(0)
    st = lib.orc_factor(n, _p(pr, ctypes.c_uint32), cap, _p(exps, ctypes.c_uint32),
                        _p(off, ctypes.c_uint64), ctypes.byref(ng), ctypes.byref(npr))
    if st != ORC_OK:
        raise RuntimeError("orc_factor failed: %d" % st)
    g = ng.value
    return exps[:g].copy(), off[: g + 1].copy(), pr[: npr.value].copy()


def mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Exact product of two LE uint32 limb vectors; len(a)+len(b) limbs."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    c = np.zeros(max(len(a) + len(b), 1), dtype=np.uint32)
    lib.orc_mul(_p(a, ctypes.c_uint32), len(a), _p(b, ctypes.c_uint32), len(b),
                _p(c, ctypes.c_uint32))
    return c[: len(a) + len(b)].copy()


def mul_batched(a_flat, a_off, b_flat, b_off):
    """c_i = a_i * b_i for a batch given as flat limb arrays with offsets."""
    lib = _load()
    a_flat = np.ascontiguousarray(a_flat, dtype=np.uint32)
    b_flat = np.ascontiguousarray(b_flat, dtype=np.uint32)
    a_off = np.ascontiguousarray(a_off, dtype=np.uint64)
    b_off = np.ascontiguousarray(b_off, dtype=np.uint64)
    batch = len(a_off) - 1
    lens = (a_off[1:] - a_off[:-1]) + (b_off[1:] - b_off[:-1])
    c_off = np.zeros(batch + 1, dtype=np.uint64)
    c_off[1:] = np.cumsum(lens)
    c = np.zeros(max(int(c_off[-1]), 1), dtype=np.uint32)
    lib.orc_mul_batched(batch, _p(a_flat, ctypes.c_uint32), _p(a_off, ctypes.c_uint64),
                        _p(b_flat, ctypes.c_uint32), _p(b_off, ctypes.c_uint64),
                        _p(c, ctypes.c_uint32), _p(c_off, ctypes.c_uint64))
    return c[: int(c_off[-1])].copy(), c_off


def catalan(n: int) -> np.ndarray:
    """C(n) as normalised LE uint32 limbs (C(0) = C(1) = [1])."""
    lib = _load()
    cap = lib.orc_catalan_limbs_bound(n)
    out = np.zeros(cap, dtype=np.uint32)
    ln = ctypes.c_size_t(0)
    st = lib.orc_catalan(n, _p(out, ctypes.c_uint32), cap, ctypes.byref(ln))
    if st != ORC_OK:
        raise RuntimeError("orc_catalan failed: %d" % st)
    return out[: ln.value].copy()


def product(items) -> np.ndarray:
    """Balanced-tree product of a list of LE uint32 limb vectors (normalised)."""
    lib = _load()
    items = [np.ascontiguousarray(x, dtype=np.uint32) for x in items]
    offs = np.zeros(len(items) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(x) for x in items]) if items else []
    flat = np.concatenate(items) if items else np.zeros(1, dtype=np.uint32)
    cap = int(offs[-1]) + 1
    out = np.zeros(cap, dtype=np.uint32)
    ln = ctypes.c_size_t(0)
    st = lib.orc_product(_p(flat, ctypes.c_uint32), _p(offs, ctypes.c_uint64), len(items),
                         _p(out, ctypes.c_uint32), cap, ctypes.byref(ln))
    if st != ORC_OK:
        raise RuntimeError("orc_product failed: %d" % st)
    return out[: ln.value].copy()


def catalan_mod_prime(n: int, q: int) -> int:
    """C(n) mod a prime q > 2n from the factorial definition, O(n)."""
    return int(_load().orc_catalan_mod_prime(n, q))


def catalan_low64(n: int) -> int:
    """C(n) mod 2^64 from odd-part products and v_2 = popcount(n+1) - 1, O(n)."""
    return int(_load().orc_catalan_low64(n))


def limbs_to_int(limbs) -> int:
    """Python integer from LE uint32 limbs (test helper)."""
    a = np.ascontiguousarray(limbs, dtype="<u4")
    return int.from_bytes(a.tobytes(), "little")


def int_to_limbs(x: int, length: int | None = None) -> np.ndarray:
    """LE uint32 limbs of a non-negative Python integer (test helper)."""
    nb = max(1, (x.bit_length() + 31) // 32)
    if length is not None:
        nb = max(nb, length)
    return np.frombuffer(x.to_bytes(4 * nb, "little"), dtype="<u4").astype(np.uint32)


class OracleError(RuntimeError):
    pass


def _args(xs):
    return np.ascontiguousarray(np.asarray([int(x) for x in xs], dtype=np.uint64).reshape(-1))


def ratio_factor(num, den=()):
    """(primes uint32[], exponents uint64[]) of prod(num!) / prod(den!), p ascending,
    exponent > 0 (Sec. 6.3, extended Legendre formula)."""
    lib = _load()
    a, b = _args(num), _args(den)
    cnt = ctypes.c_size_t()
    st = lib.orc_ratio_factor(_p(a, ctypes.c_uint64), len(a), _p(b, ctypes.c_uint64), len(b), None, None, 0,
                              ctypes.byref(cnt))
    if st:
        raise OracleError("orc_ratio_factor: %d" % st)
    pr = np.zeros(max(cnt.value, 1), dtype=np.uint32)
    ex = np.zeros(max(cnt.value, 1), dtype=np.uint64)
    st = lib.orc_ratio_factor(_p(a, ctypes.c_uint64), len(a), _p(b, ctypes.c_uint64), len(b),
                              _p(pr, ctypes.c_uint32), _p(ex, ctypes.c_uint64), len(pr), ctypes.byref(cnt))
    if st:
        raise OracleError("orc_ratio_factor: %d" % st)
    return pr[: cnt.value], ex[: cnt.value]


def ratio(num, den=()) -> np.ndarray:
    """prod(num!) / prod(den!) as normalised uint32 limbs; raises OracleError when
    the ratio is not an integer."""
    lib = _load()
    a, b = _args(num), _args(den)
    n = ctypes.c_size_t()
    st = lib.orc_ratio(_p(a, ctypes.c_uint64), len(a), _p(b, ctypes.c_uint64), len(b), None, 0, ctypes.byref(n))
    if st:
        raise OracleError("orc_ratio: %d" % st)
    out = np.zeros(max(n.value, 1), dtype=np.uint32)
    st = lib.orc_ratio(_p(a, ctypes.c_uint64), len(a), _p(b, ctypes.c_uint64), len(b), _p(out, ctypes.c_uint32),
                       len(out), ctypes.byref(n))
    if st:
        raise OracleError("orc_ratio: %d" % st)
    return out[: n.value]


def to_decimal(limbs) -> str:
    """Decimal text of LE uint32 limbs by repeated schoolbook division by 10^9
    (Sec. 3.2, optional decimal output), O(L^2)."""
    lib = _load()
    x = np.ascontiguousarray(np.asarray(limbs, dtype=np.uint32).reshape(-1))
    if x.size == 0:
        x = np.zeros(1, dtype=np.uint32)
    n = lib.orc_to_decimal(_p(x, ctypes.c_uint32), x.size, None, 0)
    if n == 0:
        raise OracleError("orc_to_decimal: out of memory")
    buf = ctypes.create_string_buffer(n)
    m = lib.orc_to_decimal(_p(x, ctypes.c_uint32), x.size, buf, n)
    if m != n:
        raise OracleError("orc_to_decimal: %d != %d" % (m, n))
    return buf.raw[:n].decode("ascii")
