"""Python binding of the gfx950 Catalan library (``libcatalan.so``).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/catalan.h``.  PyTorch provides
device memory (limb buffers and workspace) and the current stream.  Limbs are
little-endian uint32 values held in int32 tensors (same bits).

There is no CPU fallback: importing works without a GPU, but every call that
computes raises if the library is not built or no GPU is visible.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcatalan.so")

CAT_OK, CAT_EINVAL, CAT_ERANGE, CAT_ENOMEM, CAT_EDEVICE, CAT_EINTERNAL, CAT_EAGAIN = 0, -1, -2, -3, -4, -5, -6
MODE_BATCHED, MODE_PLAIN, MODE_GRAPH = 0, 1, 2
_MODES = {"batched": MODE_BATCHED, "plain": MODE_PLAIN, "graph": MODE_BATCHED | MODE_GRAPH}
MAX_GROUPS = 32

EXPORTS = [
    "cat_init", "cat_strerror", "cat_last_device_error", "cat_get_stats", "catalan_sizes",
    "catalan_factor", "bigint_mul_workspace", "bigint_mul_batched", "bigint_mul_batched_ex",
    "catalan_exact", "catalan_exact_ex", "cat_mul_plan_create", "cat_mul_plan_exec",
    "cat_mul_plan_check", "cat_mul_plan_destroy", "bigint_residues", "cat_timer_set", "cat_timer_get",
    "catalan_begin", "cat_ticket_query", "catalan_continue", "catalan_end", "cat_ticket_release",
    "cat_tune_set", "cat_tune_get", "cat_lookback_polls_set",
    "factorial_ratio_sizes", "factorial_ratio_factor", "factorial_ratio_exact",
    "prime_power_product_sizes", "prime_power_product", "bigint_compare",
    "decimal_sizes", "bigint_to_decimal", "catalan_exact_noalloc", "catalan_noalloc_max_bytes",
    "cat_fused_levels_set", "cat_lazy_primes_set", "cat_outer_node_set", "bigint_decimal_digits_workspace", "bigint_decimal_digits", "bigint_mul_check",
    "catalan_batch_sizes", "catalan_batch_begin", "catalan_batch_continue", "catalan_batch_end",
    "cat_valu_rate",
]


class CatalanError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = "%s failed: %s (%d)" % (what, _strerror(status), status)
        if status == CAT_EDEVICE and _lib is not None:
            msg += " [hip error %d]" % _lib.cat_last_device_error()
        super().__init__(msg)


class cat_tuning(ctypes.Structure):
    _fields_ = [("school_max", ctypes.c_uint32), ("cls", ctypes.c_uint8 * 28),
                ("log_row", ctypes.c_uint8 * 28), ("log_pass", ctypes.c_uint8 * 28)]


class cat_stats(ctypes.Structure):
    _fields_ = [("products", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("product_limbs", ctypes.c_uint64), ("n_primes", ctypes.c_uint64),
                ("levels", ctypes.c_uint32), ("graph_replayed", ctypes.c_uint32),
                ("outer_level", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


_lib = None


def _strerror(s: int) -> str:
    if _lib is None:
        return "status %d" % s
    return _lib.cat_strerror(s).decode()


def load(path: str = LIB_PATH):
    """Load libcatalan.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libcatalan.so is not built (run __graft_entry__.build()); "
                           "there is no fallback path")
    lib = ctypes.CDLL(path)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    szp = ctypes.POINTER(ctypes.c_size_t)
    vp = ctypes.c_void_p
    st = ctypes.c_int32
    sig = {
        "cat_init": ([ctypes.c_int], st),
        "cat_strerror": ([st], ctypes.c_char_p),
        "cat_last_device_error": ([], ctypes.c_int),
        "cat_get_stats": ([ctypes.POINTER(cat_stats)], st),
        "catalan_sizes": ([ctypes.c_uint64, szp, szp, szp], st),
        "catalan_factor": ([ctypes.c_uint64, vp, ctypes.c_size_t, u32p, u64p, u32p, szp, vp,
                            ctypes.c_size_t, vp], st),
        "bigint_mul_workspace": ([ctypes.c_uint32, u64p, u64p, szp], st),
        "bigint_mul_batched": ([ctypes.c_uint32, vp, u64p, vp, u64p, vp, u64p, vp, ctypes.c_size_t, vp], st),
        "bigint_mul_batched_ex": ([ctypes.c_uint32, vp, u64p, vp, u64p, vp, u64p, vp, ctypes.c_size_t, vp,
                                   ctypes.c_uint32], st),
        "catalan_exact": ([ctypes.c_uint64, vp, ctypes.c_size_t, szp, vp, ctypes.c_size_t, vp], st),
        "catalan_exact_ex": ([ctypes.c_uint64, vp, ctypes.c_size_t, szp, vp, ctypes.c_size_t, vp,
                              ctypes.c_uint32], st),
        "cat_mul_plan_create": ([ctypes.c_uint32, u64p, u64p, u64p, ctypes.c_uint32,
                                 ctypes.POINTER(vp), szp], st),
        "cat_mul_plan_exec": ([vp, vp, vp, vp, vp, ctypes.c_size_t, vp], st),
        "cat_mul_plan_check": ([vp, vp, vp], st),
        "cat_mul_plan_destroy": ([vp], st),
        "bigint_residues": ([vp, ctypes.c_size_t, u64p, vp, ctypes.c_size_t, vp], st),
        "cat_timer_set": ([ctypes.c_char_p], st),
        "cat_timer_get": ([ctypes.POINTER(ctypes.c_double), u64p, ctypes.POINTER(ctypes.c_double)], st),
        "cat_valu_rate": ([ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double)], st),
        "catalan_begin": ([ctypes.c_uint64, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], st),
        "cat_ticket_query": ([vp], st),
        "catalan_continue": ([vp, vp, ctypes.c_size_t], st),
        "catalan_end": ([vp, szp], st),
        "cat_ticket_release": ([vp], st),
        "cat_tune_set": ([ctypes.POINTER(cat_tuning)], st),
        "cat_lookback_polls_set": ([ctypes.c_uint32], st),
        "factorial_ratio_sizes": ([u64p, ctypes.c_uint32, u64p, ctypes.c_uint32, szp, szp, szp], st),
        "prime_power_product_sizes": ([u32p, u64p, ctypes.c_uint32, ctypes.c_uint32, szp, szp], st),
        "bigint_compare": ([vp, ctypes.c_size_t, ctypes.c_uint64, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32),
                            vp, ctypes.c_size_t, vp], st),
        "prime_power_product": ([vp, u32p, u64p, ctypes.c_uint32, ctypes.c_uint32, vp, ctypes.c_size_t, szp, vp,
                                 ctypes.c_size_t, vp, ctypes.c_uint32], st),
        "factorial_ratio_factor": ([u64p, ctypes.c_uint32, u64p, ctypes.c_uint32, vp, ctypes.c_size_t, u32p, u64p,
                                    u32p, szp, vp, ctypes.c_size_t, vp], st),
        "factorial_ratio_exact": ([u64p, ctypes.c_uint32, u64p, ctypes.c_uint32, vp, ctypes.c_size_t, szp, vp,
                                   ctypes.c_size_t, vp, ctypes.c_uint32], st),
        "cat_tune_get": ([ctypes.POINTER(cat_tuning)], st),
        "decimal_sizes": ([ctypes.c_size_t, szp, szp], st),
        "bigint_to_decimal": ([vp, ctypes.c_size_t, vp, ctypes.c_size_t, szp, vp, ctypes.c_size_t, vp], st),
        "catalan_exact_noalloc": ([ctypes.c_uint64, vp, ctypes.c_size_t, szp, vp], st),
        "catalan_noalloc_max_bytes": ([szp], st),
        "cat_fused_levels_set": ([ctypes.c_uint32], st),
        "cat_lazy_primes_set": ([ctypes.c_uint32], st),
        "cat_outer_node_set": ([ctypes.c_uint32], st),
        "bigint_decimal_digits_workspace": ([ctypes.c_size_t, szp], st),
        "bigint_decimal_digits": ([vp, ctypes.c_size_t, u64p, vp, ctypes.c_size_t, vp], st),
        "bigint_mul_check": ([vp, vp], st),
        "catalan_batch_sizes": ([ctypes.c_uint32, u64p, szp], st),
        "catalan_batch_begin": ([ctypes.c_uint32, u64p, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], st),
        "catalan_batch_continue": ([vp, ctypes.POINTER(vp), szp], st),
        "catalan_batch_end": ([vp, szp, ctypes.POINTER(ctypes.c_int32)], st),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != CAT_OK:
        raise CatalanError(status, what)


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the Catalan library runs only on the GPU")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


_work = {}


def workspace(nbytes: int, key: str = "default"):
    """A reusable device scratch buffer (kept, so graph caches see one address)."""
    torch = _torch()
    buf = _work.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
        _work[key] = buf
    return buf


def release_workspaces() -> None:
    """Drop the cached scratch buffers (the next call allocates afresh)."""
    _work.clear()


TUNING_FILE = os.path.join(_HERE, "tuning", "gfx950.json")


def get_tuning() -> dict:
    t = cat_tuning()
    _check(load().cat_tune_get(ctypes.byref(t)), "cat_tune_get")
    return {"school_max": t.school_max, "cls": list(t.cls), "log_row": list(t.log_row),
            "log_pass": list(t.log_pass)}


POLLS_AUTO = 0xFFFFFFFF


def set_lookback_polls(polls: Optional[int]) -> None:
    """Polls of a predecessor's carry flag before a CRT block recomputes it
    (0: always recompute; None: the library's per-launch choice).  Same
    results either way."""
    _check(load().cat_lookback_polls_set(POLLS_AUTO if polls is None else int(polls)), "cat_lookback_polls_set")


FUSED_DEFAULT = 0xFFFFFFFF


def set_fused_levels(max_logn: Optional[int] = 12) -> None:
    """Fuse the tree levels, and the buckets of a generic batch, with
    transforms of up to 2^max_logn coefficients into one launch (0: every
    level or bucket is a transform and a carry launch; None: the library's
    defaults, generic batches fused up to 2^12 and tree levels not fused).
    Same results either way."""
    v = FUSED_DEFAULT if max_logn is None else int(max_logn)
    _check(load().cat_fused_levels_set(v), "cat_fused_levels_set")


def set_lazy_primes(max_logn: int = 23) -> None:
    """Transforms of up to 2^max_logn points use the three primes below 2^30
    with unreduced butterfly ranges (0: the primes above 2^31 everywhere).
    The results are the same bit for bit either way."""
    _check(load().cat_lazy_primes_set(int(max_logn)), "cat_lazy_primes_set")


def set_outer_node(on: bool = True) -> None:
    """R, the product of the powers P_e with e >= 2, as a node of Q_1's
    product tree (True) or multiplied onto Q_1 after the tree (False).  The
    results are the same bit for bit either way."""
    _check(load().cat_outer_node_set(1 if on else 0), "cat_outer_node_set")


def set_tuning(d: Optional[dict]) -> None:
    """Install a schedule table (None: the library defaults)."""
    if d is None:
        _check(load().cat_tune_set(None), "cat_tune_set")
        return
    t = cat_tuning()
    t.school_max = int(d["school_max"])
    for k in range(28):
        t.cls[k] = int(d["cls"][k])
        t.log_row[k] = int(d["log_row"][k])
        t.log_pass[k] = int(d["log_pass"][k])
    _check(load().cat_tune_set(ctypes.byref(t)), "cat_tune_set")


def load_tuning(path: str = TUNING_FILE) -> bool:
    """Install the autotuner's table for this GPU if one was written."""
    import json

    if not os.path.exists(path):
        return False
    with open(path) as f:
        d = json.load(f)
    set_tuning(d["table"])
    return True


_inited = False


def init(device: int = -1, tuned: bool = True) -> None:
    global _inited
    _torch()
    _check(load().cat_init(device), "cat_init")
    if tuned and not _inited:
        load_tuning()
    _inited = True


def sizes(n: int):
    """(max_primes, max_limbs, workspace_bytes) for n (host-only)."""
    lib = load()
    a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.catalan_sizes(n, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "catalan_sizes")
    return a.value, b.value, c.value


def stats() -> dict:
    s = cat_stats()
    _check(load().cat_get_stats(ctypes.byref(s)), "cat_get_stats")
    return {f: getattr(s, f) for f, _ in cat_stats._fields_}


def factor(n: int, stream=None):
    """Phase 1 on the GPU: (exps uint32[g], off uint64[g+1], primes int32 device tensor)."""
    torch = _torch()
    lib = load()
    max_primes, _, wbytes = sizes(n)
    primes = torch.empty(max(max_primes, 1), dtype=torch.int32, device="cuda")
    w = workspace(wbytes)
    exps = np.zeros(MAX_GROUPS, dtype=np.uint32)
    off = np.zeros(MAX_GROUPS + 1, dtype=np.uint64)
    ng = ctypes.c_uint32()
    npr = ctypes.c_size_t()
    st = lib.catalan_factor(n, _ptr(primes), primes.numel(), exps.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                            _p64(off), ctypes.byref(ng), ctypes.byref(npr), _ptr(w), w.numel(), _stream(stream))
    _check(st, "catalan_factor")
    g = ng.value
    return exps[:g].copy(), off[: g + 1].copy(), primes[: npr.value]


def exact(n: int, mode: str = "graph", stream=None, out=None):
    """C(n) as normalised limbs in an int32 device tensor (uint32 bits)."""
    torch = _torch()
    lib = load()
    _, max_limbs, wbytes = sizes(n)
    w = workspace(wbytes)
    if out is None:
        out = torch.empty(max_limbs, dtype=torch.int32, device="cuda")
    nl = ctypes.c_size_t()
    st = lib.catalan_exact_ex(n, _ptr(out), out.numel(), ctypes.byref(nl), _ptr(w), w.numel(), _stream(stream),
                              _MODES[mode])
    _check(st, "catalan_exact")
    return out[: nl.value]


def exact_noalloc(n: int, out, stream=None):
    """C(n) into the caller's int32 device tensor `out` by the allocation-free
    entry point (the library's static device scratch); returns out[:limbs]."""
    lib = load()
    nl = ctypes.c_size_t()
    _check(lib.catalan_exact_noalloc(n, _ptr(out), out.numel(), ctypes.byref(nl), _stream(stream)),
           "catalan_exact_noalloc")
    return out[: nl.value]


def noalloc_max_bytes() -> int:
    """Size of the static scratch behind exact_noalloc (host only)."""
    b = ctypes.c_size_t()
    _check(load().catalan_noalloc_max_bytes(ctypes.byref(b)), "catalan_noalloc_max_bytes")
    return b.value


BATCH_MAX = 32


def batch_sizes(ns) -> int:
    """Workspace bytes of one batch of C(n) requests (host only)."""
    a = _u64(ns)
    wb = ctypes.c_size_t()
    _check(load().catalan_batch_sizes(len(a), _p64(a), ctypes.byref(wb)), "catalan_batch_sizes")
    return wb.value


def exact_batch(ns, stream=None):
    """C(n) for every n of ns (at most BATCH_MAX) as one batch: Phase 1 per
    request, Phase 2 of all of them planned and launched together.  Returns
    a list of limb tensors (bit-identical to exact(n))."""
    torch = _torch()
    lib = load()
    a = _u64(ns)
    k = len(a)
    w = workspace(batch_sizes(a), key="batch")
    outs = [torch.empty(max(sizes(int(n))[1], 1), dtype=torch.int32, device="cuda") for n in a]
    t = ctypes.c_void_p()
    _check(lib.catalan_batch_begin(k, _p64(a), _ptr(w), w.numel(), _stream(stream), ctypes.byref(t)),
           "catalan_batch_begin")
    ptrs = (ctypes.c_void_p * k)(*[o.data_ptr() for o in outs])
    caps = (ctypes.c_size_t * k)(*[o.numel() for o in outs])
    st = lib.catalan_batch_continue(t, ptrs, caps)
    if st != CAT_OK:
        lib.cat_ticket_release(t)
        _check(st, "catalan_batch_continue")
    nl = (ctypes.c_size_t * k)()
    rs = (ctypes.c_int32 * k)()
    _check(lib.catalan_batch_end(t, nl, rs), "catalan_batch_end")
    return [o[: nl[i]] for i, o in enumerate(outs)]


def _terms(xs):
    arr = np.ascontiguousarray(np.asarray([int(x) for x in xs], dtype=np.uint64))
    return arr, len(arr)


def ratio_sizes(num, den=()):
    """(max_primes, max_limbs, workspace_bytes) for prod(num!) / prod(den!) (host-only)."""
    lib = load()
    a, k = _terms(num)
    b, m = _terms(den)
    x, y, z = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.factorial_ratio_sizes(_p64(a), k, _p64(b), m, ctypes.byref(x), ctypes.byref(y), ctypes.byref(z)),
           "factorial_ratio_sizes")
    return x.value, y.value, z.value


def ratio_factor(num, den=(), stream=None):
    """Phase 1 of prod(num!) / prod(den!) on the GPU: (exps uint32[g] = 2^bit,
    off uint64[g+1], grouped primes int32 device tensor)."""
    torch = _torch()
    lib = load()
    a, k = _terms(num)
    b, m = _terms(den)
    max_primes, _, wbytes = ratio_sizes(num, den)
    primes = torch.empty(max(max_primes, 1), dtype=torch.int32, device="cuda")
    w = workspace(wbytes)
    exps = np.zeros(MAX_GROUPS, dtype=np.uint32)
    off = np.zeros(MAX_GROUPS + 1, dtype=np.uint64)
    ng = ctypes.c_uint32()
    npr = ctypes.c_size_t()
    st = lib.factorial_ratio_factor(_p64(a), k, _p64(b), m, _ptr(primes), primes.numel(),
                                    exps.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _p64(off), ctypes.byref(ng),
                                    ctypes.byref(npr), _ptr(w), w.numel(), _stream(stream))
    _check(st, "factorial_ratio_factor")
    g = ng.value
    return exps[:g].copy(), off[: g + 1].copy(), primes[: npr.value]


def ratio_exact(num, den=(), mode: str = "batched", stream=None, out=None):
    """prod(num!) / prod(den!) as normalised limbs in an int32 device tensor."""
    torch = _torch()
    lib = load()
    a, k = _terms(num)
    b, m = _terms(den)
    _, max_limbs, wbytes = ratio_sizes(num, den)
    w = workspace(wbytes)
    if out is None:
        out = torch.empty(max(max_limbs, 1), dtype=torch.int32, device="cuda")
    nl = ctypes.c_size_t()
    st = lib.factorial_ratio_exact(_p64(a), k, _p64(b), m, _ptr(out), out.numel(), ctypes.byref(nl), _ptr(w),
                                   w.numel(), _stream(stream), _MODES[mode] & ~MODE_GRAPH)
    _check(st, "factorial_ratio_exact")
    return out[: nl.value]


def product_sizes(exps, off, max_entry_bits: int = 32):
    """(max_limbs, workspace_bytes) of prod_g (entries of g)^exps[g] (host-only)."""
    lib = load()
    e = np.ascontiguousarray(np.asarray(exps, dtype=np.uint32))
    o = _u64(off)
    x, y = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.prime_power_product_sizes(e.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _p64(o), len(e),
                                         max_entry_bits, ctypes.byref(x), ctypes.byref(y)), "prime_power_product_sizes")
    return x.value, y.value


def product(exps, off, entries, max_entry_bits: int = 32, mode: str = "batched", stream=None, out=None):
    """Phase 2 alone: prod_g (prod entries[off[g]:off[g+1]])^exps[g] as normalised
    limbs; `entries` is a device tensor (int32 bits) or a host array."""
    torch = _torch()
    lib = load()
    e = np.ascontiguousarray(np.asarray(exps, dtype=np.uint32))
    o = _u64(off)
    if not isinstance(entries, torch.Tensor):
        entries = from_numpy(np.ascontiguousarray(np.asarray(entries, dtype=np.uint32)))
    max_limbs, wbytes = product_sizes(e, o, max_entry_bits)
    w = workspace(wbytes)
    if out is None:
        out = torch.empty(max(max_limbs, 1), dtype=torch.int32, device="cuda")
    nl = ctypes.c_size_t()
    st = lib.prime_power_product(_ptr(entries), e.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _p64(o), len(e),
                                 max_entry_bits, _ptr(out), out.numel(), ctypes.byref(nl), _ptr(w), w.numel(),
                                 _stream(stream), _MODES[mode] & ~MODE_GRAPH)
    _check(st, "prime_power_product")
    return out[: nl.value]


def compare(x, y, shift_bits: int = 0, stream=None) -> int:
    """sign(floor(x / 2^shift_bits) - y) of two limb tensors, on the GPU."""
    lib = load()
    w = workspace(256, key="cmp")
    sgn = ctypes.c_int32()
    _check(lib.bigint_compare(_ptr(x), x.numel(), int(shift_bits), _ptr(y), y.numel(), ctypes.byref(sgn), _ptr(w),
                              w.numel(), _stream(stream)), "bigint_compare")
    return sgn.value


def decimal_digits(x, stream=None) -> int:
    """The exact number of decimal digits of a limb tensor x, settled on the
    GPU by the library (bigint_decimal_digits)."""
    lib = load()
    n = int(x.numel())
    wb = ctypes.c_size_t()
    _check(lib.bigint_decimal_digits_workspace(n, ctypes.byref(wb)), "bigint_decimal_digits_workspace")
    w = workspace(wb.value, key="digits")
    d = ctypes.c_uint64()
    _check(lib.bigint_decimal_digits(_ptr(x) if n else None, n, ctypes.byref(d), _ptr(w), w.numel(),
                                     _stream(stream)), "bigint_decimal_digits")
    return d.value


def decimal_sizes(n_limbs: int):
    """(upper bound on the decimal digits, workspace bytes) for n_limbs limbs; host only."""
    lib = load()
    mc, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.decimal_sizes(int(n_limbs), ctypes.byref(mc), ctypes.byref(wb)), "decimal_sizes")
    return mc.value, wb.value


def to_decimal_device(x, stream=None):
    """Decimal digits of the limb tensor x as a uint8 device tensor of ASCII
    characters, most significant first (the radix conversion runs on the GPU)."""
    torch = _torch()
    lib = load()
    n = int(x.numel())
    mc, wb = decimal_sizes(n)
    w = workspace(wb, key="dec")
    out = torch.empty(max(mc, 1), dtype=torch.uint8, device="cuda")
    nc = ctypes.c_size_t()
    _check(lib.bigint_to_decimal(_ptr(x) if n else None, n, _ptr(out), out.numel(), ctypes.byref(nc), _ptr(w),
                                 w.numel(), _stream(stream)), "bigint_to_decimal")
    return out[: nc.value]


def to_decimal(x, stream=None) -> str:
    """Decimal text of the limb tensor x (converted on the GPU, copied to the host)."""
    return to_decimal_device(x, stream).cpu().numpy().tobytes().decode("ascii")


def mul_batched(a_flat, a_off, b_flat, b_off, mode: str = "batched", stream=None):
    """c_i = a_i * b_i; returns (c_flat int32 device tensor, c_off uint64[batch+1])."""
    torch = _torch()
    lib = load()
    a_off = _u64(a_off)
    b_off = _u64(b_off)
    batch = len(a_off) - 1
    lens = (a_off[1:] - a_off[:-1]) + (b_off[1:] - b_off[:-1])
    c_off = np.zeros(batch + 1, dtype=np.uint64)
    c_off[1:] = np.cumsum(lens)
    c = torch.empty(max(int(c_off[-1]), 1), dtype=torch.int32, device="cuda")
    wb = ctypes.c_size_t()
    _check(lib.bigint_mul_workspace(batch, _p64(a_off), _p64(b_off), ctypes.byref(wb)), "bigint_mul_workspace")
    w = workspace(wb.value, key="mul")
    st = lib.bigint_mul_batched_ex(batch, _ptr(a_flat), _p64(a_off), _ptr(b_flat), _p64(b_off), _ptr(c),
                                   _p64(c_off), _ptr(w), w.numel(), _stream(stream), _MODES[mode] & ~MODE_GRAPH)
    _check(st, "bigint_mul_batched")
    if batch:
        # the call only queued the products; wait for them and read the device check
        _check(lib.bigint_mul_check(_ptr(w), _stream(stream)), "bigint_mul_check")
    return c[: int(c_off[-1])], c_off


class MulPlan:
    """A reusable plan for batches of one shape (see cat_mul_plan_* in catalan.h)."""

    def __init__(self, a_off, b_off, c_off=None, mode: str = "graph"):
        lib = load()
        _torch()
        self.a_off = _u64(a_off)
        self.b_off = _u64(b_off)
        batch = len(self.a_off) - 1
        if c_off is None:
            lens = (self.a_off[1:] - self.a_off[:-1]) + (self.b_off[1:] - self.b_off[:-1])
            c_off = np.zeros(batch + 1, dtype=np.uint64)
            c_off[1:] = np.cumsum(lens)
        self.c_off = _u64(c_off)
        self.batch = batch
        self._h = ctypes.c_void_p()
        wb = ctypes.c_size_t()
        _check(lib.cat_mul_plan_create(batch, _p64(self.a_off), _p64(self.b_off), _p64(self.c_off), _MODES[mode],
                                       ctypes.byref(self._h), ctypes.byref(wb)), "cat_mul_plan_create")
        self.workspace_bytes = wb.value
        self._w = None

    def __call__(self, a_flat, b_flat, c_flat, stream=None):
        torch = _torch()
        if self._w is None:
            self._w = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device="cuda")
        _check(load().cat_mul_plan_exec(self._h, _ptr(a_flat), _ptr(b_flat), _ptr(c_flat), _ptr(self._w),
                                        self._w.numel(), _stream(stream)), "cat_mul_plan_exec")
        return c_flat

    def check(self, stream=None):
        if self._w is not None:
            _check(load().cat_mul_plan_check(self._h, _ptr(self._w), _stream(stream)), "cat_mul_plan_check")

    def close(self):
        if self._h:
            load().cat_mul_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timer_set(kernel: Optional[str]) -> None:
    """Bracket every later launch of `kernel` with HIP events (None stops)."""
    _check(load().cat_timer_set(kernel.encode() if kernel else None), "cat_timer_set")


def timer_get():
    """(summed kernel ms, launches, algorithmic work) since timer_set."""
    ms = ctypes.c_double()
    ln = ctypes.c_uint64()
    wk = ctypes.c_double()
    _check(load().cat_timer_get(ctypes.byref(ms), ctypes.byref(ln), ctypes.byref(wk)), "cat_timer_get")
    return ms.value, ln.value, wk.value


# instruction forms of the issue-rate probe, in the C ABI's order
VALU_OPS = ("v_add_u32", "v_min_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32", "v_fma_f32")


def valu_rate(op: str, iters: int = 4096):
    """(lane operations per second, launch ms) of one VALU instruction form."""
    rate = ctypes.c_double()
    ms = ctypes.c_double()
    _check(load().cat_valu_rate(VALU_OPS.index(op), iters, ctypes.byref(rate), ctypes.byref(ms)), "cat_valu_rate")
    return rate.value, ms.value


def residues(x, stream=None):
    """(x mod 2^32-5, x mod 2^32+1, x mod 2^32-1) of a limb tensor, on the GPU."""
    lib = load()
    n = x.numel()
    w = workspace(24 * ((n + 4095) // 4096) + 256, key="residues")
    out = np.zeros(3, dtype=np.uint64)
    _check(lib.bigint_residues(_ptr(x), n, _p64(out), _ptr(w), w.numel(), _stream(stream)), "bigint_residues")
    return tuple(int(v) for v in out)


def to_numpy(t) -> np.ndarray:
    """Device limb tensor -> numpy uint32 array."""
    return t.detach().cpu().numpy().view(np.uint32)


def to_int(t) -> int:
    """Device limb tensor -> Python integer."""
    return int.from_bytes(to_numpy(t).astype("<u4").tobytes(), "little")


def from_numpy(a: np.ndarray):
    torch = _torch()
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32).copy()).to("cuda")
