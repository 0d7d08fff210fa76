"""The allocation-free entry point catalan_exact_noalloc, through the C ABI:
its output equals catalan_exact's bit for bit on two calls in a row (the
second with a smaller n, so the static scratch still holds the first call's
contents), sizes beyond its static scratch are refused, and the call leaves
torch's device allocations unchanged."""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cat():
    import torch

    import paper_2601_11621_amd as c

    torch.cuda.set_device(0)
    c.init(0)
    return c


def _noalloc(cat, n, cap, out=None):
    import torch

    lib = cat.load()
    if out is None:
        out = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    nl = ctypes.c_size_t()
    st = lib.catalan_exact_noalloc(n, cat._ptr(out), cap, ctypes.byref(nl),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, nl.value, out


def test_noalloc_equals_catalan_exact_twice(cat):
    import torch

    for n in (10**6, 3 * 10**4):                     # the second call smaller
        print("noalloc C(%d)" % n, flush=True)
        _, max_limbs, _ = cat.sizes(n)
        ref = cat.to_numpy(cat.exact(n, mode="graph"))
        out = torch.full((max_limbs,), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        st, nl, out = _noalloc(cat, n, max_limbs, out)
        torch.cuda.synchronize()
        assert st == cat.CAT_OK
        assert torch.cuda.memory_allocated() == before
        got = cat.to_numpy(out[:nl])
        assert nl == len(ref) and np.array_equal(got, ref), n
        if n <= 10**5:
            assert np.array_equal(got, oracle.catalan(n))


def test_noalloc_limits_and_small_cases(cat):
    lim = cat.noalloc_max_bytes()
    _, _, w7 = cat.sizes(10**7)
    assert w7 <= lim
    _, _, w8 = cat.sizes(10**8)
    assert w8 > lim
    st, _, _ = _noalloc(cat, 10**8, 16)
    assert st == cat.CAT_ENOMEM                     # beyond the static scratch: refused
    for n in (0, 1, 2, 13):
        st, nl, out = _noalloc(cat, n, 4)
        assert st == cat.CAT_OK and np.array_equal(cat.to_numpy(out[:nl]), oracle.catalan(n)), n
    st, nl, _ = _noalloc(cat, 1000, 3)               # capacity too small: the length is reported
    assert st == cat.CAT_ERANGE and nl == len(oracle.catalan(1000))
