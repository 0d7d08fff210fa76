"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and its host-only size queries behave (no GPU work)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "catalan.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_2601_11621_amd as cat

    if not os.path.exists(cat.LIB_PATH):
        from paper_2601_11621_amd import build

        build.build(force=True)
    return cat.load()


def test_header_declares_the_boundary():
    names = _declared()
    for need in ["catalan_factor", "bigint_mul_batched", "catalan_exact", "catalan_sizes", "cat_init",
                 "cat_strerror", "bigint_residues"]:
        assert need in names


def test_library_exports_every_declared_symbol(lib):
    import paper_2601_11621_amd as cat

    for name in _declared():
        assert hasattr(lib, name), name
        assert name in cat.EXPORTS, name


def test_header_compiles_as_c99(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "catalan.h"\nint main(void){ cat_stats s; (void)s; return CAT_OK; }\n')
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                           "-c", str(src), "-o", str(tmp_path / "t.o")])


def test_strerror_and_sizes(lib):
    import paper_2601_11621_amd as cat

    assert lib.cat_strerror(0) == b"ok"
    assert lib.cat_strerror(-2) == b"capacity too small"
    mp, ml, wb = cat.sizes(10**7)
    assert mp >= 1270607 and mp < 1.01 * 1270607       # Dusart's bound is tight here
    assert ml >= 624999
    assert wb > 0
    mp, ml, wb = cat.sizes(2050572903)
    assert mp >= 194532825
    assert ml >= 128160805
    a = ctypes.c_size_t()
    assert lib.catalan_sizes(2**31, ctypes.byref(a), None, None) == cat.CAT_EINVAL


def test_size_query_needs_no_device(lib):
    import paper_2601_11621_amd as cat

    n = ctypes.c_size_t()
    st = lib.catalan_exact(10**6, None, 0, ctypes.byref(n), None, 0, None)
    assert st == cat.CAT_OK and n.value >= 62500
    assert lib.catalan_exact(2**31, None, 0, ctypes.byref(n), None, 0, None) == cat.CAT_EINVAL


def test_binding_refuses_without_gpu():
    import torch

    import paper_2601_11621_amd as cat

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        cat.exact(10)


def test_ratio_sizes_host_only():
    """factorial_ratio_sizes needs no GPU: bounds grow with the arguments; bad
    arguments and results beyond the longest transform are refused."""
    import paper_2601_11621_amd as cat

    p1, l1, w1 = cat.ratio_sizes([1000], [400, 600])
    p2, l2, w2 = cat.ratio_sizes([10**6], [400000, 600000])
    assert 0 < p1 < p2 and 0 < l1 < l2 and 0 < w1 < w2
    # C(1000, 400) has 992 bits: 31 limbs, the bound is a little above
    assert 31 <= l1 <= 40
    with pytest.raises(cat.CatalanError) as e:
        cat.ratio_sizes([2**28])             # 2^28! needs more than 2^27 limbs
    assert e.value.status == cat.CAT_ERANGE
    with pytest.raises(cat.CatalanError) as e:
        cat.ratio_sizes([2**32])
    assert e.value.status == cat.CAT_EINVAL
    with pytest.raises(cat.CatalanError) as e:
        cat.ratio_sizes(list(range(33)))
    assert e.value.status == cat.CAT_EINVAL


def test_decimal_sizes_host_only():
    """decimal_sizes needs no GPU: the digit bound covers 2^(32 L) - 1, the
    workspace grows with L, and inputs beyond the longest transform are refused."""
    import math

    import paper_2601_11621_amd as cat

    prev = 0
    for L in [0, 1, 4, 5, 1000, 624999, 6249999]:
        mc, wb = cat.decimal_sizes(L)
        assert mc >= math.floor(32 * L * math.log10(2)) + 1
        assert wb >= prev
        prev = wb
    mc, wb = cat.decimal_sizes(128160805)         # C(2,050,572,903): 1,234,567,890 digits
    assert mc >= 1234567890 and wb < 64 * 2**30
    with pytest.raises(cat.CatalanError) as e:
        cat.decimal_sizes(2**27 + 1)
    assert e.value.status == cat.CAT_ERANGE
