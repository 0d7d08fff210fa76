"""Factorial ratios on the GPU (Sec. 6.3): the device factorisation against the
oracle's exponents, and N = prod a_i! / prod b_j! bit for bit against the
oracle, against catalan_exact through (2n)!/(n!(n+1)!), and in both forms."""
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


def _say(*a):
    print(*a, flush=True)


CASES = [
    ([10], [3, 7]), ([100], [37, 63]), ([5000], [1234, 3766]), ([30], [10, 10, 10]),
    ([400], []), ([1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12], []), ([10], [4, 4]), ([3000, 17], [2999, 5, 12]),
    ([2 * 777], [777, 778]), ([123457], [23456, 100001]), ([65536], [32768, 32768]), ([65537], []),
]


@pytest.mark.parametrize("num,den", CASES)
def test_ratio_factor_matches_oracle(cat, num, den):
    """Bit groups: every group ascending, exps[g] = 2^b, and summing
    exps[g] over the groups holding p gives the oracle's exponent of p."""
    _say("ratio_factor", num, den)
    exps, off, pr = cat.ratio_factor(num, den)
    grouped = cat.to_numpy(pr)
    opr, oex = oracle.ratio_factor(num, den)
    want = dict(zip(opr.tolist(), oex.tolist()))
    got = {}
    for g in range(len(exps)):
        e = int(exps[g])
        assert e & (e - 1) == 0 and (g == 0 or e > int(exps[g - 1]))
        part = grouped[int(off[g]):int(off[g + 1])]
        assert np.all(np.diff(part.astype(np.int64)) > 0)
        for p in part.tolist():
            got[p] = got.get(p, 0) + e
    assert got == want


@pytest.mark.parametrize("num,den", CASES + [([0], []), ([1], [1]), ([], [])])
def test_ratio_exact_matches_oracle(cat, num, den):
    _say("ratio_exact", num, den)
    want = oracle.ratio(num, den)
    for mode in ("batched", "plain"):
        got = cat.to_numpy(cat.ratio_exact(num, den, mode=mode))
        assert np.array_equal(got, want), mode


@pytest.mark.parametrize("num,den", [([200000], [70000, 130000]), ([100000], []), ([60000], [20000, 20000, 20000])])
def test_ratio_exact_larger_vs_oracle(cat, num, den):
    _say("ratio_exact", num, den)
    assert np.array_equal(cat.to_numpy(cat.ratio_exact(num, den)), oracle.ratio(num, den))


@pytest.mark.parametrize("n", [0, 1, 13, 4097, 100000, 10**6, 10**7])
def test_ratio_route_equals_catalan_exact(cat, n):
    """Different grouping (exponent bits vs exponent values), same integer."""
    _say("catalan via ratio", n)
    a = cat.to_numpy(cat.ratio_exact([2 * n], [n, n + 1]))
    b = cat.to_numpy(cat.exact(n, mode="batched"))
    assert np.array_equal(a, b)


def test_ratio_not_integral_is_refused(cat):
    for num, den in [([3], [4]), ([4], [3, 3]), ([6], [4, 4])]:
        with pytest.raises(cat.CatalanError) as e:
            cat.ratio_exact(num, den)
        assert e.value.status == cat.CAT_EINVAL
