"""Pins for the CPU oracle: every check here comes from something other than
the oracle itself (brute force, textbook values, a library routine, Kummer's
and Lucas' theorems, closed forms, the log-gamma function, or the paper's own
Table 1)."""
import json
import math
import os
import random

import numpy as np
import pytest

import oracle
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ primes
def test_prime_list_matches_library_sieve():
    from sympy import primerange

    for lim in [0, 1, 2, 3, 4, 10, 97, 100, 1000, 200000]:
        got = oracle.primes(lim)
        exp = np.array(list(primerange(0, lim + 1)), dtype=np.uint32)
        assert np.array_equal(got, exp), lim


@pytest.mark.parametrize("x,pi", [(10, 4), (100, 25), (1000, 168), (10**4, 1229),
                                  (10**5, 9592), (10**6, 78498), (2 * 10**5, 17984)])
def test_prime_counts_textbook(x, pi):
    assert len(oracle.primes(x)) == pi


@pytest.mark.slow
def test_prime_count_2e7_textbook():
    # pi(2*10^7) = 1,270,607 (tabulated value of the prime-counting function)
    assert len(oracle.primes(2 * 10**7)) == 1270607


# ------------------------------------------------------------------ exponents
def test_legendre_small_factorials():
    for m in range(0, 60):
        f = math.factorial(m)
        for p in [2, 3, 5, 7, 11, 13]:
            assert oracle.legendre(m, p) == pins.vp_int(f, p) if f > 0 else True


def test_exponents_match_kummer_all_small_n():
    for n in range(0, 700):
        pr = oracle.primes(2 * n)
        if len(pr) == 0:
            continue
        e = oracle.exponents(n, pr)
        for p, ep in zip(pr.tolist(), e.tolist()):
            assert ep == pins.kummer_exponent(n, p), (n, p)


@pytest.mark.parametrize("n", [12, 13, 100000, 2 * 50021 - 1, 999999])
def test_exponents_match_kummer_selected_n(n):
    # 13: n+1 = 14 = 2*7, the cofactor case; 2q-1 with q prime: n+1 = 2q
    pr = oracle.primes(2 * n)
    e = oracle.exponents(n, pr)
    for p, ep in zip(pr.tolist(), e.tolist()):
        assert ep == pins.kummer_exponent(n, p), (n, p)


def test_factor_groups_reproduce_catalan_exactly():
    for n in list(range(0, 300)) + [1000, 4097]:
        exps, off, pr = oracle.factor(n)
        x = 1
        for g, e in enumerate(exps.tolist()):
            for p in pr[int(off[g]):int(off[g + 1])].tolist():
                x *= p ** e
        assert x == pins.catalan_comb(n), n
        # exponent ascending, primes ascending inside a group, no e = 0 group
        assert list(exps) == sorted(set(exps.tolist())) and (len(exps) == 0 or exps[0] >= 1)
        for g in range(len(exps)):
            seg = pr[int(off[g]):int(off[g + 1])]
            assert np.all(np.diff(seg.astype(np.int64)) > 0)


def test_v2_is_popcount_rule():
    for n in [5, 100, 12345, 10**5]:
        exps, off, pr = oracle.factor(n)
        v2 = 0
        for g, e in enumerate(exps.tolist()):
            if 2 in pr[int(off[g]):int(off[g + 1])].tolist():
                v2 = e
        assert v2 == bin(n + 1).count("1") - 1


# ------------------------------------------------------------------ multiply
def _rand_limbs(rng, n, kind="rand"):
    if kind == "ones":
        return np.full(n, 0xFFFFFFFF, dtype=np.uint32)
    if kind == "zero":
        return np.zeros(n, dtype=np.uint32)
    return rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)


def test_mul_matches_python_integers():
    rng = np.random.default_rng(1)
    sizes = [1, 2, 3, 31, 32, 33, 63, 64, 65, 100, 257, 1000, 2049]
    for la in sizes:
        for lb in [1, 7, 32, 33, 64, 500, la]:
            for kind in ["rand", "ones"]:
                a = _rand_limbs(rng, la, kind)
                b = _rand_limbs(rng, lb, kind)
                c = oracle.mul(a, b)
                assert len(c) == la + lb
                assert pins.limbs_int(c) == pins.limbs_int(a) * pins.limbs_int(b), (la, lb, kind)


def test_mul_closed_form_all_ones():
    # (2^{32k} - 1)^2 = 2^{64k} - 2^{32k+1} + 1, the longest carry chains
    for k in [1, 5, 32, 33, 100, 1024]:
        a = np.full(k, 0xFFFFFFFF, dtype=np.uint32)
        c = oracle.mul(a, a)
        exp = np.zeros(2 * k, dtype=np.uint32)
        exp[0] = 1
        exp[k] = 0xFFFFFFFE
        exp[k + 1:] = 0xFFFFFFFF
        assert np.array_equal(c, exp), k


def test_mul_batched_matches_single():
    rng = np.random.default_rng(2)
    la = [1, 40, 300, 5]
    lb = [3, 40, 7, 600]
    a = [_rand_limbs(rng, x) for x in la]
    b = [_rand_limbs(rng, x) for x in lb]
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    c, c_off = oracle.mul_batched(np.concatenate(a), a_off, np.concatenate(b), b_off)
    for i in range(4):
        got = pins.limbs_int(c[int(c_off[i]):int(c_off[i + 1])])
        assert got == pins.limbs_int(a[i]) * pins.limbs_int(b[i])


def test_product_tree_matches_python():
    rng = random.Random(3)
    items = [rng.getrandbits(rng.randint(1, 3000)) | 1 for _ in range(37)]
    got = pins.limbs_int(oracle.product([oracle.int_to_limbs(x) for x in items]))
    assert got == math.prod(items)
    assert pins.limbs_int(oracle.product([])) == 1


# ------------------------------------------------------------------ C(n)
@pytest.mark.parametrize("n", range(0, 12))
def test_catalan_dyck_bruteforce(n):
    assert pins.limbs_int(oracle.catalan(n)) == pins.dyck_bruteforce(n)


@pytest.mark.parametrize("n", range(0, 16))
def test_catalan_dyck_dp(n):
    assert pins.limbs_int(oracle.catalan(n)) == pins.dyck_dp(n)


def test_catalan_zero_one_single_limb():
    assert list(oracle.catalan(0)) == [1]
    assert list(oracle.catalan(1)) == [1]


def test_catalan_matches_math_comb_and_recurrence():
    prev = None
    for n in range(0, 1201):
        c = pins.limbs_int(oracle.catalan(n))
        assert c == pins.catalan_comb(n), n
        if prev is not None:
            # C(n)(n+1) = 2(2n-1) C(n-1)
            assert c * (n + 1) == 2 * (2 * n - 1) * prev, n
        prev = c


def test_catalan_normalised():
    for n in [2, 17, 100, 1000, 4096]:
        c = oracle.catalan(n)
        assert c[-1] != 0


def test_catalan_1e5_vs_math_comb():
    n = 10**5
    assert pins.limbs_int(oracle.catalan(n)) == pins.catalan_comb(n)


@pytest.mark.parametrize("n", [10**5, 10**6])
def test_catalan_residue_and_size_pins(n):
    c = oracle.catalan(n)
    # 2-adic low 64 bits
    low = int(c[0]) | (int(c[1]) << 32)
    assert low == pins.catalan_low64(n)
    # modulo the prime 2^32 - 5 > 2n, by the product formula
    q = 2**32 - 5
    assert pins.limbs_mod(c, q) == pins.catalan_mod_prime_product(n, q)
    # Lucas residues modulo small primes and modulo 2^32 +- 1 via their factors
    for q in [3, 5, 7, 11, 13, 17, 41, 109, 127, 65537]:
        assert pins.limbs_mod(c, q) == pins.catalan_mod_prime_lucas(n, q), q
    assert pins.limbs_mod(c, 2**32 + 1) == pins.catalan_mod_composite(n, [641, 6700417])
    # bit length, digits, top two limbs from log-gamma
    bits, digits, top, margin = pins.log_pins(n)
    L = len(c)
    assert 32 * (L - 1) + int(c[-1]).bit_length() == bits
    assert L == (bits + 31) // 32
    assert margin > 1e-9
    assert (int(c[-1]) << 32 | int(c[-2])) == top
    if n <= 10**5:
        x = pins.limbs_int(c)
        assert 10 ** (digits - 1) <= x < 10 ** digits


def test_table1_size_pins_from_log_gamma():
    """The paper's Table 1 (n = 2,050,572,903): the log-gamma route used to pin
    the device result reproduces the printed bit length, digit count and file
    size."""
    with open(os.path.join(GOLDEN, "table1_n2050572903.json")) as f:
        t1 = json.load(f)
    bits, digits, top, margin = pins.log_pins(t1["n"], dps=80)
    assert bits == t1["bit_length"]
    assert digits == t1["decimal_digits"]
    assert (bits + 7) // 8 == t1["result_file_bytes"]
    assert margin > 1e-6


# ------------------------------------------------------------------ planted mistakes
@pytest.mark.parametrize("fault", [1, 2, 3])
def test_pins_reject_planted_mistakes(fault):
    """A plausible mistake planted in the oracle (dropping v_p(n+1), dropping a
    schoolbook carry, halving the v_p(n!) term) must fail the pins."""
    try:
        oracle.set_fault(fault)
        bad = False
        for n in [13, 40, 300]:
            try:
                c = pins.limbs_int(oracle.catalan(n))
            except RuntimeError:
                bad = True  # negative exponent detected
                break
            if c != pins.catalan_comb(n):
                bad = True
                break
        assert bad
    finally:
        oracle.set_fault(0)


# ------------------------------------------------------------------ large-n residue routines
def test_residue_routines_match_python_definitions():
    """The O(n) C routines used to check the largest n agree with the Python
    forms and with exact integers."""
    for n in [0, 1, 2, 3, 10, 77, 1000, 12345]:
        c = pins.catalan_comb(n)
        for q in [2**32 - 5, 4294967311, 2**61 - 1]:
            if q > 2 * n:
                assert oracle.catalan_mod_prime(n, q) == c % q
        assert oracle.catalan_low64(n) == c % (1 << 64)
    n = 10**5
    assert oracle.catalan_mod_prime(n, 2**32 - 5) == pins.catalan_mod_prime_product(n, 2**32 - 5)
    assert oracle.catalan_low64(n) == pins.catalan_low64(n)


# ------------------------------------------------------------ factorial ratios (Sec. 6.3)
RATIOS = [
    ([10], [3, 7]), ([100], [37, 63]), ([1000], [1, 999]), ([5000], [1234, 3766]),
    ([30], [10, 10, 10]), ([25], [4, 5, 6, 10]),                  # multinomials
    ([400], []), ([1], []), ([0], []), ([], []),                  # factorials, empty product
    ([1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12], []),                # super-factorial sf(12)
    ([10], [4, 4]), ([2 * 777], [777, 778]),                      # an integral non-binomial; C(777)
    ([3000, 17], [2999, 5, 12]),
]


@pytest.mark.parametrize("num,den", RATIOS)
def test_ratio_exponents_match_digit_sum_formula(num, den):
    """Every exponent of the oracle's ratio factorisation against Legendre's
    digit-sum form; primes absent from the list have exponent 0."""
    import sympy

    A = max(list(num) + list(den) + [1])
    plist = list(sympy.primerange(2, A + 1))
    want = pins.ratio_exponents(num, den, plist)
    pr, ex = oracle.ratio_factor(num, den)
    got = dict(zip(pr.tolist(), ex.tolist()))
    for p, e in zip(plist, want):
        assert got.get(p, 0) == e, (p, e)
    assert all(e > 0 for e in ex.tolist())


@pytest.mark.parametrize("num,den", RATIOS)
def test_ratio_values_match_python_integers(num, den):
    assert oracle.limbs_to_int(oracle.ratio(num, den)) == pins.ratio_value(num, den)


def test_ratio_binomials_all_small():
    import math

    for n in range(0, 90):
        for k in range(0, n + 1):
            assert oracle.limbs_to_int(oracle.ratio([n], [k, n - k])) == math.comb(n, k), (n, k)


def test_ratio_large_binomial_and_factorial():
    import math

    assert oracle.limbs_to_int(oracle.ratio([100000], [31415, 68585])) == math.comb(100000, 31415)
    assert oracle.limbs_to_int(oracle.ratio([20000])) == math.factorial(20000)


@pytest.mark.parametrize("n", [0, 1, 2, 13, 1000, 100000])
def test_ratio_reproduces_catalan(n):
    """C(n) = (2n)! / (n! (n+1)!) through the ratio route equals the Catalan oracle."""
    assert np.array_equal(oracle.ratio([2 * n], [n, n + 1]), oracle.catalan(n))


@pytest.mark.parametrize("num,den", [([3], [4]), ([4], [3, 3]), ([6], [4, 4])])
def test_ratio_not_integral_rejected(num, den):
    with pytest.raises(oracle.OracleError):
        oracle.ratio(num, den)
    with pytest.raises(ValueError):
        pins.ratio_value(num, den)


# ------------------------------------------------------------------ decimal text (Sec. 3.2, optional output)
def _dec_cases():
    import random

    rng = random.Random(11621)
    xs = [0, 1, 9, 10, 99, 100, 2**32 - 1, 2**32, 10**9 - 1, 10**9, 10**9 + 1, 10**18, 2**64 - 1, 2**64]
    xs += [10**k for k in (17, 18, 19, 26, 27, 28, 100, 333)] + [10**k - 1 for k in (9, 18, 27, 100, 333)]
    xs += [rng.getrandbits(rng.randint(1, 4000)) for _ in range(120)]
    return xs


def test_decimal_oracle_closed_forms():
    """10^k is a one and k zeros, 10^k - 1 is k nines, zero is "0", and leading
    zero limbs change nothing."""
    for k in [0, 1, 8, 9, 10, 17, 18, 19, 45, 200, 1001]:
        assert oracle.to_decimal(oracle.int_to_limbs(10**k)) == "1" + "0" * k
        if k:
            assert oracle.to_decimal(oracle.int_to_limbs(10**k - 1)) == "9" * k
    assert oracle.to_decimal(np.zeros(0, dtype=np.uint32)) == "0"
    assert oracle.to_decimal(np.zeros(7, dtype=np.uint32)) == "0"
    assert oracle.to_decimal(oracle.int_to_limbs(12345, length=9)) == "12345"


def test_decimal_oracle_against_python_conversion():
    """Against CPython's own integer-to-text conversion and parsed back by int()."""
    import sys

    if hasattr(sys, "set_int_max_str_digits"):
        sys.set_int_max_str_digits(0)
    for x in _dec_cases():
        s = oracle.to_decimal(oracle.int_to_limbs(x))
        assert s == str(x)
        assert int(s) == x and (s == "0" or s[0] != "0")


def test_decimal_pins_reject_planted_mistake():
    """Dropping the zero padding of inner nine-digit groups fails the parse-back."""
    try:
        oracle.set_fault(4)
        bad = any(int(oracle.to_decimal(oracle.int_to_limbs(x))) != x for x in [10**9, 10**20 + 7, 2**200])
        assert bad
    finally:
        oracle.set_fault(0)


def test_leading_digits_and_trailing_zeros_pins():
    """The log-gamma leading digits and the Legendre count of trailing zeros
    (min(v_2, v_5)) agree with the exact decimal text for moderate n."""
    import sys

    if hasattr(sys, "set_int_max_str_digits"):
        sys.set_int_max_str_digits(0)
    for n in [50, 777, 5000, 30011]:
        s = str(pins.catalan_comb(n))
        lead, margin = pins.leading_decimal(n, 25)
        assert margin > 1e-30 and s[:25] == lead
        z = min(pins.catalan_valuation(n, 2), pins.catalan_valuation(n, 5))
        assert len(s) - len(s.rstrip("0")) == z
