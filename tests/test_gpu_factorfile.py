"""Phase 2 as a reusable engine on the GPU: rebuilding from a factorisation
file (the paper's text format) equals catalan_exact, and products of powers
of arbitrary 32-bit entries equal Python integers."""
import numpy as np
import pytest

import oracle
from paper_2601_11621_amd import factorfile

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cat():
    import torch

    import paper_2601_11621_amd as c

    torch.cuda.set_device(0)
    c.init(0)
    return c


@pytest.mark.parametrize("n", [2, 1000, 100000, 10**6, 10**7])
def test_file_round_trip_equals_catalan_exact(cat, tmp_path, n):
    print("factorisation file", n, flush=True)
    path = str(tmp_path / ("catalan_%d_factorization.txt" % n))
    factorfile.factorize_to_file(cat, n, path)
    for mode in (["batched", "plain"] if n <= 1000 else ["batched"]):
        got = cat.to_numpy(factorfile.reconstruct_from_file(cat, path, mode=mode))
        assert np.array_equal(got, cat.to_numpy(cat.exact(n, mode="batched"))), mode
    if n <= 10**6:
        assert np.array_equal(got, oracle.catalan(n))


def test_oracle_factorisation_file(cat, tmp_path):
    n = 13337
    exps, off, primes = oracle.factor(n)
    path = str(tmp_path / "o.txt")
    factorfile.write_factorization(path, exps, off, primes, "Catalan(%d)" % n)
    assert np.array_equal(cat.to_numpy(factorfile.reconstruct_from_file(cat, path)), oracle.catalan(n))


def test_product_of_powers_of_arbitrary_entries(cat):
    rng = np.random.default_rng(31)
    sizes = [5000, 300, 17, 1]
    exps = [1, 3, 7, 40]
    ent = rng.integers(1, 2**32, size=sum(sizes), dtype=np.uint64).astype(np.uint32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    want = 1
    for g, e in enumerate(exps):
        q = 1
        for v in ent[int(off[g]):int(off[g + 1])].tolist():
            q *= v
        want *= q ** e
    got = cat.product(exps, off, ent)
    assert oracle.limbs_to_int(cat.to_numpy(got)) == want


def test_product_argument_checks(cat):
    ent = np.array([3, 5, 7], dtype=np.uint32)
    with pytest.raises(cat.CatalanError) as e:
        cat.product([2, 1], [0, 1, 3], ent)                 # exponents must ascend
    assert e.value.status == cat.CAT_EINVAL
    with pytest.raises(cat.CatalanError) as e:
        cat.product([1], [0, 3], ent, max_entry_bits=2)     # 5 and 7 need 3 bits
    assert e.value.status == cat.CAT_EINVAL
    assert oracle.limbs_to_int(cat.to_numpy(cat.product([], [0], np.zeros(0, np.uint32)))) == 1


def test_compare_with_shift_against_python(cat):
    rng = np.random.default_rng(5)
    for trial in range(30):
        lx, ly = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        x = rng.integers(0, 2**32, size=lx, dtype=np.uint64).astype(np.uint32)
        y = rng.integers(0, 2**32, size=ly, dtype=np.uint64).astype(np.uint32)
        s = int(rng.integers(0, 40 * 32))
        if trial % 3 == 0:                     # equal values: y = x >> s
            xi = oracle.limbs_to_int(x) >> s
            y = oracle.int_to_limbs(xi, max(1, (xi.bit_length() + 31) // 32))
        X, Y = oracle.limbs_to_int(x) >> s, oracle.limbs_to_int(y)
        want = (X > Y) - (X < Y)
        assert cat.compare(cat.from_numpy(x), cat.from_numpy(y), s) == want, trial


@pytest.mark.parametrize("n", [1, 2, 13, 1000, 100000, 10**7])
def test_decimal_digits_of_catalan(cat, n):
    from tests import pins

    t = cat.exact(n, mode="batched")
    d = cat.decimal_digits(t)
    if n <= 1000:
        assert d == len(str(oracle.limbs_to_int(cat.to_numpy(t))))
    else:
        assert d == pins.log_pins(n)[1]


def test_decimal_text_file(cat, tmp_path):
    """The decimal text file of C(10^5) equals the oracle's text."""
    path = str(tmp_path / "catalan_100000.txt")
    d = factorfile.write_decimal(cat, cat.exact(10**5), path, chunk=4096)
    with open(path, "rb") as f:
        s = f.read().decode("ascii")
    assert d == len(s) == 60199
    assert s == oracle.to_decimal(oracle.catalan(10**5))


def test_command_line_two_phases(cat, tmp_path, capsys):
    """factor -> rebuild through the command line: the binary file, its
    SHA-256 and the decimal text equal the oracle's C(10^5)."""
    import hashlib
    import json

    from paper_2601_11621_amd import cli

    f, b, t = str(tmp_path / "f.txt"), str(tmp_path / "c.bin"), str(tmp_path / "c.txt")
    assert cli.main(["factor", "100000", "--out", f]) == 0
    capsys.readouterr()
    assert cli.main(["rebuild", f, "--bin", b, "--txt", t]) == 0
    info = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    want = oracle.catalan(100000)
    assert np.array_equal(factorfile.read_bin(b), want)
    with open(b, "rb") as fh:
        assert hashlib.sha256(fh.read()).hexdigest() == info["sha256"]
    with open(t) as fh:
        assert fh.read() == oracle.to_decimal(want)
    assert info["digits"] == 60199 and info["bits"] == 199975
