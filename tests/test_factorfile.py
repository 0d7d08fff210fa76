"""The two-phase file interface on the CPU: the factorisation text file round
trip with the paper's layout, and the binary result (ceil(B/8) bytes)."""
import hashlib
import math

import numpy as np

import oracle
from paper_2601_11621_amd import factorfile


def test_factorization_text_round_trip(tmp_path):
    exps, off, primes = oracle.factor(1000)
    path = str(tmp_path / "catalan_1000_factorization.txt")
    factorfile.write_factorization(path, exps, off, primes, "Catalan(1000)")
    text = open(path).read().splitlines()
    assert text[0] == "# Prime factorization of Catalan(1000)"
    assert text[1] == "# exponent=%d count=%d" % (exps[0], off[1] - off[0])
    title, e2, o2, p2 = factorfile.read_factorization(path)
    assert title == "Catalan(1000)"
    assert np.array_equal(e2, exps) and np.array_equal(o2, off) and np.array_equal(p2, primes)


def test_factorization_file_rebuilds_catalan_on_cpu(tmp_path):
    """Alg. 2 on the groups read back (Python integers) gives C(n)."""
    n = 777
    exps, off, primes = oracle.factor(n)
    path = str(tmp_path / "f.txt")
    factorfile.write_factorization(path, exps, off, primes, "Catalan(%d)" % n)
    _, e, o, p = factorfile.read_factorization(path)
    x = 1
    for g in range(len(e)):
        q = 1
        for v in p[int(o[g]):int(o[g + 1])].tolist():
            q *= v
        x *= q ** int(e[g])
    assert x == math.comb(2 * n, n) // (n + 1)


def test_long_groups_wrap_and_counts_are_checked(tmp_path):
    primes = np.arange(3, 3 + 2 * 250_001, 2, dtype=np.uint32)    # entries need not be prime
    path = str(tmp_path / "w.txt")
    factorfile.write_factorization(path, [1], [0, len(primes)], primes, "x")
    assert len(open(path).read().splitlines()) == 2 + 3            # 100,000 per line
    _, e, o, p = factorfile.read_factorization(path)
    assert np.array_equal(p, primes)
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        f.write("# Prime factorization of y\n# exponent=2 count=3\n5 7\n")
    try:
        factorfile.read_factorization(bad)
        raise AssertionError("count mismatch not detected")
    except ValueError:
        pass


def test_binary_result_size_and_hash(tmp_path):
    n = 5000
    limbs = oracle.catalan(n)
    x = oracle.limbs_to_int(limbs)
    nbytes = (x.bit_length() + 7) // 8
    path = str(tmp_path / "c.bin")
    h = factorfile.write_bin(path, limbs)
    data = open(path, "rb").read()
    assert len(data) == nbytes and data == x.to_bytes(nbytes, "little")
    assert h == hashlib.sha256(x.to_bytes(nbytes, "little")).hexdigest()
    hb = factorfile.write_bin(str(tmp_path / "c_be.bin"), limbs, byteorder="big")
    assert hb == hashlib.sha256(x.to_bytes(nbytes, "big")).hexdigest()
    assert np.array_equal(factorfile.read_bin(path), limbs)
    assert np.array_equal(factorfile.read_bin(str(tmp_path / "c_be.bin"), "big"), limbs)
