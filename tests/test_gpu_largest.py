"""GPU checks at sizes the oracle cannot multiply out: products up to the
largest transform length (2^27) by closed forms and by the fingerprint
identity (a*b mod q = (a mod q)(b mod q) mod q), and C(2,050,572,903) — the
paper's result — against Table 1 and residue pins."""
import hashlib
import json
import os

import numpy as np
import pytest

from tests import pins

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MODS = (2**32 - 5, 2**32 + 1, 2**32 - 1)


@pytest.fixture(scope="module")
def cat():
    import torch

    import paper_2601_11621_amd as c

    torch.cuda.set_device(0)
    c.init(0)
    return c


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("la,lb", [(1 << 23, 1 << 23), (1 << 25, (1 << 25) - 7), (1 << 26, (1 << 26) - 1),
                                   ((1 << 26) + 5, 1000)])
def test_huge_product_fingerprints(cat, la, lb):
    import torch

    _say("huge product", la, lb)
    g = torch.Generator(device="cuda")
    g.manual_seed(la ^ lb)
    a = torch.randint(-2**31, 2**31 - 1, (la,), dtype=torch.int32, device="cuda", generator=g)
    b = torch.randint(-2**31, 2**31 - 1, (lb,), dtype=torch.int32, device="cuda", generator=g)
    c, c_off = cat.mul_batched(a, [0, la], b, [0, lb])
    ra, rb, rc = cat.residues(a), cat.residues(b), cat.residues(c)
    for k, q in enumerate(MODS):
        assert rc[k] == ra[k] * rb[k] % q, q
    del a, b, c
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k", [1 << 22, (1 << 25) + 3])
def test_huge_square_all_ones_closed_form(cat, k):
    """(2^{32k} - 1)^2 = 2^{64k} - 2^{32k+1} + 1: the longest carry chains."""
    import torch

    a = torch.full((k,), -1, dtype=torch.int32, device="cuda")
    c, _ = cat.mul_batched(a, [0, k], a.clone(), [0, k])
    exp = torch.full((2 * k,), -1, dtype=torch.int32, device="cuda")
    exp[0] = 1
    exp[1:k] = 0
    exp[k] = -2          # 0xFFFFFFFE
    assert torch.equal(c, exp)
    del a, c, exp
    torch.cuda.empty_cache()


def test_catalan_2050572903_table1(cat):
    """C(2,050,572,903): bit length and file size of Table 1, the 2-adic low
    limbs and the residue modulo 2^32-5 from the oracle's definition-based
    routines, Lucas residues, and the top limbs from log-gamma."""
    import time

    import torch

    n = 2050572903
    with open(os.path.join(GOLDEN, "table1_n2050572903.json")) as f:
        t1 = json.load(f)
    with open(os.path.join(GOLDEN, "pins_n2050572903.json")) as f:
        pz = json.load(f)
    t0 = time.time()
    t = cat.exact(n, mode="graph")
    torch.cuda.synchronize()
    _say("C(%d) on the GPU: %.3f s (first call, includes planning and capture)" % (n, time.time() - t0))
    L = t.numel()
    top = int(t[-1].item()) & 0xFFFFFFFF
    bits = 32 * (L - 1) + top.bit_length()
    assert bits == t1["bit_length"]
    assert (bits + 7) // 8 == t1["result_file_bytes"]
    low = cat.to_numpy(t[:2])
    assert int(low[0]) == pz["limb0"] and int(low[1]) == pz["limb1"]
    r = cat.residues(t)
    assert r[0] == pz["mod_2p32_minus_5"]
    assert r[1] == pins.catalan_mod_composite(n, [641, 6700417])
    assert r[2] == pins.catalan_mod_composite(n, [3, 5, 17, 257, 65537])
    limbs = cat.to_numpy(t)
    # primes q with e_q = 0 (q does not divide C(n)): Lucas residues
    for q in [61, 193, 281, 347, 349, 383]:
        assert pins.limbs_mod_small(limbs, q) == pins.catalan_mod_prime_lucas(n, q), q
    b2, digits, top64, margin = pins.log_pins(n, dps=80)
    assert b2 == bits and digits == t1["decimal_digits"]
    assert margin > 1e-6
    assert (int(limbs[-1]) << 32 | int(limbs[-2])) == top64
    # SHA-256 of the result file in Table 1: the byte order is not stated, so
    # both magnitudes are hashed; a match pins every bit of the result.
    nbytes = t1["result_file_bytes"]
    le = limbs.astype("<u4").tobytes()[:nbytes]
    h_le = hashlib.sha256(le).hexdigest()
    h_be = hashlib.sha256(le[::-1]).hexdigest()
    _say("sha256 LE %s BE %s (paper %s)" % (h_le, h_be, t1["sha256_of_output_file"]))
    # the decimal digit count of Table 1, settled exactly on the GPU:
    # 10^(d-1) <= C(n) < 10^d as floor(C / 2^(d-1)) >= 5^(d-1), floor(C / 2^d) < 5^d
    t0 = time.time()
    assert cat.decimal_digits(t) == t1["decimal_digits"]
    _say("digit count settled in %.3f s" % (time.time() - t0))
    # the decimal text itself (the optional output of Sec. 3.2), converted on
    # the GPU: 1,234,567,890 characters whose nine-digit groups agree with the
    # limbs modulo 10^9 - 1, 10^9 + 1 and 10^9
    t0 = time.time()
    text = cat.to_decimal_device(t)
    torch.cuda.synchronize()
    _say("decimal text in %.3f s" % (time.time() - t0))
    assert text.numel() == t1["decimal_digits"]
    s1, s2, g0 = pins.decimal_group_residues(text)
    assert s1 == pins.limbs_mod_torch(t, 10**9 - 1)
    assert s2 == pins.limbs_mod_torch(t, 10**9 + 1)
    assert g0 == pins.limbs_mod_torch(t, 10**9)
    lead, margin = pins.leading_decimal(n, 30)
    assert margin > 1e-30 and text[:30].cpu().numpy().tobytes().decode() == lead
    z = min(pins.catalan_valuation(n, 2), pins.catalan_valuation(n, 5))
    tail = text[-(z + 1):].cpu().numpy().tobytes().decode()
    assert tail == tail[0] + "0" * z and tail[0] != "0"
    # the SHA-256 of Table 1 does not cover the bare text either (reading in
    # the design notes); printed for the record
    _say("sha256 of the decimal text %s" % hashlib.sha256(text.cpu().numpy().tobytes()).hexdigest())
    del text
    torch.cuda.empty_cache()
