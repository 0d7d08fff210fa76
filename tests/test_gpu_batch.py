"""The synthetic level-batch of 4,096 uneven products (lengths log-uniform in
[64, 65536] limbs): every product checked by the fingerprint identity
a*b = c modulo three moduli (computed independently on the host), a sample
checked bit-exact against the CPU oracle, in the batched, graph and plain
forms, which must also agree with each other bit for bit."""
import numpy as np
import pytest

import oracle
from tests import batch_inputs, pins

pytestmark = pytest.mark.gpu
MODS = (2**32 - 5, 2**32 - 1, 2**31 - 1)   # host fingerprints need q < 2^32


@pytest.fixture(scope="module")
def cat():
    import torch

    import paper_2601_11621_amd as c

    torch.cuda.set_device(0)
    c.init(0)
    return c


_PW = {}


def _host_mod(x: np.ndarray, q: int) -> int:
    """sum_i x_i (2^32)^i mod q for q < 2^32 (vectorised; x up to 2^17 limbs)."""
    pw = _PW.get(q)
    if pw is None:
        pw = np.empty(1 << 17, dtype=np.uint64)
        v, base = 1, (1 << 32) % q
        for i in range(len(pw)):
            pw[i] = v
            v = v * base % q
        _PW[q] = pw
    xs = x.astype(np.uint64) % np.uint64(q)
    return int(np.sum((xs * pw[: len(x)]) % np.uint64(q)) % q)


def test_level_batch_4096(cat):
    import torch

    a, a_off, b, b_off = batch_inputs.level_batch(seed=0)
    la = (a_off[1:] - a_off[:-1]).astype(np.int64)
    lb = (b_off[1:] - b_off[:-1]).astype(np.int64)
    da, db = cat.from_numpy(a), cat.from_numpy(b)
    plan = cat.MulPlan(a_off, b_off, mode="graph")
    c = torch.empty(int((la + lb).sum()), dtype=torch.int32, device="cuda")
    plan(da, db, c)
    plan.check()
    got = cat.to_numpy(c)
    c_off = plan.c_off
    # fingerprints of every product, computed on the host from the inputs
    rng = np.random.default_rng(123)
    sample = set(rng.choice(4096, 48, replace=False).tolist())
    for i in range(4096):
        ai = a[int(a_off[i]):int(a_off[i + 1])]
        bi = b[int(b_off[i]):int(b_off[i + 1])]
        ci = got[int(c_off[i]):int(c_off[i + 1])]
        if i in sample:
            assert np.array_equal(ci, oracle.mul(ai, bi)), i
        for q in MODS:
            assert _host_mod(ci, q) == _host_mod(ai, q) * _host_mod(bi, q) % q, (i, q)
    # the plain form (one product per launch) and a second graph replay agree bit for bit
    plain = cat.MulPlan(a_off, b_off, mode="plain")
    c2 = torch.zeros_like(c)
    plain(da, db, c2)
    plain.check()
    assert torch.equal(c, c2)
    c.zero_()
    plan(da, db, c)
    assert torch.equal(c, c2)
    plan.close()
    plain.close()
