"""The synthetic level-batch of 4,096 uneven products (lengths log-uniform in
[64, 65536] limbs) and its balanced variant (lb = la): every product checked
bit for bit against the CPU oracle through the digests of its products
(tests/golden/batch4096_digests.json, written by a script that calls only the
oracle), in the graph, batched and plain forms, which must also agree with
each other bit for bit; a sample is compared limb for limb as well."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from tests import batch_inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch4096_digests.json")


@pytest.fixture(scope="module")
def cat():
    import torch

    import paper_2601_11621_amd as c

    torch.cuda.set_device(0)
    c.init(0)
    return c


def _digests(got, c_off):
    return [hashlib.sha256(got[int(c_off[i]):int(c_off[i + 1])].astype("<u4").tobytes()).hexdigest()[:32]
            for i in range(len(c_off) - 1)]


@pytest.mark.parametrize("variant", ["uneven", "balanced"])
def test_level_batch_4096_every_product(cat, variant):
    import torch

    with open(GOLDEN) as f:
        want = json.load(f)[variant]["sha256_128"]
    a, a_off, b, b_off = batch_inputs.level_batch(seed=0, balanced=(variant == "balanced"))
    la = (a_off[1:] - a_off[:-1]).astype(np.int64)
    lb = (b_off[1:] - b_off[:-1]).astype(np.int64)
    da, db = cat.from_numpy(a), cat.from_numpy(b)
    limbs = int((la + lb).sum())
    for mode in ("graph", "batched", "plain"):
        print("level batch", variant, mode, flush=True)
        plan = cat.MulPlan(a_off, b_off, mode=mode)
        c = torch.full((limbs,), -1, dtype=torch.int32, device="cuda")
        for rep in range(2 if mode == "graph" else 1):
            if rep:
                c.fill_(-1)
            plan(da, db, c)
            plan.check()
            got = cat.to_numpy(c)
            d = _digests(got, plan.c_off)
            bad = [i for i in range(len(want)) if d[i] != want[i]]
            assert not bad, (mode, rep, bad[:10])
        plan.close()
    # a sample limb for limb, so that a digest file and the data behind it cannot drift apart
    rng = np.random.default_rng(123)
    for i in rng.choice(4096, 8, replace=False).tolist():
        ai = a[int(a_off[i]):int(a_off[i + 1])]
        bi = b[int(b_off[i]):int(b_off[i + 1])]
        ci = got[int(plan.c_off[i]):int(plan.c_off[i + 1])]
        assert np.array_equal(ci, oracle.mul(ai, bi)), i
