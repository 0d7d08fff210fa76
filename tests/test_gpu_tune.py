"""The autotuner on a few small buckets: every candidate schedule (schoolbook
threshold, one-workgroup tiles of 2^12..2^14 slots, four-step rows) must give
the default schedule's bits (tune.py raises otherwise), the table it picks is
valid for the library, and C(n) under it equals the oracle's."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def test_tuner_small_buckets_bit_identical():
    import torch

    import paper_2601_11621_amd as cat
    from paper_2601_11621_amd import tune

    torch.cuda.set_device(0)
    try:
        res = tune.autotune(max_k=10, min_k=7, reps=1, total_log2=15, verbose=True)
        assert set(res["ms"]) == {7, 8, 9, 10}
        for k in (7, 8, 9, 10):
            assert any(name.startswith("lds_t") for name in res["ms"][k]), k
        cat.set_tuning(res["table"])               # accepted by the library
        assert cat.get_tuning()["school_max"] == res["table"]["school_max"]
        for n in (3000, 40000):
            assert np.array_equal(cat.to_numpy(cat.exact(n, mode="graph")), oracle.catalan(n)), n
    finally:
        cat.set_tuning(None)
        cat.load_tuning()
