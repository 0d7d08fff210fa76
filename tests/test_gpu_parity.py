"""GPU parity: the HIP path through the C ABI against the CPU oracle,
bit-exact (all arithmetic is exact integer work)."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from tests import pins

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def cat():
    import torch

    import paper_2601_11621_amd as c

    torch.cuda.set_device(0)
    c.init(0)
    return c


def _say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ Phase 1
def test_factor_small_n_all(cat):
    for n in range(0, 400):
        exps, off, pr = cat.factor(n)
        oe, oo, op = oracle.factor(n)
        assert np.array_equal(exps, oe), n
        assert np.array_equal(off, oo), n
        assert np.array_equal(cat.to_numpy(pr), op), n


@pytest.mark.parametrize("n", [401, 1000, 2047, 2048, 2049, 4096, 65535, 65536, 100000, 262143, 1000000, 3000000])
def test_factor_selected(cat, n):
    _say("factor", n)
    exps, off, pr = cat.factor(n)
    oe, oo, op = oracle.factor(n)
    assert np.array_equal(exps, oe)
    assert np.array_equal(off, oo)
    assert np.array_equal(cat.to_numpy(pr), op)


def test_factor_1e7(cat):
    n = 10**7
    exps, off, pr = cat.factor(n)
    oe, oo, op = oracle.factor(n)
    assert np.array_equal(exps, oe) and np.array_equal(off, oo)
    assert np.array_equal(cat.to_numpy(pr), op)
    # group sizes of the paper's workload family: |G_1| = 867,378 at n = 10^7
    assert int(off[1] - off[0]) == 867378


# ------------------------------------------------------------------ products
def _rand(rng, n, kind="rand"):
    if kind == "ones":
        return np.full(n, 0xFFFFFFFF, dtype=np.uint32)
    if kind == "zero":
        return np.zeros(n, dtype=np.uint32)
    return rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)


def _run_batch(cat, la, lb, kinds, mode, seed=0):
    rng = np.random.default_rng(seed)
    a = [_rand(rng, x, k) for x, k in zip(la, kinds)]
    b = [_rand(rng, x, k) for x, k in zip(lb, kinds)]
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    af, bf = np.concatenate(a), np.concatenate(b)
    c, c_off = cat.mul_batched(cat.from_numpy(af), a_off, cat.from_numpy(bf), b_off, mode=mode)
    oc, oc_off = oracle.mul_batched(af, a_off, bf, b_off)
    assert np.array_equal(c_off, oc_off)
    got = cat.to_numpy(c)
    for i in range(len(la)):
        s, e = int(c_off[i]), int(c_off[i + 1])
        assert np.array_equal(got[s:e], oc[s:e]), (i, la[i], lb[i], kinds[i], mode)


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_mul_edges(cat, mode):
    la, lb, kinds = [], [], []
    # bucket edges of the schoolbook / LDS / four-step classes, ragged tails
    for x, y in [(1, 1), (1, 128), (128, 128), (129, 1), (129, 129), (64, 65), (255, 256), (2047, 2049),
                 (2048, 2048), (2049, 2048), (4095, 2), (3000, 1100), (4097, 4096), (5000, 3), (1, 9000)]:
        for k in ["rand", "ones", "zero"]:
            la.append(x)
            lb.append(y)
            kinds.append(k)
    _run_batch(cat, la, lb, kinds, mode)


def test_mul_large_fourstep(cat):
    la = [40000, 65536, 70000, 1, 131072]
    lb = [30000, 65536, 100, 100000, 131071]
    kinds = ["rand", "ones", "rand", "rand", "ones"]
    _run_batch(cat, la, lb, kinds, "batched", seed=5)


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_mul_long_by_short(cat, mode):
    """Long-by-short products (the shorter operand up to 1,024 limbs) that the
    schedule may take by exact column sums: the all-ones worst case for the
    column sums (1,024 full products of (2^32 - 1)^2 per column), both operand
    orders, ragged ends of the 768-column blocks, and a random mix beside
    products of other classes in the same batch."""
    rng = np.random.default_rng(21)
    la = [65536, 1024, 8199, 50000, 9000, 1, 30000, 12345, 769, 40000]
    lb = [1024, 65536, 1024, 513, 1, 9001, 1000, 1000, 20000, 40]
    kinds = ["ones", "ones", "rand", "rand", "ones", "rand", "ones", "rand", "rand", "zero"]
    for _ in range(24):
        x = int(np.rint(2 ** rng.uniform(13, 16)))
        y = int(np.rint(2 ** rng.uniform(0, 10)))
        if rng.random() < 0.5:
            x, y = y, x
        la.append(x)
        lb.append(y)
        kinds.append("rand")
    # neighbours of other classes (schoolbook, one-workgroup, four-step)
    la += [100, 3000, 70000]
    lb += [90, 2500, 60000]
    kinds += ["rand", "rand", "rand"]
    _run_batch(cat, la, lb, kinds, mode, seed=22)


def test_mul_random_batch_uneven(cat):
    rng = np.random.default_rng(7)
    la = np.rint(2 ** rng.uniform(0, 13, 300)).astype(np.int64).tolist()
    lb = np.rint(2 ** rng.uniform(0, 13, 300)).astype(np.int64).tolist()
    _run_batch(cat, la, lb, ["rand"] * 300, "batched", seed=8)


def test_mul_wide_tiles(cat):
    """Products of 2^12 .. 2^14 coefficient slots, enough of them that the
    one-workgroup transforms of 2^13 and 2^14 slots run (when the schedule
    selects them) next to the 2^12 tiles and the four-step form."""
    rng = np.random.default_rng(12)
    la = np.rint(2 ** rng.uniform(11, 13, 240)).astype(np.int64).tolist()
    lb = np.rint(2 ** rng.uniform(11, 13, 240)).astype(np.int64).tolist()
    la[:3], lb[:3] = [8192, 4097, 1], [8192, 4096, 16383]
    _run_batch(cat, la, lb, ["ones", "rand", "rand"] + ["rand"] * 237, "batched", seed=13)


def test_mul_plan_graph_replays(cat):
    import torch

    rng = np.random.default_rng(9)
    la = np.rint(2 ** rng.uniform(6, 12, 64)).astype(np.int64)
    lb = np.rint(2 ** rng.uniform(6, 12, 64)).astype(np.int64)
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    af = _rand(rng, int(a_off[-1]))
    bf = _rand(rng, int(b_off[-1]))
    plan = cat.MulPlan(a_off, b_off, mode="graph")
    c = torch.zeros(int((la + lb).sum()), dtype=torch.int32, device="cuda")
    da, db = cat.from_numpy(af), cat.from_numpy(bf)
    oc, _ = oracle.mul_batched(af, a_off, bf, b_off)
    for rep in range(4):
        c.zero_()
        torch.cuda.synchronize()
        plan(da, db, c)
        plan.check()
        assert np.array_equal(cat.to_numpy(c), oc), rep
    plan.close()


# ------------------------------------------------------------------ C(n)
def test_exact_small_n_all_modes(cat):
    for n in range(0, 300):
        exp = oracle.catalan(n)
        for mode in (["batched", "plain", "graph"] if n % 7 == 0 else ["graph"]):
            got = cat.to_numpy(cat.exact(n, mode=mode))
            assert np.array_equal(got, exp), (n, mode)


@pytest.mark.parametrize("n", [1000, 4097, 13337, 100000])
def test_exact_vs_oracle(cat, n):
    _say("exact", n)
    exp = oracle.catalan(n)
    for mode in ["batched", "graph", "plain"]:
        got = cat.to_numpy(cat.exact(n, mode=mode))
        assert np.array_equal(got, exp), mode


def test_exact_random_n_vs_oracle(cat):
    """Seeded random n spread over the sizes where the schedule changes
    (schoolbook, LDS tiles, four-step levels, small and large column tiles,
    the column-sum product by R)."""
    rng = np.random.default_rng(20260)
    ns = sorted(set(int(x) for x in np.exp(rng.uniform(np.log(300), np.log(400000), 24)).astype(np.int64)))
    for n in ns:
        _say("exact random", n)
        assert np.array_equal(cat.to_numpy(cat.exact(n, mode="graph")), oracle.catalan(n)), n


def test_exact_1e6_vs_oracle(cat):
    exp = oracle.catalan(10**6)
    got = cat.to_numpy(cat.exact(10**6, mode="graph"))
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("n", [10**7, 10**8])
def test_exact_full_size_digest(cat, n):
    """Full benchmark size: the SHA-256 of the limbs against the oracle's
    digest (written by tests/golden/make_oracle_golden.py), plus residue pins."""
    with open(os.path.join(GOLDEN, "oracle_catalan.json")) as f:
        gold = json.load(f)[str(n)]
    t = cat.exact(n, mode="graph")
    got = cat.to_numpy(t)
    assert len(got) == gold["n_limbs"]
    assert hashlib.sha256(got.astype("<u4").tobytes()).hexdigest() == gold["sha256_le_limbs"]
    r = cat.residues(t)
    assert r[0] == gold["mod_2p32_minus_5"]
    assert r[1] == pins.catalan_mod_composite(n, [641, 6700417])


def test_exact_graph_replays_are_identical(cat):
    """The whole-call graph (cached plan) replayed several times, with other
    work in between, gives the oracle's result every time."""
    import torch

    n = 250000
    exp = oracle.catalan(n)
    for rep in range(4):
        got = cat.to_numpy(cat.exact(n, mode="graph"))
        assert np.array_equal(got, exp), rep
        cat.exact(1000 + rep, mode="graph")          # other n in between
        torch.cuda.synchronize()


def test_residues_kernel(cat):
    rng = np.random.default_rng(3)
    for n in [1, 5, 255, 256, 257, 4095, 4096, 4097, 8192 + 300, 100000, 1 << 20]:
        x = _rand(rng, n)
        v = pins.limbs_int(x)
        r = cat.residues(cat.from_numpy(x))
        assert r == (v % (2**32 - 5), v % (2**32 + 1), v % (2**32 - 1)), n
    # all-ones limbs: the largest partial sums of every block
    for n in [4096, 3 * 4096 + 17]:
        x = np.full(n, 0xFFFFFFFF, dtype=np.uint32)
        v = (1 << (32 * n)) - 1
        assert cat.residues(cat.from_numpy(x)) == (v % (2**32 - 5), v % (2**32 + 1), v % (2**32 - 1)), n


@pytest.mark.parametrize("polls", [0, 1, 16])
def test_carry_lookback_recompute(cat, polls):
    """With no (or one) poll of the predecessor's published carry pair, CRT
    blocks recompute it from the residues: same products, same C(n).  All-ones
    operands give blocks that propagate a carry across their whole length."""
    try:
        cat.set_lookback_polls(polls)
        la = [5000, 70000, 9000, 4096, 131072, 3000]
        lb = [5000, 70000, 2, 4096, 131071, 12000]
        kinds = ["ones", "ones", "rand", "ones", "ones", "rand"]
        _run_batch(cat, la, lb, kinds, "batched", seed=21)
        for n in (13337, 250000):
            assert np.array_equal(cat.to_numpy(cat.exact(n, mode="graph")), oracle.catalan(n)), n
    finally:
        cat.set_lookback_polls(None)


def _carry_run(runs):
    """limbs 5, 3, 3, ..., 3 per run: times 2^32 - 1, the position after the
    first 3 of a run generates a carry and every later position of the run
    propagates it (pre-carry value 2^32 - 1)"""
    a = []
    for r in runs:
        a += [5] + [3] * r
    return np.array(a, dtype=np.uint32)


@pytest.mark.parametrize("polls", [None, 0, 16])
def test_carry_runs_across_blocks(cat, polls):
    """Carries that cross many whole CRT blocks: the positions just below a
    block do not decide its carry in, so the block looks back over its
    predecessors (or recomputes them).  Products from every transform class
    and from exact column sums, against the oracle."""
    mixed = [10, 12, 13, 14, 20, 767, 768, 769, 2000] * 4
    cases = [
        (_carry_run([300000]), 5000),     # four-step transform, one carry through 300,000 limbs
        (_carry_run([40000]), 5000),
        (_carry_run(mixed), 5000),        # runs ending at every offset around the block edges
        (_carry_run([8000]), 100),        # one-workgroup transform
        (_carry_run([40000]), 1),         # column sums (long times one limb)
        (np.full(50000, 0xFFFFFFFF, dtype=np.uint32), 3000),   # propagate everywhere, no carry
    ]
    a = [x for x, _ in cases]
    b = [np.concatenate([[0xFFFFFFFF], np.zeros(lb - 1, dtype=np.uint32)]).astype(np.uint32) for _, lb in cases]
    la = [len(x) for x in a]
    lb = [len(x) for x in b]
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    af, bf = np.concatenate(a), np.concatenate(b)
    oc, oc_off = oracle.mul_batched(af, a_off, bf, b_off)
    try:
        cat.set_lookback_polls(polls)
        for mode in ("batched", "plain"):
            c, c_off = cat.mul_batched(cat.from_numpy(af), a_off, cat.from_numpy(bf), b_off, mode=mode)
            assert np.array_equal(c_off, oc_off)
            got = cat.to_numpy(c)
            for i in range(len(cases)):
                s, e = int(c_off[i]), int(c_off[i + 1])
                assert np.array_equal(got[s:e], oc[s:e]), (i, la[i], lb[i], mode)
    finally:
        cat.set_lookback_polls(None)


def _schedule_short(t):
    """small schoolbook threshold, four-step transforms with short rows and
    short column passes from 2^11 up"""
    t["school_max"] = 32
    for k in range(11, 28):
        t["cls"][k] = 2
        t["log_row"][k] = 10
        t["log_pass"][k] = 6


def _schedule_wide(t):
    """one-workgroup transforms of 2^13 and 2^14 slots (512 and 1024 threads),
    four-step rows of 2^13 or 2^14 words above"""
    t["cls"][13] = t["cls"][14] = 1
    for k in range(15, 28):
        t["cls"][k] = 2
        t["log_row"][k] = 13 + (k & 1)
        t["log_pass"][k] = 8


def _schedule_rows11(t):
    """four-step transforms with rows of 2^11 words (the 128-thread row tile)
    from 2^12 up"""
    for k in range(12, 28):
        t["cls"][k] = 2
        t["log_row"][k] = 11
        t["log_pass"][k] = 10 if k < 24 else 8


def _schedule_tiles14(t):
    """one-workgroup transforms of 2^9 .. 2^14 points all in 2^14-slot tiles
    (1,024 threads, up to 32 products per tile)"""
    for k in range(9, 15):
        t["cls"][k] = 1
        t["log_row"][k] = 14


@pytest.mark.parametrize("schedule", [_schedule_short, _schedule_wide, _schedule_rows11, _schedule_tiles14],
                         ids=["short", "wide", "rows11", "tiles14"])
def test_schedules_change_speed_not_bits(cat, schedule):
    """A non-default product schedule gives the same C(n) and the same
    products as the default one."""
    import torch

    base = cat.get_tuning()
    ns = [5000, 100000, 10**6]
    ref = {n: cat.to_numpy(cat.exact(n, mode="batched")) for n in ns}
    rng = np.random.default_rng(4)
    la = np.rint(2 ** rng.uniform(3, 15, 40)).astype(np.int64)
    lb = np.rint(2 ** rng.uniform(3, 15, 40)).astype(np.int64)
    # and transforms of 2^19 and 2^20 points (two column passes under the
    # short schedule, the first applying its own twiddles)
    la = np.concatenate([la, [(1 << 18) - 5, 300000]])
    lb = np.concatenate([lb, [(1 << 18) - 3, 70000]])
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    da = cat.from_numpy(_rand(rng, int(a_off[-1])))
    db = cat.from_numpy(_rand(rng, int(b_off[-1])))
    c0, c_off = cat.mul_batched(da, a_off, db, b_off)
    c0 = c0.clone()
    if schedule is _schedule_short:
        # the two large products of the default schedule against the oracle
        av, bv, cv = cat.to_numpy(da), cat.to_numpy(db), cat.to_numpy(c0)
        for i in (len(la) - 2, len(la) - 1):
            xa = av[int(a_off[i]):int(a_off[i + 1])]
            xb = bv[int(b_off[i]):int(b_off[i + 1])]
            oc, _ = oracle.mul_batched(xa, np.array([0, len(xa)], dtype=np.uint64), xb,
                                       np.array([0, len(xb)], dtype=np.uint64))
            assert np.array_equal(cv[int(c_off[i]):int(c_off[i + 1])], oc), i
    t = cat.get_tuning()
    schedule(t)
    try:
        cat.set_tuning(t)
        for n in ns:
            assert np.array_equal(cat.to_numpy(cat.exact(n, mode="batched")), ref[n]), n
        c1, _ = cat.mul_batched(da, a_off, db, b_off)
        assert torch.equal(c0, c1)
    finally:
        cat.set_tuning(base)


@pytest.mark.parametrize("logn", [0, 9, 10, 12])
def test_fused_levels_same_bits(cat, logn):
    """The lower tree levels fused into one launch (tiles of 4,096 leaves kept
    in LDS across levels, carries inside the workgroup) give the same C(n) as
    one transform launch and one carry launch per level: ragged last tiles,
    groups whose tree ends inside the fused levels, and sizes where the fused
    range is cut short by the tree height."""
    try:
        cat.set_fused_levels(logn)
        for n in (300, 2500, 5000, 13337, 65536, 100000, 262147, 1000003):
            _say("fused", logn, n)
            got = cat.to_numpy(cat.exact(n, mode="graph"))
            assert np.array_equal(got, oracle.catalan(n)), (logn, n)
            assert np.array_equal(cat.to_numpy(cat.exact(n, mode="batched")), got), (logn, n)
        # a generic batch: the one-workgroup buckets in one fused launch (or
        # one launch pair per bucket), products of N and N + 1 limbs included
        rng = np.random.default_rng(logn + 100)
        la = np.rint(2 ** rng.uniform(0, 12, 150)).astype(np.int64).tolist() + [64, 2049, 1024, 2048, 129]
        lb = np.rint(2 ** rng.uniform(0, 12, 150)).astype(np.int64).tolist() + [65, 2048, 1025, 2048, 128]
        kinds = ["rand"] * 150 + ["ones", "ones", "rand", "ones", "rand"]
        _run_batch(cat, la, lb, kinds, "batched", seed=logn)
        with open(os.path.join(GOLDEN, "oracle_catalan.json")) as f:
            gold = json.load(f)["10000000"]
        got = cat.to_numpy(cat.exact(10**7, mode="graph"))
        assert hashlib.sha256(got.astype("<u4").tobytes()).hexdigest() == gold["sha256_le_limbs"]
    finally:
        cat.set_fused_levels(None)


@pytest.mark.parametrize("lazy", [0, 12, 23])
@pytest.mark.parametrize("fused", [0, 12])
def test_lazy_primes_same_bits(cat, lazy, fused):
    """Transform products on the three primes below 2^30 with unreduced
    butterfly ranges give the same products and C(n) as the three primes above
    2^31: both against the oracle, with all-ones operands (the largest
    coefficients, which the second set's CRT range must cover), ragged tiles
    and products of N + 1 limbs, with the lower tree levels fused or not."""
    try:
        cat.set_lazy_primes(lazy)
        cat.set_fused_levels(fused)
        la, lb, kinds = [], [], []
        for x, y in [(1, 1), (129, 129), (255, 256), (2047, 2049), (2048, 2048), (2049, 2048), (4095, 2),
                     (3000, 1100), (4097, 4096), (8192, 8192), (8193, 8192), (5000, 3)]:
            for k in ["rand", "ones", "zero"]:
                la.append(x)
                lb.append(y)
                kinds.append(k)
        _say("lazy", lazy, "fused", fused, "edges")
        _run_batch(cat, la, lb, kinds, "batched", seed=lazy + fused)
        _run_batch(cat, la, lb, kinds, "plain", seed=lazy + fused + 1)
        _say("lazy", lazy, "fused", fused, "four-step")
        _run_batch(cat, [40000, 65536, 70000, 131072, 1 << 17], [30000, 65536, 100, 131071, 1 << 17],
                   ["rand", "ones", "rand", "ones", "ones"], "batched", seed=9)
        for n in (300, 5000, 13337, 100000, 1000003):
            _say("lazy", lazy, "fused", fused, "C", n)
            got = cat.to_numpy(cat.exact(n, mode="graph"))
            assert np.array_equal(got, oracle.catalan(n)), (lazy, fused, n)
        with open(os.path.join(GOLDEN, "oracle_catalan.json")) as f:
            gold = json.load(f)["10000000"]
        got = cat.to_numpy(cat.exact(10**7, mode="graph"))
        assert hashlib.sha256(got.astype("<u4").tobytes()).hexdigest() == gold["sha256_le_limbs"]
    finally:
        cat.set_lazy_primes(23)
        cat.set_fused_levels(None)


@pytest.mark.parametrize("fused", [0, 12])
@pytest.mark.parametrize("on", [False, True])
def test_outer_node_same_bits(cat, on, fused):
    """R, the product of the powers P_e with e >= 2, entering Q_1's product
    tree as one more node (on) or multiplied onto Q_1 after the tree (off):
    the same C(n) in every mode against the oracle, at sizes where the node is
    taken and where Q_1's tree is too short for it, with the lower levels
    fused or not, and the full-size digest at 10^7."""
    try:
        cat.set_outer_node(on)
        cat.set_fused_levels(fused)
        for n in (2000, 5000, 13337, 100000, 262147, 524287, 1000003):
            _say("outer node", on, "fused", fused, n)
            exp = oracle.catalan(n)
            for mode in (["graph", "batched", "plain"] if n <= 100000 else ["graph", "batched"]):
                got = cat.to_numpy(cat.exact(n, mode=mode))
                assert np.array_equal(got, exp), (on, fused, n, mode)
                lvl = cat.stats()["outer_level"]
                if not on:
                    assert lvl == -1, (n, lvl)
                if on and n >= 100000:
                    assert lvl >= 6, (n, lvl)
        with open(os.path.join(GOLDEN, "oracle_catalan.json")) as f:
            gold = json.load(f)["10000000"]
        got = cat.to_numpy(cat.exact(10**7, mode="graph"))
        assert hashlib.sha256(got.astype("<u4").tobytes()).hexdigest() == gold["sha256_le_limbs"]
        assert (cat.stats()["outer_level"] >= 6) == on
    finally:
        cat.set_outer_node(True)
        cat.set_fused_levels(None)


def _ones_square(a):
    """(B^a - 1)^2 = B^(2a) - 2 B^a + 1, B = 2^32: limb 0 is 1, limbs 1..a-1
    are 0, limb a is B - 2 and limbs a+1..2a-1 are B - 1."""
    c = np.zeros(2 * a, dtype=np.uint32)
    c[0] = 1
    c[a] = 0xFFFFFFFE
    c[a + 1:] = 0xFFFFFFFF
    return c


@pytest.mark.parametrize("a", [1 << 22, (1 << 22) + 1, 1 << 23])
def test_largest_coefficients_closed_form(cat, a):
    """The all-ones square has the largest convolution coefficients a product
    of its size can have, (B - 1)^2 times the overlap; at a = 2^22 (the last
    size of the primes below 2^30, N = 2^23), 2^22 + 1 and 2^23 (the primes
    above 2^31) it must still come out exactly, against the closed form."""
    x = np.full(a, 0xFFFFFFFF, dtype=np.uint32)
    off = np.array([0, a], dtype=np.uint64)
    d = cat.from_numpy(x)
    c, c_off = cat.mul_batched(d, off, d, off, mode="batched")
    got = cat.to_numpy(c)
    assert int(c_off[-1]) == 2 * a
    assert np.array_equal(got, _ones_square(a))


def test_mul_batched_is_asynchronous(cat):
    """bigint_mul_batched returns once the products are queued; the device
    check comes from bigint_mul_check.  The same shape again (plan from the
    library's cache) on a second stream, and a new shape, give the oracle's
    products bit for bit."""
    import ctypes

    import torch

    lib = cat.load()
    rng = np.random.default_rng(41)
    la = np.rint(2 ** rng.uniform(0, 13, 40)).astype(np.int64)
    lb = np.rint(2 ** rng.uniform(0, 13, 40)).astype(np.int64)
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    c_off = np.concatenate([[0], np.cumsum(la + lb)]).astype(np.uint64)
    af, bf = _rand(rng, int(a_off[-1])), _rand(rng, int(b_off[-1]))
    oc, _ = oracle.mul_batched(af, a_off, bf, b_off)
    wb = ctypes.c_size_t()
    cat._check(lib.bigint_mul_workspace(40, cat._p64(a_off), cat._p64(b_off), ctypes.byref(wb)), "workspace")
    da, db = cat.from_numpy(af), cat.from_numpy(bf)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for s in streams + streams[:1]:
        c = torch.full((int(c_off[-1]),), -1, dtype=torch.int32, device="cuda")
        w = torch.empty(wb.value, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        vs = ctypes.c_void_p(s.cuda_stream)
        st = lib.bigint_mul_batched(40, cat._ptr(da), cat._p64(a_off), cat._ptr(db), cat._p64(b_off), cat._ptr(c),
                                    cat._p64(c_off), cat._ptr(w), w.numel(), vs)
        assert st == cat.CAT_OK
        outs.append((c, w, vs))
    for c, w, vs in outs:
        assert lib.bigint_mul_check(cat._ptr(w), vs) == cat.CAT_OK
        assert np.array_equal(cat.to_numpy(c), oc)
    # a different shape (one product more) is planned afresh
    c2, c2_off = cat.mul_batched(da, a_off[:31], db, b_off[:31])
    assert np.array_equal(cat.to_numpy(c2), oc[: int(c2_off[-1])])


def test_valu_rate_probe(cat):
    """The instruction issue-rate probe runs every form it names and rejects
    bad arguments; no form issues faster than two lane-ops per lane per clock
    at 2.4 GHz (a loose bound that catches a timing or counting slip)."""
    import ctypes

    import torch

    lib = cat.load()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for op in cat.VALU_OPS:
        r, ms = cat.valu_rate(op, 64)
        assert ms > 0 and 0 < r < 2 * cus * 64 * 2.4e9, (op, r, ms)
    rate = ctypes.c_double()
    assert lib.cat_valu_rate(len(cat.VALU_OPS), 64, ctypes.byref(rate), None) == cat.CAT_EINVAL
    assert lib.cat_valu_rate(-1, 64, ctypes.byref(rate), None) == cat.CAT_EINVAL
    assert lib.cat_valu_rate(0, 0, ctypes.byref(rate), None) == cat.CAT_EINVAL
    assert lib.cat_valu_rate(0, (1 << 20) + 1, ctypes.byref(rate), None) == cat.CAT_EINVAL
    assert lib.cat_valu_rate(0, 64, None, None) == cat.CAT_EINVAL
