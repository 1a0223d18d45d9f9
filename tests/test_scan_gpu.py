"""Parity: vrprpd_insert_scan on the GPU vs the CPU oracle (bit-exact)."""
import numpy as np
import pytest

import synth
from cases import destroy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

INT64_MAX = 2**63 - 1


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_23685_amd as P
    P.load()
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_scan(P, S, bops, brt, tuples, seg_off, blocks_per_seg=None):
    mk, st, top = P.vrprpd_insert_scan(S, dev(bops), dev(brt), dev(seg_off),
                                       dev(tuples.view(np.uint8)), blocks_per_seg=blocks_per_seg)
    torch.cuda.synchronize()
    return mk.cpu().numpy(), st.cpu().numpy().view(np.uint32), top.cpu().numpy()


def make_base(inst, seed, q):
    ops, rt = synth.random_candidates(inst, 1, seed)
    fo, off, frt = destroy(inst, ops, rt, seed=seed, q=q)
    return fo, frt[0]


SCAN_CASES = [
    # n, m, k, R, rule, lm, q, T, segs
    (16, 2, 2, 4, "base", 0, 4, 3000, 7),
    (100, 4, 5, 20, "2x", 0, 5, 4000, 20),
    (1000, 10, 10, 100, "1R20d10", 0, 40, 600, 6),
    (60, 17, 3, 60, "1R10", 1, 6, 1500, 5),
    (40, 40, 2, 80, "5x", 0, 4, 800, 3),
]


@pytest.mark.parametrize("case", SCAN_CASES, ids=lambda c: f"n{c[0]}m{c[1]}")
def test_scan_parity(orc, P, case):
    n, m, k, R, rule, lm, q, T, nseg = case
    inst = synth.make_instance(n, m, k, R, rule, seed=5000 + n, load_model=lm)
    bops, brt = make_base(inst, n, q)
    tuples = synth.random_tuples(bops, brt, n, m, T, seed=n, invalid_frac=0.05)
    cuts = np.sort(synth.rng(n).integers(0, T + 1, size=nseg - 1))
    seg_off = np.concatenate([[0], cuts, [T]]).astype(np.int64)
    S = P.InstanceSet([inst])
    mk, st, top = run_scan(P, S, bops, brt, tuples, seg_off)
    omk, ost, otop = orc.insert_scan(inst, bops, brt, tuples, seg_off)
    bad = np.nonzero((mk != omk) | (st != ost))[0]
    assert bad.size == 0, f"{bad.size} mismatches; first {bad[0]}: gpu ({mk[bad[0]]},{st[bad[0]]}) " \
                          f"oracle ({omk[bad[0]]},{ost[bad[0]]}) tuple {tuples[bad[0]]}"
    assert np.array_equal(top, otop)
    assert (ost == 32).any()
    if n <= 100 and lm == 0:
        assert (ost == 0).any()


def test_scan_parity_wide_distances(orc, P):
    """Travel times above 65535: the int32 op store (separate code and leg
    arrays, its own padding) in the scan."""
    inst = synth.make_instance(70, 4, 5, 20, "2x", seed=5301)
    inst.d = (inst.d.astype(np.int64) * 500).astype(np.int32)
    inst.p = (inst.p.astype(np.int64) * 500).astype(np.int32)
    S = P.InstanceSet([inst])
    assert S.dist16 == 0
    bops, brt = make_base(inst, 7, 6)
    T = 2000
    tuples = synth.random_tuples(bops, brt, 70, 4, T, seed=8, invalid_frac=0.05)
    seg_off = np.array([0, 700, 1300, T], np.int64)
    mk, st, top = run_scan(P, S, bops, brt, tuples, seg_off)
    omk, ost, otop = orc.insert_scan(inst, bops, brt, tuples, seg_off)
    assert np.array_equal(mk, omk) and np.array_equal(st, ost)
    assert np.array_equal(top, otop)
    assert (omk < 2**31 - 1).sum() > T // 2       # most tuples were swept to a makespan


def test_scan_deadlock_tuples_and_reuse(orc, P):
    """Pickups placed before their own drop on another vehicle deadlock; the
    group must reset its state and evaluate the following tuples exactly."""
    inst = synth.make_instance(30, 3, 4, 12, "5x", seed=11)
    bops, brt = make_base(inst, 3, 3)
    T = 900
    tuples = synth.random_tuples(bops, brt, 30, 3, T, seed=4)
    S = P.InstanceSet([inst])
    seg_off = np.array([0, T], np.int64)
    mk, st, top = run_scan(P, S, bops, brt, tuples, seg_off)
    omk, ost, otop = orc.insert_scan(inst, bops, brt, tuples, seg_off)
    assert np.array_equal(mk, omk) and np.array_equal(st, ost) and np.array_equal(top, otop)
    assert (ost & 8).any()


def test_scan_served_customer_tuples(orc, P):
    """Tuples that re-insert a customer the base already serves are tuple
    errors (valid positions or not), mixed with ordinary tuples."""
    inst = synth.make_instance(40, 3, 4, 12, "2x", seed=13)
    bops, brt = make_base(inst, 7, 4)
    ok = synth.random_tuples(bops, brt, 40, 3, 300, seed=8)
    served = sorted({int(x) >> 1 for x in bops[:int(brt[-1])]})
    bad = np.zeros(len(served), dtype=ok.dtype)
    for i, c in enumerate(served):
        bad[i]["c"], bad[i]["vD"], bad[i]["pD"], bad[i]["vP"], bad[i]["pP"] = c, 0, 0, 0, 1
    tuples = np.concatenate([ok, bad])[synth.rng(9).permutation(len(ok) + len(bad))]
    seg_off = np.array([0, 150, len(tuples)], np.int64)
    S = P.InstanceSet([inst])
    mk, st, top = run_scan(P, S, bops, brt, tuples, seg_off)
    omk, ost, otop = orc.insert_scan(inst, bops, brt, tuples, seg_off)
    assert np.array_equal(mk, omk) and np.array_equal(st, ost) and np.array_equal(top, otop)
    assert (ost == 32).sum() >= len(served)


def test_scan_bad_base(orc, P):
    inst = synth.make_instance(20, 2, 3, 6, "base", seed=12)
    bops, brt = make_base(inst, 5, 3)
    tuples = synth.random_tuples(bops, brt, 20, 2, 200, seed=6)
    S = P.InstanceSet([inst])
    seg_off = np.array([0, 100, 200], np.int64)
    dup = bops.copy()
    dup[1] = dup[0]                                      # duplicate op in the base
    for b_ops, b_rt in [(dup, brt), (bops, np.array([brt[1], brt[0]], np.uint16))]:
        mk, st, top = run_scan(P, S, b_ops, b_rt, tuples, seg_off)
        omk, ost, otop = orc.insert_scan(inst, b_ops, b_rt, tuples, seg_off)
        assert np.array_equal(mk, omk) and np.array_equal(st, ost) and np.array_equal(top, otop)
        assert np.all(top == INT64_MAX)


def test_scan_empty_segments(orc, P):
    inst = synth.make_instance(16, 2, 2, 4, "base", seed=13)
    bops, brt = make_base(inst, 7, 4)
    tuples = synth.random_tuples(bops, brt, 16, 2, 50, seed=8)
    seg_off = np.array([0, 0, 25, 25, 50, 50], np.int64)
    S = P.InstanceSet([inst])
    mk, st, top = run_scan(P, S, bops, brt, tuples, seg_off)
    omk, ost, otop = orc.insert_scan(inst, bops, brt, tuples, seg_off)
    assert np.array_equal(top, otop) and np.all(top[[0, 2, 4]] == INT64_MAX)


@pytest.mark.parametrize("bps", [1, 3, 40])
def test_scan_split_segments(orc, P, bps):
    """Several workgroups per segment merge their top-3 keys atomically; the
    result must not depend on how many share a segment."""
    inst = synth.make_instance(50, 3, 4, 12, "2x", seed=14)
    bops, brt = make_base(inst, 9, 5)
    tuples = synth.random_tuples(bops, brt, 50, 3, 2500, seed=10)
    seg_off = np.array([0, 1, 700, 2000, 2500], np.int64)
    S = P.InstanceSet([inst])
    mk, st, top = run_scan(P, S, bops, brt, tuples, seg_off, blocks_per_seg=bps)
    omk, ost, otop = orc.insert_scan(inst, bops, brt, tuples, seg_off)
    assert np.array_equal(mk, omk) and np.array_equal(st, ost) and np.array_equal(top, otop)
