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


def test_scan_two_million_tuples_in_one_launch(orc, P):
    """2^21 tuples in 2,048 segments over 8 bases of the 100-customer workload
    (1 to 5 customers removed; each base admits feasible insertions) in one
    launch.  The launch is 512 copies of the bases' tuple lists (4,096 tuples
    in 4 uneven segments each) at random positions; every tuple's makespan
    and status, and every segment's top-3 (keys carry the tuple's index in
    the launch), against the oracle."""
    inst = synth.make_instance(100, 4, 5, 20, "2x", seed=9650)
    S = P.InstanceSet([inst])
    picks = [(9660, 1), (9660, 3), (9661, 1), (9662, 1), (9663, 1), (9664, 1), (9665, 1), (9665, 5)]
    nb, per = len(picks), 4096
    bases, lists = [], []
    for b, (seed, q) in enumerate(picks):
        bops, brt = make_base(inst, seed, q)
        tuples = synth.random_tuples(bops, brt, 100, 4, per, seed=9670 + b, invalid_frac=0.05)
        cuts = np.sort(synth.rng(9680 + b).integers(1, per, size=3))
        seg = np.concatenate([[0], cuts, [per]]).astype(np.int64)
        omk, ost, otop = orc.insert_scan(inst, bops, brt, tuples, seg)
        assert (ost == 0).sum() > 50 and (otop != INT64_MAX).any()
        bases.append((bops, brt))
        lists.append((tuples, seg, omk, ost, otop))
    pick = synth.rng(9690).integers(0, nb, size=512)
    T = per * len(pick)
    tup = np.concatenate([lists[b][0] for b in pick])
    seg_off = np.concatenate([[0]] + [lists[b][1][1:] + i * per for i, b in enumerate(pick)]).astype(np.int64)
    seg_base = np.repeat(pick, 4).astype(np.int32)
    b_off = np.concatenate([[0], np.cumsum([len(o) for o, _ in bases])[:-1]]).astype(np.int64)
    b_ops = np.concatenate([o for o, _ in bases]).astype(np.uint16)
    b_rt = np.concatenate([r for _, r in bases]).astype(np.uint16)
    print(f"[scan large] T={T} segments={len(seg_off) - 1}", flush=True)
    mk, st, top = P.vrprpd_insert_scan(S, dev(b_ops), dev(b_rt), dev(seg_off), dev(tup.view(np.uint8)),
                                       num_bases=nb, base_inst=dev(np.zeros(nb, np.int32)),
                                       base_op_off=dev(b_off), base_rt_off=dev(np.arange(nb, dtype=np.int64) * 4),
                                       seg_base=dev(seg_base))
    torch.cuda.synchronize()
    mk, st, top = mk.cpu().numpy(), st.cpu().numpy().view(np.uint32), top.cpu().numpy()
    emk = np.concatenate([lists[b][2] for b in pick])
    est = np.concatenate([lists[b][3] for b in pick])
    bad = np.nonzero((mk != emk) | (st != est))[0]
    assert bad.size == 0, (bad.size, int(bad[0]))
    for i, b in enumerate(pick):
        otop = lists[b][4].copy()
        real = otop != INT64_MAX
        otop[real] += i * per           # the tuple index in the low 32 bits moves with the copy
        assert np.array_equal(top[4 * i:4 * i + 4], otop), i
