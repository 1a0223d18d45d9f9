"""Parity: solution statistics (Cross-Agent, Interleaved; Section 5.2) on the
GPU against the oracle, per solution and bit-exact."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_23685_amd as P
    P.load()
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def expect(orc, inst, ops, rt):
    out = []
    for b in range(len(ops)):
        s = orc.solution_stats(inst, ops[b][:int(rt[b][-1])], rt[b])
        out.append(s if s is not None else (-1, -1))
    return np.array(out, np.int32).reshape(-1, 2)


CASES = [
    # n, m, k, R, rule, B
    (16, 2, 2, 4, "base", 3000),           # more solutions than blocks
    (100, 4, 5, 20, "5x", 200),
    (1000, 10, 10, 100, "1R20d10", 16),
    (20, 17, 2, 40, "1R10", 64),
    (1, 3, 1, 3, "base", 8),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}m{c[1]}")
def test_stats_parity(orc, P, case):
    n, m, k, R, rule, B = case
    inst = synth.make_instance(n, m, k, R, rule, seed=8000 + n)
    ops, rt = synth.random_candidates(inst, B, seed=n)
    S = P.InstanceSet([inst])
    cross, inter = P.vrprpd_solution_stats(S, dev(ops), dev(rt))
    got = np.stack([cross.cpu().numpy(), inter.cpu().numpy()], axis=1)
    assert np.array_equal(got, expect(orc, inst, ops, rt))


def test_stats_hand_worked_boundaries(orc, P):
    """The oracle's hand-worked line schedules on the GPU, the time-equality
    boundary of Interleaved among them (p1 = 10: the drop vehicle's next op
    and the pickup both at time 20, not interleaved)."""
    D, Pk = 0, 1
    cases = [([100, 100], [[(1, D), (1, Pk)], [(2, D), (2, Pk)]], (0, 0)),
             ([100, 100], [[(1, D), (2, D), (2, Pk), (1, Pk)], []], (0, 1)),
             ([100, 100], [[(1, D), (2, D)], [(1, Pk), (2, Pk)]], (2, 1)),
             ([0, 100], [[(1, D), (2, Pk)], [(2, D), (1, Pk)]], (2, 1)),
             ([10, 0], [[(1, D), (2, D)], [(1, Pk), (2, Pk)]], (2, 0))]
    for p, routes, want in cases:
        x = np.arange(3) * 10
        d = np.abs(x[:, None] - x[None, :]).astype(np.int32)
        inst = synth.instance_from_matrix(d, np.array([0] + p, np.int32), 2, k=2, R=4)
        ops = np.array([[(c << 1) | t for r in routes for c, t in r]], np.uint16)
        rt = np.array([np.cumsum([len(r) for r in routes])], np.uint16)
        cross, inter = P.vrprpd_solution_stats(P.InstanceSet([inst]), dev(ops), dev(rt))
        got = (int(cross[0]), int(inter[0]))
        assert got == want == orc.solution_stats(inst, ops[0], rt[0]), (p, routes)


def test_stats_of_constructions_and_bad_inputs(orc, P):
    insts = [synth.make_instance(60, 5, 4, 20, "2x", seed=8101), synth.make_instance(30, 3, 3, 9, "5x", seed=8102)]
    S = P.InstanceSet(insts)
    N, M = S.n_max, S.m_max
    rows_o, rows_r, ids = [], [], []
    for h in range(4):
        o, r = P.vrprpd_construct(S, h)
        for i in range(2):
            rows_o.append(o[i].cpu().numpy())
            rows_r.append(r[i].cpu().numpy())
            ids.append(i)
    # an incomplete solution, a wait cycle, bad route ends, a bad instance index
    o = rows_o[0].copy()
    r = rows_r[0].copy()
    r2 = r.copy()
    r2[-1] -= 2
    rows_o.append(o), rows_r.append(r2), ids.append(0)
    cyc = np.zeros(2 * N, np.uint16)
    cyc[:4] = [(2 << 1) | 1, 1 << 1, (1 << 1) | 1, 2 << 1]         # P2 D1 | P1 D2 ...
    rest = [((c << 1), (c << 1) | 1) for c in range(3, 61)]
    cyc[4:4 + 2 * len(rest)] = [x for pr in rest for x in pr]
    rc = np.zeros(M, np.uint16)
    rc[0], rc[1:5] = 2, 120
    rows_o.append(cyc), rows_r.append(rc), ids.append(0)
    rb = r.copy()
    rb[0] = 5000
    rows_o.append(o), rows_r.append(rb), ids.append(0)
    rows_o.append(o), rows_r.append(r), ids.append(7)
    ops = np.stack(rows_o)
    rts = np.stack(rows_r)
    cross, inter = P.vrprpd_solution_stats(S, dev(ops), dev(rts), inst=dev(np.array(ids, np.int32)),
                                           op_off=dev(np.arange(len(ids), dtype=np.int64) * 2 * N),
                                           rt_off=dev(np.arange(len(ids), dtype=np.int64) * M))
    cross, inter = cross.cpu().numpy(), inter.cpu().numpy()
    for b, i in enumerate(ids):
        if i >= len(insts) or rts[b][0] > 2 * insts[min(i, 1)].n:
            assert (cross[b], inter[b]) == (-1, -1), b
            continue
        inst = insts[i]
        s = orc.solution_stats(inst, ops[b][:int(rts[b][inst.m - 1])], rts[b][:inst.m])
        assert (cross[b], inter[b]) == (s if s is not None else (-1, -1)), b
    assert (cross[-4], cross[-3]) == (-1, -1)           # incomplete cover, wait cycle
