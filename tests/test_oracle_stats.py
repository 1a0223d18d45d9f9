"""Pins for the oracle's solution statistics (Section 5.2: Cross-Agent and
Interleaved), CPU only: hand-worked schedules on a line, and invariants."""
import numpy as np

import synth
from oracle import solution_stats


def line_instance(p, m):
    """Depot and customers at x = 0, 10, 20, ... on a line."""
    n = len(p)
    x = np.arange(n + 1) * 10
    d = np.abs(x[:, None] - x[None, :]).astype(np.int32)
    return synth.instance_from_matrix(d, np.array([0] + list(p), np.int32), m, k=2, R=4)


def pack(routes):
    ops = np.array([(c << 1) | isP for r in routes for c, isP in r], np.uint16)
    rt = np.cumsum([len(r) for r in routes]).astype(np.uint16)
    return ops, rt


D, P_ = 0, 1


def test_hand_worked_schedules():
    inst = line_instance([100, 100], m=2)
    # each vehicle serves one customer, pickup right after drop
    assert solution_stats(inst, *pack([[(1, D), (1, P_)], [(2, D), (2, P_)]])) == (0, 0)
    # one vehicle: D1 D2 P2 P1 -- c1 has D2, P2 between its ops, c2 none
    assert solution_stats(inst, *pack([[(1, D), (2, D), (2, P_), (1, P_)], []])) == (0, 1)
    # v0 drops both (D1 at 10, D2 at 20), v1 picks both up (P1 waits to 110,
    # P2 at 120): both cross; after D1, v0 drops c2 at 20 < 110 (interleaved);
    # D2 is v0's last op (not interleaved)
    assert solution_stats(inst, *pack([[(1, D), (2, D)], [(1, P_), (2, P_)]])) == (2, 1)
    # p1 = 0, p2 = 100: v0 = D1 (10), P2 (waits to 120); v1 = D2 (20), P1 (30).
    # c1: v0's next op after D1 is at 120 >= 30: not interleaved;
    # c2: v1's next op after D2 is at 30 < 120: interleaved
    inst = line_instance([0, 100], m=2)
    assert solution_stats(inst, *pack([[(1, D), (2, P_)], [(2, D), (1, P_)]])) == (2, 1)
    # the boundary: p1 = 10, p2 = 0; v0 = D1 (10), D2 (20); v1 = P1 (arrives
    # 10, waits to 10 + 10 = 20), P2 (30).  v0's op after D1 is at 20, the same
    # time as P1: not before it, so c1 is not interleaved; D2 is v0's last op
    inst = line_instance([10, 0], m=2)
    assert solution_stats(inst, *pack([[(1, D), (2, D)], [(1, P_), (2, P_)]])) == (2, 0)


def test_unschedulable_solutions_have_no_statistics():
    inst = line_instance([5, 5], m=2)
    assert solution_stats(inst, *pack([[(1, D), (1, P_)], []])) is None                   # c2 missing
    assert solution_stats(inst, *pack([[(2, P_), (1, D)], [(1, P_), (2, D)]])) is None      # wait cycle


def test_invariants():
    inst = synth.make_instance(40, 5, 4, 20, "5x", seed=12)
    ops, rt = synth.random_candidates(inst, 20, seed=13)
    g = np.random.Generator(np.random.Philox(key=14))
    for b in range(20):
        st = solution_stats(inst, ops[b], rt[b])
        assert st is not None
        x, i = st
        assert 0 <= x <= inst.n and 0 <= i <= inst.n
        # vehicles relabelled: same counts
        routes = []
        s = 0
        for e in rt[b]:
            routes.append([(int(v) >> 1, int(v) & 1) for v in ops[b][s:int(e)]])
            s = int(e)
        perm = g.permutation(inst.m)
        assert solution_stats(inst, *pack([routes[v] for v in perm])) == st
    # one vehicle: nothing is cross-vehicle
    one = synth.make_instance(12, 1, 12, 12, "base", seed=15)
    o, r = synth.round_robin_solution(one)
    assert solution_stats(one, o, r) == (0, 0)       # drop-then-pickup pairs: no interleaving either
