"""Pins for the oracle evaluator (CPU only).

Every expected value here comes from the paper's definitions worked by hand,
from a closed form, from brute force over all timings or all solutions, or
from an independent second evaluator — never from the oracle itself.
"""
import numpy as np
import pytest

import synth
from oracle import brute

BAD_COVER, LOAD, RES, DEADLOCK = 1, 2, 4, 8
INT32_MAX = 2**31 - 1


def line_instance(xs, p, m, k, R, load_model=0):
    """Customers on a line at integer positions xs (xs[0] = depot): d = |xi - xj|
    is a metric with integer values."""
    xs = np.asarray(xs)
    d = np.abs(xs[:, None] - xs[None, :]).astype(np.int32)
    return synth.instance_from_matrix(d, p, m, k, R, load_model)


def packed(routes, m):
    ops, off, rt = synth.pack_candidates([routes], m)
    return ops, rt[0]


# ---------------------------------------------------------------- hand vectors
def test_closed_form_single_customer(orc):
    # one vehicle: drive out, drop, wait p, pick up, drive back (Eq. 7-12, 21)
    for d01, d10, p1 in [(5, 5, 7), (3, 9, 0), (1, 1, 100)]:
        d = np.array([[0, d01], [d10, 0]], dtype=np.int32)
        inst = synth.instance_from_matrix(d, [0, p1], 1, 1, 1)
        ops, rt = packed([[(1, "D"), (1, "P")]], 1)
        assert orc.eval_one(inst, ops, rt) == (d01 + p1 + d10, 0)


def test_h1_cross_route_wait(orc):
    # depot at 0, customer 1 at 3, customer 2 at 10; p1 = 4, p2 = 2.
    # v0 = [D1, P2], v1 = [P1, D2]:  D1 at 3 (ready 7); v1 reaches 1 at 3, waits
    # to 7, reaches 2 at 14 (ready 16); v0 reaches 2 at 10, waits to 16, back 26.
    inst = line_instance([0, 3, 10], [0, 4, 2], m=2, k=1, R=1)
    ops, rt = packed([[(1, "D"), (2, "P")], [(1, "P"), (2, "D")]], 2)
    mk, st, t = orc.eval_one(inst, ops, rt, times=True)
    assert (mk, st) == (26, 0)
    assert list(t) == [3, 16, 7, 14]
    # the paper's capacity model (every vehicle leaves full, q_0 = k): v1 picks
    # up while full, and 2 vehicles x k=1 exceed R=1
    inst_f = line_instance([0, 3, 10], [0, 4, 2], m=2, k=1, R=1, load_model=1)
    assert orc.eval_one(inst_f, ops, rt) == (26, LOAD | RES)


def test_h2_pickup_by_other_vehicle_waits(orc):
    inst = line_instance([0, 3, 10], [0, 20, 1], m=2, k=2, R=2)
    ops, rt = packed([[(1, "D"), (2, "D"), (2, "P")], [(1, "P")]], 2)
    mk, st, t = orc.eval_one(inst, ops, rt, times=True)
    assert (mk, st) == (26, 0)
    assert list(t) == [3, 10, 11, 23]


def test_h3_deadlocks(orc):
    inst = line_instance([0, 3, 10], [0, 4, 2], m=2, k=2, R=4)
    ops, rt = packed([[(1, "P"), (2, "D")], [(2, "P"), (1, "D")]], 2)
    assert orc.eval_one(inst, ops, rt) == (INT32_MAX, DEADLOCK)
    ops, rt = packed([[(1, "P"), (1, "D")], [(2, "D"), (2, "P")]], 2)
    assert orc.eval_one(inst, ops, rt) == (INT32_MAX, DEADLOCK)
    # zero processing does not break a cycle: still a wait on itself
    inst0 = line_instance([0, 3, 10], [0, 0, 0], m=2, k=2, R=4)
    assert orc.eval_one(inst0, ops, rt) == (INT32_MAX, DEADLOCK)


def test_cover_rules(orc):
    inst = line_instance([0, 3, 10], [0, 4, 2], m=2, k=2, R=4)
    bad = [
        [[(1, "D"), (1, "P")], [(2, "D")]],                 # P2 missing
        [[(1, "D"), (1, "P"), (1, "P")], [(2, "D"), (2, "P")]],  # P1 twice
        [[(1, "D"), (1, "P")], [(3, "D"), (3, "P")]],       # customer 3 does not exist
        [[(1, "D"), (1, "P")], []],                         # customer 2 absent
    ]
    for routes in bad:
        ops, rt = packed(routes, 2)
        assert orc.eval_one(inst, ops, rt) == (INT32_MAX, BAD_COVER), routes
    # a destroyed solution (customer 2 absent) is fine when partial is allowed
    ops, rt = packed([[(1, "D"), (1, "P")], []], 2)
    assert orc.eval_one(inst, ops, rt, allow_partial=True) == (3 + 4 + 3, 0)
    # route ends must be non-decreasing and within 2n
    ops, _ = packed([[(1, "D"), (1, "P")], [(2, "D"), (2, "P")]], 2)
    assert orc.eval_one(inst, ops, np.array([3, 2], np.uint16))[1] == BAD_COVER


def test_empty_routes_contribute_zero(orc):
    inst = line_instance([0, 3, 10], [0, 4, 2], m=4, k=2, R=4)
    ops, rt = packed([[], [(1, "D"), (2, "D"), (1, "P"), (2, "P")], [], []], 4)
    # D1@3 (r 7), D2@10 (r 12), P1: arrive 17 -> 17, P2: arrive 24 -> 24, back 34
    assert orc.eval_one(inst, ops, rt) == (34, 0)


def test_load_models(orc):
    inst = line_instance([0, 1, 2, 3], [0, 1, 1, 1], m=1, k=2, R=2)
    routes = [[(1, "D"), (2, "D"), (3, "D"), (1, "P"), (2, "P"), (3, "P")]]
    ops, rt = packed(routes, 1)
    # needs 3 resources on board at the start: over k = 2
    assert orc.eval_one(inst, ops, rt)[1] == LOAD | RES
    inst3 = line_instance([0, 1, 2, 3], [0, 1, 1, 1], m=1, k=3, R=3)
    assert orc.eval_one(inst3, ops, rt)[1] == 0
    inst3r = line_instance([0, 1, 2, 3], [0, 1, 1, 1], m=1, k=3, R=2)
    assert orc.eval_one(inst3r, ops, rt)[1] == RES
    # FULL_START: pickups before any drop overflow a full vehicle
    inst_f = line_instance([0, 1, 2], [0, 1, 1], m=2, k=1, R=2, load_model=1)
    ops, rt = packed([[(1, "D"), (2, "P")], [(2, "D"), (1, "P")]], 2)
    assert orc.eval_one(inst_f, ops, rt)[1] == 0
    ops, rt = packed([[(1, "D"), (2, "D"), (1, "P"), (2, "P")], []], 2)
    assert orc.eval_one(inst_f, ops, rt)[1] == LOAD


# ------------------------------------------------------- brute force over timings
@pytest.mark.parametrize("case", range(12))
def test_sweep_is_minimum_over_all_timings(orc, case):
    """For fixed routes, the oracle's makespan equals the minimum over every
    integer timing that satisfies the MILP's timing constraints (Eq. 7-12, 21-22)."""
    g = synth.rng(100 + case)
    xs = [0] + list(g.integers(1, 5, size=2))
    while len(set(xs)) < 3:
        xs = [0] + list(g.integers(1, 5, size=2))
    # p >= 1: every wait cycle then has positive length and no timing can
    # satisfy it, so "no feasible timing" and DEADLOCK must coincide
    p = [0] + list(g.integers(1, 4, size=2))
    inst = line_instance(xs, p, m=2, k=2, R=4)
    ops_all, rt_all = brute.enumerate_batch(2, 2)
    pick = g.choice(len(ops_all), size=6, replace=False)
    for i in pick:
        routes = synth.unpack_candidate(ops_all[i], rt_all[i])
        mk, st = orc.eval_one(inst, ops_all[i], rt_all[i])
        ref = brute.min_makespan_by_times(inst.d, inst.p, routes, horizon=16)
        if ref is None:
            assert st & DEADLOCK
        else:
            assert not (st & DEADLOCK) and mk == ref, (routes, mk, ref)


# -------------------------------------------------------- second evaluator
def _adversarial(inst, g, count):
    n, m = inst.n, inst.m
    out = []
    for _ in range(count):
        codes = [(c << 1) | b for c in range(1, n + 1) for b in (0, 1)]
        g.shuffle(codes)
        cuts = np.sort(g.integers(0, 2 * n + 1, size=m - 1))
        out.append((np.array(codes, np.uint16), np.array(list(cuts) + [2 * n], np.uint16)))
    return out


@pytest.mark.parametrize("n,m,seed", [(6, 2, 1), (16, 2, 2), (30, 4, 3), (100, 4, 4), (60, 10, 5)])
def test_sweep_agrees_with_graph_longest_path(orc, n, m, seed):
    inst = synth.make_instance(n, m, 5, 5 * m, "1R10", seed=seed)
    g = synth.rng(seed)
    cands = _adversarial(inst, g, 300)               # mostly deadlocked, random order
    ops, rt = synth.random_candidates(inst, 200, seed)  # never deadlocked
    cands += [(ops[b], rt[b]) for b in range(len(ops))]
    n_dead = 0
    for o, r in cands:
        mk, st, t = orc.eval_one(inst, o, r, times=True)
        mk2, st2, t2 = orc.eval_one(inst, o, r, dag=True, times=True)
        assert (st & DEADLOCK) == st2
        if not st2:
            assert mk == mk2
            assert np.array_equal(t, t2)
        n_dead += bool(st2)
    assert 0 < n_dead < len(cands)


# ------------------------------------------------------------- invariants
@pytest.mark.parametrize("rule", ["base", "5x", "1R20"])
def test_schedule_invariants(orc, rule):
    """Each op starts as early as its constraints allow (tightness), pickups
    wait for drop + p (Eq. 9), and z >= T_drop + p + shortest path home."""
    inst = synth.make_instance(40, 4, 5, 20, rule, seed=7)
    n, d, p = inst.n, inst.d.astype(np.int64), inst.p.astype(np.int64)
    # shortest-path closure to the depot (EUC_2D rounding breaks the triangle inequality)
    sp = d.copy()
    for k in range(n + 1):
        sp = np.minimum(sp, sp[:, k:k + 1] + sp[k:k + 1, :])
    ops, rt = synth.random_candidates(inst, 50, 9)
    for b in range(len(ops)):
        mk, st, t = orc.eval_one(inst, ops[b], rt[b], times=True)
        assert not (st & (DEADLOCK | BAD_COVER))
        drop = {}
        for j, x in enumerate(ops[b]):
            if not x & 1:
                drop[x >> 1] = t[j]
        s = 0
        for v in range(inst.m):
            prev_loc, prev_t = 0, 0
            for j in range(s, int(rt[b][v])):
                c, isP = int(ops[b][j]) >> 1, int(ops[b][j]) & 1
                arr = prev_t + d[prev_loc, c]
                expect = max(arr, drop[c] + p[c]) if isP else arr
                assert t[j] == expect
                prev_loc, prev_t = c, t[j]
            s = int(rt[b][v])
        for c in range(1, n + 1):
            assert mk >= drop[c] + p[c] + sp[c, 0]


# --------------------------------------------------- brute force over solutions
def test_special_case_reduces_to_minmax_vrp(orc):
    """Section 3.2: with p = 0, k >= n and metric travel times the optimum equals
    the min-max VRP optimum.  Both sides found by exhaustive enumeration."""
    for seed in range(3):
        g = synth.rng(500 + seed)
        n, m = 3, 2
        pts = g.integers(0, 6, size=(n + 1, 2))
        d = np.abs(pts[:, None, :] - pts[None, :, :]).sum(-1).astype(np.int32)  # Manhattan
        inst = synth.instance_from_matrix(d, np.zeros(n + 1, np.int32), m, n, n * m)
        ops, rt = brute.enumerate_batch(n, m)
        mk, st = orc.eval_batch(inst, ops, rt)
        best = int(mk[st == 0].min())
        assert best == brute.minmax_vrp_optimum(d, m)


def test_brute_force_optimum_counts(orc):
    """Exhaustive n=3, m=2: every solution is classified, at least one is
    feasible, and the optimum is no worse than serving each customer alone."""
    inst = synth.make_instance(3, 2, 2, 4, "base", seed=11)
    ops, rt = brute.enumerate_batch(3, 2)
    assert len(ops) == 720 * 7
    mk, st = orc.eval_batch(inst, ops, rt)
    assert np.all((st == 0) | (st & (DEADLOCK | LOAD | RES)).astype(bool))
    feas = mk[st == 0]
    assert feas.size > 0
    d, p = inst.d, inst.p
    lone = max(d[0, c] + p[c] + d[c, 0] for c in range(1, 4))
    assert feas.min() >= lone
    assert np.all(mk[(st & DEADLOCK) > 0] == INT32_MAX)


def test_euc2d_rounding():
    # exact integer nearest-integer rounding of sqrt(dx^2 + dy^2)
    inst = synth.make_instance(200, 2, 2, 4, seed=3)
    xy = inst.coords.astype(np.float64)
    ref = np.floor(np.sqrt(((xy[:, None] - xy[None]) ** 2).sum(-1)) + 0.5).astype(np.int32)
    assert np.array_equal(inst.d, ref)
    assert np.all(inst.d[~np.eye(201, dtype=bool)] >= 1)
