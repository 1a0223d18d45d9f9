"""Pins for the oracle's construction heuristics (the initial solution of
Section 4.2 and the warm-start seeds of Section 4.4.4), CPU only.

* the pseudo-angle order recovered from the distance matrix equals the polar
  order of the underlying points (atan2 on the coordinates), both ways round;
* the sector cut and the balancing rule on a hand-worked example, and the
  balancing's stopping condition on random instances;
* every heuristic's output is a complete feasible solution (the exact
  evaluator), over load models, scarce resources and degenerate sizes;
* each greedy step took a least-key feasible choice (replayed per step);
* the load-balanced assignment keeps Graham's list-scheduling bound
  W_max - W_min <= max w_c;
* the refinement ends in a local optimum of both local-search moves
  (brute force, as in the local-search pins) and never worsens;
* the several-source warm start places each source's encoding and its
  perturbed variants in the slots the cycle assigns.
"""
import math

import numpy as np
import pytest

import synth
from test_oracle_local_search import brute_force


def coords_instance(pts, p=None, m=2, k=3, R=6, load_model=0):
    coords = np.array(pts, dtype=np.int64)
    d = synth._euc2d_nint(coords)
    n = len(pts) - 1
    pp = np.zeros(n + 1, np.int32)
    if p is not None:
        pp[1:] = p
    return synth.Instance(n, m, k, R, d, pp, coords=coords, load_model=load_model)


def polar_points(seed, n, mirror):
    """Depot at the origin (shifted), customer 1 the farthest (angle 0),
    customer 2 the farthest from the axis (at +-90 degrees), the rest at
    angles >= 3 degrees apart and >= 3 degrees off the axis."""
    g = np.random.Generator(np.random.Philox(key=seed))
    angs = [0.0, 90.0]
    while len(angs) < n:
        a = float(g.uniform(3.0, 357.0))
        if abs(a - 180.0) < 3.0 or min(abs(a - b) for b in angs) < 3.0 or min(abs(a - b) for b in angs) > 357:
            continue
        if abs(a - 90.0) < 20.0 or abs(a - 270.0) < 20.0:
            continue                      # keeps customer 2 the unique farthest from the axis
        angs.append(a)
    radii = [4500.0, 4400.0] + [float(g.uniform(2000.0, 4000.0)) for _ in range(n - 2)]
    sgn = -1.0 if mirror else 1.0
    pts = [(6000, 6000)]
    for a, r in zip(angs, radii):
        t = math.radians(a)
        pts.append((6000 + int(round(r * math.cos(t))), 6000 + int(round(sgn * r * math.sin(t)))))
    return pts


@pytest.mark.parametrize("mirror", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_angle_order_is_the_polar_order(orc, seed, mirror):
    pts = polar_points(seed, 40, mirror)
    inst = coords_instance(pts)
    got = orc.cons_angle_order(inst)
    xy = np.array(pts[1:], dtype=np.float64) - np.array(pts[0], dtype=np.float64)
    ang = np.arctan2(xy[:, 1], xy[:, 0]) - np.arctan2(xy[0, 1], xy[0, 0])
    if mirror:
        ang = -ang                        # angles grow towards customer 2's side
    ang = np.mod(ang, 2 * np.pi)
    want = np.argsort(ang, kind="stable") + 1
    assert list(got) == list(want)


def test_sectors_hand_example(orc):
    # depot, c1 at angle 0 (farthest), c2 at 90, c3 at 180, c4 at 270 degrees
    inst = coords_instance([(0, 0), (100, 0), (0, 10), (-10, 0), (0, -10)], m=2, k=2, R=4)
    assert list(orc.cons_angle_order(inst)) == [1, 2, 3, 4]
    s0, s1, moves = orc.cons_sectors(inst)
    # cut: {1, 2} | {3, 4}; workloads 2 d0c + p: 200 + 20 | 20 + 20; gap 180.
    # Only c2 (w = 20 < 180) qualifies and moves; then W = 200 | 60 and
    # nothing in sector 0 is lighter than the gap 140.
    assert list(s0[1:]) == [0, 0, 1, 1]
    assert list(s1[1:]) == [0, 1, 1, 1] and moves == 1
    # with p_3 = 160 the sectors start within 10%: 220 | 200, no move
    inst = coords_instance([(0, 0), (100, 0), (0, 10), (-10, 0), (0, -10)], p=[0, 0, 160, 0], m=2, k=2, R=4)
    s0, s1, moves = orc.cons_sectors(inst)
    assert list(s1[1:]) == [0, 0, 1, 1] and moves == 0
    # p_3 = 150: 220 | 190 is 13.6% apart; c2 (w = 20 < 30) moves: 200 | 210
    inst = coords_instance([(0, 0), (100, 0), (0, 10), (-10, 0), (0, -10)], p=[0, 0, 150, 0], m=2, k=2, R=4)
    s0, s1, moves = orc.cons_sectors(inst)
    assert list(s1[1:]) == [0, 1, 1, 1] and moves == 1


def test_balancing_moves_the_customer_closest_to_half_the_gap(orc):
    """Worked by hand: c1 at distance 100 (angle 0), c2..c6 at distance 10 at
    90, 135, 225, 270, 315 degrees; p = (0, 40, 110, 0, 0, 0); w = 2 d + p =
    200, 60, 130, 20, 20, 20.  Cut {1,2,3} | {4,5,6}: W = 390 | 60, gap 330.
    |gap - 2w|: c1 70, c2 210, c3 70 -> tie, lower index: c1 moves (190 | 260).
    Gap 70 from sector 1: c4, c5, c6 all at |70 - 40| = 30 -> c4 (210 | 240).
    Gap 30: c5, c6 at 10 -> c5 (230 | 220).  Gap 10, 10 x 10 < 230: stop."""
    pts = [(0, 0), (100, 0), (0, 10), (-7, 7), (-7, -7), (0, -10), (7, -7)]
    inst = coords_instance(pts, p=[0, 40, 110, 0, 0, 0], m=2, k=3, R=6)
    assert list(orc.cons_angle_order(inst)) == [1, 2, 3, 4, 5, 6]
    assert [int(inst.d[0][c]) for c in range(1, 7)] == [100, 10, 10, 10, 10, 10]
    s0, s1, moves = orc.cons_sectors(inst)
    assert list(s0[1:]) == [0, 0, 0, 1, 1, 1]
    assert list(s1[1:]) == [1, 0, 0, 0, 0, 1] and moves == 3


def workloads(inst, sector, mv):
    w = 2 * inst.d[0, 1:].astype(np.int64) + inst.p[1:]
    W = np.zeros(mv, np.int64)
    np.add.at(W, sector[1:], w)
    return w, W


INSTANCES = [
    # n, m, k, R, rule, load model
    (100, 4, 5, 20, "base", 0),
    (100, 4, 5, 20, "2x", 0),
    (60, 6, 4, 24, "1R20", 0),
    (50, 10, 8, 50, "5x", 0),
    (40, 5, 3, 15, "1R10", 1),            # FULL_START (R = m k)
    (30, 6, 3, 4, "base", 0),             # fewer resources than vehicles
    (17, 2, 5, 1, "base", 0),             # one resource
    (8, 12, 2, 24, "base", 0),            # more vehicles than customers
    (1, 3, 1, 3, "base", 0),
    (2, 1, 1, 1, "5x", 0),
]


@pytest.mark.parametrize("case", INSTANCES, ids=lambda c: f"n{c[0]}m{c[1]}R{c[3]}lm{c[5]}")
def test_balancing_stops_at_its_condition(orc, case):
    n, m, k, R, rule, lm = case
    inst = synth.make_instance(n, m, k, R, rule, seed=300 + n, load_model=lm)
    mv = orc.cons_vehicles(inst)
    assert mv == (m if lm == 1 else max(1, min(m, R)))
    order = orc.cons_angle_order(inst)
    assert sorted(order) == list(range(1, n + 1))
    s0, s1, _ = orc.cons_sectors(inst)
    sizes = [n // mv + (v < n % mv) for v in range(mv)]
    assert list(s0[order]) == [v for v in range(mv) for _ in range(sizes[v])]
    assert np.all((s1[1:] >= 0) & (s1[1:] < mv))
    w, W = workloads(inst, s1, mv)
    hi, lo = int(np.argmax(W)), int(np.argmin(W))
    gap = W[hi] - W[lo]
    movable = [c for c in range(1, n + 1) if s1[c] == hi and 0 < w[c - 1] < gap]
    assert 10 * gap < W[hi] or not movable


def cap_of(inst, mv, v):
    if inst.load_model == 1:
        return inst.k
    return min(inst.k, inst.R // mv + (v < inst.R % mv))


def check_own_routes(inst, ops, rt, seq, sector, mv):
    """Each vehicle serves its own customers alone, and each of its steps took
    the feasible op of least (completion, op index)."""
    n, d, p = inst.n, inst.d, inst.p
    by_v = {}
    for v, o in seq:
        by_v.setdefault(v, []).append(o)
    for v in range(inst.m):
        mine = [c for c in range(1, n + 1) if sector[c] == v]
        steps = by_v.get(v, [])
        assert sorted(steps) == sorted([2 * (c - 1) for c in mine] + [2 * (c - 1) + 1 for c in mine])
        cap = cap_of(inst, mv, v) if v < mv else 0
        t, loc, out, state, ready = 0, 0, 0, {c: 0 for c in mine}, {}
        for o in steps:
            opts = []
            for c in mine:
                arr = t + int(d[loc, c])
                if state[c] == 0 and out < cap:
                    opts.append((arr, 2 * (c - 1)))
                elif state[c] == 1:
                    opts.append((max(arr, ready[c]), 2 * (c - 1) + 1))
            best = min(opts)
            assert best[1] == o, (v, o, best)
            c = o // 2 + 1
            t, loc = best[0], c
            if o & 1:
                state[c], out = 2, out - 1
            else:
                state[c], out, ready[c] = 1, out + 1, t + int(p[c])
            assert out <= cap


@pytest.mark.parametrize("case", INSTANCES, ids=lambda c: f"n{c[0]}m{c[1]}R{c[3]}lm{c[5]}")
def test_constructions_are_feasible_and_greedy(orc, case):
    n, m, k, R, rule, lm = case
    inst = synth.make_instance(n, m, k, R, rule, seed=300 + n, load_model=lm)
    mv = orc.cons_vehicles(inst)
    for h in range(4):
        ops, rt, seq = orc.construct(inst, h, order=True)
        assert len(ops) == 2 * n and int(rt[-1]) == 2 * n
        z, st = orc.eval_one(inst, ops, rt)
        assert st == 0, (h, st)
        # routes are the placement order grouped by vehicle
        for v in range(m):
            s = int(rt[v - 1]) if v else 0
            mine = [((o // 2 + 1) << 1) | (o & 1) for vv, o in seq if vv == v]
            assert list(ops[s:int(rt[v])]) == mine
        if h == orc.CONS_SWEEP:
            _, sector, _ = orc.cons_sectors(inst)
            check_own_routes(inst, ops, rt, seq, sector, mv)
        elif h == orc.CONS_LB:
            sector = np.full(n + 1, -1)
            for v, o in seq:
                sector[o // 2 + 1] = v
            check_own_routes(inst, ops, rt, seq, sector, mv)
            w, W = workloads(inst, sector, mv)
            assert W.max() - W.min() <= w.max()          # Graham's bound for list scheduling
        else:
            check_dispatch(inst, h, seq)


def check_dispatch(inst, h, seq):
    """Replays NN / SPT: the load rules of the decoder, and at every step the
    chosen pair is a least-key feasible pair."""
    n, m, k, R, d, p = inst.n, inst.m, inst.k, inst.R, inst.d, inst.p
    full = inst.load_model == 1
    t, loc = [0] * m, [0] * m
    q, M = [k if full else 0] * m, [k if full else 0] * m
    Lsum, state, ready = 0, [0] * (n + 1), [0] * (n + 1)
    spt = sorted(range(1, n + 1), key=lambda c: (int(p[c]), c))
    for v_got, o_got in seq:
        nxt = next(c for c in spt if state[c] == 0) if any(state[c] == 0 for c in spt) else None
        pairs = []
        for v in range(m):
            canD = q[v] > 0 or (not full and M[v] < k and Lsum < R)
            canP = q[v] < k
            for c in range(1, n + 1):
                if state[c] == 2:
                    continue
                isP = state[c] == 1
                if (isP and not canP) or (not isP and not canD):
                    continue
                if not isP and h == orc_cons_spt() and c != nxt:
                    continue
                arr = t[v] + int(d[loc[v], c])
                comp = max(arr, ready[c]) if isP else arr
                pairs.append((v, 2 * (c - 1) + int(isP), comp, int(d[loc[v], c])))
        assert pairs
        if h == orc_cons_spt():
            best = min(pairs, key=lambda x: (x[2], x[1], x[0]))
        else:
            vs = sorted({x[0] for x in pairs}, key=lambda v: (t[v], v))
            best = min((x for x in pairs if x[0] == vs[0]), key=lambda x: (x[3], x[1]))
        assert (v_got, o_got) == (best[0], best[1])
        v, o = best[0], best[1]
        c = o // 2 + 1
        t[v], loc[v] = best[2], c
        if o & 1:
            state[c] = 2
            q[v] += 1
            M[v] = max(M[v], q[v])
        else:
            if q[v] == 0:
                M[v] += 1
                Lsum += 1
                q[v] += 1
            q[v] -= 1
            state[c], ready[c] = 1, t[v] + int(p[c])
        assert 0 <= q[v] <= k and Lsum <= R


def orc_cons_spt():
    import oracle
    return oracle.CONS_SPT


def test_spt_drops_follow_processing_order(orc):
    inst = synth.make_instance(60, 4, 3, 12, "1R20", seed=9)
    _, _, seq = orc.construct(inst, orc.CONS_SPT, order=True)
    drops = [o // 2 + 1 for _, o in seq if not o & 1]
    assert drops == sorted(range(1, 61), key=lambda c: (int(inst.p[c]), c))


@pytest.mark.parametrize("case", [(14, 3, 2, 6, "base", 0), (12, 3, 3, 6, "5x", 0), (10, 2, 2, 4, "1R10", 1)],
                         ids=lambda c: f"n{c[0]}{c[4]}")
def test_refinement_reaches_a_local_optimum(orc, case):
    n, m, k, R, rule, lm = case
    if lm == 1:
        R = m * k
    inst = synth.make_instance(n, m, k, R, rule, seed=500 + n, load_model=lm)
    ops, rt = orc.construct(inst, orc.CONS_SWEEP)
    z0, st = orc.eval_one(inst, ops, rt)
    assert st == 0
    rounds, z, ops2, rt2 = orc.refine(inst, ops, rt, budget=1 << 20)
    assert z <= z0 and orc.eval_one(inst, ops2, rt2) == (z, 0)
    assert rounds >= 1
    for kind in (0, 1):
        best, _ = brute_force(inst, kind, ops2, rt2)
        assert best == z, (kind, best, z)


def test_warm_start_from_several_sources(orc):
    inst = synth.make_instance(20, 3, 4, 12, "2x", seed=4)
    srcs = [orc.construct(inst, h) for h in (orc.CONS_SWEEP, orc.CONS_NN, orc.CONS_LB, orc.CONS_SPT)]
    n_var = [3, 1, 2, 1]                  # 7 variants: slots cycle through them
    po, ho = orc.brkga_warm_start_multi(inst, srcs, n_var, 30, 16, seed=5)
    first = [0, 3, 4, 6]                  # slot of each source's variant 0
    for s, (o, r) in enumerate(srcs):
        ep, eh = orc.brkga_warm_start(inst, o, r, 1, 1, 1, seed=5)
        assert np.array_equal(po[first[s]], ep[0]) and np.array_equal(ho[first[s]], eh[0])
        assert np.array_equal(po[first[s] + 7], ep[0])          # the cycle repeats
    for slot, src0 in ((1, 0), (2, 0), (5, 4)):
        assert np.all(np.abs(po[slot] - po[src0]) <= 0.03 + 1e-6)
        assert not np.array_equal(po[slot], po[src0])
    assert not np.array_equal(po[1], po[2])
    # one source: the single-source warm start
    a = orc.brkga_warm_start_multi(inst, srcs[:1], [5], 12, 9, seed=8)
    b = orc.brkga_warm_start(inst, srcs[0][0], srcs[0][1], 12, 9, 5, seed=8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.all((po >= 0) & (po < 1) & (ho >= 0) & (ho < 1))
