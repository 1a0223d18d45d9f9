"""Pins for the oracle's ALNS operators (CPU only).

Each destroy operator (Section 4.2.2), the insertion enumeration and each
repair rule (Section 4.2.3), and the acceptance, scoring, cooling, reheat and
weight update of Algorithm 1 (Sections 4.2.1 and 4.2.4, Table 2) are checked
on hand-worked examples and against brute force on tiny instances.  Random
words are Philox4x32-10 outputs (pinned by the Random123 known-answer
vectors in the decoder tests): word a of iteration it, chain ch is word a % 4
of the block {a / 4, it, ch, 'ALNS'}; the destroy operators draw from a = 16.
"""
import math

import numpy as np
import pytest

import synth
from alns_brute import decode, encode, insert, insertions, priced, rule_choice, without

TAG = 0x414C4E53


def word(orc, seed, a, it, ch):
    out = orc.philox([a >> 2, it, ch, TAG], [seed & 0xFFFFFFFF, seed >> 32])
    return int(out[a & 3])


def below(w, n):
    """U_int[0, n) from a 32-bit word: floor(w n / 2^32)."""
    return (w * n) >> 32


D = lambda c: (c, 0)
P = lambda c: (c, 1)

# A line instance: the depot at x = 0 and customers 1..6 at x = 2, 5, 9, -3,
# -8, 14 (travel time = distance); p = 4, 1, 6, 2, 3, 5; m = 2, k = 3, R = 6.
X = np.array([0, 2, 5, 9, -3, -8, 14])
LINE_D = np.abs(X[:, None] - X[None, :]).astype(np.int32)
LINE_P = np.array([0, 4, 1, 6, 2, 3, 5], np.int32)
# v0 = D1 D2 P1 D3 P2 P3 P6, v1 = D4 D5 P4 D6 P5.  Worked by hand (Eq. 7-12):
# v0: D1 at 2, D2 at 5, P1 at 8 (ready 6), D3 at 15, P2 at 19, P3 at 23
#     (ready 21), P6 arrives 28 and waits for D6 + p6 = 35, returns 49;
# v1: D4 at 3, D5 at 8, P4 at 13 (ready 5), D6 at 30, P5 at 52, returns 60.
LINE_ROUTES = [[D(1), D(2), P(1), D(3), P(2), P(3), P(6)], [D(4), D(5), P(4), D(6), P(5)]]
LINE_TIMES = [2, 5, 8, 15, 19, 23, 35, 3, 8, 13, 30, 52]
LINE_Z = 60
# Removal gains z(S) - z(S without c), by hand: without c5 v1 is D4 3, P4 5,
# D6 22, back at 36, and v0's P6 leaves at 28 and is back at 42: gain 18;
# without c6 v1 is back at 26 and v0 at 32: gain 28; removing c1..c4 leaves
# v1's return at 60: gain 0.
LINE_GAINS = {1: 0, 2: 0, 3: 0, 4: 0, 5: 18, 6: 28}


@pytest.fixture(scope="module")
def line():
    inst = synth.instance_from_matrix(LINE_D, LINE_P, 2, 3, 6)
    ops, rt = encode(LINE_ROUTES)
    return inst, ops, rt


def test_line_instance_schedule(orc, line):
    inst, ops, rt = line
    z, st, t = orc.eval_one(inst, ops, rt, times=True)
    assert (z, st) == (LINE_Z, 0)
    assert list(t) == LINE_TIMES
    for c, g in LINE_GAINS.items():
        o, r = encode(without(LINE_ROUTES, [c]))
        assert LINE_Z - orc.eval_one(inst, o, r, allow_partial=True)[0] == g


def _find_it(orc, seed, pred, a=16, ch=0):
    """First iteration whose word a satisfies pred."""
    for it in range(10000):
        if pred(word(orc, seed, a, it, ch)):
            return it
    raise AssertionError("no such draw")


def test_random_removal_fisher_yates(orc, line):
    """Random removal: a Fisher-Yates shuffle of 1..n stopped after q swaps,
    swap partner i + U_int[0, n - i) from word 16 + i."""
    inst, ops, rt = line
    seed = 77
    for it in range(6):
        a = list(range(1, 7))
        for i in range(4):
            j = i + below(word(orc, seed, 16 + i, it, 3), 6 - i)
            a[i], a[j] = a[j], a[i]
        assert orc.alns_destroy(inst, 0, ops, rt, 4, 4, seed, it, 3) == a[:4]


def test_random_removal_uniform(orc):
    """Every customer equally likely: each of n = 12 appears in a 3-removal
    with probability 1/4 (binomial, 1,200 draws; bounds at 5 sigma)."""
    inst = synth.make_instance(12, 3, 4, 12, "base", seed=41)
    ops, rt = synth.round_robin_solution(inst)
    cnt = np.zeros(13)
    for it in range(1200):
        rem = orc.alns_destroy(inst, 0, ops, rt, 3, 3, 5, it, 0)
        assert len(set(rem)) == 3
        cnt[rem] += 1
    sd = math.sqrt(1200 * 0.25 * 0.75)
    assert np.all(np.abs(cnt[1:] - 300) < 5 * sd)


def test_worst_removal_hand(orc, line):
    """Worst removal: ranks by gain, largest first, ties by customer
    (c6 28, c5 18, then c1..c4 at 0); rank r drawn with weight
    floor(2^60 / r^6) without replacement."""
    inst, ops, rt = line
    ranked = [6, 5, 1, 2, 3, 4]
    wts = [(1 << 60) // (r ** 6) for r in range(1, 7)]
    seed = 123
    for it in range(40):
        w = list(wts)
        exp = []
        for s in range(3):
            target = (word(orc, seed, 16 + s, it, 1) * sum(w)) >> 32
            acc = 0
            for i in range(6):
                acc += w[i]
                if w[i] and target < acc:
                    break
            exp.append(ranked[i])
            w[i] = 0
        assert orc.alns_destroy(inst, 1, ops, rt, 3, 3, seed, it, 1) == exp


def test_worst_removal_favours_largest_gain(orc):
    """The first pick is the largest-gain customer with probability
    1 / sum_r r^-6 (0.9830 for n = 30); over 600 draws at least 95%."""
    inst = synth.make_instance(30, 3, 5, 15, "2x", seed=8)
    ops, rt = synth.round_robin_solution(inst)
    z = orc.eval_one(inst, ops, rt)[0]
    routes = decode(ops, rt)
    gain = {}
    for c in range(1, 31):
        o, r = encode(without(routes, [c]))
        gain[c] = z - orc.eval_one(inst, o, r, allow_partial=True)[0]
    top = min(gain, key=lambda c: (-gain[c], c))
    firsts = [orc.alns_destroy(inst, 1, ops, rt, 4, 4, 9, it, 0)[0] for it in range(600)]
    assert sum(f == top for f in firsts) >= 570


def test_shaw_removal_hand(orc, line):
    """Shaw removal from seed c2 (x = 5, drop at 5, both ops on v0), with
    R = 9 d + 3 |dT_drop| + 2.5 [drop vehicles differ] + 2.5 [pickup
    vehicles differ]:
      c1: 9*3 + 3*3            = 36
      c3: 9*4 + 3*10           = 66
      c4: 9*8 + 3*2 + 2.5 + 2.5 = 83
      c5: 9*13 + 3*3 + 5        = 131
      c6: 9*9 + 3*25 + 2.5      = 158.5 (drop on v1, pickup on v0)
    so q = 5 removes c2, c1, c3, c4, c5."""
    inst, ops, rt = line
    seed = 31
    it = _find_it(orc, seed, lambda w: 1 + below(w, 6) == 2)
    assert orc.alns_destroy(inst, 2, ops, rt, 5, 4, seed, it, 0) == [2, 1, 3, 4, 5]
    assert orc.alns_destroy(inst, 2, ops, rt, 3, 3, seed, it, 0) == [2, 1, 3]
    # from seed c6 (drop at 30 on v1, pickup on v0):
    #   c1 9*12+3*28+2.5 = 194.5, c2 9*9+3*25+2.5 = 158.5, c3 9*5+3*15+2.5 = 92.5,
    #   c4 9*17+3*27+2.5 = 236.5, c5 9*22+3*22+2.5 = 266.5
    it = _find_it(orc, seed, lambda w: 1 + below(w, 6) == 6)
    assert orc.alns_destroy(inst, 2, ops, rt, 6, 4, seed, it, 0) == [6, 3, 2, 1, 4, 5]


def test_cluster_removal_hand(orc, line):
    """Cluster removal from centre c2: the q - 1 customers nearest by travel
    time (c1 3, c3 4, c4 8, c6 9, c5 13)."""
    inst, ops, rt = line
    seed = 5
    it = _find_it(orc, seed, lambda w: 1 + below(w, 6) == 2)
    assert orc.alns_destroy(inst, 3, ops, rt, 5, 4, seed, it, 0) == [2, 1, 3, 4, 6]
    # centre c5 (x = -8): c4 5, c1 10, c2 13, c3 17, c6 22
    it = _find_it(orc, seed, lambda w: 1 + below(w, 6) == 5)
    assert orc.alns_destroy(inst, 3, ops, rt, 4, 4, seed, it, 0) == [5, 4, 1, 2]


def test_cluster_removal_nearest(orc):
    """On random instances the removed customers other than the centre are
    never farther from it than any customer kept."""
    for s in range(4):
        inst = synth.make_instance(40, 4, 5, 20, "base", seed=300 + s)
        ops, rt = synth.round_robin_solution(inst)
        for it in range(10):
            rem = orc.alns_destroy(inst, 3, ops, rt, 6, 4, 11, it, s)
            cen, rest = rem[0], rem[1:]
            kept = [c for c in range(1, 41) if c not in rem]
            assert max(inst.d[cen, c] for c in rest) <= min(inst.d[cen, c] for c in kept)


def test_route_removal_hand(orc, line):
    """Route removal: a random non-empty route's customers in order of first
    appearance; below q_min, topped up with the customers nearest to those
    taken (ties by index)."""
    inst, ops, rt = line
    seed = 3
    it = _find_it(orc, seed, lambda w: below(w, 2) == 0)
    assert orc.alns_destroy(inst, 4, ops, rt, 4, 4, seed, it, 0) == [1, 2, 3, 6]
    assert orc.alns_destroy(inst, 4, ops, rt, 5, 4, seed, it, 0) == [1, 2, 3, 6]
    # v1 holds c4, c5, c6; the nearest other customer to them: c1 (5 from c4)
    # and c3 (5 from c6) tie, c1 has the lower index.
    it = _find_it(orc, seed, lambda w: below(w, 2) == 1)
    assert orc.alns_destroy(inst, 4, ops, rt, 4, 4, seed, it, 0) == [4, 5, 6, 1]
    assert orc.alns_destroy(inst, 4, ops, rt, 4, 5, seed, it, 0) == [4, 5, 6, 1, 3]


def test_critical_path_removal_hand(orc, line):
    """Critical path removal: the vehicle with the latest return (v1, back
    at 60 against v0's 49), its customers by descending gain (c6 28, c5 18,
    c4 0); below q_min, the others by descending gain (ties by index)."""
    inst, ops, rt = line
    assert orc.alns_destroy(inst, 5, ops, rt, 4, 4, 1, 0, 0) == [6, 5, 4, 1]
    assert orc.alns_destroy(inst, 5, ops, rt, 2, 2, 1, 0, 0) == [6, 5]
    assert orc.alns_destroy(inst, 5, ops, rt, 4, 3, 1, 0, 0) == [6, 5, 4]


# ----------------------------------------------------------------- enumeration

def test_enumeration_detour_hand(orc):
    """Depot at 0, c1 at 10, c2 at 5 on a line; v0 = D1 P1, v1 empty;
    inserting c2.  Drop slots by detour d[a][c] + d[c][b] - d[a][b]:
    (v0, 0) 5+5-10 = 0, (v0, 2) 0, (v0, 1) 5+5-0 = 10, (v1, 0) 10.  With
    K_D = K_P = 2: after a drop at (v0, 0) the pickup slots rank (v0, 1)
    0+5-5 = 0, (v0, 3) 0, (v0, 2) 10, (v1, 0) 10; after (v0, 2): (v0, 3) 0,
    (v1, 0) 10."""
    x = np.array([0, 10, 5])
    d = np.abs(x[:, None] - x[None, :]).astype(np.int32)
    inst = synth.instance_from_matrix(d, np.array([0, 3, 2], np.int32), 2, 2, 4)
    ops, rt = encode([[D(1), P(1)], []])
    t = orc.alns_enumerate(inst, ops, rt, 2, KD=2, KP=2)
    got = [(int(a["vD"]), int(a["pD"]), int(a["vP"]), int(a["pP"])) for a in t]
    assert got == [(0, 0, 0, 1), (0, 0, 0, 3), (0, 2, 0, 3), (0, 2, 1, 0)]
    assert all(int(a["c"]) == 2 for a in t)


def test_enumeration_complete_when_unbounded(orc):
    """K_D = K_P = 0 lists every valid (vD, pD, vP, pP) exactly once."""
    for s in range(5):
        inst = synth.make_instance(9, 3, 3, 9, "base", seed=50 + s)
        ops, rt = synth.random_candidates(inst, 1, seed=s)
        routes = without(decode(ops[0], rt[0]), [4, 7])
        o, r = encode(routes)
        t = orc.alns_enumerate(inst, o, r, 4)
        got = [(int(a["vD"]), int(a["pD"]), int(a["vP"]), int(a["pP"])) for a in t]
        assert len(got) == len(set(got))
        assert set(got) == set(insertions(routes, 4))


def _det(d, route, p, c, after=None):
    a = route[p - 1][0] if p > 0 else 0
    b = route[p][0] if p < len(route) else 0
    return int(d[a, c]) + int(d[c, b]) - int(d[a, b])


def test_enumeration_keeps_least_detours(orc):
    """Under a budget, the drop slots kept have no larger detour than any
    slot left out, and for each kept drop the same holds for its pickups."""
    for s in range(4):
        inst = synth.make_instance(12, 3, 4, 12, "2x", seed=70 + s)
        ops, rt = synth.random_candidates(inst, 1, seed=s)
        routes = without(decode(ops[0], rt[0]), [3, 9])
        o, r = encode(routes)
        t = orc.alns_enumerate(inst, o, r, 3, KD=3, KP=2)
        drops = sorted({(int(a["vD"]), int(a["pD"])) for a in t})
        assert len(drops) == 3
        all_d = [(v, p) for v in range(3) for p in range(len(routes[v]) + 1)]
        det = {vp: _det(inst.d, routes[vp[0]], vp[1], 3) for vp in all_d}
        assert max(det[x] for x in drops) <= min(det[x] for x in all_d if x not in drops)
        for vD, pD in drops:
            after = [list(x) for x in routes]
            after[vD].insert(pD, D(3))
            picks = [(int(a["vP"]), int(a["pP"])) for a in t if (a["vD"], a["pD"]) == (vD, pD)]
            allp = [(v, p) for v in range(3) for p in range((pD + 1 if v == vD else 0), len(after[v]) + 1)]
            pdet = {vp: _det(inst.d, after[vp[0]], vp[1], 3) for vp in allp}
            assert len(picks) == 2
            assert max(pdet[x] for x in picks) <= min(pdet[x] for x in allp if x not in picks)


# ----------------------------------------------------------------- repair

def _replay(orc, inst, routes0, rem, rule):
    """Runs one oracle repair with every slot pair and checks each step
    against brute force: the customer inserted is the rule's choice over all
    waiting customers, and the partial solution after it has the least
    makespan over all of that customer's insertions."""
    o, r = encode(routes0)
    ok, z, fo, fr, order = orc.alns_repair(inst, rule, o, r, rem)
    assert ok
    final = decode(fo, fr)
    assert sorted(order) == sorted(rem)
    waiting = list(rem)
    for j, c in enumerate(order):
        state = without(final, order[j:])
        nxt = without(final, order[j + 1:])
        choice = rule_choice(orc, inst, state, waiting, rule)
        assert choice is not None and choice[0] == c, (rule, j, choice, c)
        on, rn = encode(nxt)
        mk, st = orc.eval_one(inst, on, rn, allow_partial=True)
        assert st == 0 and mk == choice[1]
        waiting.remove(c)
    assert z == orc.eval_one(inst, fo, fr)[0]
    return order


@pytest.mark.parametrize("rule", [0, 1, 2, 3])
def test_repair_rules_brute_force(orc, rule):
    """Seeds whose first step has customers of different best makespans (on
    most random starts one untouched route fixes the makespan and every
    customer ties, which would not tell the rules apart)."""
    for s in (7, 9, 11):
        inst = synth.make_instance(7, 3, 2, 6, ["5x", "1R20", "base"][s % 3], seed=200 + s)
        ops, rt = synth.random_candidates(inst, 1, seed=s)
        g = synth.rng(s)
        rem = [int(x) for x in g.choice(np.arange(1, 8), 3, replace=False)]
        base = without(decode(ops[0], rt[0]), rem)
        c1 = [min(mk for mk, _ in priced(orc, inst, base, c)) for c in rem]
        assert len(set(c1)) > 1
        _replay(orc, inst, base, rem, rule)


def _diff_case(seed, rules):
    n, m = 8, 5
    inst = synth.make_instance(n, m, 3, 10, ["5x", "1R20", "2x", "base"][seed % 4], seed=900 + seed)
    ops, rt = synth.random_candidates(inst, 1, seed=seed)
    g = synth.rng(seed)
    rem = [int(x) for x in g.choice(np.arange(1, n + 1), 5, replace=False)]
    return inst, without(decode(ops[0], rt[0]), rem), rem


def test_repair_rules_choose_differently(orc):
    """Two instances on which the rules' first insertions differ: greedy
    against regret-2 (and the regrets) on the first; regret-2, regret-3 and
    regret-m on the second.  Each whole repair is replayed by brute force."""
    inst, routes, rem = _diff_case(23, None)
    firsts = [_replay(orc, inst, routes, rem, r)[0] for r in range(4)]
    assert firsts[0] != firsts[1] and firsts[1] == firsts[2] == firsts[3]
    inst, routes, rem = _diff_case(159, None)
    firsts = [_replay(orc, inst, routes, rem, r)[0] for r in range(4)]
    assert len({firsts[1], firsts[2], firsts[3]}) == 3


def test_repair_fails_without_feasible_insertion(orc):
    """One vehicle, k = 1: with R = 1 the route D1 P1 takes c2 as the pair
    D2 P2 (its preload stays 1); with R = 0 every drop needs a resource the
    fleet does not have, so no insertion is feasible and the repair fails."""
    x = np.array([0, 3, 6])
    d = np.abs(x[:, None] - x[None, :]).astype(np.int32)
    inst = synth.instance_from_matrix(d, np.array([0, 1, 1], np.int32), 1, 1, 1)
    ops, rt = encode([[D(1), P(1)]])
    ok, z, fo, fr, _ = orc.alns_repair(inst, 0, ops, rt, [2])
    assert ok and orc.eval_one(inst, fo, fr) == (z, 0)
    inst0 = synth.instance_from_matrix(d, np.array([0, 1, 1], np.int32), 1, 1, 0)
    ok0, _, _, _, _ = orc.alns_repair(inst0, 0, *encode([[]]), [2])
    assert not ok0


# ----------------------------------------------------------------- Algorithm 1 bookkeeping

def test_acceptance_scores_weights_trace(orc):
    """Three iterations by hand, tau = 3 (Table 2 otherwise):
      start z = z* = 100, T = 0.3 * 100 = 30;
      it 0: destroy 2, repair 1, z' = 90 < z* -> new best, both score
            sigma1 = 33 (sigma2 = 9 plus sigma1 - sigma2 = 24);
      it 1: destroy 2, repair 0, z' = 95 > z = 90, T = 30 * 0.9998 = 29.994:
            exp(-5 / 29.994) = 0.8465 > u = 0.5 -> accepted worse, sigma3 = 13;
      it 2: destroy 0, repair 0, z' = 94 < z = 95 but > z* -> improving, 9;
      then the weight update (iteration 3 is a multiple of tau):
            w = max(0.1, 0.9 w + 0.1 s / a):
            destroy 2: s = 33 + 13 = 46, a = 2 -> 0.9 + 2.3 = 3.2
            destroy 0: s = 9, a = 1 -> 0.9 + 0.9 = 1.8
            repair 1: s = 33, a = 1 -> 0.9 + 3.3 = 4.2
            repair 0: s = 13 + 9 = 22, a = 2 -> 0.9 + 1.1 = 2.0
            operators without attempts keep w = 1."""
    prm = orc.alns_params(tau=3)
    c = orc.alns_chain(100)
    assert c.T == pytest.approx(30.0, rel=1e-15)
    assert orc.alns_update(prm, c, 2, 1, True, 90, 0.99, 0) == 2
    assert (c.z, c.zb, c.sD[2], c.sR[1], c.stag) == (90, 90, 33, 33, 1)
    assert orc.alns_update(prm, c, 2, 0, True, 95, 0.5, 1) == 3
    assert (c.z, c.zb, c.sD[2], c.sR[0], c.stag) == (95, 90, 46, 13, 2)
    assert orc.alns_update(prm, c, 0, 0, True, 94, 0.99, 2) == 1
    assert (c.z, c.zb, c.stag) == (94, 90, 3)
    assert list(c.wD) == pytest.approx([1.8, 1.0, 3.2, 1.0, 1.0, 1.0], rel=1e-14)
    assert list(c.wR) == pytest.approx([2.0, 4.2, 1.0, 1.0], rel=1e-14)
    assert list(c.sD) == [0] * 6 and list(c.aD) == [0] * 6 and list(c.aR) == [0] * 4
    assert c.T == pytest.approx(30.0 * 0.9998 ** 3, rel=1e-14)


def test_annealing_threshold(orc):
    """A worse candidate is accepted iff u < exp(-(z' - z) / T): with z = 100
    and T = 30, z' = 130 gives exp(-1) = 0.3679; u = 0.36 accepts, u = 0.37
    rejects; z' = z is always accepted (exp(0) = 1) and scores sigma3; a
    failed repair is never accepted."""
    prm = orc.alns_params()
    for u, exp in ((0.36, 3), (0.37, 0)):
        c = orc.alns_chain(100)
        assert orc.alns_update(prm, c, 0, 0, True, 130, u, 0) == exp
        assert c.z == (130 if exp else 100)
        assert c.sD[0] == (13 if exp else 0)
    c = orc.alns_chain(100)
    assert orc.alns_update(prm, c, 1, 2, True, 100, 0.999999, 0) == 3
    assert (c.sD[1], c.sR[2]) == (13, 13)
    c = orc.alns_chain(100)
    assert orc.alns_update(prm, c, 1, 2, False, 50, 0.0, 0) == 0
    assert (c.z, c.zb, c.sD[1], c.aD[1], c.aR[2]) == (100, 100, 0, 1, 1)


def test_weight_floor_and_idle_operators(orc):
    """With tau = 1 and nothing accepted, the chosen operators' weights decay
    by 0.9 per period and stop at the minimum weight 0.1; an operator with no
    attempt keeps its weight."""
    prm = orc.alns_params(tau=1)
    c = orc.alns_chain(100)
    for it in range(30):
        orc.alns_update(prm, c, 4, 3, True, 10**6, 0.9, it)
        expect = max(0.1, 0.9 ** (it + 1))
        assert c.wD[4] == pytest.approx(expect, rel=1e-12)
        assert c.wR[3] == pytest.approx(expect, rel=1e-12)
    assert c.wD[4] == 0.1 and c.wR[3] == 0.1
    assert list(c.wD)[:4] == [1.0] * 4 and c.wD[5] == 1.0


def test_reheat_needs_stagnation_and_cold(orc):
    """Reheat (Section 4.2.4): after stag_limit iterations without a new best
    and only once T < gate * T_init, T = 0.5 * T0 * z*, and the stagnation
    counter restarts."""
    prm = orc.alns_params(stag_limit=2, gate=1.0)
    c = orc.alns_chain(100)
    orc.alns_update(prm, c, 0, 0, True, 10**6, 0.9, 0)
    assert c.stag == 1 and c.T == pytest.approx(30 * 0.9998, rel=1e-15)
    orc.alns_update(prm, c, 0, 0, True, 10**6, 0.9, 1)
    assert c.stag == 0 and c.T == pytest.approx(0.5 * 0.3 * 100, rel=1e-15)
    prm = orc.alns_params(stag_limit=2, gate=0.01)
    c = orc.alns_chain(100)
    for it in range(3):
        orc.alns_update(prm, c, 0, 0, True, 10**6, 0.9, it)
    assert c.stag == 3 and c.T == pytest.approx(30 * 0.9998 ** 3, rel=1e-14)
    # a new best restarts the count
    orc.alns_update(prm, c, 0, 0, True, 50, 0.9, 3)
    assert c.stag == 1 and c.zb == 50


def test_budget_split(orc):
    """T_c = max(1, B / (q(q+1)/2)), K_D = max(1, floor(sqrt T_c)),
    K_P = max(1, T_c / K_D): B = 16,384 and q = 37 give T_c = 23, K_D = 4,
    K_P = 5; q = 25 gives T_c = 50, K_D = 7, K_P = 7; B = 0 lists all."""
    assert orc.alns_budget_split(16384, 37) == (4, 5)
    assert orc.alns_budget_split(16384, 25) == (7, 7)
    assert orc.alns_budget_split(10, 50) == (1, 1)
    assert orc.alns_budget_split(0, 5) == (0, 0)
