"""Pins for the oracle decoder, insertion scan and BRKGA operators (CPU only)."""
import numpy as np
import pytest

import synth

BAD_COVER, LOAD, RES, DEADLOCK, BAD_KEY, BAD_TUPLE = 1, 2, 4, 8, 16, 32
INT32_MAX, INT64_MAX = 2**31 - 1, 2**63 - 1


def inst2(load_model):
    d = np.array([[0, 5], [5, 0]], dtype=np.int32)
    return synth.instance_from_matrix(d, [0, 7], m=2, k=1, R=1, load_model=load_model)


# ----------------------------------------------------------------- decoder
def test_h4_hint_tie_break(orc):
    """n=1, d01=5, p1=7, m=2, k=1.  pi=(0.1, 0.2), alpha=(0.9, 0.2).
    FULL_START (Algorithm 2's q = k): both vehicles full; the drop ties at 5 and
    the hint floor(2*0.9)=1 picks v1; only v1 has room for the pickup, which
    waits to 12; return at 17.
    MIN_PRELOAD: the pickup ties at 12 on both vehicles; hint floor(2*0.2)=0
    picks v0; return 12+5 = 17."""
    prio = np.array([0.1, 0.2], np.float32)
    hint = np.array([0.9, 0.2], np.float32)
    r = orc.decode(inst2(1), prio, hint, want_ops=True)
    assert (r["fitness"], r["makespan"], r["unscheduled"]) == (17, 17, 0)
    assert list(r["rt_end"]) == [0, 2]
    r = orc.decode(inst2(0), prio, hint, want_ops=True)
    assert (r["fitness"], r["makespan"], r["unscheduled"]) == (17, 17, 0)
    assert list(r["rt_end"]) == [1, 2] and list(r["ops"]) == [3, 2]


def test_hint_rotation_three_vehicles(orc):
    """Ties go to the first vehicle counting upward (cyclically) from the
    hint vehicle.  Line: depot 0, c1 at -4, c2 at 6 (d01 = 4, d02 = 6,
    d12 = 10), p = (3, 5), m = 3, k = 1, R = 3, MIN_PRELOAD.  Priorities put
    the ops in the order D1, D2, P1, P2; hints floor(3 alpha) = 0, 1, 0, 0 for
    D1, P1, D2, P2.
      D1: all three vehicles tie at 4, hint 0 -> v0 (drop at 4, ready 7);
      D2: v0 holds its one resource and may not load another; v1 and v2 tie
          at 6, hint 0 -> v1 (the next after v0; counting down would give v2);
          ready 11;
      P1: v0 max(4, 7) = 7, v1 max(16, 7) = 16, v2 max(4, 7) = 7; hint 1,
          tie v0 / v2 -> v2 (after v1 comes v2, then v0);
      P2: v2 is full; v0 max(14, 11) = 14, v1 max(6, 11) = 11 -> v1.
    Returns: v0 4 + 4 = 8, v1 11 + 6 = 17, v2 7 + 4 = 11; z = 17."""
    x = np.array([0, -4, 6])
    d = np.abs(x[:, None] - x[None, :]).astype(np.int32)
    inst = synth.instance_from_matrix(d, np.array([0, 3, 5], np.int32), m=3, k=1, R=3)
    prio = np.array([0.1, 0.8, 0.2, 0.9], np.float32)
    hint = np.array([0.1, 0.5, 0.1, 0.1], np.float32)
    r = orc.decode(inst, prio, hint, want_ops=True)
    assert (r["fitness"], r["makespan"], r["unscheduled"]) == (17, 17, 0)
    assert list(r["rt_end"]) == [1, 3, 4]
    assert list(r["ops"]) == [2, 4, 5, 3]


def _line2():
    """Line: depot 0, c1 at 3, c2 at 10 (d01 = 3, d02 = 10, d12 = 7)."""
    x = np.array([0, 3, 10])
    return np.abs(x[:, None] - x[None, :]).astype(np.int32)


def test_hint_first_keeps_the_hint_vehicle(orc):
    """Hint-first rule (Section 4.4.1: the hint is the vehicle unless
    feasibility overrides it) against SelectVehicle's least completion time
    (Section 4.4.2).  p = (4, 2), m = 2, k = 2, R = 4, MIN_PRELOAD; order D1,
    P1, D2, P2; every hint floor(2 * 0.75) = 1.
    Hint-first: v1 takes all four: D1 at 3 (ready 7), P1 waits to 7, D2 at
      7 + 7 = 14 (ready 16), P2 waits to 16, return 16 + 10 = 26.
    Least completion: D1 ties at 3 -> hint v1; P1 ties at 7 -> v1; D2: v0
      arrives at 10, v1 at 14 -> v0 (ready 12); P2: v0 max(10, 12) = 12, v1
      max(14, 12) = 14 -> v0; returns v0 12 + 10 = 22, v1 7 + 3 = 10."""
    inst = synth.instance_from_matrix(_line2(), np.array([0, 4, 2], np.int32), m=2, k=2, R=4)
    prio = np.array([0.1, 0.2, 0.3, 0.4], np.float32)
    hint = np.full(4, 0.75, np.float32)
    r = orc.decode(inst, prio, hint, want_ops=True, flags=orc.DECODE_HINT_FIRST)
    assert (r["fitness"], r["makespan"], r["unscheduled"], r["status"]) == (26, 26, 0, 0)
    assert list(r["rt_end"]) == [0, 4] and list(r["ops"]) == [2, 3, 4, 5]
    r = orc.decode(inst, prio, hint, want_ops=True)
    assert (r["fitness"], r["makespan"], r["unscheduled"]) == (22, 22, 0)
    assert list(r["rt_end"]) == [2, 4] and list(r["ops"]) == [4, 5, 2, 3]
    assert orc.eval_one(inst, np.array([2, 3, 4, 5], np.uint16), np.array([0, 4], np.uint16)) == (26, 0)


def test_hint_first_override_and_rotation(orc):
    """Hint-first when the hint vehicle cannot take the op: SelectVehicle
    over the others, ties counted cyclically from the hint.  Same line,
    p = (4, 2), m = 3, k = 1, R = 3, FULL_START (every vehicle leaves with
    one resource); order D1, D2, P1, P2; hints floor(3 alpha) = 0 (D1), 0
    (D2), 2 (P1), 1 (P2).
      D1: v0 can drop -> v0 at 3 (ready 7);
      D2: v0 is empty; v1 and v2 tie at 10, counting from 0 -> v1 (ready 12);
      P1: v2 is full; v0 max(3, 7) = 7, v1 max(17, 7) = 17 -> v0;
      P2: v1 has room -> v1, max(10, 12) = 12.
    Returns v0 7 + 3 = 10, v1 12 + 10 = 22; v2 unused."""
    inst = synth.instance_from_matrix(_line2(), np.array([0, 4, 2], np.int32), m=3, k=1, R=3, load_model=1)
    prio = np.array([0.1, 0.3, 0.2, 0.4], np.float32)
    hint = np.array([0.1, 0.9, 0.1, 0.5], np.float32)
    r = orc.decode(inst, prio, hint, want_ops=True, flags=orc.DECODE_HINT_FIRST)
    assert (r["fitness"], r["makespan"], r["unscheduled"], r["status"]) == (22, 22, 0, 0)
    assert list(r["rt_end"]) == [2, 4, 4] and list(r["ops"]) == [2, 3, 4, 5]


def test_hint_first_reproduces_warm_encoding(orc):
    """Under hint-first every op of an encoded solution goes to its own
    vehicle when the encoding's priority order is a time order of the
    schedule: the one-vehicle-per-route solution of a round-robin start
    (drop then own pickup, customers in turn) decodes back to itself."""
    inst = synth.make_instance(30, 3, 3, 9, "base", seed=44)
    ops, rt = synth.round_robin_solution(inst)
    po, ho = orc.brkga_warm_start(inst, ops, rt, 1, 1, 1, 5)
    r = orc.decode(inst, po[0], ho[0], want_ops=True, flags=orc.DECODE_HINT_FIRST)
    assert r["unscheduled"] == 0
    assert list(r["rt_end"]) == list(rt) and list(r["ops"]) == list(ops)
    assert r["makespan"] == orc.eval_one(inst, ops, rt)[0]


def test_single_vehicle_closed_form(orc):
    """m = 1 with room for everything: pass 1 takes ops in priority order,
    skipping pickups whose drop comes later; pass 2 takes those pickups in
    priority order.  So the route is known without simulation."""
    for seed in range(5):
        inst = synth.make_instance(12, 1, 12, 12, "base", seed=seed)
        g = synth.rng(seed)
        prio = g.random(24, dtype=np.float32)
        r = orc.decode(inst, prio, want_ops=True)
        order = list(np.argsort(prio, kind="stable"))
        done, first, later = set(), [], []
        for o in order:
            if o & 1 and (o - 1) not in done:
                later.append(o)
            else:
                first.append(o)
                done.add(o)
        expect = [((o // 2 + 1) << 1) | (o & 1) for o in first + later]
        assert list(r["ops"]) == expect
        assert r["unscheduled"] == 0
        assert orc.eval_one(inst, r["ops"], r["rt_end"]) == (r["makespan"], 0)


def test_hint_decides_on_full_ties(orc):
    """All travel times equal and no processing: every vehicle offers the same
    completion time for every op, so each op lands on its hint vehicle
    floor(m * alpha) when capacity allows."""
    n, m = 6, 3
    d = np.full((n + 1, n + 1), 4, np.int32)
    np.fill_diagonal(d, 0)
    inst = synth.instance_from_matrix(d, np.zeros(n + 1, np.int32), m, k=n, R=n * m)
    g = synth.rng(3)
    # drops first in priority, then pickups; hints spread over vehicles
    prio = np.array([0.1 + 0.01 * i if i % 2 == 0 else 0.6 + 0.01 * i for i in range(2 * n)],
                    np.float32)
    hint = g.random(2 * n, dtype=np.float32)
    r = orc.decode(inst, prio, hint, want_ops=True)
    # the first drop is placed at time 4 on its hint vehicle
    first_v = int(np.floor(np.float32(m) * hint[0]))
    rt = [0] + list(r["rt_end"])
    routes = [list(r["ops"][rt[v]:rt[v + 1]]) for v in range(m)]
    assert 2 in routes[first_v]


def test_decoder_output_is_a_feasible_schedule(orc):
    """Complete decodes re-evaluate to the decoder's own makespan, status 0."""
    for (n, m, k, R, rule, lm) in [(16, 2, 2, 4, "base", 0), (40, 4, 5, 20, "2x", 0),
                                   (40, 4, 5, 20, "5x", 1), (60, 6, 3, 10, "1R20", 0)]:
        inst = synth.make_instance(n, m, k, R, rule, seed=n, load_model=lm)
        prio, hint = synth.random_keys(30, n, seed=n)
        done = 0
        for b in range(30):
            r = orc.decode(inst, prio[b], hint[b], want_ops=True)
            if r["unscheduled"] == 0:
                assert r["fitness"] == r["makespan"]
                assert orc.eval_one(inst, r["ops"], r["rt_end"]) == (r["makespan"], 0)
                done += 1
            else:
                assert r["fitness"] == r["makespan"] + 10**6 * r["unscheduled"]
        assert done > 0


def test_infeasible_penalty(orc):
    """No resources at all: no drop can be made, so nothing schedules and the
    fitness is the penalty lambda * 2n with lambda = 1e6."""
    inst = synth.make_instance(5, 2, 2, 0, "base", seed=1)
    prio, hint = synth.random_keys(1, 5, seed=1)
    r = orc.decode(inst, prio[0], hint[0])
    assert (r["makespan"], r["unscheduled"], r["fitness"]) == (0, 10, 10 * 10**6)


def test_bad_keys(orc):
    inst = synth.make_instance(4, 2, 2, 4, "base", seed=1)
    prio, hint = synth.random_keys(1, 4, seed=1)
    for bad in [np.nan, 1.0, -0.25, np.inf]:
        p2 = prio[0].copy()
        p2[3] = bad
        r = orc.decode(inst, p2, hint[0])
        assert r["status"] == BAD_KEY and r["fitness"] == INT64_MAX
    p2 = prio[0].copy()
    p2[:] = -0.0            # negative zero is a valid key (equal to 0)
    assert orc.decode(inst, p2, hint[0])["status"] == 0


# ------------------------------------------------------------- insert scan
def _insert(routes, c, vD, pD, vP, pP):
    out = [list(r) for r in routes]
    out[vD].insert(pD, (c, "D"))
    out[vP].insert(pP, (c, "P"))
    return out


def test_insert_scan_matches_hand_built_solutions(orc):
    inst = synth.make_instance(12, 3, 3, 9, "2x", seed=4)
    ops, rt = synth.random_candidates(inst, 1, 5)
    routes = synth.unpack_candidate(ops[0], rt[0])
    removed = {3, 7}
    base = [[x for x in r if x[0] not in removed] for r in routes]
    bops, _, brt = synth.pack_candidates([base], 3)
    tuples = synth.random_tuples(bops, brt[0], 12, 3, 200, seed=6, invalid_frac=0.1)
    seg_off = np.array([0, 50, 50, 120, 200], np.int64)
    mk, st, top = orc.insert_scan(inst, bops, brt[0], tuples, seg_off)
    nbad = 0
    for i, t in enumerate(tuples):
        c, vD, vP, pD, pP = int(t["c"]), int(t["vD"]), int(t["vP"]), int(t["pD"]), int(t["pP"])
        lens = [len(r) for r in base]
        valid = (1 <= c <= 12 and c in removed and vD < 3 and vP < 3 and pD <= lens[vD] and
                 ((pD + 1 <= pP <= lens[vD] + 1) if vP == vD else pP <= lens[vP]))
        if not valid:
            assert (mk[i], st[i]) == (INT32_MAX, BAD_TUPLE)
            nbad += 1
            continue
        full = _insert(base, c, vD, pD, vP, pP)
        o2, _, r2 = synth.pack_candidates([full], 3)
        assert (mk[i], st[i]) == orc.eval_one(inst, o2, r2[0], allow_partial=True)
    assert nbad > 0
    for s in range(4):
        lo, hi = seg_off[s], seg_off[s + 1]
        keys = sorted((int(mk[i]) << 32) | i for i in range(lo, hi) if st[i] == 0)
        keys = (keys + [INT64_MAX] * 3)[:3]
        assert list(top[s]) == keys
    # a customer the base already serves cannot be inserted again, whatever
    # the positions (a tuple error, not a cover error of the result)
    served = sorted({x[0] for r in base for x in r})
    extra = np.zeros(len(served), dtype=tuples.dtype)
    for i, c in enumerate(served):
        extra[i]["c"], extra[i]["vD"], extra[i]["pD"], extra[i]["vP"], extra[i]["pP"] = c, 0, 0, 0, 1
    mk2, st2, _ = orc.insert_scan(inst, bops, brt[0], extra, np.array([0, len(extra)], np.int64))
    assert np.all(st2 == BAD_TUPLE) and np.all(mk2 == INT32_MAX)


def test_insert_position_semantics(orc):
    """pP counts positions after the drop went in: on the same vehicle
    pP = pD + 1 puts the pickup right after the drop (the vehicle waits p_c)."""
    d = np.abs(np.subtract.outer([0, 2, 5], [0, 2, 5])).astype(np.int32)
    inst = synth.instance_from_matrix(d, [0, 3, 4], m=1, k=2, R=2)
    base = [[(1, "D"), (1, "P")]]
    bops, _, brt = synth.pack_candidates([base], 1)
    tup = np.zeros(3, dtype=synth.TUPLE_DTYPE)
    tup[0] = (2, 0, 0, 2, 3)   # [D1, P1, D2, P2]: 2 -> wait 3 -> 5 -> wait 4 -> back 5: 2+3+3+4+5
    tup[1] = (2, 0, 0, 0, 1)   # [D2, P2, D1, P1]: 5+4+3+3+2 = 17
    tup[2] = (2, 0, 0, 1, 3)   # [D1, D2, P1, P2]: D1@2 D2@5 P1@8 P2@11(ready 9) back 16
    mk, st, top = orc.insert_scan(inst, bops, brt[0], tup, np.array([0, 3], np.int64))
    assert list(mk) == [17, 17, 16] and list(st) == [0, 0, 0]
    assert top[0][0] == (16 << 32) | 2


# ------------------------------------------------------------------- BRKGA
def test_philox_known_answers(orc):
    """Known-answer vectors of Philox4x32-10 from the Random123 distribution."""
    assert list(orc.philox([0, 0, 0, 0], [0, 0])) == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert list(orc.philox([0xffffffff] * 4, [0xffffffff] * 2)) == \
        [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert list(orc.philox([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344],
                           [0xa4093822, 0x299f31d0])) == [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_brkga_sizes(orc):
    # Table 3 proportions, rounded down
    assert orc.brkga_sizes(1024) == (153, 153)
    assert orc.brkga_sizes(4096) == (614, 614)
    assert orc.brkga_sizes(30000) == (4500, 4500)
    assert orc.rho_threshold(0.7) == 11744051


def test_brkga_evolve_structure(orc):
    n, Np = 10, 200
    ne, nm = orc.brkga_sizes(Np)
    prio, hint = synth.random_keys(Np, n, seed=8)
    fit = synth.rng(9).integers(0, 50, size=Np).astype(np.int64)   # many ties
    po, ho, rank = orc.brkga_evolve(prio, hint, fit, ne, nm, orc.rho_threshold(0.7), 1234, 3)
    order = sorted(range(Np), key=lambda i: (fit[i], i))
    assert list(rank) == order
    for i in range(ne):                                   # elites copied unchanged
        assert np.array_equal(po[i], prio[order[i]]) and np.array_equal(ho[i], hint[order[i]])
    mut = np.concatenate([po[ne:ne + nm].ravel(), ho[ne:ne + nm].ravel()])
    assert mut.min() >= 0 and mut.max() < 1 and len(np.unique(mut)) > 0.9 * mut.size
    full = np.concatenate([prio, hint], axis=1)          # all 4n genes per individual
    child = np.concatenate([po, ho], axis=1)
    frac = []
    for i in range(ne + nm, Np):
        # each gene equals the same position of an elite or a non-elite parent
        found = None
        for e in order[:ne]:
            me = child[i] == full[e]
            if me.mean() < 0.4:
                continue
            for x in order[ne:]:
                mx = child[i] == full[x]
                if np.all(me | mx) and mx.any():
                    found = me
                    break
            if found is not None:
                break
        assert found is not None
        frac.append(found.mean())
    assert 0.6 < np.mean(frac) < 0.8


def test_warm_start_encoding(orc):
    inst = synth.make_instance(8, 3, 4, 12, "base", seed=2)
    ops, rt = synth.random_candidates(inst, 1, 3)
    po, ho = orc.brkga_warm_start(inst, ops[0], rt[0], 20, 6, 4, seed=77)
    # slot 0 is the seed encoding: position (r-1)/L_v and hint (v + 1/2)/m
    s = 0
    for v in range(3):
        e = int(rt[0][v])
        for j in range(s, e):
            o = 2 * ((int(ops[0][j]) >> 1) - 1) + (int(ops[0][j]) & 1)
            assert po[0][o] == np.float32((j - s) / (e - s))
            assert ho[0][o] == np.float32((v + 0.5) / 3)
            assert int(np.floor(np.float32(3) * ho[0][o])) == v
        s = e
    assert np.array_equal(po[4], po[0])                   # variants cycle (4 variants)
    assert np.all(np.abs(po[1] - po[0]) <= 0.03 + 1e-6)
    assert np.all((po >= 0) & (po < 1) & (ho >= 0) & (ho < 1))
    assert not np.array_equal(po[1], po[2])
