"""Pins for the learned proposal's feature oracle (CPU only): the hand vector
H1 worked out from the timing rules, and invariances of the definition."""
import os
from fractions import Fraction

import numpy as np

import synth
from oracle import features as of

GOLD = os.path.join(os.path.dirname(__file__), "golden", "features_h1.txt")


def h1():
    d = [[0, 3, 10], [3, 0, 7], [10, 7, 0]]
    inst = synth.instance_from_matrix(d, [0, 4, 2], m=2, k=1, R=2)
    ops = np.array([2 * 1, 2 * 2 + 1, 2 * 1 + 1, 2 * 2], np.uint16)   # [D1, P2] [P1, D2]
    return inst, ops, np.array([2, 4], np.uint16)


def test_h1_features_match_hand_values():
    inst, ops, rt = h1()
    F = of.customer_features(inst, ops, rt)
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for r in rows:
        c = int(r[0])
        for i, tok in enumerate(r[1:]):
            want = np.float32(float(Fraction(tok)))
            assert F[c, i] == want, (c, i, F[c, i], want)
            assert F[c, 32 + i] == want          # gate = 1 for both
    assert np.all(F[0] == 0)


def test_invariant_under_vehicle_relabeling():
    inst = synth.make_instance(12, 3, 3, 9, "base", seed=4)
    ops, rt = synth.round_robin_solution(inst)
    F = of.customer_features(inst, ops, rt)
    routes = synth.unpack_candidate(ops, rt)
    perm = [2, 0, 1]
    ops2, _, rt2 = synth.pack_candidates([[routes[v] for v in perm]], inst.m)
    F2 = of.customer_features(inst, ops2, rt2[0])
    assert np.array_equal(F, F2)
    assert np.all(np.isfinite(F))
    # the gated half is the base half times a 0/1 gate per customer
    gate = F[1:, 32] / F[1:, 0]
    assert set(np.unique(gate)) <= {0.0, 1.0}
    assert np.array_equal(F[1:, 32:], F[1:, :32] * gate[:, None])
    # a customer on a vehicle finishing at the makespan has the gate set
    assert gate.max() == 1.0


def test_gains_are_direct_evaluations():
    inst = synth.make_instance(9, 2, 3, 6, "base", seed=8)
    ops, rt = synth.round_robin_solution(inst)
    from oracle import eval_one
    z, st = eval_one(inst, ops, rt)
    g = of.removal_gains(inst, ops, rt, z)
    # removing a customer never lengthens a schedule here (metric-ish
    # distances, no new waits): check one by hand-built partial solution
    c = 5
    routes = synth.unpack_candidate(ops, rt)
    red = [[x for x in r if x[0] != c] for r in routes]
    o2, _, r2 = synth.pack_candidates([red], inst.m)
    zc, st2 = eval_one(inst, o2, r2[0], allow_partial=True)
    assert st == 0 and st2 == 0 and g[c] == z - zc
