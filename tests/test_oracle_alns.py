"""Pins for the oracle ALNS (CPU only)."""
import math

import numpy as np
import pytest

import synth
from oracle import brute


def test_removal_size_examples(orc):
    """Section 4.2.2 prints q in [5, 10] at n = 202, [10, 21] at n = 431 and a
    constant 4 for small instances (n below about 80)."""
    assert orc.alns_qrange(202) == (5, 10)
    assert orc.alns_qrange(431) == (10, 21)
    for n in (17, 24, 51, 79):
        assert orc.alns_qrange(n) == (4, 4)
    assert orc.alns_qrange(1000) == (25, 50)


def test_det_exp_matches_libm(orc):
    xs = np.concatenate([np.linspace(-700, 0, 20001), -np.logspace(-12, 2, 500), [0.0]])
    for x in xs:
        ref = math.exp(x)
        assert abs(orc.det_exp(x) - ref) <= 1e-13 * ref + 1e-300
    assert orc.det_exp(0.0) == 1.0
    assert orc.det_exp(-800.0) == 0.0


def _run(orc, inst, iters, chains=2, seed=5, **kw):
    ops, rt = synth.round_robin_solution(inst)
    prm = orc.alns_params(**kw)
    return orc.alns_run(inst, prm, chains, iters, seed, ops, rt, trace=True), ops, rt


@pytest.mark.parametrize("n,m,k,R,rule,budget", [(16, 2, 2, 4, "base", 0), (40, 4, 5, 20, "5x", 400),
                                                 (30, 3, 3, 9, "1R20", 0)])
def test_alns_invariants(orc, n, m, k, R, rule, budget):
    inst = synth.make_instance(n, m, k, R, rule, seed=n)
    out, ops0, rt0 = _run(orc, inst, 150, tuple_budget=budget, import_interval=50)
    z0 = orc.eval_one(inst, ops0, rt0)[0]
    tr = out["trace"]
    for ch in range(tr.shape[0]):
        best = tr[ch, :, 2]
        assert np.all(np.diff(best) <= 0)
        cur = tr[ch, :, 1]
        assert np.all(cur >= best)
        assert best[-1] <= z0
        info = tr[ch, :, 3]
        nrem = info >> 24
        qmin, qmax = orc.alns_qrange(n)
        d_op = info & 0xFF
        # removal sizes stay in [q_min, q_max] except route removal's own size
        assert np.all((nrem >= 1) & (nrem <= max(qmax, n)))
        assert np.all(nrem[(d_op != 4) & (d_op != 5)] >= qmin)
        assert np.all(nrem[(d_op != 4) & (d_op != 5)] <= qmax)
        # every operator gets used
        assert set(np.unique(d_op)) == set(range(6))
        assert set(np.unique((info >> 8) & 0xFF)) == set(range(4))
    for ch in range(tr.shape[0]):
        mk, st = orc.eval_one(inst, out["best_ops"][ch], out["best_rt"][ch])
        assert st == 0 and mk == out["best_mk"][ch]


def test_best_never_increases_and_import(orc):
    inst = synth.make_instance(20, 2, 3, 6, "2x", seed=3)
    out, _, _ = _run(orc, inst, 120, chains=4, import_interval=40)
    tr = out["trace"]
    assert np.all(np.diff(tr[:, :, 2], axis=1) <= 0)
    # the import after iteration 40 (and 80) hands every chain the best of all
    for it in (39, 79):
        assert tr[:, it + 1, 2].max() <= tr[:, it, 2].min()
        assert tr[:, it + 1, 1].max() <= max(tr[:, it, 2].min(), tr[:, it + 1, 0].max())


def test_alns_finds_brute_force_optimum(orc):
    """n = 4, m = 2: exhaustive enumeration of every op-sequence solution gives
    the optimum; ALNS destroying 2 of 4 customers per iteration reaches it."""
    for seed in range(2):
        inst = synth.make_instance(4, 2, 2, 4, "base", seed=600 + seed)
        ops, rt = brute.enumerate_batch(4, 2)
        mk, st = orc.eval_batch(inst, ops, rt)
        opt = int(mk[st == 0].min())
        out, _, _ = _run(orc, inst, 400, chains=2, seed=seed, q_min=2, q_max=2, import_interval=0)
        assert int(out["best_mk"].min()) == opt


def test_special_case_minmax_vrp(orc):
    """p = 0 and ample capacity: the ALNS optimum equals the min-max VRP
    optimum found by enumeration (Section 3.2)."""
    g = synth.rng(9)
    n, m = 5, 2
    pts = g.integers(0, 8, size=(n + 1, 2))
    while len({tuple(x) for x in pts}) < n + 1:
        pts = g.integers(0, 8, size=(n + 1, 2))
    d = np.abs(pts[:, None, :] - pts[None, :, :]).sum(-1).astype(np.int32)
    inst = synth.instance_from_matrix(d, np.zeros(n + 1, np.int32), m, n, n * m)
    out, _, _ = _run(orc, inst, 600, chains=2, seed=1, q_min=2, q_max=3)
    assert int(out["best_mk"].min()) == brute.minmax_vrp_optimum(d, m)
