"""Pins for the periodic local search of the ALNS oracle (Section 4.2.6):
with a budget above every neighbourhood's size, one pass equals the best move
found by brute force over the moves the paper describes (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import alns_local_search, eval_one


def routes_of(ops, rt):
    out, s = [], 0
    for e in rt:
        out.append([int(x) for x in ops[s:int(e)]])
        s = int(e)
    return out


def pack(routes):
    ops = np.array([x for r in routes for x in r], np.uint16)
    rt = np.cumsum([len(r) for r in routes]).astype(np.uint16)
    return ops, rt


def finishes(inst, ops, rt):
    z, st, times = eval_one(inst, ops, rt, times=True)
    fin, s = [], 0
    for e in rt:
        e = int(e)
        fin.append(int(times[e - 1]) + int(inst.d[int(ops[e - 1]) >> 1][0]) if e > s else 0)
        s = e
    return z, fin


def brute_force(inst, kind, ops, rt):
    z, fin = finishes(inst, ops, rt)
    routes = routes_of(ops, rt)
    m = inst.m
    best = z
    if kind == 0:
        cands = [x >> 1 for v in range(m) if 20 * fin[v] >= 19 * z for x in routes[v] if x & 1]
    else:
        b = int(np.argmax(fin))
        cands = []
        for x in routes[b]:
            if x >> 1 not in cands:
                cands.append(x >> 1)
    for c in cands:
        if kind == 0:
            base = [[x for x in r if x != 2 * c + 1] for r in routes]
            vD = next(v for v in range(m) if 2 * c in base[v])
            pD = base[vD].index(2 * c)
            for v in range(m):
                lo = pD + 1 if v == vD else 0
                for p in range(lo, len(base[v]) + 1):
                    new = [list(r) for r in base]
                    new[v].insert(p, 2 * c + 1)
                    zz, st = eval_one(inst, *pack(new))
                    if st == 0 and zz < best:
                        best = zz
        else:
            base = [[x for x in r if x >> 1 != c] for r in routes]
            for v in range(m):
                if v == b:
                    continue
                for pD in range(len(base[v]) + 1):
                    for pP in range(pD + 1, len(base[v]) + 2):
                        new = [list(r) for r in base]
                        new[v].insert(pD, 2 * c)
                        new[v].insert(pP, 2 * c + 1)
                        zz, st = eval_one(inst, *pack(new))
                        if st == 0 and zz < best:
                            best = zz
    return z, best


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_one_pass_equals_brute_force(kind, seed):
    inst = synth.make_instance(9, 3, 3, 9, "base", seed=600 + seed)
    ops, rt = synth.random_candidates(inst, 1, seed=700 + seed)
    ops, rt = ops[0], rt[0]
    z0, st = eval_one(inst, ops, rt)
    assert st == 0
    z, best = brute_force(inst, kind, ops, rt)
    k, z1, o1, r1 = alns_local_search(inst, kind, ops, rt, budget=1 << 20, passes=1)
    assert z1 == best, (z, best, z1)
    assert k == (1 if best < z else 0)
    assert eval_one(inst, o1, r1) == (z1, 0)


def test_passes_improve_monotonically():
    inst = synth.make_instance(30, 4, 4, 16, "2x", seed=31)
    ops, rt = synth.round_robin_solution(inst)
    z0 = eval_one(inst, ops, rt)[0]
    prev = z0
    for passes in (1, 2, 3):
        for kind in (0, 1):
            k, z, o, r = alns_local_search(inst, kind, ops, rt, budget=2000, passes=passes)
            assert k <= passes and z <= z0
            assert eval_one(inst, o, r) == (z, 0)
    k0, z0b, _, _ = alns_local_search(inst, 0, ops, rt, budget=2000, passes=1)
    k3, z3, _, _ = alns_local_search(inst, 0, ops, rt, budget=2000, passes=3)
    assert z3 <= z0b <= prev
