"""Brute-force helpers for the ALNS pins (CPU only, test infrastructure).

Written from the position semantics of an insertion tuple (the drop goes
before index p_D of its vehicle's route, the pickup before index p_P of the
route after the drop went in, after the drop when on the same vehicle) and
from the readings of the repair rules; every candidate is priced by the
oracle's evaluator, which is pinned on its own.
"""
import numpy as np

BIGC = 1 << 40


def encode(routes):
    """[[(c, isP), ...] per vehicle] -> (ops uint16, rt_end uint16)."""
    ops, rt = [], []
    for r in routes:
        ops += [(c << 1) | isP for c, isP in r]
        rt.append(len(ops))
    return np.array(ops, np.uint16), np.array(rt, np.uint16)


def decode(ops, rt):
    routes, s = [], 0
    for e in rt:
        routes.append([(int(o) >> 1, int(o) & 1) for o in ops[s:int(e)]])
        s = int(e)
    return routes


def without(routes, customers):
    gone = set(customers)
    return [[x for x in r if x[0] not in gone] for r in routes]


def insertions(routes, c):
    """Every valid (vD, pD, vP, pP) insertion of customer c."""
    m = len(routes)
    out = []
    for vD in range(m):
        for pD in range(len(routes[vD]) + 1):
            for vP in range(m):
                L = len(routes[vP]) + (1 if vP == vD else 0)
                lo = pD + 1 if vP == vD else 0
                for pP in range(lo, L + 1):
                    out.append((vD, pD, vP, pP))
    return out


def insert(routes, c, t):
    vD, pD, vP, pP = t
    r = [list(x) for x in routes]
    r[vD].insert(pD, (c, 0))
    r[vP].insert(pP, (c, 1))
    return r


def priced(orc, inst, routes, c):
    """[(makespan, tuple)] of every feasible insertion of c (partial solutions allowed)."""
    res = []
    for t in insertions(routes, c):
        o, rt = encode(insert(routes, c, t))
        mk, st = orc.eval_one(inst, o, rt, allow_partial=True)
        if st == 0:
            res.append((mk, t))
    return res


def rule_choice(orc, inst, routes, waiting, rule):
    """The customer a repair rule inserts next (rule 0 greedy, 1 regret-2,
    2 regret-3, 3 regret-m) and its best makespan, from every insertion of
    every waiting customer; None if some customer has no feasible one."""
    m = inst.m
    k = {1: 2, 2: 3, 3: m}.get(rule)
    best = None
    for i, c in enumerate(waiting):
        pr = priced(orc, inst, routes, c)
        if not pr:
            return None
        c1 = min(mk for mk, _ in pr)
        reg = 0
        if rule:
            opt = sorted(min([mk for mk, t in pr if t[0] == v], default=BIGC) for v in range(m))
            reg = sum(opt[h] - opt[0] for h in range(1, min(k, m)))
            reg += sum(BIGC - opt[0] for h in range(m, k))
        key = (c1,) if rule == 0 else (-reg, c1)
        if best is None or key < best[0]:
            best = (key, c, c1)
    return best[1], best[2]
