"""Brute-force references for tiny instances (test infrastructure only).

These enumerate solutions outright, so they pin the oracle's evaluator and
search results on instances small enough to cover every case.
"""
from __future__ import annotations

import itertools

import numpy as np


def all_sequence_solutions(n: int, m: int):
    """Every way to place the 2n ops (D_c, P_c for c = 1..n) into m ordered
    vehicle sequences.  Yields flat (ops uint16 [2n], rt_end uint16 [m])."""
    codes = [(c << 1) | isP for c in range(1, n + 1) for isP in (0, 1)]
    L = len(codes)
    for perm in itertools.permutations(codes):
        # bars: choose m-1 cut points with repetition in [0, L]
        for cuts in itertools.combinations_with_replacement(range(L + 1), m - 1):
            ends = list(cuts) + [L]
            yield np.array(perm, dtype=np.uint16), np.array(ends, dtype=np.uint16)


def enumerate_batch(n: int, m: int):
    ops, rts = [], []
    for o, r in all_sequence_solutions(n, m):
        ops.append(o)
        rts.append(r)
    return np.stack(ops), np.stack(rts)


def minmax_vrp_optimum(d: np.ndarray, m: int) -> int:
    """Min-max VRP by enumeration: split customers 1..n among m vehicles, order
    each group, minimise the longest closed tour from the depot (node 0)."""
    n = d.shape[0] - 1
    best = None

    def tour_best(group):
        if not group:
            return 0
        b = None
        for perm in itertools.permutations(group):
            length = d[0, perm[0]] + sum(d[perm[i], perm[i + 1]] for i in range(len(perm) - 1)) \
                + d[perm[-1], 0]
            b = length if b is None or length < b else b
        return b

    for assign in itertools.product(range(m), repeat=n):
        groups = [[c + 1 for c in range(n) if assign[c] == v] for v in range(m)]
        z = max(tour_best(g) for g in groups)
        best = z if best is None or z < best else best
    return int(best)


def min_makespan_by_times(d, p, routes, horizon):
    """Minimum makespan of fixed routes by enumerating integer op times.

    The constraints are those of the MILP (Section 3.1) restricted to a fixed
    routing: along each route the vehicle's clock never runs backwards and
    covers each travel time (Eq. 10, 12); a drop's time is the vehicle's
    arrival-or-later clock (Eq. 7); a pickup happens no earlier than its drop
    plus processing (Eq. 9); the makespan covers every return (Eq. 21-22).
    Waiting is allowed anywhere, so the minimum over all feasible integer
    timings is the earliest-start makespan.  Returns None when no timing in
    [0, horizon] is feasible (a cyclic wait)."""
    ops = [(v, j, c, op) for v, r in enumerate(routes) for j, (c, op) in enumerate(r)]
    K = len(ops)
    best = None
    for times in itertools.product(range(horizon + 1), repeat=K):
        T = {}
        ok = True
        for idx, (v, j, c, op) in enumerate(ops):
            T[(v, j)] = times[idx]
        for (v, j, c, op) in ops:
            prev_loc = 0 if j == 0 else routes[v][j - 1][0]
            prev_t = 0 if j == 0 else T[(v, j - 1)]
            if T[(v, j)] < prev_t + d[prev_loc, c]:
                ok = False
                break
        if not ok:
            continue
        drop_t = {c: T[(v, j)] for (v, j, c, op) in ops if op == "D"}
        for (v, j, c, op) in ops:
            if op == "P" and T[(v, j)] < drop_t[c] + p[c]:
                ok = False
                break
        if not ok:
            continue
        z = 0
        for v, r in enumerate(routes):
            if r:
                z = max(z, T[(v, len(r) - 1)] + d[r[-1][0], 0])
        best = z if best is None or z < best else best
    return best
