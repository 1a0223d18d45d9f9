"""Seeded synthetic inputs for VRP-RPD: instances, candidate solutions,
insertion tuples and random-key chromosomes.

This module is the only code shared by the CPU oracle's tests and the GPU
path's tests and benchmark. It draws inputs; it computes no makespan, no load
check, no schedule and no decoder step.

Instances follow the benchmark design of the paper's experimental setup
(Section 5.1, "Benchmark Instances and Problem Variants"): a depot plus n
customers, travel times taken as integer edge weights, and processing times
drawn by one of the five variants (base, 2x, 5x, 1R10, 1R20).  The paper uses
TSPLIB instances, which are not available here; these generators stand in for
them with integer points uniform in [0, 1000]^2 and TSPLIB EUC_2D rounding
(nearest integer of the Euclidean distance).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "RULES", "Instance", "make_instance", "random_candidates", "pack_candidates",
    "random_tuples", "random_keys", "round_robin_solution", "rng",
]

RULES = ("base", "2x", "5x", "1R10", "1R20", "1R20d10", "paper_base", "zero")

MIN_PRELOAD = 0
FULL_START = 1


def rng(seed: int) -> np.random.Generator:
    """Philox4x32-10 stream keyed by ``seed`` (numpy's implementation)."""
    return np.random.Generator(np.random.Philox(key=int(seed) & ((1 << 64) - 1)))


class Instance:
    """One VRP-RPD instance: node 0 is the depot, nodes 1..n are customers."""

    def __init__(self, n, m, k, R, d, p, coords=None, load_model=MIN_PRELOAD, rule=""):
        self.n, self.m, self.k, self.R = int(n), int(m), int(k), int(R)
        self.d = np.ascontiguousarray(d, dtype=np.int32)
        self.p = np.ascontiguousarray(p, dtype=np.int32)
        self.coords = coords
        self.load_model = int(load_model)
        self.rule = rule
        assert self.d.shape == (n + 1, n + 1) and self.p.shape == (n + 1,)
        assert self.p[0] == 0

    def __repr__(self):
        return (f"Instance(n={self.n}, m={self.m}, k={self.k}, R={self.R}, "
                f"rule={self.rule!r}, load_model={self.load_model})")


def _euc2d_nint(coords: np.ndarray) -> np.ndarray:
    """TSPLIB EUC_2D: nearest integer of the Euclidean distance, computed in
    exact integer arithmetic.  With S = dx^2 + dy^2 and r = isqrt(S), the
    distance rounds up iff sqrt(S) >= r + 1/2, i.e. iff S > r^2 + r (S and r
    are integers, so no tie is possible)."""
    x = coords[:, 0].astype(np.int64)
    y = coords[:, 1].astype(np.int64)
    S = (x[:, None] - x[None, :]) ** 2 + (y[:, None] - y[None, :]) ** 2
    r = np.floor(np.sqrt(S.astype(np.float64))).astype(np.int64)
    r[(r + 1) * (r + 1) <= S] += 1
    r[r * r > S] -= 1
    return (r + ((S - r * r) > r)).astype(np.int32)


def make_instance(n: int, m: int, k: int, R: int, rule: str = "base", seed: int = 0,
                  load_model: int = MIN_PRELOAD, grid: int = 1000) -> Instance:
    """Synthetic TSPLIB-shaped instance.

    Points: n+1 distinct integer points uniform in [0, grid]^2, node 0 = depot.
    Processing rules (dbar = floor(mean depot distance)):
      base      p ~ U_int[floor(dbar/2), 2*dbar]
      2x, 5x    base times 2 or 5
      1R10/1R20 base times U_int[1,10] / U_int[1,20]
      1R20d10   U_int[1,20] * floor(dbar/10)   (the full-scale n=1000 workload)
      paper_base  U_int[d_min, d_max] over off-diagonal edge weights
      zero      p = 0 (the special case of the NP-hardness reduction)
    """
    if rule not in RULES:
        raise ValueError(f"unknown processing rule {rule!r}")
    g = rng(seed)
    seen = set()
    pts = []
    while len(pts) < n + 1:
        x, y = (int(v) for v in g.integers(0, grid + 1, size=2))
        if (x, y) not in seen:
            seen.add((x, y))
            pts.append((x, y))
    coords = np.array(pts, dtype=np.int64)
    d = _euc2d_nint(coords)
    dbar = int(d[0, 1:].sum()) // n
    lo, hi = dbar // 2, 2 * dbar
    base = g.integers(lo, hi + 1, size=n, dtype=np.int64)
    if rule == "base":
        pc = base
    elif rule == "2x":
        pc = 2 * base
    elif rule == "5x":
        pc = 5 * base
    elif rule == "1R10":
        pc = base * g.integers(1, 11, size=n, dtype=np.int64)
    elif rule == "1R20":
        pc = base * g.integers(1, 21, size=n, dtype=np.int64)
    elif rule == "1R20d10":
        pc = g.integers(1, 21, size=n, dtype=np.int64) * (dbar // 10)
    elif rule == "paper_base":
        off = d[~np.eye(n + 1, dtype=bool)]
        pc = g.integers(int(off.min()), int(off.max()) + 1, size=n, dtype=np.int64)
    else:
        pc = np.zeros(n, dtype=np.int64)
    p = np.zeros(n + 1, dtype=np.int32)
    p[1:] = pc
    return Instance(n, m, k, R, d, p, coords=coords, load_model=load_model, rule=rule)


def instance_from_matrix(d, p, m, k, R, load_model=MIN_PRELOAD) -> Instance:
    d = np.asarray(d, dtype=np.int32)
    n = d.shape[0] - 1
    return Instance(n, m, k, R, d, np.asarray(p, dtype=np.int32), load_model=load_model)


def random_candidates(inst: Instance, B: int, seed: int, respect_load: bool = True,
                      chunk: int = 8192, outstanding_frac: float = 0.5):
    """B candidate solutions as per-vehicle drop/pickup sequences.

    Each candidate is a random linear extension of the drop-before-pickup
    order: at every step the next op is a drop of a not-yet-dropped customer
    (customers in a random order) or the pickup of a random dropped one, so
    the sequences never contain a precedence cycle.  At most
    ``outstanding_frac * R`` resources are out at any time.  Each op then goes
    to a random vehicle; with ``respect_load`` the vehicle is drawn among those
    whose running drop-minus-pickup window stays within k and whose summed
    peaks stay within R (a sampling filter that keeps most candidates
    load-feasible; nothing in the tests relies on it).

    Returns (ops [B, 2n] uint16 with code = (c << 1) | isPickup, grouped by
    vehicle; rt_end [B, m] uint16 cumulative route ends).
    """
    n, m, k, R = inst.n, inst.m, inst.k, inst.R
    g = rng(seed)
    lim = max(1, int(outstanding_frac * R)) if R > 0 else 1
    ops_all = np.empty((B, 2 * n), dtype=np.uint16)
    rt_all = np.empty((B, m), dtype=np.uint16)
    for s in range(0, B, chunk):
        b = min(chunk, B - s)
        rows = np.arange(b)
        dorder = np.argsort(g.random((b, n)), axis=1) + 1          # drop order of customers
        dptr = np.zeros(b, dtype=np.int64)
        out = np.zeros((b, n), dtype=np.int64)                      # dropped, not picked up
        cnt = np.zeros(b, dtype=np.int64)
        code = np.empty((b, 2 * n), dtype=np.int64)
        veh = np.empty((b, 2 * n), dtype=np.int64)
        w = np.zeros((b, m), dtype=np.int64)
        wmax = np.zeros((b, m), dtype=np.int64)
        wmin = np.zeros((b, m), dtype=np.int64)
        for step in range(2 * n):
            can_d = (dptr < n) & (cnt < lim)
            can_p = cnt > 0
            coin = g.random(b)
            is_d = can_d & (~can_p | (coin < 0.5))
            c = np.where(is_d, dorder[rows, np.minimum(dptr, n - 1)], 0)
            pick = (g.random(b) * np.maximum(cnt, 1)).astype(np.int64)
            pc = out[rows, pick]
            last = out[rows, np.maximum(cnt - 1, 0)]
            # pickups: swap-remove the chosen customer from the outstanding list
            out[rows, pick] = np.where(is_d, out[rows, pick], last)
            cnt = np.where(is_d, cnt, cnt - 1)
            c = np.where(is_d, c, pc)
            out[rows, cnt] = np.where(is_d, c, out[rows, cnt])
            cnt = np.where(is_d, cnt + 1, cnt)
            dptr = np.where(is_d, dptr + 1, dptr)
            code[:, step] = (c << 1) | (~is_d).astype(np.int64)
            delta = np.where(is_d, 1, -1)[:, None]
            score = g.random((b, m))
            if respect_load:
                w2 = w + delta
                nmax = np.maximum(wmax, w2)
                nmin = np.minimum(wmin, w2)
                ok = (nmax - nmin) <= k
                lsum = wmax.sum(axis=1, keepdims=True) - wmax + nmax
                ok &= lsum <= R
                score = np.where(ok, score + 1.0, score)
            v = np.argmax(score, axis=1)
            veh[:, step] = v
            w[rows, v] += delta[:, 0]
            wmax[rows, v] = np.maximum(wmax[rows, v], w[rows, v])
            wmin[rows, v] = np.minimum(wmin[rows, v], w[rows, v])
        # group by vehicle, keeping the global order inside each route
        pos = np.argsort(veh * (2 * n) + np.arange(2 * n)[None, :], axis=1, kind="stable")
        ops_all[s:s + b] = np.take_along_axis(code, pos, axis=1).astype(np.uint16)
        counts = np.stack([(veh == v).sum(axis=1) for v in range(m)], axis=1)
        rt_all[s:s + b] = np.cumsum(counts, axis=1).astype(np.uint16)
    return ops_all, rt_all


def pack_candidates(routes_list, m):
    """Pack a list of candidates, each a list of m routes of (c, 'D'|'P'),
    into flat (ops uint16, op_off int64, rt_end uint16 [B, m])."""
    ops, off, rts = [], [], []
    cur = 0
    for routes in routes_list:
        assert len(routes) == m
        off.append(cur)
        ends, e = [], 0
        for r in routes:
            for c, op in r:
                ops.append((int(c) << 1) | (1 if op in ("P", 1, True) else 0))
            e += len(r)
            ends.append(e)
        rts.append(ends)
        cur += e
    return (np.array(ops, dtype=np.uint16), np.array(off, dtype=np.int64),
            np.array(rts, dtype=np.uint16).reshape(len(routes_list), m))


def unpack_candidate(ops, rt_end):
    routes, s = [], 0
    for e in rt_end:
        e = int(e)
        routes.append([(int(x) >> 1, "P" if int(x) & 1 else "D") for x in ops[s:e]])
        s = e
    return routes


def round_robin_solution(inst: Instance, vehicles: int | None = None):
    """A simple structural starting solution: customers 1..n dealt to the
    first ``vehicles`` vehicles in turn, each served as a drop immediately
    followed by its own pickup.  Returns (ops [2n] uint16, rt_end [m] uint16)."""
    n, m = inst.n, inst.m
    nv = m if vehicles is None else max(1, min(m, vehicles))
    routes = [[] for _ in range(m)]
    for c in range(1, n + 1):
        routes[(c - 1) % nv] += [(c, "D"), (c, "P")]
    ops, _, rt = pack_candidates([routes], m)
    return ops, rt[0]


def random_tuples(base_ops, base_rt, n, m, T, seed, absent=None, invalid_frac=0.0):
    """T insertion tuples against one base partial solution.

    Tuple = (c, vD, pD, vP, pP): insert D_c before index pD of route vD, then
    P_c before index pP of route vP counted after the drop insertion.  ``absent``
    lists customers missing from the base (default: those whose ops are not in
    it).  A fraction ``invalid_frac`` is drawn without the position rules to
    exercise the BAD_TUPLE path.  Returns a structured array with fields
    c (u2), vD (u1), vP (u1), pD (u2), pP (u2).
    """
    g = rng(seed)
    lens = np.diff(np.concatenate([[0], base_rt.astype(np.int64)]))
    if absent is None:
        present = set(int(x) >> 1 for x in base_ops[: int(base_rt[-1])])
        absent = [c for c in range(1, n + 1) if c not in present]
    absent = np.asarray(absent, dtype=np.int64)
    out = np.zeros(T, dtype=TUPLE_DTYPE)
    for i in range(T):
        c = int(absent[g.integers(0, len(absent))])
        vD = int(g.integers(0, m))
        vP = int(g.integers(0, m))
        pD = int(g.integers(0, lens[vD] + 1))
        if vP == vD:
            pP = int(g.integers(pD + 1, lens[vD] + 2))
        else:
            pP = int(g.integers(0, lens[vP] + 1))
        if invalid_frac and g.random() < invalid_frac:
            kind = int(g.integers(0, 4))
            if kind == 0:
                pD = int(lens[vD]) + 1 + int(g.integers(0, 3))
            elif kind == 1 and vP == vD:
                pP = int(g.integers(0, pD + 1))
            elif kind == 2:
                vD = m + int(g.integers(0, 3))
            else:
                c = int(g.integers(n + 1, n + 10))
        out[i] = (c, vD, vP, pD, pP)
    return out


TUPLE_DTYPE = np.dtype([("c", "<u2"), ("vD", "u1"), ("vP", "u1"), ("pD", "<u2"), ("pP", "<u2")])


def random_keys(B, n, seed, special=False):
    """BRKGA random keys: priorities and vehicle hints, each [B, 2n] fp32 in
    [0, 1).  With ``special`` some rows carry ties, 0.0, -0.0, the largest
    float below 1 and (in the last row) a NaN and a 1.0."""
    g = rng(seed)
    prio = g.random((B, 2 * n), dtype=np.float32)
    hint = g.random((B, 2 * n), dtype=np.float32)
    if special and B >= 4:
        prio[0, : 2 * n // 2] = 0.5                      # many exact ties
        prio[1, ::3] = 0.0
        prio[1, 1::3] = -0.0
        prio[2, :] = np.float32(0.99999994)
        hint[2, ::2] = np.float32(0.99999994)
        hint[3, :] = 0.0
        prio[B - 1, 0] = np.nan
        hint[B - 1, 1] = 1.0
    return prio, hint


def relabel_candidates(ops, rt_end, n, B, seed):
    """B candidates made from a pool by renaming customers: candidate i takes
    pool row i % len(pool) and applies a fresh random permutation sigma of
    1..n to every op (c -> sigma(c), op type kept).  Route shapes, op types
    and the drop-before-pickup structure are kept, so load feasibility and
    freedom from wait cycles carry over, while the visited customers (and so
    the travel times and the makespan) change."""
    g = rng(seed)
    P = ops.shape[0]
    out = np.empty((B, ops.shape[1]), dtype=np.uint16)
    rt = np.empty((B, rt_end.shape[1]), dtype=np.uint16)
    step = 4096
    for s in range(0, B, step):
        b = min(step, B - s)
        src = (np.arange(s, s + b) % P)
        sigma = np.argsort(g.random((b, n)), axis=1) + 1          # sigma[c-1] in 1..n
        sigma = np.concatenate([np.zeros((b, 1), np.int64), sigma], axis=1)
        o = ops[src].astype(np.int64)
        c = np.take_along_axis(sigma, o >> 1, axis=1)
        out[s:s + b] = ((c << 1) | (o & 1)).astype(np.uint16)
        rt[s:s + b] = rt_end[src]
    return out, rt


BATCH_RULES = ("base", "2x", "5x", "1R10", "1R20")


def batched_instances(count: int = 256, seed: int = 4000, n_min: int = 17, n_max: int = 1000):
    """Instances of uneven size for the batched form: n = round(exp U[ln
    n_min, ln n_max]), m = ceil(n / 100) + 1, R = floor(n / 10), k ~
    U_int[5, 10], processing rules cycled base/2x/5x/1R10/1R20; instance i
    is generated with seed + i."""
    g = rng(seed)
    out = []
    for i in range(count):
        n = int(round(np.exp(g.uniform(np.log(n_min), np.log(n_max)))))
        m = -(-n // 100) + 1
        R = max(1, n // 10)
        k = int(g.integers(5, 11))
        out.append(make_instance(n, m, k, R, BATCH_RULES[i % len(BATCH_RULES)], seed=seed + i))
    return out
