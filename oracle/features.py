"""Oracle for the learned destroy proposal's per-customer features (test
infrastructure only).

The paper leaves learned destroy operators to future work (Section 7.4); the
feature set is this project's.  For a complete, feasible solution S with its
earliest-start schedule (Section 3, Eq. 7-12) every customer c gets 64 fp32
features: 32 base features and the same 32 gated by "c's drop or pickup
vehicle finishes at the makespan" (feature 32 + i = feature i times that
indicator).  Every feature is one fp32 operation on values exact in fp32 or
an integer converted once (round to nearest), so any implementation that
performs the same operations gets the same bits.

Notation: z makespan, dbar = max(1, floor(sum_i d[0][i] / n)); for the drop
(D) and pickup (P) of c: vehicle v, position i in its route (0-based), route
length L, start time t (= departure; service is instantaneous), arrival a,
neighbours prev / next in the route (the depot 0 at either end), route finish
f = last op's time + travel home; walk = #drops - #pickups over the route's
ops up to and including the op; g = z - z(S without c).

 0  1                       16 d(prevD,c)/dbar
 1  d(0,c)/dbar             17 d(c,nextD)/dbar
 2  p_c/dbar                18 d(prevP,c)/dbar
 3  tD/z                    19 d(c,nextP)/dbar
 4  tP/z                    20 g/z
 5  (tP - tD - p_c)/z       21 walkD/k
 6  (tP - aP)/z             22 walkP/k
 7  [vD = vP]               23 (LD m)/(2n)
 8  iD/LD                   24 (LP m)/(2n)
 9  iP/LP                   25 (iP - iD)/LD if vD = vP else 0
10  fD/z                    26 nearest other node's distance / dbar
11  fP/z                    27 (sum of the 4 nearest other nodes' distances)/(4 dbar)
12  [fD = z]                28 (z - fD)/z
13  [fP = z]                29 (z - fP)/z
14  (d(prevD,c) + d(c,nextD) - d(prevD,nextD))/dbar      30 [g > 0]
15  the same for P                                       31 p_c/(tP - tD) (1 if tP = tD)
("other nodes" are all nodes but c, the depot included; fewer than 4 others:
all of them, divided by their count times dbar.)
"""
from __future__ import annotations

import numpy as np

from . import eval_one

NF = 64


def f32(x):
    return np.float32(x)


def div(a, b):
    """One correctly rounded fp32 division of two values converted to fp32."""
    return np.float32(np.float32(a) / np.float32(b))


def dbar_of(inst):
    return max(1, int(np.asarray(inst.d)[0, 1:].sum()) // inst.n)


def static_features(inst):
    """Per-customer instance features 26, 27 (independent of the solution)."""
    d = np.asarray(inst.d, np.int64)
    n = inst.n
    db = dbar_of(inst)
    out = np.zeros((n + 1, 2), np.float32)
    for c in range(1, n + 1):
        others = np.delete(d[c], c)
        srt = np.sort(others)
        cnt = min(4, len(srt))
        out[c, 0] = div(srt[0], db)
        out[c, 1] = div(int(srt[:cnt].sum()), cnt * db)
    return out


def removal_gains(inst, ops, rt_end, z):
    """g[c] = z - makespan of the solution with c's two ops taken out."""
    n, m = inst.n, inst.m
    ops = np.asarray(ops, np.uint16)
    rt_end = np.asarray(rt_end, np.int64)
    g = np.zeros(n + 1, np.int64)
    for c in range(1, n + 1):
        keep = (ops >> 1) != c
        new_rt = np.array([keep[:e].sum() for e in rt_end], np.uint16)
        zc, st = eval_one(inst, ops[keep], new_rt, allow_partial=True)
        assert st == 0
        g[c] = z - zc
    return g


def customer_features(inst, ops, rt_end):
    """[n + 1, 64] float32 features (row 0 is zero) of a complete feasible
    solution."""
    n, m, k = inst.n, inst.m, inst.k
    d = np.asarray(inst.d, np.int64)
    p = np.asarray(inst.p, np.int64)
    ops = np.asarray(ops, np.uint16)
    rt_end = np.asarray(rt_end, np.int64)
    z, st, times = eval_one(inst, ops, rt_end, times=True)
    assert st == 0 and z > 0
    db = dbar_of(inst)
    stat = static_features(inst)
    gain = removal_gains(inst, ops, rt_end, z)
    starts = np.concatenate([[0], rt_end[:-1]])
    info = {}
    finish = np.zeros(m, np.int64)
    for v in range(m):
        s, e = int(starts[v]), int(rt_end[v])
        route = [int(x) for x in ops[s:e]]
        L = e - s
        if L:
            finish[v] = times[e - 1] + d[route[-1] >> 1, 0]
        walk = 0
        for i, cd in enumerate(route):
            c, isP = cd >> 1, cd & 1
            walk += -1 if isP else 1
            prev = route[i - 1] >> 1 if i > 0 else 0
            nxt = route[i + 1] >> 1 if i + 1 < L else 0
            t_prev = times[s + i - 1] if i > 0 else 0
            info[(c, isP)] = dict(v=v, i=i, L=L, t=int(times[s + i]), a=int(t_prev + d[prev, c]),
                                  prev=prev, next=nxt, walk=walk)
    F = np.zeros((n + 1, NF), np.float32)
    for c in range(1, n + 1):
        D, P = info[(c, 0)], info[(c, 1)]
        fD, fP = finish[D["v"]], finish[P["v"]]
        same = D["v"] == P["v"]
        b = np.zeros(32, np.float32)
        b[0] = 1.0
        b[1] = div(d[0, c], db)
        b[2] = div(p[c], db)
        b[3] = div(D["t"], z)
        b[4] = div(P["t"], z)
        b[5] = div(P["t"] - D["t"] - p[c], z)
        b[6] = div(P["t"] - P["a"], z)
        b[7] = 1.0 if same else 0.0
        b[8] = div(D["i"], D["L"])
        b[9] = div(P["i"], P["L"])
        b[10] = div(fD, z)
        b[11] = div(fP, z)
        b[12] = 1.0 if fD == z else 0.0
        b[13] = 1.0 if fP == z else 0.0
        b[14] = div(d[D["prev"], c] + d[c, D["next"]] - d[D["prev"], D["next"]], db)
        b[15] = div(d[P["prev"], c] + d[c, P["next"]] - d[P["prev"], P["next"]], db)
        b[16] = div(d[D["prev"], c], db)
        b[17] = div(d[c, D["next"]], db)
        b[18] = div(d[P["prev"], c], db)
        b[19] = div(d[c, P["next"]], db)
        b[20] = div(gain[c], z)
        b[21] = div(D["walk"], k)
        b[22] = div(P["walk"], k)
        b[23] = div(D["L"] * m, 2 * n)
        b[24] = div(P["L"] * m, 2 * n)
        b[25] = div(P["i"] - D["i"], D["L"]) if same else 0.0
        b[26] = stat[c, 0]
        b[27] = stat[c, 1]
        b[28] = div(z - fD, z)
        b[29] = div(z - fP, z)
        b[30] = 1.0 if gain[c] > 0 else 0.0
        b[31] = div(p[c], P["t"] - D["t"]) if P["t"] > D["t"] else 1.0
        gate = np.float32(1.0 if (fD == z or fP == z) else 0.0)
        F[c, :32] = b
        F[c, 32:] = b * gate
    return F
