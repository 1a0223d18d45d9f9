"""Candidate families for the parity tests (shared by CPU and GPU tests).

Everything here is built from synth's seeded generators plus structural
mutations; no expected value is computed here."""
import numpy as np

import synth


def flat(ops2d, rt2d):
    """[B, L] / [B, m] blocks -> flat arrays with offsets."""
    B = ops2d.shape[0]
    L = ops2d.shape[1]
    m = rt2d.shape[1]
    return (ops2d.reshape(-1).copy(), np.arange(B, dtype=np.int64) * L,
            rt2d.reshape(-1).copy(), np.arange(B, dtype=np.int64) * m)


def mutate(inst, ops, rt, seed, count):
    """Adversarial variants of feasible candidates: deadlocks (a pickup moved in
    front of its drop, swapped ops across routes), cover errors (duplicate op,
    missing op, customer id 0 or > n), bad route ends, empty routes."""
    g = synth.rng(seed)
    n, m = inst.n, inst.m
    out_ops, out_rt = [], []
    for i in range(count):
        b = int(g.integers(0, len(ops)))
        o = ops[b].astype(np.int64).copy()
        r = rt[b].astype(np.int64).copy()
        kind = int(g.integers(0, 9))
        L = len(o)
        if kind == 0:        # move a pickup to the front of its route
            js = [j for j in range(L) if o[j] & 1]
            j = js[int(g.integers(0, len(js)))]
            v = int(np.searchsorted(r, j, side="right"))
            s = 0 if v == 0 else int(r[v - 1])
            x = o[j]
            o = np.concatenate([o[:s], [x], np.delete(o[s:], j - s)])
        elif kind == 1:      # swap two random ops (often across routes)
            a, c = g.integers(0, L, size=2)
            o[a], o[c] = o[c], o[a]
        elif kind == 2:      # duplicate op
            a, c = g.integers(0, L, size=2)
            o[a] = o[c]
        elif kind == 3:      # customer id out of range
            o[int(g.integers(0, L))] = (n + 1 + int(g.integers(0, 5))) << 1
        elif kind == 4:      # customer 0 (the depot) as an op
            o[int(g.integers(0, L))] = int(g.integers(0, 2))
        elif kind == 5 and m > 1:   # non-monotone route ends
            v = int(g.integers(0, m - 1))
            r[v] = r[v + 1] + 1 if r[v + 1] + 1 <= L else r[v]
            if r[v] <= r[v + 1]:
                r[v], r[v + 1] = r[v + 1], max(0, r[v] - 1)
        elif kind == 6:      # route ends past 2n
            r[-1] = L + 1 + int(g.integers(0, 3))
        elif kind == 7:      # move all ops to one vehicle (other routes empty)
            v = int(g.integers(0, m))
            r[:v] = 0
            r[v:] = L
        else:                # reverse one route (pickups before drops)
            v = int(g.integers(0, m))
            s = 0 if v == 0 else int(r[v - 1])
            o[s:int(r[v])] = o[s:int(r[v])][::-1]
        out_ops.append(np.clip(o, 0, 65535).astype(np.uint16))
        out_rt.append(np.clip(r, 0, 65535).astype(np.uint16))
    return np.stack(out_ops), np.stack(out_rt)


def destroy(inst, ops, rt, seed, q):
    """Remove q random customers from each candidate (partial solutions):
    returns flat ops, op_off, rt_end [B, m]."""
    g = synth.rng(seed)
    n, m = inst.n, inst.m
    fo, off, frt = [], [], []
    cur = 0
    for b in range(len(ops)):
        gone = set(int(c) for c in g.choice(np.arange(1, n + 1), size=q, replace=False))
        s = 0
        ends = []
        kept_all = []
        for v in range(m):
            e = int(rt[b][v])
            kept = [x for x in ops[b][s:e] if (int(x) >> 1) not in gone]
            kept_all += kept
            ends.append(len(kept_all))
            s = e
        off.append(cur)
        fo += kept_all
        frt.append(ends)
        cur += len(kept_all)
    return (np.array(fo, np.uint16), np.array(off, np.int64), np.array(frt, np.uint16))
