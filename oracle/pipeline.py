"""The two-stage method on the CPU oracle: ALNS, then BRKGA warm-started from
its incumbent (Section 4 opening, Section 4.4.4) -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU leg use it.  Every
stage is a call into the oracle's C core; this module only sequences them:

  start   the paper's initial solution (Section 4.2: sweep construction,
          then refinement rounds of the local searches until a round
          improves nothing), or a given solution;
  ALNS    `chains` chains of Algorithm 1 from the start; the incumbent is
          the best solution of any chain;
  seeds   the incumbent and the NN, load-balanced and SPT constructions
          (Section 4.4.4), encoded and perturbed into 14 + 2 + 2 + 2 = 20
          warm chromosomes cycled through the first floor(0.15 Np) slots,
          the rest fresh random keys;
  BRKGA   `gens` generations of decode + evolve (Section 4.4.3, Table 3),
          keeping the best decoded chromosome (lowest fitness, earliest
          generation, then lowest index); by default the decoder gives each
          op to its hint vehicle whenever that vehicle can take it (Section
          4.4.1), so the encoded incumbent decodes close to itself;
  result  the better of the ALNS incumbent and BRKGA's best complete
          schedule (the pipeline never discards the incumbent).
"""
from __future__ import annotations

import time

import numpy as np

from . import (CONS_LB, CONS_NN, CONS_SPT, CONS_SWEEP, DECODE_HINT_FIRST, alns_run, brkga_evolve, brkga_sizes,
               brkga_warm_start_multi, construct, decode, decode_batch, eval_one, refine, rho_threshold)

WARM_VARIANTS = (14, 2, 2, 2)      # ALNS incumbent, NN, LB, SPT


def paper_start(inst, ls_budget=16384):
    """Sweep construction, then refinement (Section 4.2): (ops, rt_end, z)."""
    o, r = construct(inst, CONS_SWEEP)
    _, z, o, r = refine(inst, o, r, budget=ls_budget)
    return o, r, int(z)


def warm_population(inst, alns_ops, alns_rt, Np, seed):
    """The initial population: 20 warm chromosomes from the ALNS incumbent
    and the three construction seeds in floor(0.15 Np) slots, the rest
    fresh."""
    sources = [(alns_ops, alns_rt)] + [construct(inst, h) for h in (CONS_NN, CONS_LB, CONS_SPT)]
    return brkga_warm_start_multi(inst, sources, list(WARM_VARIANTS), Np, int(0.15 * Np), seed)


def brkga_run(inst, prio, hint, gens, seed, rho_e=0.7, flags=DECODE_HINT_FIRST):
    """`gens` generations from the given population; returns (best fitness,
    best prio row, best hint row, fitness history of the best)."""
    Np = prio.shape[0]
    ne, nm = brkga_sizes(Np)
    thr = rho_threshold(rho_e)
    best_f, bp, bh, hist = np.iinfo(np.int64).max, None, None, []
    for gen in range(gens):
        fit = decode_batch(inst, prio, hint, flags=flags)[0]
        i = int(np.argmin(fit))
        if fit[i] < best_f:
            best_f, bp, bh = int(fit[i]), prio[i].copy(), hint[i].copy()
        hist.append(best_f)
        prio, hint, _ = brkga_evolve(prio, hint, fit, ne, nm, thr, seed, gen)
    return best_f, bp, bh, hist


def run(inst, alns_params, chains, iterations, alns_seed, Np, gens, brkga_seed, start=None, ls_budget=16384,
        decode_flags=DECODE_HINT_FIRST):
    """The pipeline; start = (ops, rt_end) or None for the paper's start.
    Returns a dict with each stage's result and wall time."""
    t0 = time.perf_counter()
    if start is None:
        s_ops, s_rt, z_start = paper_start(inst, ls_budget)
    else:
        s_ops, s_rt = start
        z_start = int(eval_one(inst, s_ops, s_rt)[0])
    t1 = time.perf_counter()
    a = alns_run(inst, alns_params, chains, iterations, alns_seed, s_ops, s_rt)
    c = int(np.argmin(a["best_mk"]))
    z_alns = int(a["best_mk"][c])
    a_rt = a["best_rt"][c]
    a_ops = a["best_ops"][c][:int(a_rt[-1])]
    t2 = time.perf_counter()
    prio, hint = warm_population(inst, a_ops, a_rt, Np, brkga_seed)
    bf, bp, bh, hist = brkga_run(inst, prio, hint, gens, brkga_seed, flags=decode_flags)
    d = decode(inst, bp, bh, want_ops=True, flags=decode_flags)
    t3 = time.perf_counter()
    z_brkga = int(d["makespan"]) if d["unscheduled"] == 0 and d["status"] == 0 else None
    if z_brkga is not None and z_brkga < z_alns:
        best, b_ops, b_rt = z_brkga, d["ops"], d["rt_end"]
    else:
        best, b_ops, b_rt = z_alns, a_ops, a_rt
    return dict(z_start=z_start, z_alns=z_alns, alns_ops=a_ops, alns_rt=a_rt, warm_prio=prio, warm_hint=hint,
                brkga_fitness=bf, brkga_prio=bp, brkga_hint=bh, brkga_history=hist, z_brkga=z_brkga,
                best=best, best_ops=b_ops, best_rt=b_rt, start_seconds=t1 - t0, alns_seconds=t2 - t1,
                brkga_seconds=t3 - t2)
