"""The two-stage method (Section 4 opening; Section 4.4.4): ALNS, then BRKGA
warm-started from its incumbent, as a sequence of library calls.

Every step runs in the library's kernels; this module only orders the calls
and moves device tensors between them:

  start   the paper's initial solution (Section 4.2): vrprpd_construct with
          the sweep heuristic, then alns_refine on a one-chain state (the
          refinement is deterministic, so one chain per instance suffices);
  ALNS    alns_step on `chains` chains per instance from the start;
          the incumbent is the best solution of any chain (alns_get_best);
  seeds   brkga_warm_start_multi from the incumbent and the NN, load-balanced
          and SPT constructions: 14 + 2 + 2 + 2 = 20 warm chromosomes cycled
          through the first floor(0.15 Np) slots, the rest fresh keys;
  BRKGA   brkga_state generations (decode + evolve), with the decoder's
          hint-first vehicle rule by default (the hint is the vehicle unless it
          cannot take the op: Section 4.4.1), under which the encoded
          incumbent decodes close to itself;
  result  the better of the incumbent and BRKGA's best complete schedule.
"""
from __future__ import annotations

import time

import torch

from . import _lib as L

WARM_VARIANTS = (14, 2, 2, 2)      # ALNS incumbent, NN, LB, SPT


def paper_start(S: L.InstanceSet, params, seed=0, stream=None):
    """Sweep construction and refinement for every instance of S: returns
    (ops [I][2 n_max], rt_end [I][m_max], refinement rounds)."""
    ops, rt = L.vrprpd_construct(S, L.CONS_SWEEP, stream=stream)
    ids = list(range(S.num_inst))
    one = L.AlnsState(S, ids, 1, params, seed, ops, rt, stream=stream)
    rounds = one.refine(stream=stream)
    best = [one.best(i, stream=stream) for i in ids]
    one.close()
    return torch.stack([b[1] for b in best]), torch.stack([b[2] for b in best]), rounds


def warm_population(S: L.InstanceSet, inst, ops, rt_end, Np, seed, stream=None):
    """The initial population of instance `inst` from its ALNS incumbent
    (ops [>= 2n], rt_end [>= m] device uint16) and the three construction
    seeds; returns (prio, hint) [Np][2 n_max]."""
    idx = torch.tensor([inst], dtype=torch.int32, device=ops.device)
    srcs_o, srcs_r = [ops[: 2 * S.n_max]], [rt_end[: S.m_max]]
    for h in (L.CONS_NN, L.CONS_LB, L.CONS_SPT):
        o, r = L.vrprpd_construct(S, h, inst=idx, stream=stream)
        srcs_o.append(o[0])
        srcs_r.append(r[0])
    so = torch.zeros((4, 2 * S.n_max), dtype=torch.uint16, device=ops.device)
    sr = torch.zeros((4, S.m_max), dtype=torch.uint16, device=ops.device)
    for i, (o, r) in enumerate(zip(srcs_o, srcs_r)):
        so[i, : o.numel()] = o
        sr[i, : r.numel()] = r
    return L.brkga_warm_start_multi(S, so, sr, list(WARM_VARIANTS), Np, int(0.15 * Np), seed, inst=inst,
                                    stride=2 * S.n_max, stream=stream)


def run(S: L.InstanceSet, inst, params, chains, iterations, alns_seed, Np, gens, brkga_seed, start=None,
        decode_flags=L.DECODE_HINT_FIRST, rho_e=0.7, stream=None):
    """The pipeline on instance `inst` of S (a set holding only that
    instance's size as its largest).  start: (ops, rt_end) device tensors, or
    None for the paper's start.  Returns a dict of the stages' results (device
    tensors for solutions and chromosomes) and their wall times (each stage
    ends with a device synchronisation)."""
    t0 = time.perf_counter()
    if start is None:
        s_ops, s_rt, rounds = paper_start(S, params, alns_seed, stream=stream)
        s_ops, s_rt = s_ops[inst : inst + 1], s_rt[inst : inst + 1]
    else:
        s_ops, s_rt = start[0].reshape(1, -1), start[1].reshape(1, -1)
        rounds = 0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = L.AlnsState(S, [inst], chains, params, alns_seed, s_ops, s_rt, stream=stream)
    z_start = int(st.state()["zb"][0])
    st.step(iterations, stream=stream)
    z_alns, a_ops, a_rt = st.best(-1, stream=stream)
    st.close()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    prio, hint = warm_population(S, inst, a_ops, a_rt, Np, brkga_seed, stream=stream)
    ne, nm = int(0.15 * Np), int(0.15 * Np)
    pop = L.BrkgaState(S, [inst], Np, ne, nm, rho_e, brkga_seed, prio, hint, stream=stream,
                       decode_flags=decode_flags)
    pop.step(gens, stream=stream)
    bf, bp, bh = pop.best(stream=stream)
    pop.close()
    d = L.brkga_decode_eval(S, bp[:1], bh[:1], inst=torch.tensor([inst], dtype=torch.int32, device=bp.device),
                            want_ops=True, stream=stream, flags=decode_flags)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    complete = int(d["unscheduled"][0]) == 0 and int(d["status"][0]) == 0
    z_brkga = int(d["makespan"][0]) if complete else None
    if z_brkga is not None and z_brkga < z_alns:
        best, b_ops, b_rt = z_brkga, d["ops"][0], d["rt_end"][0]
    else:
        best, b_ops, b_rt = z_alns, a_ops, a_rt
    return dict(z_start=z_start, refine_rounds=rounds, z_alns=int(z_alns), alns_ops=a_ops, alns_rt=a_rt,
                warm_prio=prio, warm_hint=hint, brkga_fitness=int(bf[0]), brkga_prio=bp[0], brkga_hint=bh[0],
                z_brkga=z_brkga, best=int(best), best_ops=b_ops, best_rt=b_rt, start_seconds=t1 - t0,
                alns_seconds=t2 - t1, brkga_seconds=t3 - t2)
