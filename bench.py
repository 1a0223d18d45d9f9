#!/usr/bin/env python3
"""Exact VRP-RPD makespan evaluation on one MI355X: throughput of the whole
hot path at n = 1000.

Workload (the full-scale configuration): one instance with n = 1000 customers,
m = 10 vehicles, capacity k = 10, R = 100 resources, processing times
U_int[1,20] * floor(mean depot distance / 10); synthetic TSPLIB-shaped points
(integer, uniform in [0,1000]^2, EUC_2D rounding).  One step runs every stage
of the path once on inputs already resident in HBM:
  1. vrprpd_eval         65,536 explicit candidate solutions
  2. vrprpd_insert_scan  16,384 insertion tuples (one ALNS iteration's budget)
                         for 37 removed customers of a destroyed solution
  3. brkga_decode_eval   a population of 4,096 chromosomes (2n keys + 2n hints)
     brkga_evolve        one generation (614 elites, 614 mutants, rho_e = 0.7)
  4. alns_step           one ALNS iteration of 32 chains (budget 16,384 tuples)
`value` is the evaluator's rate: complete n = 1000 candidates evaluated per
second by the vrprpd_eval launches of the timed steps (HIP events on their
stream); `all_evals_per_s` counts every exact schedule evaluation of the step
(explicit candidates, tuples, decoded chromosomes and the ALNS iteration's
tuples and removal gains) per second of step wall time.  In the timed steps
the ALNS iteration runs on a second stream, concurrently with stages 1, 2 and
3 on the first (the stages share no data; the streams join at the end of each
step); `components_ms` times the stages one after another in as many further
steps.  `roofline` is the evaluation kernel's (HBM bytes, with the measured
L2 random-read ceiling as the secondary bound), `roofline_components` the
scan's (LDS) and the decoder's (HBM).

Also reported, each as its own phase (--phases): races of the two-stage method
to the oracle's best makespans (16, 100 and 1000 customers), the smaller
workloads (16 and 100 customers), the construction heuristics, the batched and
learned forms, the processing-time hypothesis sweep, and the CPU baseline (the
oracle on one core and on the process's share of cores, on a bounded sample).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact makespan evals/sec at n=1000; wall time to oracle-best makespan"
HBM_PEAK = 8.0e12   # MI355X HBM3E, bytes/s
LDS_PEAK = 256 * 128 * 2.4e9   # 256 CUs x 128 B/clk of LDS x 2.4 GHz = 78.6 TB/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# the evaluation kernel of each form and the rocprofv3 summary of its HBM traffic
EVAL_KERNELS = ("eval_kernel", "eval_live_kernel")
EVAL_SOURCES = ["paper_2602_23685_amd/csrc/eval.hip", "paper_2602_23685_amd/csrc/sweep.h",
                "paper_2602_23685_amd/csrc/common.h"]


def measured_traffic(form):
    """HBM bytes per launch of the evaluation kernel of `form` (0 staged,
    1 live legs) from the committed rocprofv3 counter summary, or None when
    the kernel sources changed since it was taken."""
    import hashlib
    try:
        txt = open(os.path.join(ROOT, "profiles", f"{EVAL_KERNELS[form]}_n1000_pmc_traffic.md")).read()
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in txt.splitlines() if l.startswith(("traffic_bytes", "kernel_sources")))
    h = hashlib.sha256()
    for src in EVAL_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if vals.get("kernel_sources_sha256", "").strip() != h.hexdigest():
        return None
    return float(vals["traffic_bytes_per_launch"])


def make_workload(seed=3003, B=65536, T=16384, Np=4096):
    import synth
    inst = synth.make_instance(1000, 10, 10, 100, "1R20d10", seed=seed)
    pool_ops, pool_rt = synth.random_candidates(inst, 1024, seed=seed + 1)
    ops, rt = synth.relabel_candidates(pool_ops, pool_rt, inst.n, B, seed=seed + 2)
    # a destroyed solution: 37 customers removed from a feasible candidate
    g = synth.rng(seed + 3)
    removed = sorted(int(c) for c in g.choice(np.arange(1, inst.n + 1), size=37, replace=False))
    gone = set(removed)
    base_routes = [[x for x in r if x[0] not in gone] for r in synth.unpack_candidate(pool_ops[0], pool_rt[0])]
    bops, _, brt = synth.pack_candidates([base_routes], inst.m)
    tuples = synth.random_tuples(bops, brt[0], inst.n, inst.m, T, seed=seed + 4, absent=removed)
    order = np.argsort(tuples["c"], kind="stable")
    tuples = tuples[order]
    cs = tuples["c"].astype(np.int64)
    seg_off = np.concatenate([[0], np.nonzero(np.diff(cs))[0] + 1, [T]]).astype(np.int64)
    prio, hint = synth.random_keys(Np, inst.n, seed=seed + 5)
    return dict(inst=inst, ops=ops, rt=rt, bops=bops, brt=brt[0], tuples=tuples, seg_off=seg_off,
                prio=prio, hint=hint, pool_ops=pool_ops, pool_rt=pool_rt)


def cpu_cores():
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (the share of the host given to it)."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_baseline(inst, ops, rt, seconds):
    """The oracle's evaluator on the host: single-threaded, then one thread
    per core over disjoint slices of the same candidates (the C oracle runs
    without the interpreter lock).  Bounded to about `seconds` each."""
    import concurrent.futures as cf

    import oracle
    oracle.lib()
    chunk = 256
    done, t0, i = 0, time.perf_counter(), 0
    while time.perf_counter() - t0 < seconds and i < len(ops):
        oracle.eval_batch(inst, ops[i:i + chunk], rt[i:i + chunk])
        done += min(chunk, len(ops) - i)
        i += chunk
    dt1 = time.perf_counter() - t0
    one = done / dt1
    cores = cpu_cores()
    # every thread starts at its own slice and walks on (wrapping around the
    # candidates) for about `seconds` of work at the single-core rate
    per = max(chunk, int(one * seconds / chunk) * chunk)
    span = (len(ops) // cores) // chunk * chunk

    def work(tid):
        for j in range(per // chunk):
            lo = (tid * span + j * chunk) % (len(ops) - chunk + 1)
            oracle.eval_batch(inst, ops[lo:lo + chunk], rt[lo:lo + chunk])
        return per

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        total = sum(ex.map(work, range(cores)))
    dtn = time.perf_counter() - t0
    return {"value": total / dtn, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "value_1core": one,
            "sample": f"single-threaded: first {done} of the 65,536 explicit candidates at n=1000 in {dt1:.1f} s; "
                      f"{cores} threads: {per} candidates each, from disjoint starting slices ({total} in "
                      f"all) in {dtn:.1f} s"}


def paper_start_oracle(oracle, inst, ls_budget=16384):
    """The paper's initial solution on the CPU oracle: sweep construction,
    then refinement rounds (Section 4.2, initial solution)."""
    o, r = oracle.construct(inst, oracle.CONS_SWEEP)
    _, z, o, r = oracle.refine(inst, o, r, budget=ls_budget)
    return o, r, z


def paper_start_gpu(P, S, chains, prm, seed):
    """The same on the GPU: vrprpd_construct, then alns_refine on a one-chain
    state per instance (construction and refinement are deterministic, so
    every chain would refine the same solution), then the ALNS state of all
    chains from the refined solutions; returns it and the refinement rounds."""
    import torch
    ops, rt = P.vrprpd_construct(S, P.CONS_SWEEP)
    ids = list(range(S.num_inst))
    one = P.AlnsState(S, ids, 1, prm, seed, ops, rt)
    rounds = one.refine()
    best = [one.best(i) for i in ids]
    one.close()
    r_ops = torch.stack([b[1] for b in best])
    r_rt = torch.stack([b[2] for b in best])
    return P.AlnsState(S, ids, chains, prm, seed, r_ops, r_rt), rounds


def time_to_oracle_best(P, torch, iters_oracle=2000, chains=32, budget_iters=4000):
    """Small-instance race: the oracle's ALNS (one chain, 2000 iterations,
    every slot pair priced, from the paper's initial solution) sets the
    target; GPU ALNS with 32 chains, from the same construction and
    refinement done on the GPU, runs until its best reaches it.  Both times
    include the construction and refinement."""
    import oracle
    import synth
    inst = synth.make_instance(16, 2, 2, 4, "base", seed=1001)
    t0 = time.perf_counter()
    ops, rt, _ = paper_start_oracle(oracle, inst)
    ref = oracle.alns_run(inst, oracle.alns_params(), 1, iters_oracle, 2024, ops, rt)
    t_oracle = time.perf_counter() - t0
    z_target = int(ref["best_mk"][0])
    S = P.InstanceSet([inst])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, _ = paper_start_gpu(P, S, chains, P.alns_params(), 99)
    done, best, chunk = 0, int(st.state()["zb"].min()), 25
    while best > z_target and done < budget_iters:
        st.step(chunk)
        done += chunk
        best = int(st.state()["zb"].min())
    t_gpu = time.perf_counter() - t0
    st.close()
    return {"config": "n=16 customers, m=2, k=2, R=4, base rule; start: sweep construction + refinement",
            "z_oracle": z_target, "oracle_seconds": t_oracle, "oracle_iterations": iters_oracle,
            "oracle_chains": 1, "gpu_seconds": t_gpu, "gpu_iterations": done, "gpu_chains": chains,
            "gpu_best": best, "reached": bool(best <= z_target)}


TARGETS = os.path.join(ROOT, "tests", "golden", "oracle_targets.json")


def race_to_oracle(P, torch, chains=32, limit_s=60.0, alns_chunk=10, brkga_chunk=2):
    """The two-stage method on the GPU against the best makespan the oracle's
    two-stage method reached on the same instance from the same start
    (stored by tests/golden/make_oracle_targets.py: one ALNS chain, then
    BRKGA warm-started from its incumbent): wall time until the GPU's best is
    at least as good.  The GPU runs 32 ALNS chains for the oracle's iteration
    budget (checked every 10 iterations), then BRKGA with the oracle's
    population from its incumbent (checked every 2 generations) until the
    target or the time limit.  Start "paper": the paper's construction and
    refinement, on the GPU inside the timed region; "round_robin": a weak
    start that leaves the work to the search."""
    import synth
    from paper_2602_23685_amd import pipeline
    try:
        targets = json.load(open(TARGETS))
    except OSError:
        return None
    out = {}
    for name, c in targets.items():
        inst = synth.make_instance(c["n"], c["m"], c["k"], c["R"], c["rule"], seed=c["seed"])
        S = P.InstanceSet([inst])
        prm = P.alns_params(tuple_budget=c["budget"])
        target = c["z_oracle"]
        if c["start"] == "round_robin":
            ops, rt = synth.round_robin_solution(inst, vehicles=min(c["m"], c["R"]))
            d_ops, d_rt = torch.from_numpy(ops).cuda()[None], torch.from_numpy(rt).cuda()[None]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        rounds = 0
        if c["start"] == "paper":
            d_ops, d_rt, rounds = pipeline.paper_start(S, prm, 99)
        st = P.AlnsState(S, [0], chains, prm, 99, d_ops, d_rt)
        best = int(st.state()["zb"].min())
        t_start, hist, reached_at, stage = now(), [], None, "start"
        if best <= target:
            reached_at = t_start
        it = 0
        while reached_at is None and it < c["iterations"] and now() < limit_s:
            st.step(alns_chunk)
            it += alns_chunk
            best = int(st.state()["zb"].min())
            hist.append(("alns", it, round(now(), 4), best))
            if best <= target:
                reached_at, stage = now(), "alns"
        z_alns = best
        gens = 0
        if reached_at is None:
            _, a_ops, a_rt = st.best(-1)
            prio, hint = pipeline.warm_population(S, 0, a_ops, a_rt, c["Np"], c["brkga_seed"])
            ne = nm = int(0.15 * c["Np"])
            pop = P.BrkgaState(S, [0], c["Np"], ne, nm, 0.7, c["brkga_seed"], prio, hint,
                               decode_flags=P.DECODE_HINT_FIRST)
            while reached_at is None and now() < limit_s:
                pop.step(brkga_chunk)
                gens += brkga_chunk
                f = int(pop.best()[0][0])            # fitness = makespan for a complete schedule (< 10^6)
                best = min(best, f)
                hist.append(("brkga", gens, round(now(), 4), best))
                if best <= target:
                    reached_at, stage = now(), "brkga"
            pop.close()
        st.close()
        out[name] = {"n": c["n"], "m": c["m"], "k": c["k"], "R": c["R"], "rule": c["rule"], "start": c["start"],
                     "tuple_budget": c["budget"], "z_start": c["z_refined"], "oracle_z_alns": c["z_alns"],
                     "oracle_z_brkga": c["z_brkga"], "z_oracle": target,
                     "oracle_protocol": f"1 chain x {c['iterations']} ALNS iterations, then BRKGA "
                                        f"{c['Np']} x {c['gens']} generations",
                     "oracle_seconds": c["oracle_seconds"], "oracle_alns_seconds": c["alns_seconds"],
                     "oracle_brkga_seconds": c["brkga_seconds"], "gpu_chains": chains,
                     "gpu_refine_rounds": rounds, "gpu_start_seconds": t_start, "gpu_alns_iterations": it,
                     "gpu_z_alns": z_alns, "gpu_brkga_generations": gens, "gpu_best": best,
                     "gpu_seconds": reached_at if reached_at is not None else now(),
                     "reached": reached_at is not None, "reached_in": stage if reached_at is not None else None,
                     "speedup_vs_oracle": (c["oracle_seconds"] / reached_at) if reached_at else None,
                     "history": hist[-12:]}
    return out


def batched_form(P, torch, count=256, cpi=4, iters=40, Np=128, gens=20, chunk=10, gchunk=2, limit_s=60.0):
    """The batched form on 256 instances of uneven size against the plain
    two-stage method run instance by instance.
    Plain: for every instance in turn, the paper's start, `cpi` ALNS chains
    for `iters` iterations (graph replay) and BRKGA of `Np` x `gens` from
    the incumbent; its best is that instance's target.
    Batched: every instance of an n-bucket in one set -- one construction
    launch, one refinement state, one ALNS state (one captured iteration
    replayed for all), one BRKGA state -- advanced chunk by chunk until
    every instance has reached its plain target (or the time limit).
    Reported: both wall times, the share of instances reaching their target
    and when."""
    import synth
    from paper_2602_23685_amd import pipeline
    insts = synth.batched_instances(count)
    prm = P.alns_params(tuple_budget=2048, import_interval=0)
    edges = [0, 50, 150, 450, 10**9]
    buckets = [[i for i, x in enumerate(insts) if edges[b] <= x.n < edges[b + 1]] for b in range(4)]
    buckets = [b for b in buckets if b]
    # instance i is the pos[i]-th of its bucket: its plain run draws as its
    # chains and population do in the bucket's states, so both forms follow
    # the same trajectories and reach the same bests
    pos = {i: k for b in buckets for k, i in enumerate(b)}
    # the repair rounds' scan shape, tuned once per n-bucket set (outside the
    # timed region, as the evaluation's shape is); later states on the set use it
    sets = [P.InstanceSet([insts[i] for i in b]) for b in buckets]
    tuned = []
    for b, S in zip(buckets, sets):
        o, r = P.vrprpd_construct(S, P.CONS_SWEEP)
        tst = P.AlnsState(S, list(range(len(b))), cpi, prm, 11, o, r)
        tuned.append(tst.autotune(2))
        tst.close()
    log(f"batched form: plain two-stage method on {count} instances one by one")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    target = np.zeros(count, np.int64)
    for i, x in enumerate(insts):
        prm_i = P.alns_params(tuple_budget=2048, import_interval=0, chain_base=pos[i] * cpi)
        r = pipeline.run(P.InstanceSet([x]), 0, prm_i, cpi, iters, 11, Np, gens, P.pop_seed(13, pos[i]))
        target[i] = r["best"]
    t_plain = time.perf_counter() - t0
    # batched
    log(f"batched form: the same method on {len(buckets)} n-buckets together")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    best = np.full(count, np.iinfo(np.int64).max)
    reach_t = np.full(count, np.nan)

    def update(b, z):
        idx = np.array(buckets[b])
        better = z < best[idx]
        best[idx[better]] = z[better]
        newly = idx[(best[idx] <= target[idx]) & np.isnan(reach_t[idx])]
        reach_t[newly] = now()

    states = []
    for b, S in enumerate(sets):
        ops, rt, _ = pipeline.paper_start(S, prm, 11)
        st = P.AlnsState(S, list(range(len(buckets[b]))), cpi, prm, 11, ops, rt)
        update(b, st.state()["zb"].reshape(-1, cpi).min(axis=1))
        states.append(st)
    t_start = now()
    it = 0
    while np.isnan(reach_t).any() and it < iters:
        for st in states:
            st.step(chunk)
        it += chunk
        for b, st in enumerate(states):
            update(b, st.state()["zb"].reshape(-1, cpi).min(axis=1))
    t_alns = now()
    pops, g = [], 0
    if np.isnan(reach_t).any():
        for b, (S, st) in enumerate(zip(sets, states)):
            zb = st.state()["zb"].reshape(-1, cpi)
            P_, H_ = [], []
            for k in range(len(buckets[b])):
                _, o, r = st.best(int(k * cpi + zb[k].argmin()))
                pp, hh = pipeline.warm_population(S, k, o, r, Np, P.pop_seed(13, k))
                P_.append(pp)
                H_.append(hh)
            ne = nm = int(0.15 * Np)
            pops.append(P.BrkgaState(S, list(range(len(buckets[b]))), Np, ne, nm, 0.7, 13, torch.cat(P_),
                                     torch.cat(H_), decode_flags=P.DECODE_HINT_FIRST))
        while np.isnan(reach_t).any() and now() < limit_s:
            for pp in pops:
                pp.step(gchunk)
            g += gchunk
            for b, pp in enumerate(pops):
                update(b, pp.best()[0])
    t_batched = now()
    for st in states:
        st.close()
    for pp in pops:
        pp.close()
    ns = np.array([x.n for x in insts])
    done = ~np.isnan(reach_t)
    return {"instances": count, "n_range": [int(ns.min()), int(ns.max())], "n_buckets": len(buckets),
            "chains_per_instance": cpi, "alns_iterations": iters, "population": Np, "brkga_generations": gens,
            "tuple_budget": 2048,
            "scan_tuples_per_workgroup_by_bucket": [t[0] for t in tuned],
            "scan_ms_per_iteration_by_bucket_and_shape": [[round(x, 3) for x in t[1]] for t in tuned],
            "plain": "one instance at a time: paper's start, ALNS (graph replay), BRKGA from the incumbent",
            "plain_seconds": t_plain,
            "batched_seconds_to_all_targets": t_batched if done.all() else None,
            "batched_seconds": t_batched, "batched_start_seconds": t_start, "batched_alns_seconds": t_alns - t_start,
            "batched_alns_iterations": it, "batched_brkga_generations": g,
            "reached_fraction": float(done.mean()),
            "reached_seconds_median": float(np.nanmedian(reach_t)) if done.any() else None,
            "speedup_to_all_targets": (t_plain / t_batched) if done.all() else None,
            "mean_best_ratio_batched_vs_plain": float(np.mean(best / target)),
            "same_bests_as_plain": bool(np.array_equal(best, target))}


def construction(P, torch, oracle_instances=64):
    """The construction heuristics (the initial solution of Section 4.2 and
    the warm-start seeds of Section 4.4.4): one launch over the 256 batched
    instances per heuristic (HIP events, median of 5), and the oracle's time
    for the first `oracle_instances` of them, scaled to all."""
    import oracle
    import synth
    insts = synth.batched_instances(256)
    S = P.InstanceSet(insts)
    names = ["sweep", "nn", "lb", "spt"]
    out = {"instances": len(insts)}
    stream = torch.cuda.current_stream()
    for h, name in enumerate(names):
        P.vrprpd_construct(S, h)
        times = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            P.vrprpd_construct(S, h)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        t0 = time.perf_counter()
        for x in insts[:oracle_instances]:
            oracle.construct(x, h)
        t_orc = (time.perf_counter() - t0) * len(insts) / oracle_instances
        out[name] = {"gpu_ms": float(np.median(times)), "oracle_seconds_scaled": t_orc}
    return out


TSPLIB_NODES = [17, 21, 24, 29, 48, 51, 52, 100, 101, 202, 431, 666, 783, 1000]
VARIANTS = ["base", "2x", "5x", "1R10", "1R20"]


def signed_rank_p_greater(a, b):
    """One-sided Wilcoxon signed-rank test of a > b on paired samples: zero
    differences dropped, tied |differences| given their average rank, and
    the p-value P(W+ >= observed) from the exact distribution of W+ over
    all 2^n sign assignments (n <= 20 here)."""
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    d = d[d != 0]
    nd = len(d)
    if nd == 0:
        return 1.0
    order = np.argsort(np.abs(d), kind="stable")
    ranks = np.empty(nd)
    absd = np.abs(d)[order]
    i = 0
    while i < nd:
        j = i
        while j + 1 < nd and absd[j + 1] == absd[i]:
            j += 1
        ranks[order[i:j + 1]] = (i + j + 2) / 2.0
        i = j + 1
    w = ranks[d > 0].sum()
    signs = ((np.arange(2 ** nd)[:, None] >> np.arange(nd)) & 1).astype(np.float64)
    wplus = signs @ ranks
    return float(np.mean(wplus >= w - 1e-9))


def hypothesis(P, torch, chains=8, iters=300, Np=256, gens=30):
    """The processing-time hypothesis (Section 5.2) re-tested on synthetic
    stand-ins of the 14 benchmark sizes (depot + n customers, fleet m = 3,
    k = 5 below 24 customers, else m = 6, k = 4, R = m k) under the five
    processing variants: all 70 instances run the two-stage method as one
    batched GPU pipeline (construction, refinement, ALNS, BRKGA from each
    instance's incumbent); the statistics are those of each instance's best
    schedule (the paper takes them from BRKGA's best); paired one-sided
    Wilcoxon signed-rank tests of each variant against base over the 14
    sizes."""
    import synth
    from paper_2602_23685_amd import pipeline
    insts = []
    for v, rule in enumerate(VARIANTS):
        for s_, nodes in enumerate(TSPLIB_NODES):
            n = nodes - 1
            m, k = (3, 5) if n < 24 else (6, 4)
            insts.append(synth.make_instance(n, m, k, m * k, rule, seed=7000 + 100 * s_ + v))
    S = P.InstanceSet(insts)
    I = len(insts)
    prm = P.alns_params(tuple_budget=4096)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ops, rt, _ = pipeline.paper_start(S, prm, 17)
    st = P.AlnsState(S, list(range(I)), chains, prm, 17, ops, rt)
    st.step(iters)
    zb = st.state()["zb"].reshape(I, chains)
    z_alns = zb.min(axis=1)
    B_ops = torch.zeros((I, 2 * S.n_max), dtype=torch.uint16, device="cuda")
    B_rt = torch.zeros((I, S.m_max), dtype=torch.uint16, device="cuda")
    prios, hints = [], []
    for i in range(I):
        _, o, r = st.best(int(i * chains + zb[i].argmin()))
        B_ops[i] = o
        B_rt[i] = r
        pp, hh = pipeline.warm_population(S, i, o, r, Np, P.pop_seed(19, i))
        prios.append(pp)
        hints.append(hh)
    st.close()
    ne = nm = int(0.15 * Np)
    pop = P.BrkgaState(S, list(range(I)), Np, ne, nm, 0.7, 19, torch.cat(prios), torch.cat(hints),
                       decode_flags=P.DECODE_HINT_FIRST)
    pop.step(gens)
    bf, bp, bh = pop.best()
    pop.close()
    idx = torch.arange(I, dtype=torch.int32, device="cuda")
    d = P.brkga_decode_eval(S, bp, bh, inst=idx, want_ops=True, flags=P.DECODE_HINT_FIRST)
    unsch = d["unscheduled"].cpu().numpy()
    z_brkga = np.where(unsch == 0, d["makespan"].cpu().numpy(), np.iinfo(np.int64).max)
    for i in np.nonzero(z_brkga < z_alns)[0]:
        B_ops[i] = d["ops"][i]
        B_rt[i] = d["rt_end"][i]
    off = torch.arange(I, dtype=torch.int64, device="cuda")
    cross, inter = P.vrprpd_solution_stats(S, B_ops, B_rt, inst=idx, op_off=off * 2 * S.n_max,
                                           rt_off=off * S.m_max)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    ns = np.array([x.n for x in insts], np.float64)
    xa = 100.0 * cross.cpu().numpy() / ns
    il = 100.0 * inter.cpu().numpy() / ns
    k = len(TSPLIB_NODES)
    out = {"instances": I, "chains": chains, "alns_iterations": iters, "population": Np, "brkga_generations": gens,
           "seconds": seconds, "brkga_improved": int((z_brkga < z_alns).sum()),
           "note": "synthetic stand-ins of the 14 benchmark sizes, one instance per variant; statistics of each "
                   "instance's best schedule of the two-stage method"}
    for v, rule in enumerate(VARIANTS):
        row = {"cross_agent_pct_mean": float(xa[v * k:(v + 1) * k].mean()),
               "interleaved_pct_mean": float(il[v * k:(v + 1) * k].mean())}
        if v:
            for name, arr in (("cross_agent", xa), ("interleaved", il)):
                row[f"{name}_wilcoxon_p_greater_than_base"] = signed_rank_p_greater(arr[v * k:(v + 1) * k], arr[:k])
        out[rule] = row
    return out


def two_stage_chunked(P, torch, S, ops, rt, prm, chains, iters, seed, Np, gens, bseed, target=None, mlp=None,
                      K=8, eps=0.1, chunk=10, gchunk=2, limit_s=60.0):
    """The two-stage method on instance 0 of S from (ops, rt), advanced in
    chunks of `chunk` ALNS iterations, then `gchunk` BRKGA generations, with
    the best makespan read after each chunk.  With a target it stops as soon
    as the best reaches it (BRKGA then runs past `gens` until the time
    limit); with an ALNS network (mlp) the ALNS stage uses the learned
    proposal.  Returns the best, the time it was reached (or None) and the
    (seconds, best) history."""
    from paper_2602_23685_amd import pipeline
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    st = P.AlnsState(S, [0], chains, prm, seed, ops, rt)
    if mlp is not None:
        st.set_learned(mlp, K=K, eps=eps)
    best = int(st.state()["zb"].min())
    hist, at = [(now(), best)], None
    it = 0
    while it < iters and (target is None or best > target):
        st.step(chunk)
        it += chunk
        best = min(best, int(st.state()["zb"].min()))
        hist.append((now(), best))
    if target is not None and best <= target:
        at = now()
    g = 0
    if at is None:
        _, a_ops, a_rt = st.best(-1)
        prio, hint = pipeline.warm_population(S, 0, a_ops, a_rt, Np, bseed)
        ne = nm = int(0.15 * Np)
        pop = P.BrkgaState(S, [0], Np, ne, nm, 0.7, bseed, prio, hint, decode_flags=P.DECODE_HINT_FIRST)
        while (g < gens) if target is None else (best > target and now() < limit_s):
            pop.step(gchunk)
            g += gchunk
            best = min(best, int(pop.best()[0][0]))
            hist.append((now(), best))
        if target is not None and best <= target:
            at = now()
        pop.close()
    st.close()
    first = next(t for t, z in hist if z == best)     # when the final best was first held
    return {"best": best, "reached_at": at, "first_at_best": first, "seconds": now(), "alns_iterations": it,
            "brkga_generations": g, "history": [(round(t, 4), z) for t, z in hist[-6:]]}


def small_configs(P, torch, reps=10):
    """Throughput at the two smaller workloads (HIP events on the launch
    stream, median of `reps`):
      depot + 16 customers (m = 2, k = 2, R = 4, base rule): vrprpd_eval on
        4,096 random feasible solutions, then 2,000 ALNS iterations of 32
        chains from the paper's start (wall time);
      100 customers (m = 4, k = 5, R = 20, 2x rule): 65,536 ALNS neighbours of
        one solution as insertion tuples (vrprpd_insert_scan against a
        feasible solution with 5 customers removed), the same number of explicit
        random candidates (vrprpd_eval), and one BRKGA generation of 1,024
        chromosomes (brkga_decode_eval + brkga_evolve).
    With the evaluation's rooflines (HBM bytes 4n + 2m + 8 per candidate; the
    measured L2 random-read ceiling at 2n + 2m reads per candidate), the
    scan's (20 B of LDS per customer of base + tuple) and the generation's
    (16n + 20 B of HBM per chromosome, keys read and outputs written)."""
    import synth
    stream = torch.cuda.current_stream()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def timed(fn):
        fn()
        ev = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            ev.append((a, b))
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    out = {}
    for name, (n, m, k, R, rule, B) in {"n16": (16, 2, 2, 4, "base", 4096),
                                        "n100": (100, 4, 5, 20, "2x", 65536)}.items():
        inst = synth.make_instance(n, m, k, R, rule, seed=1001 if n == 16 else 2002)
        S = P.InstanceSet([inst])
        pool_o, pool_r = synth.random_candidates(inst, min(B, 1024), seed=n + 1)
        if B > len(pool_o):
            ops, rt = synth.relabel_candidates(pool_o, pool_r, n, B, seed=n + 2)
        else:
            ops, rt = pool_o, pool_r
        d_ops, d_rt = dev(ops), dev(rt)
        mk_ = torch.empty(B, dtype=torch.int32, device="cuda")
        st_ = torch.empty(B, dtype=torch.int32, device="cuda")
        form = P.vrprpd_autotune_eval(S, d_ops, d_rt, reps=2)[2]
        t = timed(lambda: P.vrprpd_eval(S, d_ops, d_rt, makespan=mk_, status=st_))
        rate, _ = P.vrprpd_gather_rate(S, 0)
        row = {"workload": f"{n} customers, m = {m}, k = {k}, R = {R}, {rule} rule", "eval_candidates": B,
               "eval_form": ("staged", "live legs")[form], "eval_ms": t, "eval_per_s": B / (t * 1e-3),
               "eval_hbm_frac": (4 * n + 2 * m + 8) * B / (t * 1e-3) / HBM_PEAK,
               "eval_l2_gather_frac": B / (t * 1e-3) / (rate / (2 * n + 2 * m)),
               "l2_reads_per_s": rate}
        if n == 16:
            # 2,000 ALNS iterations of 32 chains from the paper's start (every
            # slot pair priced at this size), as one timed region
            st_, _ = paper_start_gpu(P, S, 32, P.alns_params(), 77)
            ev0 = st_.state()["evals"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st_.step(2000)
            torch.cuda.synchronize()
            ta = time.perf_counter() - t0
            ev = st_.state()["evals"] - ev0
            row.update({"alns_chains": 32, "alns_iterations": 2000, "alns_seconds": ta,
                        "alns_iterations_per_s": 2000 / ta, "alns_evals_per_s": ev / ta,
                        "alns_best": int(st_.state()["zb"].min())})
            st_.close()
        if n == 100:
            g = synth.rng(n + 3)
            removed = sorted(int(c) for c in g.choice(np.arange(1, n + 1), size=5, replace=False))
            gone = set(removed)
            base = [[x for x in r if x[0] not in gone] for r in synth.unpack_candidate(pool_o[0], pool_r[0])]
            fo, _, frt = synth.pack_candidates([base], m)
            T = 65536
            tuples = synth.random_tuples(fo, frt[0], n, m, T, seed=n + 4, absent=removed)
            tuples = tuples[np.argsort(tuples["c"], kind="stable")]
            cs = tuples["c"].astype(np.int64)
            seg_off = np.concatenate([[0], np.nonzero(np.diff(cs))[0] + 1, [T]]).astype(np.int64)
            d_b, d_br, d_seg, d_t = dev(fo), dev(frt[0]), dev(seg_off), dev(tuples.view(np.uint8))
            ts = timed(lambda: P.vrprpd_insert_scan(S, d_b, d_br, d_seg, d_t))
            base_c = int(frt[0][-1]) // 2   # customers in the base
            row.update({"neighbours": T, "scan_ms": ts, "scan_per_s": T / (ts * 1e-3),
                        "scan_lds_frac": 20 * (base_c + 1) * T / (ts * 1e-3) / LDS_PEAK})
            Np = 1024
            prio, hint = synth.random_keys(Np, n, seed=n + 5)
            d_p, d_h = dev(prio), dev(hint)
            out_ = P.brkga_decode_eval(S, d_p, d_h)
            p2, h2 = torch.empty_like(d_p), torch.empty_like(d_h)
            rk = torch.empty(Np, dtype=torch.int32, device="cuda")
            ne = nm = int(0.15 * Np)

            def gen():
                P.brkga_decode_eval(S, d_p, d_h, out=out_)
                P.brkga_evolve(d_p, d_h, out_["fitness"], ne, nm, 0.7, 5, 0, prio_out=p2, hint_out=h2,
                               rank_out=rk)
            tg = timed(gen)
            row.update({"population": Np, "generation_ms": tg, "chromosomes_per_s": Np / (tg * 1e-3),
                        "generation_hbm_frac": (16 * n + 20) * Np / (tg * 1e-3) / HBM_PEAK})
        out[name] = row
    return out


MFMA_BF16_PEAK = 2.5e15   # MI355X dense bf16 matrix peak, flop/s


def mlp_roofline(P, torch, row_counts=(16384, 131072), reps=10):
    """Matrix-core rate of the network's hand-written GEMMs (gemm_kernel,
    bf16 MFMA with fp32 accumulation): forward, and forward + backward, on
    `rows` random feature rows, HIP events on the launch stream.  Flops:
    2 rows (64*256 + 256*256 + 256*256) forward; backward adds the weight
    gradients of the three layers and the input gradients of the upper two,
    2 rows (147,456 + 131,072)."""
    out = []
    stream = torch.cuda.current_stream()
    fwd_per_row = 2 * (64 * 256 + 256 * 256 + 256 * 256)
    bwd_per_row = 2 * (64 * 256 + 256 * 256 + 256 * 256 + 256 * 256 + 256 * 256)
    for rows in row_counts:
        M = P.Mlp(max_rows=rows, seed=3)
        g = torch.Generator(device="cuda").manual_seed(rows)
        x = (torch.rand((rows, 64), generator=g, device="cuda") * 2 - 1).to(torch.bfloat16)
        y = torch.empty(rows, dtype=torch.float32, device="cuda")
        dy = torch.full((rows,), 1e-3, dtype=torch.float32, device="cuda")

        def timed(fn):
            fn()
            ev = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn()
                b.record(stream)
                ev.append((a, b))
            torch.cuda.synchronize()
            return float(np.median([a.elapsed_time(b) for a, b in ev]))

        t_f = timed(lambda: M.forward(x, y))
        t_fb = timed(lambda: (M.forward(x, y), M.backward(dy)))
        M.close()
        f_f, f_fb = fwd_per_row * rows, (fwd_per_row + bwd_per_row) * rows
        out.append({"rows": rows, "forward_ms": t_f, "forward_tflops": f_f / (t_f * 1e-3) / 1e12,
                    "forward_backward_ms": t_fb, "forward_backward_tflops": f_fb / (t_fb * 1e-3) / 1e12,
                    "bound": "mfma", "peak_tflops": MFMA_BF16_PEAK / 1e12,
                    "frac_forward": f_f / (t_f * 1e-3) / MFMA_BF16_PEAK,
                    "frac_forward_backward": f_fb / (t_fb * 1e-3) / MFMA_BF16_PEAK})
    return out


def learned_form(P, torch, n=500, train_insts=8, rec_chains=128, rec_iters=1000, rec_budget=1024, epochs=1,
                 batch_sets=512, lr=1e-3, tests=5, chains=32, iters=200, Np=512, gens=20, K=8, eps=0.1):
    """The learned form on the 500-customer shape (m = 10, k = 8, R = 50,
    base rule).  Plain ALNS records (removal set, makespan change) pairs on
    `train_insts` instances (rec_chains chains x rec_iters iterations each:
    >= 1M pairs); the network trains on them with the library's kernels for
    `epochs` passes.  Then on `tests` other instances of the same shape the
    plain two-stage method (ALNS 32 chains x 200 iterations with 16,384
    tuples, BRKGA 512 x 20 from its incumbent) sets the target, and the
    two-stage method with the learned ALNS proposal runs from the same start
    until it reaches it.  Reported per instance and as medians; the
    recording and training time is reported apart and amortised over the
    test instances."""
    import synth
    from paper_2602_23685_amd import learned
    mk = lambda seed: synth.make_instance(n, 10, 8, 50, "base", seed=seed)
    train = [mk(5100 + i) for i in range(train_insts)]
    S_tr = P.InstanceSet(train)
    starts = [synth.round_robin_solution(x, vehicles=10) for x in train]
    r_ops = torch.from_numpy(np.stack([o for o, _ in starts])).cuda()
    r_rt = torch.from_numpy(np.stack([r for _, r in starts])).cuda()
    rec = P.AlnsState(S_tr, list(range(train_insts)), rec_chains, P.alns_params(tuple_budget=rec_budget), 101,
                      r_ops, r_rt)
    log(f"learned form: recording {train_insts} x {rec_chains} chains x {rec_iters} iterations")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sets = learned.record(rec, rec_iters)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    _, q = rec.record_info()
    M = P.Mlp(max_rows=max(batch_sets * q, chains * n), seed=7)
    steps = max(1, epochs * sets // batch_sets)
    log(f"learned form: training {steps} steps on {sets} sets")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    learned.train(M, rec, steps=steps, batch_sets=batch_sets, lr=lr, momentum=0.9)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    rec.close()
    prm = P.alns_params(tuple_budget=16384, import_interval=100)
    rows, held = [], []
    for t in range(tests):
        x = mk(5200 + t)
        S = P.InstanceSet([x])
        o, r = synth.round_robin_solution(x, vehicles=10)
        d_o, d_r = torch.from_numpy(o).cuda(), torch.from_numpy(r).cuda()
        if t == 0:   # held-out loss on this instance's plain records
            te = P.AlnsState(S, [0], 32, P.alns_params(tuple_budget=rec_budget), 102, d_o, d_r)
            learned.record(te, 20)
            held = learned.held_out(M, te)
            te.close()
        log(f"learned form: test instance {t}")
        plain = two_stage_chunked(P, torch, S, d_o, d_r, prm, chains, iters, 103 + t, Np, gens, 104 + t)
        lrn = two_stage_chunked(P, torch, S, d_o, d_r, prm, chains, iters, 103 + t, Np, gens, 104 + t,
                                target=plain["best"], mlp=M, K=K, eps=eps, limit_s=3 * plain["seconds"] + 5)
        rows.append({"instance_seed": 5200 + t, "plain_best": plain["best"],
                     "plain_seconds_to_its_best": plain["first_at_best"], "plain_seconds": plain["seconds"],
                     "learned_best": lrn["best"], "learned_seconds_to_plain_best": lrn["reached_at"],
                     "learned_alns_iterations": lrn["alns_iterations"],
                     "learned_brkga_generations": lrn["brkga_generations"]})
    M.close()
    mlp_roof = mlp_roofline(P, torch)
    reached = [r for r in rows if r["learned_seconds_to_plain_best"] is not None]
    ratio = [r["learned_seconds_to_plain_best"] / r["plain_seconds_to_its_best"] for r in reached]
    return {"n": n, "m": 10, "k": 8, "R": 50, "rule": "base", "train_instances": train_insts,
            "recorded_sets": sets, "record_chains": train_insts * rec_chains, "record_iterations": rec_iters,
            "record_tuple_budget": rec_budget, "record_seconds": t_rec, "train_steps": steps,
            "train_batch_sets": batch_sets, "train_seconds": t_train,
            "heldout_loss": held[0], "heldout_mean_predictor_loss": held[1],
            "test_instances": tests, "K": K, "eps": eps, "chains": chains, "alns_iterations": iters,
            "population": Np, "brkga_generations": gens,
            "reached": len(reached), "time_ratio_learned_vs_plain": ratio,
            "time_ratio_median": float(np.median(ratio)) if ratio else None,
            "time_ratio_range": [float(min(ratio)), float(max(ratio))] if ratio else None,
            "record_and_train_seconds_per_test_instance": (t_rec + t_train) / tests,
            "per_instance": rows, "mlp_roofline": mlp_roof,
            "note": "training pairs from plain ALNS on other instances of the same shape; the learned run counts "
                    "only its own search time, record_and_train_seconds_per_test_instance is the amortised cost"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-race", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and learned forms")
    ap.add_argument("--phases", default=None,
                    help="comma list of the phases after the timed steps to run (small, race, construction, "
                         "batched, hypothesis, learned, mlp, cpu); default: all not switched off by the --no-* "
                         "flags")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only copy 256 MiB three times (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_ref:
        import torch
        x = torch.ones(64 * 1024 * 1024, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copied 256 MiB three times")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2602_23685_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    P.load()
    K, W = args.steps, args.warmup
    log("generating workload")
    w = make_workload()
    inst = w["inst"]
    S = P.InstanceSet([inst])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    d_ops, d_rt = dev(w["ops"]), dev(w["rt"])
    B = d_rt.shape[0]
    mk = torch.empty(B, dtype=torch.int32, device="cuda")
    st = torch.empty(B, dtype=torch.int32, device="cuda")
    d_bops, d_brt, d_seg = dev(w["bops"]), dev(w["brt"]), dev(w["seg_off"])
    d_tup = dev(w["tuples"].view(np.uint8))
    T = len(w["tuples"])
    d_prio, d_hint = dev(w["prio"]), dev(w["hint"])
    Np = d_prio.shape[0]
    ne, nm = int(0.15 * Np), int(0.15 * Np)
    dec_out = P.brkga_decode_eval(S, d_prio, d_hint)
    p_next, h_next = torch.empty_like(d_prio), torch.empty_like(d_hint)
    rank = torch.empty(Np, dtype=torch.int32, device="cuda")
    chains = 32
    init_ops = dev(w["pool_ops"][0])
    init_rt = dev(w["pool_rt"][0])
    # two identical ALNS states (same start and seed): the sequential and the
    # concurrent pass time the same iterations
    alns_seq = P.AlnsState(S, [0], chains, P.alns_params(tuple_budget=16384), 7, init_ops, init_rt)
    alns = P.AlnsState(S, [0], chains, P.alns_params(tuple_budget=16384), 7, init_ops, init_rt)
    stream = torch.cuda.current_stream()
    log("autotuning the evaluation launch shape")
    tuned = P.vrprpd_autotune_eval(S, d_ops, d_rt, reps=2)
    names = ["vrprpd_eval", "vrprpd_insert_scan", "brkga_decode_eval+evolve", "alns_step"]
    ev = {nm_: [] for nm_ in names}

    dec_seq_ev = []

    def step_sequential(gen):
        """The stages one after another on one stream, each between events."""
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        marks[0].record(stream)
        P.vrprpd_eval(S, d_ops, d_rt, makespan=mk, status=st, stream=stream)
        marks[1].record(stream)
        P.vrprpd_insert_scan(S, d_bops, d_brt, d_seg, d_tup, stream=stream)
        marks[2].record(stream)
        P.brkga_decode_eval(S, d_prio, d_hint, out=dec_out, stream=stream)
        marks[5].record(stream)
        P.brkga_evolve(d_prio, d_hint, dec_out["fitness"], ne, nm, 0.7, 11, gen, prio_out=p_next,
                       hint_out=h_next, rank_out=rank, stream=stream)
        marks[3].record(stream)
        alns_seq.step(1, stream=stream)
        marks[4].record(stream)
        for i, nm_ in enumerate(names):
            ev[nm_].append((marks[i], marks[i + 1]))
        dec_seq_ev.append((marks[2], marks[5]))

    # The timed step: the ALNS iteration (many small latency-bound launches)
    # runs on a second stream while the first runs the evaluation, the scan
    # and BRKGA; the streams join at the end of every step.
    side = torch.cuda.Stream()   # default priority
    eval_ev, scan_ev, dec_ev = [], [], []

    def mark(record):
        if not record:
            return None
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def step_concurrent(gen, record):
        fork = torch.cuda.Event()
        fork.record(stream)
        side.wait_event(fork)
        alns.step(1, stream=side)
        e0 = mark(record)
        P.vrprpd_eval(S, d_ops, d_rt, makespan=mk, status=st, stream=stream)
        e1 = mark(record)
        P.vrprpd_insert_scan(S, d_bops, d_brt, d_seg, d_tup, stream=stream)
        e2 = mark(record)
        P.brkga_decode_eval(S, d_prio, d_hint, out=dec_out, stream=stream)
        e3 = mark(record)
        P.brkga_evolve(d_prio, d_hint, dec_out["fitness"], ne, nm, 0.7, 11, gen, prio_out=p_next,
                       hint_out=h_next, rank_out=rank, stream=stream)
        if record:
            eval_ev.append((e0, e1))
            scan_ev.append((e1, e2))
            dec_ev.append((e2, e3))
        join = torch.cuda.Event()
        join.record(side)
        stream.wait_event(join)

    log(f"per-stage times: {W} + {K} sequential steps")
    for i in range(W):
        step_sequential(i)
    torch.cuda.synchronize()
    for nm_ in names:
        ev[nm_].clear()
    dec_seq_ev.clear()
    s0 = alns_seq.state()
    for i in range(K):
        step_sequential(W + i)
    torch.cuda.synchronize()
    s1 = alns_seq.state()
    comp_ms = {nm_: float(np.mean([a.elapsed_time(b) for a, b in ev[nm_]])) for nm_ in names}
    comp_ms["brkga_decode_eval"] = float(np.mean([a.elapsed_time(b) for a, b in dec_seq_ev]))
    alns_evals_seq = (s1["evals"] - s0["evals"]) / K
    log(f"warmup {W}")
    for i in range(W):
        step_concurrent(i, False)
    torch.cuda.synchronize()
    ev0 = alns.state()
    log(f"timing {K} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        step_concurrent(W + i, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev1 = alns.state()
    alns_evals = (ev1["evals"] - ev0["evals"]) / K
    evals_per_step = B + T + Np + alns_evals
    all_rate = evals_per_step * K / wall
    # live, in the timed steps, from events on the stream the kernels run on
    ms = lambda evs: float(np.mean([a.elapsed_time(b) for a, b in evs]))
    eval_ms = ms(eval_ev)
    # the scan and the decoder alone (sequential steps): in the timed steps
    # they share the GPU with the concurrent ALNS stream
    scan_ms, dec_ms = comp_ms["vrprpd_insert_scan"], comp_ms["brkga_decode_eval"]
    scan_ms_conc, dec_ms_conc = ms(scan_ev), ms(dec_ev)
    value = B / (eval_ms * 1e-3)
    bytes_per_eval = 2 * 2 * inst.n + 2 * inst.m + 4 + 4
    achieved = bytes_per_eval * B / (eval_ms * 1e-3)
    feasible = float((st == 0).float().mean().item())
    # secondary bound: travel times read at random entries of the 2 MB
    # matrix, one per op and one per return leg (2n + m); the staged form
    # also reads the m route starts twice (the flat list's leg, then the
    # depot's)
    gather_rate, _ = P.vrprpd_gather_rate(S, 0)
    form = tuned[2]
    reads_per_eval = 2 * inst.n + (2 if form == 0 else 1) * inst.m
    # insertion scan: LDS bytes of one exact evaluation of base + tuple (per
    # customer: two op codes and two legs read, p and ready[] for the drop,
    # ready[] for the pickup = 20 B)
    base_customers = int(w["brt"][-1]) // 2 + 1
    scan_lds_per_tuple = 20 * base_customers
    # decoder: the chromosome's 2n priorities and 2n hints (fp32) and the
    # fitness, makespan, unscheduled count and status written
    dec_bytes = 16 * inst.n + 20

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "value_is": "vrprpd_eval: exact makespan evaluations of complete n=1000 candidates per second, over the "
                    "evaluation launches of the timed whole-path steps (HIP events on their stream)",
        "all_evals_per_s": all_rate,
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "ms_per_step_sequential": float(sum(comp_ms[nm_] for nm_ in names)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "n=1000 customers, m=10 vehicles, k=10, R=100, p=U_int[1,20]*floor(dbar/10); "
                        "per step: 65,536 explicit candidates, 16,384 insertion tuples, BRKGA 4,096 "
                        "decode+evolve, one ALNS iteration of 32 chains (16,384-tuple budget)",
            "n": inst.n, "m": inst.m, "k": inst.k, "R": inst.R,
            "explicit_candidates": B, "tuples": T, "population": Np, "alns_chains": chains,
            "evals_per_step": evals_per_step, "feasible_fraction": feasible,
        },
        "eval_launch_shape": {"form": ("staged", "live legs")[tuned[2]], "candidates_per_wave": tuned[0],
                              "ops_per_step": tuned[1],
                              "candidate_shapes_ms": {"staged": [round(float(x), 4) for x in tuned[3][:6]],
                                                      "live legs": [round(float(x), 4) for x in tuned[3][6:]]}},
        "components_ms": comp_ms,
        "component_evals_per_s": {
            "vrprpd_eval": B / (comp_ms["vrprpd_eval"] * 1e-3),
            "vrprpd_insert_scan": T / (comp_ms["vrprpd_insert_scan"] * 1e-3),
            "brkga_decode_eval+evolve": Np / (comp_ms["brkga_decode_eval+evolve"] * 1e-3),
            "brkga_decode_eval": Np / (comp_ms["brkga_decode_eval"] * 1e-3),
            "alns_step": alns_evals_seq / (comp_ms["alns_step"] * 1e-3),
        },
        "streams": "timed steps: the ALNS iteration on a second stream, concurrent with the evaluation, the "
                   "scan and BRKGA (joined every step); components_ms from as many sequential steps",
        "roofline": {
            "bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "traffic": measured_traffic(form),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "algorithmic_bytes_per_launch": bytes_per_eval * B,
            "kernel": EVAL_KERNELS[form], "kernel_ms": eval_ms, "bytes_per_unit": bytes_per_eval,
            "units_per_launch": B,
            "secondary": {"bound": "l2_gather", "reads_per_unit": reads_per_eval,
                          "measured_reads_per_s": gather_rate, "ceiling_units_per_s": gather_rate / reads_per_eval,
                          "frac": value / (gather_rate / reads_per_eval),
                          "how": "vrprpd_gather_rate: 2^29 random 2-byte reads of the instance's matrix, "
                                 "8192 x 256 threads, 16 in flight each"},
        },
        "roofline_components": [
            {"kernel": "scan_kernel (vrprpd_insert_scan)", "bound": "lds",
             "achieved": scan_lds_per_tuple * T / (scan_ms * 1e-3) / 1e9, "peak": LDS_PEAK / 1e9, "unit": "GB/s",
             "frac": scan_lds_per_tuple * T / (scan_ms * 1e-3) / LDS_PEAK, "bytes_per_unit": scan_lds_per_tuple,
             "units_per_launch": T, "kernel_ms": scan_ms, "kernel_ms_beside_alns": scan_ms_conc,
             "unit_is": "one exact evaluation of base + tuple (20 B of LDS traffic per customer)"},
            {"kernel": "decode_sort_kernel + decode_kernel (brkga_decode_eval)", "bound": "hbm",
             "achieved": dec_bytes * Np / (dec_ms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
             "frac": dec_bytes * Np / (dec_ms * 1e-3) / HBM_PEAK, "bytes_per_unit": dec_bytes,
             "units_per_launch": Np, "kernel_ms": dec_ms, "kernel_ms_beside_alns": dec_ms_conc,
             "unit_is": "one chromosome: 2n fp32 priorities + 2n fp32 hints read, 20 B written"},
        ],
    }
    if args.phases is not None:
        phases = set(x.strip() for x in args.phases.split(",") if x.strip())
    else:
        phases = {"small", "race", "construction", "batched", "hypothesis", "learned", "cpu"}
        if args.no_race:
            phases.discard("race")
        if args.no_forms:
            phases -= {"construction", "batched", "hypothesis", "learned"}
        if args.no_cpu_baseline:
            phases.discard("cpu")
    def phase(key, msg, fn):
        """One reported phase after the timed steps: a Python error in it is
        recorded in its place, so the line is still printed."""
        if msg:
            log(msg)
        try:
            out[key] = fn()
        except Exception as exc:   # noqa: BLE001 -- reported, not hidden
            log(f"{key} failed: {exc!r}")
            out[key] = {"error": repr(exc)}

    if "race" in phases:
        phase("time_to_oracle_best", "time to oracle-best (n=16)", lambda: time_to_oracle_best(P, torch))
        phase("time_to_oracle_best_large", "time to oracle-best (n=100, n=1000)", lambda: race_to_oracle(P, torch))
    if "small" in phases:
        phase("small_configs", "smaller workloads (16 and 100 customers)", lambda: small_configs(P, torch))
    if "construction" in phases:
        phase("construction", "construction heuristics", lambda: construction(P, torch))
    if "batched" in phases:
        phase("batched_form", None, lambda: batched_form(P, torch))
    if "hypothesis" in phases:
        phase("hypothesis", "processing-time hypothesis", lambda: hypothesis(P, torch))
    if "learned" in phases:
        phase("learned_form", None, lambda: learned_form(P, torch))
    elif "mlp" in phases:   # the network's GEMM rate alone (the learned form reports it too)
        phase("mlp_roofline", "network GEMM rate", lambda: mlp_roofline(P, torch))
    if "cpu" in phases:
        phase("cpu_baseline", "cpu baseline", lambda: cpu_baseline(inst, w["ops"], w["rt"], args.cpu_seconds))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
