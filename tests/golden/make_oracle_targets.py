"""Writes oracle_targets.json: the best makespan the CPU oracle's ALNS reaches
on the benchmark instances with a fixed seed and budget, and its wall time.
Calls only oracle/ and synth/ (the seeded input generator).

Protocol (one chain, Table 2 parameters including the periodic local search
every 200 / 500 iterations with 16,384 tuples per pass), from two starts:
  paper:        the paper's initial solution (Section 4.2): sweep
                construction, then refinement rounds of the local searches
                until one improves nothing; the time includes the start;
  round_robin:  customers dealt round-robin to min(m, R) vehicles as
                drop-then-pickup pairs (a weak start that leaves the ALNS
                iterations all the work).
  n=100:  m=4, k=5, R=20, rule 2x, tuple budget 2,000, 2,000 iterations
  n=1000: m=10, k=10, R=100, rule 1R20d10, tuple budget 16,384, 200 iterations
Run from the repository root: python tests/golden/make_oracle_targets.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CASES = [
    dict(name="n100", n=100, m=4, k=5, R=20, rule="2x", seed=2002, budget=2000, iterations=2000, alns_seed=77),
    dict(name="n1000", n=1000, m=10, k=10, R=100, rule="1R20d10", seed=3003, budget=16384, iterations=200,
         alns_seed=77),
]


def main():
    out = {}
    for c in CASES:
        inst = synth.make_instance(c["n"], c["m"], c["k"], c["R"], c["rule"], seed=c["seed"])
        for start in ("paper", "round_robin"):
            t0 = time.perf_counter()
            if start == "paper":
                ops, rt = oracle.construct(inst, oracle.CONS_SWEEP)
                z0 = oracle.eval_one(inst, ops, rt)[0]
                rounds, z1, ops, rt = oracle.refine(inst, ops, rt, budget=16384)
            else:
                ops, rt = synth.round_robin_solution(inst, vehicles=min(c["m"], c["R"]))
                z0 = z1 = oracle.eval_one(inst, ops, rt)[0]
                rounds = 0
            t1 = time.perf_counter()
            r = oracle.alns_run(inst, oracle.alns_params(tuple_budget=c["budget"]), 1, c["iterations"],
                                c["alns_seed"], ops, rt)
            dt = time.perf_counter() - t0
            name = f"{c['name']}_{start}"
            out[name] = dict(c, start=start, z_construct=int(z0), z_refined=int(z1), refine_rounds=rounds,
                             z_oracle=int(r["best_mk"][0]), start_seconds=t1 - t0, oracle_seconds=dt, chains=1)
            print(name, z0, z1, rounds, int(r["best_mk"][0]), f"{t1 - t0:.1f} s start, {dt:.1f} s", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_targets.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
