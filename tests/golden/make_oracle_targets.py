"""Writes oracle_targets.json: the best makespan the CPU oracle's two-stage
method (ALNS, then BRKGA warm-started from its incumbent) reaches on the
benchmark instances with fixed seeds and budgets, each stage's result and
wall time.  Calls only oracle/ and synth/ (the seeded input generator).

Protocol (ALNS: one chain, Table 2 parameters including the periodic local
search every 200 / 500 iterations with 16,384 tuples per pass; BRKGA: Table 3
fractions, 20 warm seeds from the incumbent and the NN / LB / SPT
constructions, the hint-first decoder rule), from two starts:
  paper:        the paper's initial solution (Section 4.2): sweep
                construction, then refinement rounds of the local searches
                until one improves nothing; the time includes the start;
  round_robin:  customers dealt round-robin to min(m, R) vehicles as
                drop-then-pickup pairs (a weak start that leaves the search
                all the work).
  n=100:  m=4, k=5, R=20, rule 2x, tuple budget 2,000, 2,000 iterations,
          then BRKGA 1,024 x 100 generations
  n=1000: m=10, k=10, R=100, rule 1R20d10, tuple budget 16,384, 200
          iterations, then BRKGA 4,096 x 60 generations (20 generations do
          not improve on the paper's start at this size; 60 do)
Run from the repository root: python tests/golden/make_oracle_targets.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import pipeline  # noqa: E402

CASES = [
    dict(name="n100", n=100, m=4, k=5, R=20, rule="2x", seed=2002, budget=2000, iterations=2000, alns_seed=77,
         Np=1024, gens=100, brkga_seed=78),
    dict(name="n1000", n=1000, m=10, k=10, R=100, rule="1R20d10", seed=3003, budget=16384, iterations=200,
         alns_seed=77, Np=4096, gens=60, brkga_seed=78),
]


def main():
    out = {}
    only = sys.argv[1:]
    for c in CASES:
        if only and c["name"] not in only:
            continue
        inst = synth.make_instance(c["n"], c["m"], c["k"], c["R"], c["rule"], seed=c["seed"])
        for start in ("paper", "round_robin"):
            st = None if start == "paper" else synth.round_robin_solution(inst, vehicles=min(c["m"], c["R"]))
            r = pipeline.run(inst, oracle.alns_params(tuple_budget=c["budget"]), 1, c["iterations"], c["alns_seed"],
                             c["Np"], c["gens"], c["brkga_seed"], start=st)
            name = f"{c['name']}_{start}"
            out[name] = dict(c, start=start, z_refined=r["z_start"], z_alns=r["z_alns"], z_brkga=r["z_brkga"],
                             z_oracle=r["best"], brkga_history=r["brkga_history"],
                             start_seconds=r["start_seconds"], alns_seconds=r["alns_seconds"],
                             brkga_seconds=r["brkga_seconds"],
                             oracle_seconds=r["start_seconds"] + r["alns_seconds"] + r["brkga_seconds"], chains=1)
            print(name, {k: out[name][k] for k in ("z_refined", "z_alns", "z_brkga", "z_oracle", "oracle_seconds")},
                  flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_targets.json")
    if only and os.path.exists(path):
        old = json.load(open(path))
        old.update(out)
        out = old
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
