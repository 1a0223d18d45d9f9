"""The oracle's two-stage pipeline (CPU): the stages compose as Section 4
and Section 4.4.4 describe -- the warm population's first slot is the
encoded ALNS incumbent, the hint-first decoder rebuilds the incumbent from
it, BRKGA's best is never worse than the best warm chromosome, and the
result is the better of the two stages and a feasible schedule."""
import numpy as np

import synth


def test_pipeline_stages(orc):
    from oracle import pipeline as opl
    inst = synth.make_instance(30, 3, 4, 12, "2x", seed=8830)
    r = opl.run(inst, orc.alns_params(tuple_budget=300, ls_budget=1000), 2, 15, 3, 64, 4, 9, ls_budget=1000)
    assert r["z_alns"] <= r["z_start"]
    # slot 0: the unperturbed encoding of the incumbent
    po, ho = orc.brkga_warm_start(inst, r["alns_ops"], r["alns_rt"], 1, 1, 1, 9)
    assert np.array_equal(r["warm_prio"][0].view(np.uint32), po[0].view(np.uint32))
    assert np.array_equal(r["warm_hint"][0].view(np.uint32), ho[0].view(np.uint32))
    d0 = orc.decode(inst, po[0], ho[0], flags=orc.DECODE_HINT_FIRST)
    assert r["brkga_history"][0] <= d0["fitness"]
    assert all(a >= b for a, b in zip(r["brkga_history"], r["brkga_history"][1:]))
    assert r["brkga_fitness"] == r["brkga_history"][-1]
    assert r["best"] == min(r["z_alns"], r["z_brkga"] if r["z_brkga"] is not None else r["z_alns"])
    L = int(r["best_rt"][-1])
    assert orc.eval_one(inst, np.asarray(r["best_ops"])[:L], r["best_rt"]) == (r["best"], 0)


def test_hint_first_decodes_the_incumbent_close_to_itself(orc):
    """On a refined start the encoded incumbent decodes, under the hint-first
    rule, to a schedule no worse than 5% above it; under the least-completion
    rule it may land far away (the reason the pipeline uses hint-first)."""
    from oracle import pipeline as opl
    inst = synth.make_instance(60, 4, 5, 20, "2x", seed=8831)
    ops, rt, z = opl.paper_start(inst, ls_budget=2000)
    po, ho = orc.brkga_warm_start(inst, ops, rt, 1, 1, 1, 1)
    hf = orc.decode(inst, po[0], ho[0], flags=orc.DECODE_HINT_FIRST)
    assert hf["unscheduled"] == 0 and hf["makespan"] <= 1.05 * z
