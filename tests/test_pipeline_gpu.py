"""The two-stage method (ALNS, then BRKGA warm-started from its incumbent) on
the GPU against the same pipeline on the oracle, stage by stage and bit for
bit: the paper's start, the ALNS incumbent, the warm population, BRKGA's
best chromosome and fitness, and the pipeline's result."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_23685_amd as P
    P.load()
    return P


CASES = [
    # n, m, k, R, rule, chains, iterations, budget, Np, gens, decoder flags
    (40, 4, 5, 20, "2x", 2, 30, 400, 128, 6, 1),
    (60, 5, 4, 15, "5x", 3, 20, 600, 96, 5, 1),
    (40, 4, 5, 20, "2x", 2, 10, 400, 64, 4, 0),     # the least-completion decoder rule
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}m{c[1]}f{c[10]}")
def test_pipeline_matches_oracle(orc, P, case):
    from oracle import pipeline as opl
    from paper_2602_23685_amd import pipeline as gpl
    n, m, k, R, rule, chains, iters, budget, Np, gens, flags = case
    inst = synth.make_instance(n, m, k, R, rule, seed=8800 + n)
    kw = dict(tuple_budget=budget, import_interval=10, ls_budget=2000)
    ref = opl.run(inst, orc.alns_params(**kw), chains, iters, 77, Np, gens, 5, ls_budget=2000, decode_flags=flags)
    S = P.InstanceSet([inst])
    got = gpl.run(S, 0, P.alns_params(**kw), chains, iters, 77, Np, gens, 5, decode_flags=flags)
    assert got["z_start"] == ref["z_start"]
    assert got["z_alns"] == ref["z_alns"]
    L = int(ref["alns_rt"][-1])
    assert np.array_equal(got["alns_rt"].cpu().numpy()[:m], ref["alns_rt"])
    assert np.array_equal(got["alns_ops"].cpu().numpy()[:L], ref["alns_ops"])
    G = 2 * n
    assert np.array_equal(got["warm_prio"].cpu().numpy()[:, :G].view(np.uint32), ref["warm_prio"].view(np.uint32))
    assert np.array_equal(got["warm_hint"].cpu().numpy()[:, :G].view(np.uint32), ref["warm_hint"].view(np.uint32))
    assert got["brkga_fitness"] == ref["brkga_fitness"]
    assert np.array_equal(got["brkga_prio"].cpu().numpy()[:G].view(np.uint32), ref["brkga_prio"].view(np.uint32))
    assert np.array_equal(got["brkga_hint"].cpu().numpy()[:G].view(np.uint32), ref["brkga_hint"].view(np.uint32))
    assert got["z_brkga"] == ref["z_brkga"] and got["best"] == ref["best"]
    Lb = int(ref["best_rt"][-1])
    assert np.array_equal(got["best_ops"].cpu().numpy()[:Lb], np.asarray(ref["best_ops"])[:Lb])
    assert orc.eval_one(inst, np.asarray(ref["best_ops"])[:Lb], ref["best_rt"]) == (ref["best"], 0)
