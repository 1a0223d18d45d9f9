"""Checkpoint and resume of the search states (alns_state_save / load,
brkga_state_save / load): a run interrupted by a save, the destruction of the
state, a new state and a load continues bit for bit as the run without the
interruption -- per-iteration records, fp64 temperatures and weights, best
solutions; for BRKGA the populations, bests and fitness."""
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


def _alns(P, S, ops, rt, prm, seed=4242, chains=3):
    return P.AlnsState(S, [0], chains, prm, seed, torch.from_numpy(ops).cuda(), torch.from_numpy(rt).cuda())


@pytest.mark.parametrize("graph", [True, False])
def test_alns_resume_equals_uninterrupted(orc, P, graph):
    """20 iterations, save, destroy, load into a fresh state, 20 more: the
    same 40 records, state and bests as 40 in one go; both match the oracle.
    The weight period (tau = 7), the import (every 15) and the local searches
    (repositioning at 25, relocation at 30) straddle the checkpoint."""
    inst = synth.make_instance(40, 4, 5, 20, "5x", seed=5151)
    ops, rt = synth.round_robin_solution(inst)
    kw = dict(tuple_budget=400, import_interval=15, tau=7, ls_repos_interval=25, ls_reloc_interval=30,
              ls_budget=2000)
    prm = P.alns_params(**kw)
    S = P.InstanceSet([inst])
    full = _alns(P, S, ops, rt, prm)
    full.set_graph(graph)
    tf = full.set_trace(40)
    full.step(40)
    first = _alns(P, S, ops, rt, prm)
    first.set_graph(graph)
    t1 = first.set_trace(20)
    first.step(20)
    blob = first.save()
    e20 = first.state()["evals"]
    first.close()
    second = _alns(P, S, ops, rt, prm)
    second.set_graph(graph)
    second.load(blob)
    s = second.state()
    assert s["iterations"] == 20 and s["evals"] == e20
    t2 = second.set_trace(20)
    second.step(20)
    torch.cuda.synchronize()
    got = np.concatenate([t1.cpu().numpy(), t2.cpu().numpy()], axis=1)
    assert np.array_equal(got, tf.cpu().numpy())
    sa, sb = second.state(), full.state()
    for key in ("iterations", "evals", "z", "zb", "T", "wD", "wR"):
        assert np.array_equal(sa[key], sb[key]), key
    for ch in range(3):
        ma, oa, ra = second.best(ch)
        mb, ob, rb = full.best(ch)
        assert ma == mb
        assert torch.equal(oa, ob) and torch.equal(ra, rb)
    ref = orc.alns_run(inst, orc.alns_params(**kw), 3, 40, 4242, ops, rt, trace=True)
    assert np.array_equal(got, ref["trace"])
    # saving again after the load reproduces the state the uninterrupted run has
    assert second.save() == full.save()


def test_alns_load_refuses_other_configurations(P):
    inst = synth.make_instance(20, 2, 3, 6, "2x", seed=77)
    ops, rt = synth.round_robin_solution(inst)
    S = P.InstanceSet([inst])
    a = _alns(P, S, ops, rt, P.alns_params(), seed=1, chains=2)
    a.step(3)
    blob = a.save()
    for other in (_alns(P, S, ops, rt, P.alns_params(), seed=2, chains=2),
                  _alns(P, S, ops, rt, P.alns_params(tau=50), seed=1, chains=2),
                  _alns(P, S, ops, rt, P.alns_params(), seed=1, chains=3)):
        with pytest.raises(P.VrpError):
            other.load(blob)
    b = _alns(P, S, ops, rt, P.alns_params(), seed=1, chains=2)
    with pytest.raises(P.VrpError):
        b.load(blob[:-1])
    b.load(blob)
    a.step(4)
    b.step(4)
    assert a.save() == b.save()


@pytest.mark.parametrize("graph", [True, False])
def test_brkga_resume_equals_uninterrupted(P, graph):
    insts = [synth.make_instance(n, 3, 4, 12, "base", seed=60 + n) for n in (30, 45)]
    S = P.InstanceSet(insts)
    Np, ne, nm = 64, 9, 9
    mk = lambda: P.BrkgaState(S, [0, 1], Np, ne, nm, 0.7, 99)
    full = mk()
    full.step(6, graph=graph)
    a = mk()
    a.step(3, graph=graph)
    blob = a.save()
    a.close()
    b = mk()
    b.load(blob)
    b.step(3, graph=graph)
    torch.cuda.synchronize()
    fa, pa, ha = b.best()
    fb, pb, hb = full.best()
    assert np.array_equal(fa, fb)
    assert torch.equal(pa, pb) and torch.equal(ha, hb)
    qa, ra = b.population()
    qb, rb = full.population()
    assert torch.equal(qa, qb) and torch.equal(ra, rb)
    assert b.save() == full.save()
    c = P.BrkgaState(S, [0, 1], Np, ne, nm, 0.7, 100)
    with pytest.raises(P.VrpError):
        c.load(blob)
