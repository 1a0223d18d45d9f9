"""Parity: alns_step on the GPU reproduces the oracle's ALNS trajectories.

Every iteration's candidate makespan, current and best makespan, operator
choice, outcome and removal size must match, and so must the final
temperatures and operator weights (fp64, bit for bit) and best solutions."""
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


ALNS_CASES = [
    # n, m, k, R, rule, load_model, chains, iters, budget, import_interval
    (16, 2, 2, 4, "base", 0, 4, 60, 0, 20),        # full enumeration (small case)
    (40, 4, 5, 20, "5x", 0, 3, 30, 400, 10),
    (100, 4, 5, 20, "2x", 0, 2, 12, 2000, 0),
    (30, 3, 3, 9, "1R20", 1, 2, 25, 300, 0),
    (20, 17, 2, 40, "1R10", 0, 2, 12, 500, 0),     # 32-lane groups
]


def _same_state(info, ref):
    """Final current makespans, fp64 temperatures and operator weights, bit
    for bit."""
    assert np.array_equal(info["z"], ref["z"])
    for key in ("T", "wD", "wR"):
        assert np.array_equal(info[key].view(np.uint64), ref[key].view(np.uint64)), key


@pytest.mark.parametrize("case", ALNS_CASES, ids=lambda c: f"n{c[0]}m{c[1]}b{c[8]}")
def test_alns_trajectory_parity(orc, P, case):
    n, m, k, R, rule, lm, chains, iters, budget, imp = case
    inst = synth.make_instance(n, m, k, R, rule, seed=9000 + n, load_model=lm)
    ops, rt = synth.round_robin_solution(inst, vehicles=min(m, R))
    assert orc.eval_one(inst, ops, rt)[1] == 0
    seed = 1234 + n
    ref = orc.alns_run(inst, orc.alns_params(tuple_budget=budget, import_interval=imp), chains, iters, seed,
                       ops, rt, trace=True)
    S = P.InstanceSet([inst])
    st = P.AlnsState(S, [0], chains, P.alns_params(tuple_budget=budget, import_interval=imp), seed,
                     torch.from_numpy(ops).cuda(), torch.from_numpy(rt).cuda())
    tr = st.set_trace(iters)
    st.step(iters)
    torch.cuda.synchronize()
    got = tr.cpu().numpy()
    exp = ref["trace"]
    for ch in range(chains):
        for it in range(iters):
            assert np.array_equal(got[ch, it], exp[ch, it]), (ch, it, got[ch, it], exp[ch, it])
    info = st.state()
    assert info["iterations"] == iters
    assert np.array_equal(info["zb"], ref["best_mk"])
    _same_state(info, ref)
    for ch in range(chains):
        mk, bops, brt = st.best(ch)
        assert mk == ref["best_mk"][ch]
        b_rt = brt.cpu().numpy()[:m]
        assert np.array_equal(b_rt, ref["best_rt"][ch])
        assert np.array_equal(bops.cpu().numpy()[:2 * n], ref["best_ops"][ch])
        assert orc.eval_one(inst, bops.cpu().numpy()[:2 * n], b_rt) == (mk, 0)


def test_alns_trajectory_parity_wide_distances(orc, P):
    """Travel times above 65535: the int32 op store in every ALNS kernel."""
    inst = synth.make_instance(30, 3, 3, 9, "2x", seed=9301)
    inst.d = (inst.d.astype(np.int64) * 500).astype(np.int32)
    inst.p = (inst.p.astype(np.int64) * 500).astype(np.int32)
    S = P.InstanceSet([inst])
    assert S.dist16 == 0
    ops, rt = synth.round_robin_solution(inst, vehicles=3)
    chains, iters, seed = 2, 20, 9302
    prm = dict(tuple_budget=300, import_interval=0)
    ref = orc.alns_run(inst, orc.alns_params(**prm), chains, iters, seed, ops, rt, trace=True)
    st = P.AlnsState(S, [0], chains, P.alns_params(**prm), seed, torch.from_numpy(ops).cuda(),
                     torch.from_numpy(rt).cuda())
    tr = st.set_trace(iters)
    st.step(iters)
    torch.cuda.synchronize()
    got = tr.cpu().numpy()
    for ch in range(chains):
        for it in range(iters):
            assert np.array_equal(got[ch, it], ref["trace"][ch, it]), (ch, it)
    assert np.array_equal(st.state()["zb"], ref["best_mk"])


def test_alns_continues_across_calls(orc, P):
    """Two calls of alns_step(k) equal one call of alns_step(2k)."""
    inst = synth.make_instance(16, 2, 2, 4, "2x", seed=77)
    ops, rt = synth.round_robin_solution(inst)
    prm = P.alns_params(import_interval=7)
    S = P.InstanceSet([inst])
    a = P.AlnsState(S, [0], 3, prm, 5, torch.from_numpy(ops).cuda(), torch.from_numpy(rt).cuda())
    b = P.AlnsState(S, [0], 3, prm, 5, torch.from_numpy(ops).cuda(), torch.from_numpy(rt).cuda())
    a.step(10)
    a.step(10)
    b.step(20)
    sa, sb = a.state(), b.state()
    for key in ("z", "zb", "T", "wD", "wR"):
        assert np.array_equal(sa[key], sb[key]), key
    ref = orc.alns_run(inst, orc.alns_params(import_interval=7), 3, 20, 5, ops, rt)
    assert np.array_equal(sa["zb"], ref["best_mk"])


def test_graph_replay_equals_eager_launches(orc, P):
    """The captured iteration replayed many times gives the eager launch
    sequence's trajectory, with other device work and host synchronisation
    between replays; every replayed iteration is compared."""
    inst = synth.make_instance(40, 4, 5, 20, "2x", seed=91)
    ops, rt = synth.round_robin_solution(inst)
    prm = P.alns_params(tuple_budget=400, import_interval=5)
    S = P.InstanceSet([inst])
    mk_state = lambda: P.AlnsState(S, [0], 3, prm, 31, torch.from_numpy(ops).cuda(), torch.from_numpy(rt).cuda())
    g, e = mk_state(), mk_state()
    e.set_graph(False)
    tg, te = g.set_trace(24), e.set_trace(24)
    cand_ops, cand_rt = synth.random_candidates(inst, 64, seed=5)
    d_ops, d_rt = torch.from_numpy(cand_ops).cuda(), torch.from_numpy(cand_rt).cuda()
    for chunk in (1, 1, 2, 5, 7, 8):
        g.step(chunk)
        P.vrprpd_eval(S, d_ops, d_rt)          # eager work between replays
        torch.cuda.synchronize()
        e.step(chunk)
        torch.cuda.synchronize()
        sg, se = g.state(), e.state()
        for key in ("z", "zb", "T", "wD", "wR"):
            assert np.array_equal(sg[key], se[key]), (chunk, key)
    assert np.array_equal(tg.cpu().numpy(), te.cpu().numpy())
    ref = orc.alns_run(inst, orc.alns_params(tuple_budget=400, import_interval=5), 3, 24, 31, ops, rt, trace=True)
    assert np.array_equal(tg.cpu().numpy(), ref["trace"])


LS_CASES = [
    # n, m, k, R, rule, chains, iters, budget, repos, reloc, ls_budget
    (30, 3, 3, 9, "base", 3, 25, 300, 4, 6, 400),
    (100, 4, 5, 20, "2x", 2, 12, 2000, 3, 5, 3000),
    (20, 17, 2, 40, "1R10", 2, 12, 500, 2, 3, 600),   # 32-lane groups
    (16, 2, 2, 4, "base", 4, 30, 0, 5, 7, 100000),      # budget above every neighbourhood
]


@pytest.mark.parametrize("case", LS_CASES, ids=lambda c: f"n{c[0]}m{c[1]}r{c[8]}x{c[9]}")
def test_alns_local_search_parity(orc, P, case):
    """Periodic pickup repositioning and cross-agent relocation (Section
    4.2.6) at short intervals: trajectories, best makespans and solutions
    bit-identical to the oracle, with graph replay and with direct launches."""
    n, m, k, R, rule, chains, iters, budget, repos, reloc, lsb = case
    inst = synth.make_instance(n, m, k, R, rule, seed=9100 + n)
    ops, rt = synth.round_robin_solution(inst, vehicles=min(m, R))
    seed = 4321 + n
    kw = dict(tuple_budget=budget, import_interval=0, ls_repos_interval=repos, ls_reloc_interval=reloc,
              ls_budget=lsb)
    ref = orc.alns_run(inst, orc.alns_params(**kw), chains, iters, seed, ops, rt, trace=True)
    S = P.InstanceSet([inst])
    for graph in (True, False):
        st = P.AlnsState(S, [0], chains, P.alns_params(**kw), seed, torch.from_numpy(ops).cuda(),
                         torch.from_numpy(rt).cuda())
        st.set_graph(graph)
        tr = st.set_trace(iters)
        st.step(iters)
        got = tr.cpu().numpy()
        for ch in range(chains):
            for it in range(iters):
                assert np.array_equal(got[ch, it], ref["trace"][ch, it]), (graph, ch, it, got[ch, it],
                                                                           ref["trace"][ch, it])
        info = st.state()
        assert np.array_equal(info["zb"], ref["best_mk"])
        _same_state(info, ref)
        for ch in range(chains):
            mk, bops, brt = st.best(ch)
            assert np.array_equal(bops.cpu().numpy()[:2 * n], ref["best_ops"][ch])
            assert orc.eval_one(inst, bops.cpu().numpy()[:2 * n], brt.cpu().numpy()[:m]) == (mk, 0)
        st.close()


FULL_SCALE = [
    # 1000 customers, 10 vehicles, k = 10, R = 100, p = U_int[1,20] floor(dbar/10), 16,384 tuples per
    # iteration: q in [25, 50], enumeration sorts of ~2,000 slot keys, gains over n customers
    ("alns", dict(tuple_budget=16384, import_interval=2)),
    # the same with both local searches due in the first iterations (16,384-tuple passes)
    ("ls", dict(tuple_budget=16384, import_interval=0, ls_repos_interval=2, ls_reloc_interval=3,
                ls_budget=16384)),
]


@pytest.mark.parametrize("name,kw", FULL_SCALE, ids=[c[0] for c in FULL_SCALE])
def test_alns_full_scale_parity(orc, P, name, kw):
    """alns_step at the full-scale configuration (the one the benchmark
    times): four chains x three iterations cover all six destroy operators;
    traces, final makespans, fp64 temperatures and weights and the best
    solutions equal the oracle's."""
    inst = synth.make_instance(1000, 10, 10, 100, "1R20d10", seed=10000)
    ops, rt = synth.round_robin_solution(inst, vehicles=10)
    chains, iters, seed = 4, 3, 77
    ref = orc.alns_run(inst, orc.alns_params(**kw), chains, iters, seed, ops, rt, trace=True)
    assert set((ref["trace"][:, :, 3] & 0xFF).ravel()) == set(range(6))
    S = P.InstanceSet([inst])
    st = P.AlnsState(S, [0], chains, P.alns_params(**kw), seed, torch.from_numpy(ops).cuda(),
                     torch.from_numpy(rt).cuda())
    tr = st.set_trace(iters)
    st.step(iters)
    torch.cuda.synchronize()
    got = tr.cpu().numpy()
    for ch in range(chains):
        for it in range(iters):
            assert np.array_equal(got[ch, it], ref["trace"][ch, it]), (ch, it, got[ch, it], ref["trace"][ch, it])
    info = st.state()
    assert np.array_equal(info["zb"], ref["best_mk"])
    _same_state(info, ref)
    for ch in range(chains):
        mk, bops, brt = st.best(ch)
        assert np.array_equal(brt.cpu().numpy()[:10], ref["best_rt"][ch])
        assert np.array_equal(bops.cpu().numpy()[:2000], ref["best_ops"][ch])
    st.close()


def test_chain_base_matches_the_chains_of_a_batched_state(orc, P):
    """A one-instance state with chain_base = k * chains draws as the k-th
    instance's chains of a state over several instances: trajectories and
    bests equal, and equal to the oracle's run with those chain ids."""
    insts = [synth.make_instance(n, m, 4, 4 * m, "2x", seed=9500 + n) for n, m in ((30, 3), (45, 4), (25, 3))]
    S = P.InstanceSet(insts)
    cpi, iters, seed = 3, 15, 606
    kw = dict(tuple_budget=300, import_interval=5)
    starts = [synth.round_robin_solution(x) for x in insts]
    N, Mx = S.n_max, S.m_max
    ops = np.zeros((3, 2 * N), np.uint16)
    rts = np.zeros((3, Mx), np.uint16)
    for i, (o, r) in enumerate(starts):
        ops[i, :len(o)] = o
        rts[i, :len(r)] = r
    big = P.AlnsState(S, [0, 1, 2], cpi, P.alns_params(**kw), seed, torch.from_numpy(ops).cuda(),
                      torch.from_numpy(rts).cuda())
    tb = big.set_trace(iters)
    big.step(iters)
    zb_big = big.state()["zb"]
    tb = tb.cpu().numpy()
    for k, x in enumerate(insts):
        one = P.AlnsState(P.InstanceSet([x]), [0], cpi, P.alns_params(chain_base=k * cpi, **kw), seed,
                          torch.from_numpy(starts[k][0]).cuda(), torch.from_numpy(starts[k][1]).cuda())
        to = one.set_trace(iters)
        one.step(iters)
        assert np.array_equal(to.cpu().numpy(), tb[k * cpi:(k + 1) * cpi]), k
        assert np.array_equal(one.state()["zb"], zb_big[k * cpi:(k + 1) * cpi]), k
        ref = orc.alns_run(x, orc.alns_params(**kw), cpi, iters, seed, starts[k][0], starts[k][1], trace=True,
                           chain0=k * cpi)
        assert np.array_equal(to.cpu().numpy(), ref["trace"]), k
        one.close()
    big.close()


def test_autotune_keeps_the_trajectory(orc, P):
    """alns_autotune tries the repair rounds' scan shapes from a checkpoint and
    restores it: the run continues exactly as one never tuned (and as the
    oracle), with the trace it had before the call."""
    inst = synth.make_instance(100, 4, 5, 20, "2x", seed=9700)
    ops, rt = synth.round_robin_solution(inst)
    kw = dict(tuple_budget=2000, import_interval=4)
    S = P.InstanceSet([inst])
    mk_state = lambda: P.AlnsState(S, [0], 3, P.alns_params(**kw), 77, torch.from_numpy(ops).cuda(),
                                   torch.from_numpy(rt).cuda())
    a, b = mk_state(), mk_state()
    ta, tb = a.set_trace(20), b.set_trace(20)
    a.step(5)
    tpb, ms = a.autotune(2)
    assert tpb in (8, 16, 32, 64) and all(x > 0 for x in ms)
    assert a.state()["iterations"] == 5
    a.step(15)
    b.step(20)
    torch.cuda.synchronize()
    assert np.array_equal(ta.cpu().numpy(), tb.cpu().numpy())
    sa, sb = a.state(), b.state()
    for key in ("z", "zb", "T", "wD", "wR"):
        assert np.array_equal(sa[key], sb[key]), key
    ref = orc.alns_run(inst, orc.alns_params(**kw), 3, 20, 77, ops, rt, trace=True)
    assert np.array_equal(ta.cpu().numpy(), ref["trace"])
    # a later state on the set starts with the tuned shape and still matches
    c = mk_state()
    tc = c.set_trace(20)
    c.step(20)
    assert np.array_equal(tc.cpu().numpy(), ref["trace"])
    a.close()
    b.close()
    c.close()


def test_batched_state_of_128_uneven_instances(orc, P):
    """One ALNS state over 128 instances of uneven size (the batched form's
    generator, n in [17, 300]; 4 chains each, best-solution import every 4
    iterations) from the paper's sweep construction: every chain's trace,
    final temperature and weights (fp64 bits) and best makespan equal the
    oracle's run of that instance with the same chain ids."""
    insts = synth.batched_instances(count=128, seed=9300, n_min=17, n_max=300)
    S = P.InstanceSet(insts)
    cpi, iters, seed = 4, 8, 321
    kw = dict(tuple_budget=1024, import_interval=4)
    N, Mx = S.n_max, S.m_max
    starts = [orc.construct(x, 0) for x in insts]
    ops = np.zeros((len(insts), 2 * N), np.uint16)
    rts = np.zeros((len(insts), Mx), np.uint16)
    for i, (o, r) in enumerate(starts):
        assert orc.eval_one(insts[i], o, r)[1] == 0
        ops[i, :len(o)] = o
        rts[i, :len(r)] = r
    print(f"[alns batched] {len(insts)} instances x {cpi} chains x {iters} iterations", flush=True)
    st = P.AlnsState(S, list(range(len(insts))), cpi, P.alns_params(**kw), seed, torch.from_numpy(ops).cuda(),
                     torch.from_numpy(rts).cuda())
    tr = st.set_trace(iters)
    st.step(iters)
    torch.cuda.synchronize()
    got, info = tr.cpu().numpy(), st.state()
    for k, x in enumerate(insts):
        ref = orc.alns_run(x, orc.alns_params(**kw), cpi, iters, seed, starts[k][0], starts[k][1], trace=True,
                           chain0=k * cpi)
        sl = slice(k * cpi, (k + 1) * cpi)
        assert np.array_equal(got[sl], ref["trace"]), k
        assert np.array_equal(info["zb"][sl], ref["best_mk"]), k
        assert np.array_equal(info["z"][sl], ref["z"]), k
        for key in ("T", "wD", "wR"):
            assert np.array_equal(info[key][sl].view(np.uint64), ref[key].view(np.uint64)), (k, key)
    st.close()
