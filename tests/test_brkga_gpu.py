"""Parity: BRKGA decode, generation and warm start on the GPU vs the oracle."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


DECODE_CASES = [
    # n, m, k, R, rule, load_model, B
    (16, 2, 2, 4, "base", 0, 1024),
    (100, 4, 5, 20, "2x", 0, 256),
    (100, 4, 5, 20, "2x", 1, 128),
    (1000, 10, 10, 100, "1R20d10", 0, 24),
    (500, 10, 8, 50, "base", 0, 24),
    (30, 3, 2, 2, "5x", 0, 256),           # scarce resources: many passes, unscheduled ops
    (1, 1, 1, 1, "base", 0, 16),
    (20, 40, 1, 10, "1R10", 0, 64),        # more vehicles than customers
    (70, 64, 2, 100, "2x", 1, 48),         # every lane a vehicle (all-ones vehicle mask)
]


@pytest.mark.parametrize("case", DECODE_CASES, ids=lambda c: f"n{c[0]}m{c[1]}lm{c[5]}")
def test_decode_parity(orc, P, case):
    n, m, k, R, rule, lm, B = case
    inst = synth.make_instance(n, m, k, R, rule, seed=7000 + n, load_model=lm)
    prio, hint = synth.random_keys(B, n, seed=n + m, special=B >= 8)
    S = P.InstanceSet([inst])
    for use_hint, flags in ((True, 0), (False, 0), (True, P.DECODE_HINT_FIRST), (False, P.DECODE_HINT_FIRST)):
        out = P.brkga_decode_eval(S, dev(prio), dev(hint) if use_hint else None, want_ops=True, flags=flags)
        torch.cuda.synchronize()
        f = out["fitness"].cpu().numpy()
        mk = out["makespan"].cpu().numpy()
        un = out["unscheduled"].cpu().numpy()
        st = out["status"].cpu().numpy().view(np.uint32)
        ops = out["ops"].cpu().numpy()
        rt = out["rt_end"].cpu().numpy()
        for b in range(B):
            r = orc.decode(inst, prio[b], hint[b] if use_hint else None, want_ops=True, flags=flags)
            assert (f[b], mk[b], un[b], st[b]) == (r["fitness"], r["makespan"], r["unscheduled"],
                                                     r["status"]), (b, use_hint, flags)
            if r["status"] & 16:
                assert np.all(rt[b] == 0)
            else:
                assert np.array_equal(rt[b], r["rt_end"]), b
                L = int(rt[b][-1])
                assert np.array_equal(ops[b][:L], r["ops"]), b


@pytest.mark.parametrize("case", [(1000, 10, 10, 100, "1R20d10", 64), (20, 40, 1, 10, "1R10", 64)],
                         ids=lambda c: f"n{c[0]}m{c[1]}")
def test_decode_parity_without_sequences(orc, P, case):
    """The launch without op sequences (no schedule log) prices the same."""
    n, m, k, R, rule, B = case
    inst = synth.make_instance(n, m, k, R, rule, seed=7100 + n)
    prio, hint = synth.random_keys(B, n, seed=n + 3, special=True)
    S = P.InstanceSet([inst])
    out = P.brkga_decode_eval(S, dev(prio), dev(hint))
    torch.cuda.synchronize()
    got = np.stack([out["fitness"].cpu().numpy(), out["makespan"].cpu().numpy(),
                    out["unscheduled"].cpu().numpy(), out["status"].cpu().numpy().view(np.uint32)], axis=1)
    for b in range(B):
        r = orc.decode(inst, prio[b], hint[b])
        assert tuple(got[b]) == (r["fitness"], r["makespan"], r["unscheduled"], r["status"]), b


@pytest.mark.parametrize("case", [c for c in DECODE_CASES if c[1] <= 16], ids=lambda c: f"n{c[0]}m{c[1]}lm{c[5]}")
def test_decode_without_sequences_all_rules(orc, P, case):
    """The launch without op sequences (the BRKGA generations' form) on every
    m <= 16 case: a batch that is not a multiple of four, both vehicle rules,
    with and without hints, a bad key in the last chromosome."""
    n, m, k, R, rule, lm, B = case
    B = min(B, 64) + 3
    inst = synth.make_instance(n, m, k, R, rule, seed=7300 + n, load_model=lm)
    prio, hint = synth.random_keys(B, n, seed=n + m + 1, special=B >= 8)
    S = P.InstanceSet([inst])
    for use_hint, flags in ((True, 0), (False, 0), (True, P.DECODE_HINT_FIRST), (False, P.DECODE_HINT_FIRST)):
        out = P.brkga_decode_eval(S, dev(prio), dev(hint) if use_hint else None, flags=flags)
        torch.cuda.synchronize()
        got = np.stack([out["fitness"].cpu().numpy(), out["makespan"].cpu().numpy(),
                        out["unscheduled"].cpu().numpy(), out["status"].cpu().numpy().view(np.uint32)], axis=1)
        for b in range(B):
            r = orc.decode(inst, prio[b], hint[b] if use_hint else None, flags=flags)
            assert tuple(got[b]) == (r["fitness"], r["makespan"], r["unscheduled"], r["status"]), \
                (b, use_hint, flags)


def test_decode_parity_wide_distances(orc, P):
    """Travel times above 65535 keep the int32 distance layout in the decoder."""
    inst = synth.make_instance(80, 5, 4, 20, "2x", seed=7201)
    inst.d = (inst.d.astype(np.int64) * 500).astype(np.int32)
    inst.p = (inst.p.astype(np.int64) * 500).astype(np.int32)
    S = P.InstanceSet([inst])
    assert S.dist16 == 0
    B = 64
    prio, hint = synth.random_keys(B, 80, seed=7202, special=True)
    for want_ops in (False, True):
        out = P.brkga_decode_eval(S, dev(prio), dev(hint), want_ops=want_ops)
        torch.cuda.synchronize()
        f = out["fitness"].cpu().numpy()
        for b in range(B):
            r = orc.decode(inst, prio[b], hint[b], want_ops=want_ops)
            assert f[b] == r["fitness"], (b, want_ops)
            if want_ops and not r["status"] & 16:
                L = int(r["rt_end"][-1])
                assert np.array_equal(out["ops"][b].cpu().numpy()[:L], r["ops"]), b


@pytest.mark.parametrize("Np", [1024, 4096, 5000, 65536], ids=lambda x: f"Np{x}")
def test_evolve_parity(orc, P, Np):
    """Ranking by the block-wide sort (Np <= 4096) and by counting (larger)."""
    n = 100
    ne, nm = orc.brkga_sizes(Np)
    prio, hint = synth.random_keys(Np, n, seed=3)
    fit = synth.rng(4).integers(0, 10**6, size=Np).astype(np.int64)
    fit[::7] = fit[0]                                       # ties resolved by index
    fit[5] = 2**63 - 1
    fit[3] = -(2**40)                                       # any int64 orders
    for gen in (0, 17):
        po, ho, rank = P.brkga_evolve(dev(prio), dev(hint), dev(fit), ne, nm, 0.7, 0xC0FFEE, gen)
        torch.cuda.synchronize()
        opo, oho, orank = orc.brkga_evolve(prio, hint, fit, ne, nm, orc.rho_threshold(0.7), 0xC0FFEE, gen)
        assert np.array_equal(rank.cpu().numpy(), orank)
        assert np.array_equal(po.cpu().numpy().view(np.uint32), opo.view(np.uint32))
        assert np.array_equal(ho.cpu().numpy().view(np.uint32), oho.view(np.uint32))
    # without hints (priorities only); genes not a multiple of 4
    prio2 = prio[:, :198].copy()
    po, ho, rank = P.brkga_evolve(dev(prio2), None, dev(fit), ne, nm, 0.7, 5, 1)
    opo, _, orank = orc.brkga_evolve(prio2, None, fit, ne, nm, orc.rho_threshold(0.7), 5, 1)
    assert np.array_equal(po.cpu().numpy().view(np.uint32), opo.view(np.uint32))


def test_warm_start_parity(orc, P):
    inst = synth.make_instance(100, 4, 5, 20, "2x", seed=9)
    ops, rt = synth.random_candidates(inst, 1, 10)
    S = P.InstanceSet([inst])
    po, ho = P.brkga_warm_start(S, dev(ops[0]), dev(rt[0]), 300, 45, 20, seed=99)
    torch.cuda.synchronize()
    opo, oho = orc.brkga_warm_start(inst, ops[0], rt[0], 300, 45, 20, 99)
    assert np.array_equal(po.cpu().numpy().view(np.uint32), opo.view(np.uint32))
    assert np.array_equal(ho.cpu().numpy().view(np.uint32), oho.view(np.uint32))


def test_generation_loop_matches_oracle(orc, P):
    """Warm start, then decode + evolve for a few generations entirely on the
    GPU; the oracle replays the same generations from the same inputs."""
    inst = synth.make_instance(40, 3, 4, 12, "5x", seed=21)
    ops, rt = synth.random_candidates(inst, 1, 22)
    S = P.InstanceSet([inst])
    Np, G = 256, 80
    ne, nm = orc.brkga_sizes(Np)
    gp, gh = P.brkga_warm_start(S, dev(ops[0]), dev(rt[0]), Np, int(0.15 * Np), 20, seed=5)
    op_, oh_ = orc.brkga_warm_start(inst, ops[0], rt[0], Np, int(0.15 * Np), 20, 5)
    for gen in range(4):
        out = P.brkga_decode_eval(S, gp, gh)
        of = orc.decode_batch(inst, op_, oh_)[0]
        assert np.array_equal(out["fitness"].cpu().numpy(), of)
        gp, gh, _ = P.brkga_evolve(gp, gh, out["fitness"], ne, nm, 0.7, 77, gen)
        op_, oh_, _ = orc.brkga_evolve(op_, oh_, of, ne, nm, orc.rho_threshold(0.7), 77, gen)
        assert np.array_equal(gp.cpu().numpy().view(np.uint32), op_.view(np.uint32))


@pytest.mark.parametrize("graph,flags", [(True, 0), (False, 0), (True, 1)], ids=["graph", "direct", "hintfirst"])
def test_batched_populations_match_oracle(orc, P, graph, flags):
    """Three instances of different size evolved as one batched state: every
    population equals the oracle's single-population run with its seed, and
    the kept best fitness is the best decoded so far."""
    insts = [synth.make_instance(16, 2, 2, 4, "base", seed=31),
             synth.make_instance(40, 4, 5, 20, "2x", seed=32),
             synth.make_instance(25, 3, 3, 9, "1R10", seed=33)]
    S = P.InstanceSet(insts)
    Np, gens, seed = 96, 5, 2024
    ne, nm = orc.brkga_sizes(Np)
    stride = 2 * 40
    g = np.random.Generator(np.random.Philox(key=77))
    p0 = np.zeros((3 * Np, stride), np.float32)
    h0 = np.zeros((3 * Np, stride), np.float32)
    for p, inst in enumerate(insts):
        p0[p * Np:(p + 1) * Np, :2 * inst.n] = g.random((Np, 2 * inst.n), dtype=np.float32)
        h0[p * Np:(p + 1) * Np, :2 * inst.n] = g.random((Np, 2 * inst.n), dtype=np.float32)
    st = P.BrkgaState(S, [0, 1, 2], Np, ne, nm, 0.7, seed, dev(p0), dev(h0), decode_flags=flags)
    st.step(2, graph=graph)
    torch.cuda.synchronize()
    st.step(gens - 2, graph=graph)
    best, _, _ = st.best()
    pop_p, pop_h = st.population()
    pop_p, pop_h = pop_p.cpu().numpy(), pop_h.cpu().numpy()
    for p, inst in enumerate(insts):
        G = 2 * inst.n
        op_ = p0[p * Np:(p + 1) * Np, :G].copy()
        oh_ = h0[p * Np:(p + 1) * Np, :G].copy()
        bf = np.iinfo(np.int64).max
        for gen in range(gens):
            fit = orc.decode_batch(inst, op_, oh_, flags=flags)[0]
            bf = min(bf, int(fit.min()))
            op_, oh_, _ = orc.brkga_evolve(op_, oh_, fit, ne, nm, orc.rho_threshold(0.7), P.pop_seed(seed, p), gen)
        assert best[p] == bf, (p, best[p], bf)
        assert np.array_equal(pop_p[p * Np:(p + 1) * Np, :G].view(np.uint32), op_.view(np.uint32)), p
        assert np.array_equal(pop_h[p * Np:(p + 1) * Np, :G].view(np.uint32), oh_.view(np.uint32)), p
    st.close()


def test_batched_populations_of_96_uneven_instances(orc, P):
    """One batched BRKGA state over 96 instances of uneven size (the batched
    form's generator, n in [17, 200]; Np = 64, 4 generations, hint-first rule,
    graph replay): every population and best fitness equals the oracle's
    single-population run of that instance with its seed."""
    insts = synth.batched_instances(count=96, seed=9400, n_min=17, n_max=200)
    S = P.InstanceSet(insts)
    Np, gens, seed, flags = 64, 4, 4242, 1
    ne, nm = orc.brkga_sizes(Np)
    stride = 2 * S.n_max
    g = np.random.Generator(np.random.Philox(key=78))
    p0 = np.zeros((len(insts) * Np, stride), np.float32)
    h0 = np.zeros((len(insts) * Np, stride), np.float32)
    for p, inst in enumerate(insts):
        p0[p * Np:(p + 1) * Np, :2 * inst.n] = g.random((Np, 2 * inst.n), dtype=np.float32)
        h0[p * Np:(p + 1) * Np, :2 * inst.n] = g.random((Np, 2 * inst.n), dtype=np.float32)
    print(f"[brkga batched] {len(insts)} instances x Np {Np} x {gens} generations", flush=True)
    st = P.BrkgaState(S, list(range(len(insts))), Np, ne, nm, 0.7, seed, dev(p0), dev(h0), decode_flags=flags)
    st.step(gens, graph=True)
    torch.cuda.synchronize()
    best, _, _ = st.best()
    pop_p, pop_h = st.population()
    pop_p, pop_h = pop_p.cpu().numpy(), pop_h.cpu().numpy()
    for p, inst in enumerate(insts):
        G = 2 * inst.n
        op_ = p0[p * Np:(p + 1) * Np, :G].copy()
        oh_ = h0[p * Np:(p + 1) * Np, :G].copy()
        bf = np.iinfo(np.int64).max
        for gen in range(gens):
            fit = orc.decode_batch(inst, op_, oh_, flags=flags)[0]
            bf = min(bf, int(fit.min()))
            op_, oh_, _ = orc.brkga_evolve(op_, oh_, fit, ne, nm, orc.rho_threshold(0.7), P.pop_seed(seed, p), gen)
        assert best[p] == bf, (p, best[p], bf)
        assert np.array_equal(pop_p[p * Np:(p + 1) * Np, :G].view(np.uint32), op_.view(np.uint32)), p
        assert np.array_equal(pop_h[p * Np:(p + 1) * Np, :G].view(np.uint32), oh_.view(np.uint32)), p
    st.close()


@pytest.mark.parametrize("flags", [0, 1], ids=["selectvehicle", "hintfirst"])
def test_packed_and_plain_vehicle_minimum_agree_on_ties(orc, P, flags):
    """The decoder's two vehicle-minimum paths (packed time << 4 | rank keys
    when every time of the set is below 2^27, a plain minimum and tie ballot
    otherwise) on the same decoding problems: a 5-vehicle instance on a small
    integer grid (many equal travel times, so many completion-time ties), decoded
    alone (packed) and inside a set whose second instance has travel times
    large enough to switch the whole set to the plain path."""
    g = np.random.Generator(np.random.Philox(key=4141))
    n, m = 40, 5
    pts = g.integers(0, 4, size=(n + 1, 2))
    d = (np.abs(pts[:, None, :] - pts[None, :, :]).sum(axis=2) * 3).astype(np.int32)   # Manhattan: ties
    d[d == 0] = 1
    np.fill_diagonal(d, 0)
    p = np.concatenate([[0], g.integers(0, 4, size=n)]).astype(np.int32)
    inst = synth.instance_from_matrix(d, p, m=m, k=3, R=10)
    big = synth.make_instance(30, 3, 4, 12, "base", seed=4142)
    big.p = (big.p.astype(np.int64) * (150_000_000 // int(big.p.sum()))).astype(np.int32)   # sum p > 2^27
    alone, mixed = P.InstanceSet([inst]), P.InstanceSet([inst, big])
    assert alone.dist16 == 1 and mixed.dist16 == 1         # same 16-bit matrix layout on both paths
    B = 256
    prio, hint = synth.random_keys(B, n, seed=4143, special=True)
    prio[B // 2:] = np.round(prio[B // 2:] * 8) / 8 * 0.99          # coarse keys: tied priorities too
    hint[B // 2:] = np.round(hint[B // 2:] * 5) / 5 * 0.99
    inst_idx = torch.zeros(B, dtype=torch.int32, device="cuda")
    pm = np.zeros((B, 2 * mixed.n_max), np.float32)
    hm = np.zeros((B, 2 * mixed.n_max), np.float32)
    pm[:, :2 * n], hm[:, :2 * n] = prio, hint
    a = P.brkga_decode_eval(alone, dev(prio), dev(hint), want_ops=True, flags=flags)
    b = P.brkga_decode_eval(mixed, dev(pm), dev(hm), inst=inst_idx, want_ops=True, flags=flags)
    torch.cuda.synchronize()
    for key in ("fitness", "makespan", "unscheduled", "status"):
        assert torch.equal(a[key], b[key]), key
    assert torch.equal(a["rt_end"], b["rt_end"][:, :m])
    assert torch.equal(a["ops"], b["ops"][:, :2 * n])
    f = a["fitness"].cpu().numpy()
    for i in range(0, B, 16):
        assert f[i] == orc.decode(inst, prio[i], hint[i], flags=flags)["fitness"], i


def test_decode_a_quarter_million_chromosomes_in_one_launch(orc, P):
    """2^18 chromosomes of the 100-customer workload (m = 4, k = 5, R = 20,
    2x rule) in one launch per vehicle rule, each a copy of one of 1,024
    oracle-decoded bases (special keys among them) at a random position:
    fitness, makespan, unscheduled count, status and the op sequences of
    every chromosome against the oracle."""
    n, m = 100, 4
    inst = synth.make_instance(n, m, 5, 20, "2x", seed=9750)
    S = P.InstanceSet([inst])
    prio, hint = synth.random_keys(1024, n, seed=9751, special=True)
    B = 1 << 18
    src = synth.rng(9752).integers(0, 1024, size=B)
    d_prio, d_hint = dev(prio[src]), dev(hint[src])
    pos = np.arange(2 * n)[None, :]
    for flags in (0, P.DECODE_HINT_FIRST):
        ref = [orc.decode(inst, prio[b], hint[b], want_ops=True, flags=flags) for b in range(1024)]
        ef = np.array([r["fitness"] for r in ref])[src]
        emk = np.array([r["makespan"] for r in ref])[src]
        eun = np.array([r["unscheduled"] for r in ref])[src]
        est = np.array([r["status"] for r in ref], np.uint32)[src]
        ert = np.stack([np.zeros(m, np.uint16) if r["status"] & 16 else r["rt_end"] for r in ref])
        eops = np.zeros((1024, 2 * n), np.uint16)
        for b, r in enumerate(ref):
            eops[b, :len(r["ops"])] = r["ops"]
        assert (est == 0).sum() > B // 4 and (est == 16).any()
        print(f"[decode large] B={B} flags={flags}", flush=True)
        out = P.brkga_decode_eval(S, d_prio, d_hint, want_ops=True, flags=flags)
        torch.cuda.synchronize()
        assert np.array_equal(out["fitness"].cpu().numpy(), ef), flags
        assert np.array_equal(out["makespan"].cpu().numpy(), emk), flags
        assert np.array_equal(out["unscheduled"].cpu().numpy(), eun), flags
        assert np.array_equal(out["status"].cpu().numpy().view(np.uint32), est), flags
        rt = out["rt_end"].cpu().numpy()
        assert np.array_equal(rt, ert[src]), flags
        ops = out["ops"].cpu().numpy()
        L = rt[:, -1].astype(np.int64)
        live = pos < L[:, None]
        assert np.array_equal(np.where(live, ops, 0), np.where(live, eops[src], 0)), flags
