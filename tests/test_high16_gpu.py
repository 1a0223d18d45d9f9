"""Travel times in [32768, 65535]: still packed as uint16 (the set's 16-bit
layout), where a signed reinterpretation of a stored time would turn it
negative.  Evaluation, insertion scan, decoder (both vehicle-minimum
variants: packed keys below the 2^27 longest-path bound, plain above) and
ALNS against the oracle, bit for bit."""
import numpy as np
import pytest

import synth
from cases import destroy, mutate

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


def high16(n, m, k, R, rule, seed):
    """An instance whose largest travel time lies in [32768, 65535]: every
    time (and processing time) scaled by floor(65535 / max d)."""
    inst = synth.make_instance(n, m, k, R, rule, seed=seed)
    f = 65535 // int(inst.d.max())
    inst.d = (inst.d.astype(np.int64) * f).astype(np.int32)
    inst.p = (inst.p.astype(np.int64) * f).astype(np.int32)
    assert 32768 <= inst.d.max() <= 65535
    assert (inst.d >= 32768).mean() > 0.05
    return inst


def time_bound(inst):
    return (2 * inst.n + 1) * int(inst.d.max()) + int(inst.p.sum())


INSTS = [(200, 6, 5, 30, "2x", 61), (1000, 10, 10, 100, "1R20d10", 62)]


@pytest.fixture(scope="module", params=INSTS, ids=lambda c: f"n{c[0]}")
def inst(request):
    return high16(*request.param)


def test_high16_layout(P, inst):
    S = P.InstanceSet([inst])
    assert S.dist16 == 1


def test_high16_eval(orc, P, inst):
    ops, rt = synth.random_candidates(inst, 384, seed=3)
    bad_ops, bad_rt = mutate(inst, ops, rt, seed=4, count=128)
    ops = np.concatenate([ops, bad_ops])
    rt = np.concatenate([rt, bad_rt])
    S = P.InstanceSet([inst])
    mk, st = P.vrprpd_eval(S, dev(ops), dev(rt))
    torch.cuda.synchronize()
    omk, ost = orc.eval_batch(inst, ops, rt)
    assert np.array_equal(mk.cpu().numpy(), omk)
    assert np.array_equal(st.cpu().numpy().view(np.uint32), ost)
    assert (ost == 0).sum() > 300 and omk[ost == 0].min() > 65535


def test_high16_scan(orc, P, inst):
    n, m = inst.n, inst.m
    ops, rt = synth.random_candidates(inst, 1, seed=5)
    bops, _, brt = destroy(inst, ops, rt, seed=6, q=min(30, n // 4))
    brt = brt[0]
    T = 3000
    tuples = synth.random_tuples(bops, brt, n, m, T, seed=7, invalid_frac=0.05)
    seg_off = np.array([0, 1000, 1700, T], np.int64)
    S = P.InstanceSet([inst])
    mk, st, top = P.vrprpd_insert_scan(S, dev(bops), dev(brt), dev(seg_off), dev(tuples.view(np.uint8)))
    torch.cuda.synchronize()
    omk, ost, otop = orc.insert_scan(inst, bops, brt, tuples, seg_off)
    assert np.array_equal(mk.cpu().numpy(), omk)
    assert np.array_equal(st.cpu().numpy().view(np.uint32), ost)
    assert np.array_equal(top.cpu().numpy(), otop)
    assert (omk < 2**31 - 1).sum() > T // 2       # most tuples were swept to a makespan


def test_high16_decode(orc, P, inst):
    S = P.InstanceSet([inst])
    B = 48
    prio, hint = synth.random_keys(B, inst.n, seed=8, special=True)
    out = P.brkga_decode_eval(S, dev(prio), dev(hint), want_ops=True)
    torch.cuda.synchronize()
    f = out["fitness"].cpu().numpy()
    for b in range(B):
        r = orc.decode(inst, prio[b], hint[b], want_ops=True)
        assert f[b] == r["fitness"], b
        if not r["status"] & 16:
            L = int(r["rt_end"][-1])
            assert np.array_equal(out["ops"][b].cpu().numpy()[:L], r["ops"]), b


def test_high16_decode_both_minimum_variants(P):
    """The two instances fall on either side of the packed-key bound."""
    bounds = [time_bound(high16(*c)) for c in INSTS]
    assert bounds[0] < 2**27 < bounds[1]


def test_high16_alns(orc, P, inst):
    n, m = inst.n, inst.m
    ops, rt = synth.round_robin_solution(inst, vehicles=m)
    big = n >= 1000
    kw = dict(tuple_budget=16384 if big else 2000, import_interval=0)
    chains, iters, seed = (2, 2, 91) if big else (3, 8, 92)
    ref = orc.alns_run(inst, orc.alns_params(**kw), chains, iters, seed, ops, rt, trace=True)
    S = P.InstanceSet([inst])
    st = P.AlnsState(S, [0], chains, P.alns_params(**kw), seed, dev(ops), dev(rt))
    tr = st.set_trace(iters)
    st.step(iters)
    torch.cuda.synchronize()
    assert np.array_equal(tr.cpu().numpy(), ref["trace"])
    info = st.state()
    assert np.array_equal(info["zb"], ref["best_mk"])
    assert np.array_equal(info["T"].view(np.uint64), ref["T"].view(np.uint64))
    st.close()
