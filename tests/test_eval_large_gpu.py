"""vrprpd_eval on batches of millions of candidates in one launch, every
output checked against the oracle: each candidate of the batch is a copy of
one of a few thousand seeded base candidates (feasible ones and adversarial
variants) that the oracle evaluates, placed at a random position of the
batch, so the whole launch is compared at the cost of the bases."""
import numpy as np
import pytest

import synth
from cases import mutate

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


def test_eval_four_million_candidates_one_instance(orc, P):
    """2^22 candidates at n = 16, m = 2 (the 16-customer workload's shape) in
    one launch per form: 2,048 bases (a quarter of them adversarial)."""
    inst = synth.make_instance(16, 2, 2, 4, "base", seed=9600)
    ops, rt = synth.random_candidates(inst, 1536, seed=9601)
    mops, mrt = mutate(inst, ops, rt, seed=9602, count=512)
    bops, brt = np.concatenate([ops, mops]), np.concatenate([rt, mrt])
    omk, ost = orc.eval_batch(inst, bops, brt)
    assert (ost != 0).sum() > 100 and (ost == 0).sum() > 1000
    B = 1 << 22
    src = synth.rng(9603).integers(0, len(bops), size=B)
    d_ops, d_rt = dev(bops[src]), dev(brt[src])
    S = P.InstanceSet([inst])
    for form in (0, 1):
        print(f"[large] n=16 B={B} form={form}", flush=True)
        P.vrprpd_eval_set_shape(S, 16, 2, 0, 4, form)
        mk, st = P.vrprpd_eval(S, d_ops, d_rt)
        torch.cuda.synchronize()
        mk, st = mk.cpu().numpy(), st.cpu().numpy().view(np.uint32)
        bad = np.nonzero((mk != omk[src]) | (st != ost[src]))[0]
        assert bad.size == 0, (form, bad.size, int(bad[0]), int(src[bad[0]]))


def test_eval_a_million_candidates_over_uneven_instances(orc, P):
    """2^20 candidates over 200 instances of uneven size (n log-uniform in
    [17, 200], m = ceil(n/100) + 1, the five processing rules) in one launch
    per form, with per-candidate instance, op and route-end offsets."""
    insts = synth.batched_instances(count=200, seed=9700, n_min=17, n_max=200)
    S = P.InstanceSet(insts)
    base_ops, base_rt, base_inst, omk, ost = [], [], [], [], []
    for i, x in enumerate(insts):
        ops, rt = synth.random_candidates(x, 6, seed=9800 + i)
        mops, mrt = mutate(x, ops, rt, seed=9900 + i, count=2)
        bo, br = np.concatenate([ops, mops]), np.concatenate([rt, mrt])
        mk, st = orc.eval_batch(x, bo, br)
        base_ops += list(bo)
        base_rt += list(br)
        base_inst += [i] * len(bo)
        omk.append(mk)
        ost.append(st)
    omk, ost = np.concatenate(omk), np.concatenate(ost)
    base_inst = np.array(base_inst, np.int32)
    blen = np.array([len(o) for o in base_ops], np.int64)
    bstart = np.concatenate([[0], np.cumsum(blen)[:-1]])
    bflat = np.concatenate(base_ops).astype(np.uint16)
    mlen = np.array([len(r) for r in base_rt], np.int64)
    mstart = np.concatenate([[0], np.cumsum(mlen)[:-1]])
    mflat = np.concatenate(base_rt).astype(np.uint16)

    B = 1 << 20
    src = synth.rng(9701).integers(0, len(base_ops), size=B)
    olen, rlen = blen[src], mlen[src]
    op_off = np.concatenate([[0], np.cumsum(olen)[:-1]])
    rt_off = np.concatenate([[0], np.cumsum(rlen)[:-1]])
    # gather the copies: position p of the flat batch reads its base's entry
    ops_idx = (np.arange(int(olen.sum()), dtype=np.int64) - np.repeat(op_off, olen) + np.repeat(bstart[src], olen))
    rt_idx = (np.arange(int(rlen.sum()), dtype=np.int64) - np.repeat(rt_off, rlen) + np.repeat(mstart[src], rlen))
    d_ops, d_rt = dev(bflat[ops_idx]), dev(mflat[rt_idx])
    del ops_idx, rt_idx
    d_inst, d_ooff, d_roff = dev(base_inst[src]), dev(op_off), dev(rt_off)
    n_max, m_max = max(x.n for x in insts), max(x.m for x in insts)
    for form in (0, 1):
        print(f"[large] uneven B={B} n_max={n_max} form={form}", flush=True)
        P.vrprpd_eval_set_shape(S, n_max, m_max, 0, 4, form)
        mk, st = P.vrprpd_eval(S, d_ops, d_rt, inst=d_inst, op_off=d_ooff, rt_off=d_roff)
        torch.cuda.synchronize()
        mk, st = mk.cpu().numpy(), st.cpu().numpy().view(np.uint32)
        bad = np.nonzero((mk != omk[src]) | (st != ost[src]))[0]
        assert bad.size == 0, (form, bad.size, int(bad[0]), int(src[bad[0]]))
