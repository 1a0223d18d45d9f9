"""Parity at the largest sizes each kernel accepts, and clean refusals just
past them (LDS per workgroup: 160 KB per CU on MI355X)."""
import numpy as np
import pytest

import synth
from cases import destroy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LDS = 160 * 1024


def a16(x):
    return (x + 15) & ~15


def staged_bytes(n):   # one candidate of the staged evaluation, 16-bit times
    return a16(4 * (n + 1)) + a16(4 * ((2 * (n + 1) + 31) // 32)) + a16(4 * (2 * n + 8))


def live_bytes(n):     # one candidate of the live-leg evaluation (16-bit codes above n = 2047;
    return a16(4 * (n + 1)) + a16(2 * (2 * n + 16))   # the cover bits share ready[]'s space)


def scan_bytes(n):     # one scan block (4 waves of four 16-lane groups), 16-bit times
    b = a16(4 * (n + 1)) + a16(4 * ((2 * (n + 1) + 31) // 32)) + a16(4 * 3 * 64)
    b += a16(4 * (2 * n + 4)) + a16(8 * 3 * 16)
    return b + 16 * a16(4 * (n + 1))


def largest(fits, hi=32767):
    n = 1
    while n + 1 <= hi and fits(n + 1):
        n += 1
    return n


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_23685_amd as P
    P.load()
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_eval_both_forms_at_the_staged_limit(orc, P):
    """n at the staged form's limit (two 16-lane candidates per wave): both
    forms against the oracle; the staged form one customer later is refused."""
    n = largest(lambda x: 2 * staged_bytes(x) <= LDS)
    assert 2 * live_bytes(n) <= LDS
    inst = synth.make_instance(n, 16, 4, 64, "2x", seed=9100)
    ops, rt = synth.random_candidates(inst, 37, seed=9101)
    S = P.InstanceSet([inst])
    omk, ost = orc.eval_batch(inst, ops, rt)
    for form in (0, 1):
        P.vrprpd_eval_set_shape(S, n, 16, 2, 4, form)
        mk, st = P.vrprpd_eval(S, dev(ops), dev(rt))
        torch.cuda.synchronize()
        assert np.array_equal(mk.cpu().numpy(), omk), form
        assert np.array_equal(st.cpu().numpy().view(np.uint32), ost), form
    with pytest.raises(RuntimeError):
        P.vrprpd_eval_set_shape(S, n + 1, 16, 2, 4, 0)
    P.vrprpd_eval_set_shape(S, n + 1, 16, 2, 4, 1)      # the live form still fits


@pytest.mark.parametrize("n", [2047, 2048])
def test_eval_live_form_code_width_switch(orc, P, n):
    """The live-leg form packs codes in 12 bits up to n = 2047 (the largest
    code, 4095, fills the field) and keeps 16 bits from n = 2048; both against
    the oracle, with partial solutions and cover errors in the batch."""
    inst = synth.make_instance(n, 12, 6, 72, "2x", seed=9400 + n)
    ops, rt = synth.random_candidates(inst, 40, seed=9401)
    top = 2 * n + 1                                    # the pickup of customer n
    assert (ops == top).any(axis=1).all()
    bad = ops.copy()
    bad[1, 5] = bad[1, 6]                              # a duplicate op
    bad[2, 0] = (n + 1) << 1                           # a customer past n
    ops2 = np.concatenate([ops, bad[1:3]])
    rt2 = np.concatenate([rt, rt[1:3]])
    S = P.InstanceSet([inst])
    omk, ost = orc.eval_batch(inst, ops2, rt2)
    assert (ost == 1).sum() == 2
    for form in (0, 1):
        P.vrprpd_eval_set_shape(S, n, 12, 0, 4, form)
        mk, st = P.vrprpd_eval(S, dev(ops2), dev(rt2))
        torch.cuda.synchronize()
        assert np.array_equal(mk.cpu().numpy(), omk), form
        assert np.array_equal(st.cpu().numpy().view(np.uint32), ost), form


def test_eval_live_form_limit_is_refused(P):
    n = largest(lambda x: 2 * live_bytes(x) <= LDS)
    S = P.InstanceSet([synth.make_instance(20, 16, 2, 20, seed=1)])
    P.vrprpd_eval_set_shape(S, n, 16, 2, 4, 1)
    with pytest.raises(RuntimeError):
        P.vrprpd_eval_set_shape(S, n + 1, 16, 2, 4, 1)


def test_eval_live_form_at_the_largest_instance(orc, P):
    """The largest instance the library accepts (n = 10,000, m = 64) in the
    live-leg form (one 64-lane candidate per wave, 78 KB of LDS), against the
    oracle, with cover errors in the batch."""
    n, m = 10000, 64
    assert 2 * live_bytes(n) <= LDS
    inst = synth.make_instance(n, m, 8, 8 * m, "2x", seed=9500)
    ops, rt = synth.random_candidates(inst, 6, seed=9501)
    bad = ops.copy()
    bad[0, 7] = bad[0, 8]                              # a duplicate op
    bad[1, 3] = (n + 1) << 1                           # a customer past n
    ops2, rt2 = np.concatenate([ops, bad[:2]]), np.concatenate([rt, rt[:2]])
    S = P.InstanceSet([inst])
    omk, ost = orc.eval_batch(inst, ops2, rt2)
    assert (ost == 1).sum() == 2
    P.vrprpd_eval_set_shape(S, n, m, 1, 4, 1)
    mk, st = P.vrprpd_eval(S, dev(ops2), dev(rt2))
    torch.cuda.synchronize()
    assert np.array_equal(mk.cpu().numpy(), omk)
    assert np.array_equal(st.cpu().numpy().view(np.uint32), ost)


def test_decode_at_the_sort_limit(orc, P):
    """2n = 8,192 ops, the most one CU sorts; one customer more is refused."""
    n = 4096
    inst = synth.make_instance(n, 16, 6, 60, "base", seed=9200)
    B = 5
    prio, hint = synth.random_keys(B, n, seed=9201)
    S = P.InstanceSet([inst])
    for flags in (0, P.DECODE_HINT_FIRST):
        out = P.brkga_decode_eval(S, dev(prio), dev(hint), flags=flags)
        torch.cuda.synchronize()
        for b in range(B):
            r = orc.decode(inst, prio[b], hint[b], flags=flags)
            got = (int(out["fitness"][b]), int(out["makespan"][b]), int(out["unscheduled"][b]))
            assert got == (r["fitness"], r["makespan"], r["unscheduled"]), (b, flags)
    big = synth.make_instance(n + 1, 4, 6, 60, "base", seed=9202)
    p2, h2 = synth.random_keys(2, n + 1, seed=9203)
    with pytest.raises(RuntimeError):
        P.brkga_decode_eval(P.InstanceSet([big]), dev(p2), dev(h2))


def test_scan_at_its_limit(orc, P):
    """The largest base the scan stages (16 ready[] arrays per block), against
    the oracle; one customer more is refused."""
    n = largest(lambda x: scan_bytes(x) <= LDS, hi=4000)
    inst = synth.make_instance(n, 16, 16, 256, "2x", seed=9300)
    ops, rt = synth.random_candidates(inst, 1, seed=9301)
    fo, _, frt = destroy(inst, ops, rt, seed=9302, q=6)
    tuples = synth.random_tuples(fo, frt[0], n, 16, 700, seed=9303, invalid_frac=0.05)
    seg_off = np.array([0, 300, 700], np.int64)
    S = P.InstanceSet([inst])
    mk, st, top = P.vrprpd_insert_scan(S, dev(fo), dev(frt[0]), dev(seg_off), dev(tuples.view(np.uint8)))
    torch.cuda.synchronize()
    omk, ost, otop = orc.insert_scan(inst, fo, frt[0], tuples, seg_off)
    assert np.array_equal(mk.cpu().numpy(), omk)
    assert np.array_equal(st.cpu().numpy().view(np.uint32), ost)
    assert np.array_equal(top.cpu().numpy(), otop)
    big = synth.make_instance(n + 1, 16, 16, 256, "2x", seed=9304)
    o2, r2 = synth.random_candidates(big, 1, seed=9305)
    f2, _, fr2 = destroy(big, o2, r2, seed=9306, q=6)
    t2 = synth.random_tuples(f2, fr2[0], n + 1, 16, 10, seed=9307)
    with pytest.raises(RuntimeError):
        P.vrprpd_insert_scan(P.InstanceSet([big]), dev(f2), dev(fr2[0]), dev(np.array([0, 10], np.int64)),
                             dev(t2.view(np.uint8)))
