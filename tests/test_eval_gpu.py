"""Parity: vrprpd_eval on the GPU vs the CPU oracle, element by element.

Makespans are integers and must match bit for bit, status bits too."""
import numpy as np
import pytest

import synth
from cases import destroy, flat, mutate

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


def gpu_eval(P, S, ops, rt, **kw):
    kw2 = {k: (dev(v) if isinstance(v, np.ndarray) else v) for k, v in kw.items()}
    mk, st = P.vrprpd_eval(S, dev(ops), dev(rt), **kw2)
    torch.cuda.synchronize()
    return mk.cpu().numpy(), st.cpu().numpy().view(np.uint32)


FORMS = ((0, "staged"), (1, "live legs"))


def check(orc, P, inst, ops, rt, label, partial=False, op_off=None):
    """Both forms of the evaluation kernel against the oracle."""
    S = P.InstanceSet([inst])
    if op_off is None:
        omk, ost = orc.eval_batch(inst, ops, rt, allow_partial=partial)
    else:
        rt_off = np.arange(len(op_off), dtype=np.int64) * inst.m
        omk, ost = orc.eval_batch(inst, ops, rt.reshape(-1), op_off=op_off, rt_off=rt_off,
                                  allow_partial=partial)
    for form, name in FORMS:
        P.vrprpd_eval_set_shape(S, inst.n, inst.m, 0, 4, form)
        if op_off is None:
            mk, st = gpu_eval(P, S, ops, rt, partial=partial)
        else:
            mk, st = gpu_eval(P, S, ops, rt.reshape(-1), op_off=op_off, rt_off=rt_off, partial=partial)
        bad = np.nonzero((mk != omk) | (st != ost))[0]
        assert bad.size == 0, (f"{label} ({name}): {bad.size} mismatches, first b={bad[0]} gpu=({mk[bad[0]]},"
                               f"{st[bad[0]]}) oracle=({omk[bad[0]]},{ost[bad[0]]})")
    return omk, ost


CONFIGS = [
    # (n, m, k, R, rule, load_model, B)
    (16, 2, 2, 4, "base", 0, 4096),        # depot + 16 customers, 2 vehicles (small parity case)
    (100, 4, 5, 20, "2x", 0, 2048),        # 100 customers, 4 vehicles
    (1000, 10, 10, 100, "1R20d10", 0, 256),  # full scale, 1000 customers, 10 vehicles
    (240, 4, 7, 24, "5x", 1, 512),
    (37, 17, 3, 30, "1R10", 0, 512),       # 17 vehicles -> 32-lane groups
    (50, 40, 2, 80, "base", 0, 256),       # 40 vehicles -> full-wave groups
    (1, 1, 1, 1, "base", 0, 8),
    (3, 64, 1, 64, "base", 0, 64),         # most vehicles empty
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: f"n{c[0]}m{c[1]}")
def test_eval_parity_random_feasible(orc, P, cfg):
    n, m, k, R, rule, lm, B = cfg
    inst = synth.make_instance(n, m, k, R, rule, seed=1000 + n, load_model=lm)
    ops, rt = synth.random_candidates(inst, B, seed=n + m)
    omk, ost = check(orc, P, inst, ops, rt, f"feasible n={n}")
    assert (ost == 0).mean() > 0.5 or lm == 1 or n == 1


@pytest.mark.parametrize("cfg", CONFIGS[:6], ids=lambda c: f"n{c[0]}m{c[1]}")
def test_eval_parity_adversarial(orc, P, cfg):
    n, m, k, R, rule, lm, B = cfg
    inst = synth.make_instance(n, m, k, R, rule, seed=2000 + n, load_model=lm)
    ops, rt = synth.random_candidates(inst, 64, seed=n)
    mops, mrt = mutate(inst, ops, rt, seed=n, count=min(B, 1024))
    omk, ost = check(orc, P, inst, mops, mrt, f"adversarial n={n}")
    assert (ost & 8).any() and (ost & 1).any()


@pytest.mark.parametrize("cfg", CONFIGS[:3], ids=lambda c: f"n{c[0]}m{c[1]}")
def test_eval_parity_partial(orc, P, cfg):
    n, m, k, R, rule, lm, B = cfg
    inst = synth.make_instance(n, m, k, R, rule, seed=3000 + n, load_model=lm)
    ops, rt = synth.random_candidates(inst, min(B, 256), seed=n + 1)
    fops, off, frt = destroy(inst, ops, rt, seed=n, q=max(1, n // 20))
    check(orc, P, inst, fops, frt, "partial", partial=True, op_off=off)
    # the same partial solutions without ALLOW_PARTIAL are cover errors
    _, ost = check(orc, P, inst, fops, frt, "partial-strict", partial=False, op_off=off)
    assert np.all(ost == 1)


def test_eval_parity_wide_distances(orc, P):
    """Travel times above 65535 keep the int32 distance layout."""
    inst = synth.make_instance(60, 4, 5, 20, "base", seed=4)
    inst.d = (inst.d.astype(np.int64) * 500).astype(np.int32)
    inst.p = (inst.p.astype(np.int64) * 500).astype(np.int32)
    S = P.InstanceSet([inst])
    assert S.dist16 == 0
    ops, rt = synth.random_candidates(inst, 512, seed=5)
    check(orc, P, inst, ops, rt, "int32 distances")


def test_eval_parity_mixed_instances(orc, P):
    """Instances of uneven size in one launch (per-candidate instance index)."""
    g = synth.rng(77)
    insts, chunks = [], []
    for i in range(12):
        n = int(np.exp(g.uniform(np.log(17), np.log(400))))
        m = int(np.ceil(n / 100)) + 1
        inst = synth.make_instance(n, m, int(g.integers(5, 11)), max(1, n // 10),
                                   ["base", "2x", "5x", "1R10", "1R20"][i % 5], seed=i)
        insts.append(inst)
        chunks.append(synth.random_candidates(inst, 40, seed=100 + i))
    S = P.InstanceSet(insts)
    ops, op_off, rt, rt_off, idx = [], [], [], [], []
    co = cr = 0
    order = g.permutation(sum(len(c[0]) for c in chunks))
    flat_list = [(i, b) for i, c in enumerate(chunks) for b in range(len(c[0]))]
    for t in order:
        i, b = flat_list[t]
        o, r = chunks[i][0][b], chunks[i][1][b]
        ops.append(o); rt.append(r); idx.append(i)
        op_off.append(co); rt_off.append(cr)
        co += len(o); cr += len(r)
    ops = np.concatenate(ops); rt = np.concatenate(rt)
    op_off = np.array(op_off, np.int64); rt_off = np.array(rt_off, np.int64)
    idx = np.array(idx, np.int32)
    refs = [orc.eval_one(insts[idx[t]], ops[op_off[t]:op_off[t] + 2 * insts[idx[t]].n],
                         rt[rt_off[t]:rt_off[t] + insts[idx[t]].m]) for t in range(len(idx))]
    for form, name in FORMS:
        P.vrprpd_eval_set_shape(S, max(x.n for x in insts), max(x.m for x in insts), 0, 4, form)
        mk, st = gpu_eval(P, S, ops, rt, inst=idx, op_off=op_off, rt_off=rt_off)
        for t in range(len(idx)):
            assert (mk[t], st[t]) == refs[t], (name, t)


def test_eval_full_scale_sampled(orc, P):
    """The benchmark's launch: 65,536 candidates at n = 1000, m = 10; the oracle
    re-evaluates a seeded sample of 200 of them."""
    inst = synth.make_instance(1000, 10, 10, 100, "1R20d10", seed=3003)
    base_ops, base_rt = synth.random_candidates(inst, 2048, seed=3)
    reps = 32
    perm = synth.rng(5).permutation(2048 * reps)
    ops = np.tile(base_ops, (reps, 1))[perm]
    rt = np.tile(base_rt, (reps, 1))[perm]
    S = P.InstanceSet([inst])
    pick = synth.rng(6).choice(len(ops), size=200, replace=False)
    omk, ost = orc.eval_batch(inst, ops[pick], rt[pick])
    src = perm % 2048
    first = np.full(2048, -1)
    for i, s_ in enumerate(src):
        if first[s_] < 0:
            first[s_] = i
    for form, name in FORMS:
        P.vrprpd_eval_set_shape(S, 1000, 10, 0, 4, form)
        mk, st = gpu_eval(P, S, ops, rt)
        assert np.array_equal(mk[pick], omk) and np.array_equal(st[pick], ost), name
        # copies of one candidate agree wherever they sit in the batch
        assert np.array_equal(mk, mk[first[src]]), name


def test_eval_set_shape_refuses_bad_options(P):
    inst = synth.make_instance(30, 3, 4, 12, seed=2)
    S = P.InstanceSet([inst])
    for args in [(30, 3, 5, 4, 1), (30, 3, 0, 3, 1), (30, 3, 0, 4, 2), (0, 3, 0, 4, 0), (30, 40, 2, 4, 0)]:
        with pytest.raises(RuntimeError):
            P.vrprpd_eval_set_shape(S, *args)
    P.vrprpd_eval_set_shape(S, 30, 3, 3, 2, 0)


def test_eval_empty_batch(P):
    inst = synth.make_instance(5, 2, 2, 4, seed=1)
    S = P.InstanceSet([inst])
    e16 = torch.empty(0, dtype=torch.uint16, device="cuda")
    mk, st = P.vrprpd_eval(S, e16, e16, B=0)
    assert mk.numel() == 0


@pytest.mark.parametrize("n,m,B", [(100, 4, 4096), (37, 17, 2048), (1000, 10, 2048)])
def test_autotuned_shapes_agree_with_oracle(orc, P, n, m, B):
    """The autotuner runs every launch shape (it checks that they agree bit for
    bit) and later launches use the chosen one; the oracle checks a sample."""
    inst = synth.make_instance(n, m, max(2, n // m), n, "2x", seed=8800 + n)
    ops, rt = synth.random_candidates(inst, B, seed=n)
    S = P.InstanceSet([inst])
    d_ops, d_rt = torch.from_numpy(ops).cuda(), torch.from_numpy(rt).cuda()
    w, k, form, ms = P.vrprpd_autotune_eval(S, d_ops, d_rt, reps=2)
    opts = [2, 3, 4] if m <= 16 else ([1, 2] if m <= 32 else [1])
    assert w in opts and k in (2, 4) and form in (0, 1)
    assert ms[6 * form + 2 * opts.index(w) + (k == 4)] > 0
    for f in (0, 1):   # both forms; the smallest option always fits
        assert np.all(ms[6 * f:6 * f + 2] > 0)
        assert np.all(ms[6 * f + 2 * len(opts):6 * f + 6] == -1)
    mk, st = gpu_eval(P, S, ops, rt)
    pick = synth.rng(n).choice(B, size=min(B, 300), replace=False)
    omk, ost = orc.eval_batch(inst, ops[pick], rt[pick])
    assert np.array_equal(mk[pick], omk) and np.array_equal(st[pick], ost)


def test_gather_rate_measurement(P):
    """vrprpd_gather_rate runs (16-bit and 32-bit matrices) and reports a
    positive rate; bad arguments are refused."""
    inst = synth.make_instance(200, 4, 5, 20, "base", seed=12)
    rate, ms = P.vrprpd_gather_rate(P.InstanceSet([inst]), 0, blocks=64, per_thread=32)
    assert rate > 0 and ms > 0
    inst.d = (inst.d.astype(np.int64) * 500).astype(np.int32)
    S = P.InstanceSet([inst])
    assert S.dist16 == 0
    assert P.vrprpd_gather_rate(S, 0, blocks=64, per_thread=32)[0] > 0
    with pytest.raises(P.VrpError):
        P.vrprpd_gather_rate(S, 1, blocks=64, per_thread=32)
    with pytest.raises(P.VrpError):
        P.vrprpd_gather_rate(S, 0, blocks=64, per_thread=20)
