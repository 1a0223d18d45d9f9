"""brkga_decode_eval_noalloc (the decoder on the library's fixed workspace)
against brkga_decode_eval, bit for bit, through the C-ABI: two calls in a
row on one GPU, the second smaller than the first (the fixed workspace keeps
the first call's contents), with and without sequences and instance arrays;
batches beyond the workspace are rejected."""
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


def _same(a, b, keys):
    for k in keys:
        assert torch.equal(a[k], b[k]), k


KEYS = ("fitness", "makespan", "unscheduled", "status")


def test_noalloc_matches_allocating_decoder_twice(orc, P):
    big = synth.make_instance(1000, 10, 10, 100, "1R20d10", seed=3003)
    small = synth.make_instance(120, 4, 5, 20, "2x", seed=4004)
    for inst, B, seed in ((big, 1024, 11), (small, 200, 12)):
        S = P.InstanceSet([inst])
        prio, hint = synth.random_keys(B, inst.n, seed=seed, special=True)
        p, h = dev(prio), dev(hint)
        ref = P.brkga_decode_eval(S, p, h, want_ops=True)
        got = P.brkga_decode_eval_noalloc(S, p, h, want_ops=True)
        torch.cuda.synchronize()
        _same(got, ref, KEYS + ("ops", "rt_end"))
        # and without sequences (no schedule log in the workspace)
        got2 = P.brkga_decode_eval_noalloc(S, p, None)
        ref2 = P.brkga_decode_eval(S, p, None)
        torch.cuda.synchronize()
        _same(got2, ref2, KEYS)
        # the hint-first vehicle rule
        got3 = P.brkga_decode_eval_noalloc(S, p, h, want_ops=True, flags=P.DECODE_HINT_FIRST)
        ref3 = P.brkga_decode_eval(S, p, h, want_ops=True, flags=P.DECODE_HINT_FIRST)
        torch.cuda.synchronize()
        _same(got3, ref3, KEYS + ("ops", "rt_end"))
        # a few against the oracle as well
        f = got["fitness"].cpu().numpy()
        for b in range(0, B, max(1, B // 6)):
            assert f[b] == orc.decode(inst, prio[b], hint[b])["fitness"], b


def test_noalloc_instance_array_and_output_reuse(P):
    insts = [synth.make_instance(n, m, 5, 4 * m, "base", seed=500 + n) for n, m in ((300, 6), (40, 3), (17, 2))]
    S = P.InstanceSet(insts)
    B = 600
    g = np.random.default_rng(5)
    ids = g.integers(0, 3, B).astype(np.int32)
    prio, hint = synth.random_keys(B, S.n_max, seed=21)
    p, h, i = dev(prio), dev(hint), dev(ids)
    ref = P.brkga_decode_eval(S, p, h, inst=i, want_ops=True)
    out = P.brkga_decode_eval(S, p, h, inst=i, want_ops=True)   # preallocated outputs, overwritten
    for t in out.values():
        t.fill_(-1) if t.dtype != torch.uint16 else t.zero_()
    got = P.brkga_decode_eval_noalloc(S, p, h, inst=i, out=out)
    torch.cuda.synchronize()
    _same(got, ref, KEYS + ("ops", "rt_end"))
    # second, smaller call on the same outputs' prefix
    sub = {k: v[:100] for k, v in out.items()}
    got = P.brkga_decode_eval_noalloc(S, p[:100], h[:100], inst=i[:100], out=sub)
    ref = P.brkga_decode_eval(S, p[:100], h[:100], inst=i[:100], want_ops=True)
    torch.cuda.synchronize()
    _same(got, ref, KEYS + ("ops", "rt_end"))


def test_noalloc_rejects_batches_beyond_the_workspace(P):
    assert P.brkga_decode_noalloc_max_bytes() == 32 << 20
    inst = synth.make_instance(1000, 10, 10, 100, "1R20d10", seed=3003)
    S = P.InstanceSet([inst])
    for B, want_ops in ((8191, False), (2731, True)):
        prio = torch.zeros((B, 2 * inst.n), dtype=torch.float32, device="cuda")
        with pytest.raises(P.VrpError, match="fixed one holds"):
            P.brkga_decode_eval_noalloc(S, prio, None, want_ops=want_ops)
    # the largest batches that fit still run, and match
    prio, hint = synth.random_keys(8190, inst.n, seed=31)
    p, h = dev(prio), dev(hint)
    got = P.brkga_decode_eval_noalloc(S, p, h)
    ref = P.brkga_decode_eval(S, p, h)
    torch.cuda.synchronize()
    _same(got, ref, KEYS)
    # empty batch: nothing to do
    P.brkga_decode_eval_noalloc(S, p[:0], h[:0])
