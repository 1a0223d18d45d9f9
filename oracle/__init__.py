"""CPU oracle for VRP-RPD — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference implementations of everything the
GPU path computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP library (``paper_2602_23685_amd``) and never imports it.

The C core (``oracle/*.c``) is built with gcc into ``oracle/liboracle.so`` by
:func:`build`; these wrappers marshal numpy arrays into it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["eval.c", "decode.c", "scan.c", "brkga.c", "alns.c", "construct.c", "stats.c"]

BAD_COVER, LOAD, RES, DEADLOCK, BAD_KEY, BAD_TUPLE = 1, 2, 4, 8, 16, 32
MIN_PRELOAD, FULL_START = 0, 1
INT32_MAX = 2**31 - 1
INT64_MAX = 2**63 - 1

TUPLE_DTYPE = np.dtype([("c", "<u2"), ("vD", "u1"), ("vP", "u1"), ("pD", "<u2"), ("pP", "<u2")])


def build(verbose: bool = False, out: str | None = None, opt: str = "-O2", extra: tuple = ()) -> str:
    """Compile the oracle's C sources with gcc (plain -O2, no FP contraction)
    into ``out`` (default: the library :func:`lib` loads); ``opt`` and
    ``extra`` change the optimisation level and add flags (the sanitizer
    test builds a checked copy this way)."""
    out = out or LIB_PATH
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = out + ".tmp"
    cmd = ["gcc", opt, "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", *extra,
           "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


class _Inst(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("k", C.c_int32), ("R", C.c_int32),
                ("load_model", C.c_int32), ("d", C.c_void_p), ("p", C.c_void_p)]


_lib = None


def lib():
    """The oracle's C core: ``liboracle.so`` (built on first use), or the
    library named by VRPRPD_ORACLE_LIB (the sanitizer test's checked copy)."""
    global _lib
    if _lib is None:
        path = os.environ.get("VRPRPD_ORACLE_LIB") or LIB_PATH
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(path)
        _declare(_lib)
    return _lib


def _declare(L):
    P = C.c_void_p
    L.orc_eval.restype = C.c_uint32
    L.orc_eval.argtypes = [P, C.c_int, P, P, P, P]
    L.orc_eval_dag.restype = C.c_uint32
    L.orc_eval_dag.argtypes = [P, P, P, P, P]
    L.orc_eval_batch.restype = None
    L.orc_eval_batch.argtypes = [P, C.c_int, C.c_int64, P, P, P, P, P, P]
    L.orc_insert_scan.restype = None
    L.orc_insert_scan.argtypes = [P, P, P, C.c_int64, P, C.c_int32, P, P, P, P]
    L.orc_decode.restype = C.c_uint32
    L.orc_decode.argtypes = [P, P, P, P, P, P, P, P]
    L.orc_decode_ex.restype = C.c_uint32
    L.orc_decode_ex.argtypes = [P, P, P, P, P, P, P, P, C.c_int32]
    L.orc_philox.restype = None
    L.orc_philox.argtypes = [P, P, P]
    L.orc_brkga_evolve.restype = None
    L.orc_brkga_evolve.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_int32, C.c_int32,
                                   C.c_uint32, C.c_uint64, C.c_uint32, P, P, P]
    L.orc_brkga_warm_start.restype = None
    L.orc_brkga_warm_start.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, P, P]
    L.orc_brkga_warm_start_multi.restype = None
    L.orc_brkga_warm_start_multi.argtypes = [P, C.c_int32, P, C.c_int64, P, C.c_int64, P, C.c_int32, C.c_int32,
                                             C.c_uint64, P, P]
    L.orc_construct.restype = C.c_int32
    L.orc_construct.argtypes = [P, C.c_int32, P, P, P, P]
    L.orc_cons_vehicles.restype = C.c_int32
    L.orc_cons_vehicles.argtypes = [P]
    L.orc_cons_angle_order.restype = None
    L.orc_cons_angle_order.argtypes = [P, P]
    L.orc_cons_sectors.restype = C.c_int32
    L.orc_cons_sectors.argtypes = [P, P, P]
    L.orc_solution_stats.restype = C.c_int32
    L.orc_solution_stats.argtypes = [P, P, P, P, P]
    if hasattr(L, "orc_alns_run"):
        _declare_alns(L)


class AlnsParams(C.Structure):
    """Table 2 hyper-parameters (Section 4.2.7) plus this build's repair budget."""
    _fields_ = [("T0", C.c_double), ("alpha", C.c_double), ("reheat", C.c_double), ("gate", C.c_double),
                ("stag_limit", C.c_int32), ("tau", C.c_int32), ("r", C.c_double),
                ("sigma1", C.c_int32), ("sigma2", C.c_int32), ("sigma3", C.c_int32),
                ("w_min", C.c_double), ("q_min", C.c_int32), ("q_max", C.c_int32),
                ("tuple_budget", C.c_int32), ("import_interval", C.c_int32), ("op_mask", C.c_uint32),
                ("ls_repos_interval", C.c_int32), ("ls_reloc_interval", C.c_int32), ("ls_budget", C.c_int32)]


def alns_params(**kw):
    """Table 2 defaults: T0 = 0.30, alpha = 0.9998, reheat 0.50 after 2000
    stagnant iterations (temperature gate 1% of T_init), tau = 100, r = 0.1,
    sigma = (33, 9, 13), minimum weight 0.1, intra-GPU import every 1000."""
    d = dict(T0=0.30, alpha=0.9998, reheat=0.50, gate=0.01, stag_limit=2000, tau=100, r=0.1,
             sigma1=33, sigma2=9, sigma3=13, w_min=0.1, q_min=0, q_max=0, tuple_budget=0,
             import_interval=1000, op_mask=0x0F3F,
             ls_repos_interval=200, ls_reloc_interval=500, ls_budget=16384)
    d.update(kw)
    return AlnsParams(**d)


def _declare_alns(L):
    P = C.c_void_p
    L.orc_alns_run.restype = C.c_int32
    L.orc_alns_run.argtypes = [P, P, C.c_int32, C.c_int64, C.c_uint64, P, P, P, P, P, P]
    L.orc_alns_run_from.restype = C.c_int32
    L.orc_alns_run_from.argtypes = [P, P, C.c_int32, C.c_int64, C.c_uint64, P, P, P, P, P, P, C.c_uint32]
    L.orc_alns_run_ex.restype = C.c_int32
    L.orc_alns_run_ex.argtypes = [P, P, C.c_int32, C.c_int64, C.c_uint64, P, P, P, P, P, P, C.c_uint32, P, P]
    L.orc_det_exp.restype = C.c_double
    L.orc_det_exp.argtypes = [C.c_double]
    L.orc_alns_qrange.restype = None
    L.orc_alns_qrange.argtypes = [C.c_int, P, P]
    L.orc_alns_local_search.restype = C.c_int32
    L.orc_alns_local_search.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P]
    L.orc_alns_destroy.restype = C.c_int32
    L.orc_alns_destroy.argtypes = [P, C.c_int32, P, P, C.c_int32, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32,
                                   C.c_int32, P]
    L.orc_alns_update.restype = C.c_int32
    L.orc_alns_update.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_int64]
    L.orc_alns_enumerate.restype = C.c_int32
    L.orc_alns_enumerate.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int32, P]
    L.orc_alns_repair.restype = C.c_int32
    L.orc_alns_repair.argtypes = [P, C.c_int32, P, P, P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P]
    L.orc_alns_budget_split.restype = None
    L.orc_alns_budget_split.argtypes = [C.c_int32, C.c_int32, P, P]


class AlnsChain(C.Structure):
    """The scalars Algorithm 1 keeps per chain (current and best makespan,
    temperature, weights, scores, attempts, stagnation)."""
    _fields_ = [("z", C.c_int32), ("zb", C.c_int32), ("T", C.c_double), ("T_init", C.c_double),
                ("wD", C.c_double * 6), ("wR", C.c_double * 4), ("sD", C.c_int64 * 6), ("sR", C.c_int64 * 4),
                ("aD", C.c_int32 * 6), ("aR", C.c_int32 * 4), ("stag", C.c_int32)]


def alns_chain(z, zb=None, T=None, T0=0.30):
    """A chain as Algorithm 1 initialises it from a solution of makespan z."""
    c = AlnsChain()
    c.z = z
    c.zb = z if zb is None else zb
    c.T = T0 * c.zb if T is None else T
    c.T_init = c.T
    for i in range(6):
        c.wD[i] = 1.0
    for i in range(4):
        c.wR[i] = 1.0
    return c


def alns_update(params, chain, di, ri, repaired, zn, u, it):
    """Algorithm 1 after one repair on `chain` (updated in place); returns 0
    rejected, 1 improving, 2 new best, 3 accepted by annealing."""
    return int(lib().orc_alns_update(C.byref(params), C.byref(chain), di, ri, int(repaired), zn, float(u), it))


def alns_enumerate(inst, ops, rt_end, c, KD=0, KP=0):
    """Ranked insertion tuples of customer c against a partial solution."""
    oi = _oinst(inst)
    ops = np.ascontiguousarray(ops, dtype=np.uint16)
    rt = np.ascontiguousarray(rt_end, dtype=np.uint16)
    cap = (2 * oi.n + oi.m + 2) ** 2
    out = np.zeros(cap, dtype=TUPLE_DTYPE)
    T = lib().orc_alns_enumerate(oi.ref, _ptr(ops), _ptr(rt), c, KD, KP, _ptr(out))
    return out[:T]


def alns_repair(inst, op, ops, rt_end, removed, KD=0, KP=0):
    """One repair (0 greedy, 1 regret-2, 2 regret-3, 3 regret-m) of a partial
    solution; returns (ok, makespan, ops, rt_end, insertion order)."""
    oi = _oinst(inst)
    ops = np.ascontiguousarray(ops, dtype=np.uint16)
    rt = np.ascontiguousarray(rt_end, dtype=np.uint16)
    rem = np.ascontiguousarray(removed, dtype=np.int32)
    oo = np.zeros(2 * oi.n + 2, np.uint16)
    orr = np.zeros(oi.m, np.uint16)
    z = np.zeros(1, np.int32)
    order = np.zeros(max(len(rem), 1), np.int32)
    ok = lib().orc_alns_repair(oi.ref, op, _ptr(ops), _ptr(rt), _ptr(rem), len(rem), KD, KP, _ptr(oo), _ptr(orr),
                               _ptr(z), _ptr(order))
    return bool(ok), int(z[0]), oo[:int(orr[-1])], orr, [int(x) for x in order[:len(rem)]]


def alns_budget_split(budget, nrem):
    a, b = C.c_int32(), C.c_int32()
    lib().orc_alns_budget_split(budget, nrem, C.byref(a), C.byref(b))
    return a.value, b.value


def det_exp(x):
    return lib().orc_det_exp(float(x))


def alns_qrange(n):
    a, b = C.c_int(), C.c_int()
    lib().orc_alns_qrange(n, C.byref(a), C.byref(b))
    return a.value, b.value


def alns_destroy(inst, op, ops, rt_end, q, q_min, seed, it, chain, cand=0):
    """Removed customers (list) of destroy operator `op` on a complete
    solution, as in iteration `it` of chain `chain`, candidate `cand`."""
    oi = _oinst(inst)
    ops = np.ascontiguousarray(ops, dtype=np.uint16)
    rt = np.ascontiguousarray(rt_end, dtype=np.uint16)
    rem = np.zeros(oi.n + 1, dtype=np.int32)
    cnt = lib().orc_alns_destroy(oi.ref, op, _ptr(ops), _ptr(rt), q, q_min, seed & (2**64 - 1), it, chain, cand,
                                 _ptr(rem))
    if cnt < 0:
        raise ValueError("solution is not feasible")
    return [int(x) for x in rem[:cnt]]


def alns_local_search(inst, kind, ops, rt_end, budget=16384, passes=3):
    """(improving passes, makespan, ops, rt_end) of the periodic local search
    (kind 0 pickup repositioning, 1 cross-agent relocation)."""
    oi = _oinst(inst)
    ops = np.ascontiguousarray(ops, dtype=np.uint16)
    rt = np.ascontiguousarray(rt_end, dtype=np.uint16)
    oo = np.zeros(2 * oi.n, np.uint16)
    orr = np.zeros(oi.m, np.uint16)
    z = np.zeros(1, np.int32)
    k = lib().orc_alns_local_search(oi.ref, kind, budget, passes, _ptr(ops), _ptr(rt), _ptr(oo), _ptr(orr), _ptr(z))
    if k < 0:
        raise ValueError("solution is not feasible")
    return int(k), int(z[0]), oo[:int(orr[-1])], orr


def alns_run(inst, params, chains, iterations, seed, init_ops, init_rt, trace=False, chain0=0):
    """Run ALNS chains from one initial solution.  Returns dict(best_mk [chains],
    best_ops [chains, 2n], best_rt [chains, m], z [chains] (final current
    makespans), T [chains], wD [chains, 6], wR [chains, 4] (final temperatures
    and operator weights), trace [chains, iters, 4]).
    chain0: index of the first chain in the random-draw counters."""
    oi = _oinst(inst)
    init_ops = np.ascontiguousarray(init_ops, dtype=np.uint16)
    init_rt = np.ascontiguousarray(init_rt, dtype=np.uint16)
    bo = np.zeros((chains, 2 * oi.n), dtype=np.uint16)
    br = np.zeros((chains, oi.m), dtype=np.uint16)
    bm = np.zeros(chains, dtype=np.int32)
    z = np.zeros(chains, dtype=np.int32)
    fs = np.zeros((chains, 11), dtype=np.float64)
    tr = np.zeros((chains, iterations, 4), dtype=np.int64) if trace else None
    lib().orc_alns_run_ex(oi.ref, C.byref(params), chains, iterations, seed & (2**64 - 1), _ptr(init_ops),
                          _ptr(init_rt), _ptr(bo), _ptr(br), _ptr(bm), _ptr(tr), chain0, _ptr(z), _ptr(fs))
    out = dict(best_mk=bm, best_ops=bo, best_rt=br, z=z, T=fs[:, 0].copy(), wD=fs[:, 1:7].copy(),
               wR=fs[:, 7:11].copy())
    if trace:
        out["trace"] = tr
    return out


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OInst:
    """Holds the instance arrays alive for the duration of oracle calls."""

    def __init__(self, inst):
        self.n, self.m, self.k, self.R = inst.n, inst.m, inst.k, inst.R
        self.load_model = inst.load_model
        self.d = np.ascontiguousarray(inst.d, dtype=np.int32)
        self.p = np.ascontiguousarray(inst.p, dtype=np.int32)
        self.s = _Inst(self.n, self.m, self.k, self.R, self.load_model,
                       self.d.ctypes.data, self.p.ctypes.data)

    @property
    def ref(self):
        return C.byref(self.s)


def _oinst(inst):
    return inst if isinstance(inst, OInst) else OInst(inst)


def eval_one(inst, ops, rt_end, allow_partial=False, times=False, dag=False):
    """Evaluate one candidate.  Returns (makespan, status) or, with times,
    (makespan, status, op_time[L])."""
    oi = _oinst(inst)
    ops = np.ascontiguousarray(ops, dtype=np.uint16)
    rt = np.ascontiguousarray(rt_end, dtype=np.uint16)
    mk = np.zeros(1, dtype=np.int32)
    L = int(rt[-1]) if len(rt) else 0
    tt = np.full(max(L, 1), -1, dtype=np.int64) if times else None
    if dag:
        st = lib().orc_eval_dag(oi.ref, _ptr(ops), _ptr(rt), _ptr(mk), _ptr(tt))
    else:
        st = lib().orc_eval(oi.ref, int(allow_partial), _ptr(ops), _ptr(rt), _ptr(mk), _ptr(tt))
    if times:
        return int(mk[0]), int(st), tt[:L]
    return int(mk[0]), int(st)


def eval_batch(inst, ops, rt_end, op_off=None, rt_off=None, allow_partial=False):
    """Evaluate B candidates.  ops: [B, 2n] (or flat with op_off), rt_end: [B, m]
    (or flat with rt_off).  Returns (makespan int32[B], status uint32[B])."""
    oi = _oinst(inst)
    ops = np.ascontiguousarray(ops, dtype=np.uint16)
    rt = np.ascontiguousarray(rt_end, dtype=np.uint16)
    if op_off is None:
        B = ops.shape[0] if ops.ndim == 2 else len(ops) // (2 * oi.n)
    else:
        op_off = np.ascontiguousarray(op_off, dtype=np.int64)
        B = len(op_off)
    if rt_off is not None:
        rt_off = np.ascontiguousarray(rt_off, dtype=np.int64)
    mk = np.zeros(B, dtype=np.int32)
    st = np.zeros(B, dtype=np.uint32)
    lib().orc_eval_batch(oi.ref, int(allow_partial), B, _ptr(op_off), _ptr(ops), _ptr(rt_off),
                         _ptr(rt), _ptr(mk), _ptr(st))
    return mk, st


def insert_scan(inst, base_ops, base_rt, tuples, seg_off):
    oi = _oinst(inst)
    base_ops = np.ascontiguousarray(base_ops, dtype=np.uint16)
    base_rt = np.ascontiguousarray(base_rt, dtype=np.uint16)
    tuples = np.ascontiguousarray(tuples).astype(TUPLE_DTYPE, copy=False)
    seg_off = np.ascontiguousarray(seg_off, dtype=np.int64)
    T, S = len(tuples), len(seg_off) - 1
    mk = np.zeros(max(T, 1), dtype=np.int32)
    st = np.zeros(max(T, 1), dtype=np.uint32)
    top = np.zeros((max(S, 1), 3), dtype=np.int64)
    lib().orc_insert_scan(oi.ref, _ptr(base_ops), _ptr(base_rt), T, _ptr(tuples), S,
                          _ptr(seg_off), _ptr(mk), _ptr(st), _ptr(top))
    return mk[:T], st[:T], top[:S]


DECODE_HINT_FIRST = 1


def decode(inst, prio, hint=None, want_ops=False, flags=0):
    """Decode one chromosome.  Returns dict(fitness, makespan, unscheduled,
    status[, ops, rt_end]).  flags: DECODE_HINT_FIRST (the hint vehicle takes
    an op whenever it can)."""
    oi = _oinst(inst)
    prio = np.ascontiguousarray(prio, dtype=np.float32)
    hint = None if hint is None else np.ascontiguousarray(hint, dtype=np.float32)
    f = np.zeros(1, dtype=np.int64)
    mk = np.zeros(1, dtype=np.int32)
    un = np.zeros(1, dtype=np.int32)
    ops = np.zeros(2 * oi.n, dtype=np.uint16) if want_ops else None
    rt = np.zeros(oi.m, dtype=np.uint16) if want_ops else None
    st = lib().orc_decode_ex(oi.ref, _ptr(prio), _ptr(hint), _ptr(f), _ptr(mk), _ptr(un),
                             _ptr(ops), _ptr(rt), int(flags))
    out = dict(fitness=int(f[0]), makespan=int(mk[0]), unscheduled=int(un[0]), status=int(st))
    if want_ops:
        out["ops"] = ops[: int(rt[-1])] if rt[-1] else ops[:0]
        out["rt_end"] = rt
    return out


def decode_batch(inst, prio, hint=None, flags=0):
    oi = _oinst(inst)
    B = prio.shape[0]
    f = np.zeros(B, dtype=np.int64)
    mk = np.zeros(B, dtype=np.int32)
    un = np.zeros(B, dtype=np.int32)
    st = np.zeros(B, dtype=np.uint32)
    for b in range(B):
        r = decode(oi, prio[b], None if hint is None else hint[b], flags=flags)
        f[b], mk[b], un[b], st[b] = r["fitness"], r["makespan"], r["unscheduled"], r["status"]
    return f, mk, un, st


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def rho_threshold(rho: float) -> int:
    """Integer threshold of the Bernoulli(rho) draw: (w >> 8) < floor(rho * 2^24)."""
    return int(np.floor(rho * 16777216.0))


def brkga_sizes(Np, elite_frac=0.15, mutant_frac=0.15):
    return int(np.floor(elite_frac * Np)), int(np.floor(mutant_frac * Np))


def brkga_evolve(prio, hint, fitness, n_elite, n_mutant, rho_thr24, seed, generation):
    prio = np.ascontiguousarray(prio, dtype=np.float32)
    Np, G = prio.shape
    hint = None if hint is None else np.ascontiguousarray(hint, dtype=np.float32)
    fitness = np.ascontiguousarray(fitness, dtype=np.int64)
    po = np.zeros_like(prio)
    ho = None if hint is None else np.zeros_like(hint)
    rank = np.zeros(Np, dtype=np.int32)
    lib().orc_brkga_evolve(Np, G, _ptr(prio), _ptr(hint), _ptr(fitness), n_elite, n_mutant,
                           rho_thr24, seed & (2**64 - 1), generation, _ptr(po), _ptr(ho),
                           _ptr(rank))
    return po, ho, rank


def brkga_warm_start(inst, ops, rt_end, Np, n_warm, n_variants, seed):
    oi = _oinst(inst)
    ops = np.ascontiguousarray(ops, dtype=np.uint16)
    rt = np.ascontiguousarray(rt_end, dtype=np.uint16)
    G = 2 * oi.n
    po = np.zeros((Np, G), dtype=np.float32)
    ho = np.zeros((Np, G), dtype=np.float32)
    lib().orc_brkga_warm_start(oi.ref, _ptr(ops), _ptr(rt), Np, n_warm, n_variants,
                               seed & (2**64 - 1), _ptr(po), _ptr(ho))
    return po, ho


def brkga_warm_start_multi(inst, sources, n_var, Np, n_warm, seed):
    """Warm start from several solutions: sources = [(ops, rt_end), ...],
    n_var[s] variants of source s (Section 4.4.4)."""
    oi = _oinst(inst)
    S = len(sources)
    ops = np.zeros((S, 2 * oi.n), np.uint16)
    rt = np.zeros((S, oi.m), np.uint16)
    for s, (o, r) in enumerate(sources):
        ops[s, :len(o)] = o
        rt[s] = r
    nv = np.ascontiguousarray(n_var, dtype=np.int32)
    G = 2 * oi.n
    po = np.zeros((Np, G), dtype=np.float32)
    ho = np.zeros((Np, G), dtype=np.float32)
    lib().orc_brkga_warm_start_multi(oi.ref, S, _ptr(ops), 2 * oi.n, _ptr(rt), oi.m, _ptr(nv), Np, n_warm,
                                     seed & (2**64 - 1), _ptr(po), _ptr(ho))
    return po, ho


CONS_SWEEP, CONS_NN, CONS_LB, CONS_SPT = 0, 1, 2, 3


def construct(inst, heuristic, order=False):
    """One construction heuristic (0 sweep + balance + per-vehicle nearest
    neighbour, 1 nearest neighbour, 2 load balanced, 3 shortest processing
    time).  Returns (ops, rt_end), plus the placement order [(vehicle, op)]
    when order is set."""
    oi = _oinst(inst)
    ops = np.zeros(2 * oi.n, np.uint16)
    rt = np.zeros(oi.m, np.uint16)
    sv = np.zeros(2 * oi.n, np.int32)
    so = np.zeros(2 * oi.n, np.int32)
    cnt = lib().orc_construct(oi.ref, heuristic, _ptr(ops), _ptr(rt), _ptr(sv), _ptr(so))
    res = (ops[:cnt], rt)
    if order:
        return res + (list(zip(sv[:cnt].tolist(), so[:cnt].tolist())),)
    return res


def cons_vehicles(inst):
    return int(lib().orc_cons_vehicles(_oinst(inst).ref))


def cons_angle_order(inst):
    oi = _oinst(inst)
    order = np.zeros(oi.n, np.int32)
    lib().orc_cons_angle_order(oi.ref, _ptr(order))
    return order


def cons_sectors(inst):
    """(sectors before balancing, after balancing, moves); index 0 unused."""
    oi = _oinst(inst)
    s0 = np.zeros(oi.n + 1, np.int32)
    s1 = np.zeros(oi.n + 1, np.int32)
    moves = lib().orc_cons_sectors(oi.ref, _ptr(s0), _ptr(s1))
    return s0, s1, int(moves)


def refine(inst, ops, rt_end, budget=16384, max_rounds=1000):
    """The construction's refinement (Section 4.2, initial solution, last
    phase): rounds of pickup repositioning then cross-agent relocation (up
    to three passes each, Section 4.2.6) until a round improves nothing.
    Returns (rounds run, makespan, ops, rt_end)."""
    z = eval_one(inst, ops, rt_end)[0]
    rounds = 0
    while rounds < max_rounds:
        rounds += 1
        k0, z, ops, rt_end = alns_local_search(inst, 0, ops, rt_end, budget=budget, passes=3)
        k1, z, ops, rt_end = alns_local_search(inst, 1, ops, rt_end, budget=budget, passes=3)
        if k0 == 0 and k1 == 0:
            break
    return rounds, int(z), ops, rt_end


def solution_stats(inst, ops, rt_end):
    """(cross-vehicle customers, interleaved customers) of a solution
    (Section 5.2), or None when its cover is incomplete or it deadlocks."""
    oi = _oinst(inst)
    ops = np.ascontiguousarray(ops, dtype=np.uint16)
    rt = np.ascontiguousarray(rt_end, dtype=np.uint16)
    x = np.zeros(2, np.int32)
    rc = lib().orc_solution_stats(oi.ref, _ptr(ops), _ptr(rt), _ptr(x[:1]), _ptr(x[1:]))
    return None if rc < 0 else (int(x[0]), int(x[1]))


def int32_safe(inst) -> bool:
    """Whether every time of every schedule fits in int32: a longest path
    has at most one incoming edge per op (travel or processing) plus the
    return leg."""
    dmax = int(np.max(inst.d))
    return (2 * inst.n + 1) * dmax + int(np.sum(inst.p, dtype=np.int64)) < 2**31 - 1
