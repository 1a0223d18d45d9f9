"""ctypes binding of libvrprpd.so: argument marshalling only.

Every computation runs in the library's HIP kernels.  Tensors passed here must
be device tensors; the functions hand their pointers and the current torch
stream to the C-ABI (include/vrprpd.h) and return device tensors.  There is no
fallback: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvrprpd.so")

OK, EINVAL, ERANGE, ENOMEM, EHIP = 0, -1, -2, -3, -4
ST_BAD_COVER, ST_LOAD, ST_RES, ST_DEADLOCK, ST_BAD_KEY, ST_BAD_TUPLE = 1, 2, 4, 8, 16, 32
MIN_PRELOAD, FULL_START = 0, 1
ALLOW_PARTIAL = 1

TUPLE_DTYPE = np.dtype([("c", "<u2"), ("vD", "u1"), ("vP", "u1"), ("pD", "<u2"), ("pP", "<u2")])


class VrpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vrprpd error {code}: {msg}")
        self.code = code


class _Desc(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("k", C.c_int32), ("R", C.c_int32),
                ("load_model", C.c_int32), ("dist", C.c_void_p), ("proc", C.c_void_p)]


_lib = None

# name -> (restype, argtypes); every symbol declared in include/vrprpd.h
_P, _I32, _I64, _U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
SIGNATURES = {
    "vrprpd_last_error": (C.c_char_p, []),
    "vrprpd_set_create": (C.c_int, [C.POINTER(C.c_void_p), _I32, _P]),
    "vrprpd_set_destroy": (C.c_int, [_P]),
    "vrprpd_set_info": (C.c_int, [_P, _P, _P, _P, _P]),
    "vrprpd_eval": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _I32, _P, _P, _P]),
    "vrprpd_autotune_eval": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _I32, _P, _P, _I32, _P, _P, _P, _P]),
    "vrprpd_gather_rate": (C.c_int, [_P, _I32, _I32, _I32, _P, _P, _P]),
    "vrprpd_eval_set_shape": (C.c_int, [_P, _I32, _I32, _I32, _I32, _I32]),
    "vrprpd_insert_scan": (C.c_int, [_P, _I32, _P, _P, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _I32, _P]),
    "brkga_decode_eval": (C.c_int, [_P, _I64, _P, _P, _P, _I64, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "brkga_decode_eval_noalloc": (C.c_int, [_P, _I64, _P, _P, _P, _I64, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "brkga_decode_noalloc_max_bytes": (C.c_int64, []),
    "brkga_evolve": (C.c_int, [_I32, _I32, _I64, _P, _P, _P, _I32, _I32, C.c_double, _U64, C.c_uint32,
                               _P, _P, _P, _P]),
    "brkga_warm_start": (C.c_int, [_P, _I32, _P, _P, _I32, _I32, _I32, _U64, _I64, _P, _P, _P]),
    "alns_state_create": (C.c_int, [C.POINTER(C.c_void_p), _P, _I32, _P, _I32, _P, _U64, _P, _P, _P]),
    "alns_step": (C.c_int, [_P, _I32, _P]),
    "alns_set_trace": (C.c_int, [_P, _P, _I64]),
    "alns_get_best": (C.c_int, [_P, _I32, _P, _P, _P, _P]),
    "alns_get_state": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "alns_state_destroy": (C.c_int, [_P]),
    "alns_state_save": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
    "alns_state_load": (C.c_int, [_P, _P, C.c_int64, _P]),
    "brkga_state_save": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
    "brkga_state_load": (C.c_int, [_P, _P, C.c_int64, _P]),
    "brkga_state_create": (C.c_int, [C.POINTER(C.c_void_p), _P, _I32, _P, _I32, _I32, _I32, C.c_double, _U64,
                                     _I32, _P, _P, _P]),
    "brkga_state_step": (C.c_int, [_P, _I32, _I32, _P]),
    "brkga_state_get": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "brkga_state_destroy": (C.c_int, [_P]),
    "alns_set_graph": (C.c_int, [_P, _I32]),
    "alns_autotune": (C.c_int, [_P, _I32, _P, _P, _P]),
    "alns_set_learned": (C.c_int, [_P, _P, _I32, C.c_double, _P]),
    "alns_record": (C.c_int, [_P, _I64, _P]),
    "alns_record_info": (C.c_int, [_P, _P, _P]),
    "alns_record_batch": (C.c_int, [_P, _I32, _U64, _P, _P, _P, _P]),
    "alns_get_learned": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "vrprpd_mlp_create": (C.c_int, [C.POINTER(C.c_void_p), _I64, _P, _U64]),
    "vrprpd_mlp_destroy": (C.c_int, [_P]),
    "vrprpd_mlp_get_params": (C.c_int, [_P, _P, _P, _P]),
    "vrprpd_mlp_set_params": (C.c_int, [_P, _P, _P]),
    "vrprpd_mlp_forward": (C.c_int, [_P, _I64, _P, _P, _P]),
    "vrprpd_mlp_set_scores": (C.c_int, [_P, _I32, _P, _P, _P]),
    "vrprpd_mlp_loss": (C.c_int, [_P, _I32, _P, _P, _P, _P]),
    "vrprpd_mlp_backward": (C.c_int, [_P, _P, _P]),
    "vrprpd_mlp_sgd_step": (C.c_int, [_P, C.c_float, C.c_float, _P]),
    "vrprpd_mlp_hidden": (C.c_int, [_P, _I32, _P, _P]),
    "vrprpd_construct": (C.c_int, [_P, _I32, _P, _I32, _I64, _P, _I64, _P, _P]),
    "brkga_warm_start_multi": (C.c_int, [_P, _I32, _I32, _P, _I64, _P, _I64, _P, _I32, _I32, _U64, _I64, _P, _P,
                                         _P]),
    "alns_refine": (C.c_int, [_P, _I32, _P, _P]),
    "vrprpd_solution_stats": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
}

CONS_SWEEP, CONS_NN, CONS_LB, CONS_SPT = 0, 1, 2, 3
DECODE_HINT_FIRST = 1

MLP_IN, MLP_HIDDEN, MLP_NUM_PARAMS = 64, 256, 148481


def load():
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2602_23685_amd/build.py "
                              "(or __graft_entry__.build())")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if hasattr(lib, name):
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
        _lib = lib
    return _lib


def _check(rc):
    if rc != OK:
        raise VrpError(rc, load().vrprpd_last_error().decode())


def _stream(stream=None):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _dptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


class InstanceSet:
    """Instances copied to the current device (vrprpd_set_create)."""

    def __init__(self, instances):
        if not isinstance(instances, (list, tuple)):
            instances = [instances]
        lib = load()
        self._keep = []
        descs = (_Desc * len(instances))()
        for i, inst in enumerate(instances):
            d = np.ascontiguousarray(inst.d, dtype=np.int32)
            p = np.ascontiguousarray(inst.p, dtype=np.int32)
            self._keep += [d, p]
            descs[i] = _Desc(inst.n, inst.m, inst.k, inst.R, inst.load_model,
                             d.ctypes.data, p.ctypes.data)
        h = C.c_void_p()
        _check(lib.vrprpd_set_create(C.byref(h), len(instances), descs))
        self.handle = h
        self.instances = list(instances)
        self._keep = None
        info = [C.c_int32() for _ in range(4)]
        _check(lib.vrprpd_set_info(h, *[C.byref(x) for x in info]))
        self.num_inst, self.n_max, self.m_max, self.dist16 = (x.value for x in info)

    def close(self):
        if getattr(self, "handle", None):
            load().vrprpd_set_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vrprpd_eval(S: InstanceSet, ops, rt_end, inst=None, op_off=None, rt_off=None,
                partial=False, makespan=None, status=None, B=None, stream=None):
    """Exact makespan and status of B candidates (see vrprpd_eval in vrprpd.h).

    ops: uint16 codes (device); rt_end: uint16 route ends (device).  With
    op_off/rt_off None the candidates are [B, 2n] and [B, m] blocks."""
    if B is None:
        if op_off is not None:
            B = op_off.numel()
        else:
            B = rt_end.numel() // S.instances[0].m
    dev = ops.device
    if makespan is None:
        makespan = torch.empty(B, dtype=torch.int32, device=dev)
    if status is None:
        status = torch.empty(B, dtype=torch.int32, device=dev)
    _check(load().vrprpd_eval(
        S.handle, B, _dptr(inst, torch.int32, "inst"), _dptr(op_off, torch.int64, "op_off"),
        _dptr(ops, torch.uint16, "ops"), _dptr(rt_off, torch.int64, "rt_off"),
        _dptr(rt_end, torch.uint16, "rt_end"), ALLOW_PARTIAL if partial else 0,
        _dptr(makespan, torch.int32, "makespan"), _dptr(status, None, "status"), _stream(stream)))
    return makespan, status


def vrprpd_autotune_eval(S: InstanceSet, ops, rt_end, inst=None, op_off=None, rt_off=None, partial=False,
                         reps=3, stream=None):
    """Tune vrprpd_eval's launch shape on this batch; returns (candidates
    per wave, ops per step, live-leg form (0 or 1), mean ms of the twelve
    shapes indexed 6 * form + 2 * option + (step == 4))."""
    B = rt_end.shape[0]
    mk = torch.empty(B, dtype=torch.int32, device="cuda")
    st = torch.empty(B, dtype=torch.int32, device="cuda")
    w, k = C.c_int32(), C.c_int32()
    ms = np.zeros(12, np.float32)
    _check(load().vrprpd_autotune_eval(S.handle, B, _dptr(inst, torch.int32, "inst"),
                                       _dptr(op_off, torch.int64, "op_off"), _dptr(ops, torch.uint16, "ops"),
                                       _dptr(rt_off, torch.int64, "rt_off"), _dptr(rt_end, torch.uint16, "rt_end"),
                                       ALLOW_PARTIAL if partial else 0, _dptr(mk), _dptr(st), reps, C.byref(w),
                                       C.byref(k), ms.ctypes.data, _stream(stream)))
    valid = np.where(ms > 0, ms, np.inf)
    return w.value, k.value, int(np.argmin(valid)) // 6, ms


def vrprpd_eval_set_shape(S: InstanceSet, n, m, ng=0, step=4, live=1):
    """Pin vrprpd_eval's launch shape for (n, m) (see vrprpd_eval_set_shape
    in vrprpd.h): ng candidates per wave (0: default), step 2 or 4, live 0
    (staged travel times) or 1 (live legs)."""
    _check(load().vrprpd_eval_set_shape(S.handle, n, m, ng, step, live))


def vrprpd_gather_rate(S: InstanceSet, inst=0, blocks=8192, per_thread=256, stream=None):
    """Random reads of instance inst's travel-time matrix per second (see
    vrprpd_gather_rate in vrprpd.h): (reads per second, milliseconds)."""
    sink = torch.empty(blocks, dtype=torch.int32, device="cuda")
    ms = C.c_float()
    _check(load().vrprpd_gather_rate(S.handle, inst, blocks, per_thread, _dptr(sink), C.byref(ms), _stream(stream)))
    reads = blocks * 256 * per_thread
    return reads / (ms.value * 1e-3), ms.value


def vrprpd_insert_scan(S: InstanceSet, base_ops, base_rt, seg_off, tuples, num_bases=1,
                       base_inst=None, base_op_off=None, base_rt_off=None, seg_base=None,
                       want_each=True, blocks_per_seg=None, stream=None):
    """Exact makespan of insertion tuples against base partial solutions (see
    vrprpd_insert_scan in vrprpd.h).  tuples: device uint8 tensor holding the
    packed 8-byte tuples (TUPLE_DTYPE).  Returns (mk, status, seg_top3)."""
    dev = base_ops.device
    S_ = seg_off.numel() - 1
    T = tuples.numel() // 8
    mk = torch.empty(T, dtype=torch.int32, device=dev) if want_each else None
    st = torch.empty(T, dtype=torch.int32, device=dev) if want_each else None
    top = torch.empty((max(S_, 0), 3), dtype=torch.int64, device=dev)
    if blocks_per_seg is None:      # about 16 tuples per workgroup
        blocks_per_seg = max(1, min(65535, -(-T // max(1, S_ * 16))))
    _check(load().vrprpd_insert_scan(
        S.handle, num_bases, _dptr(base_inst, torch.int32, "base_inst"),
        _dptr(base_op_off, torch.int64, "base_op_off"), _dptr(base_ops, torch.uint16, "base_ops"),
        _dptr(base_rt_off, torch.int64, "base_rt_off"), _dptr(base_rt, torch.uint16, "base_rt"),
        S_, _dptr(seg_off, torch.int64, "seg_off"), _dptr(seg_base, torch.int32, "seg_base"),
        _dptr(tuples, torch.uint8, "tuples"), _dptr(mk, torch.int32, "mk"), _dptr(st, None, "st"),
        _dptr(top, torch.int64, "seg_top3"), blocks_per_seg, _stream(stream)))
    return mk, st, top


def _decode_out(S: InstanceSet, B, dev, inst, want_ops):
    out = dict(fitness=torch.empty(B, dtype=torch.int64, device=dev),
               makespan=torch.empty(B, dtype=torch.int32, device=dev),
               unscheduled=torch.empty(B, dtype=torch.int32, device=dev),
               status=torch.empty(B, dtype=torch.int32, device=dev))
    if want_ops:
        n_max = S.n_max if inst is not None else S.instances[0].n
        m_max = S.m_max if inst is not None else S.instances[0].m
        out["ops"] = torch.zeros((B, 2 * n_max), dtype=torch.uint16, device=dev)
        out["rt_end"] = torch.zeros((B, m_max), dtype=torch.uint16, device=dev)
    return out


def _decode_call(fn, S, prio, hint, inst, out, stream, flags):
    B, stride = prio.shape
    _check(fn(
        S.handle, B, _dptr(inst, torch.int32, "inst"), _dptr(prio, torch.float32, "prio"),
        _dptr(hint, torch.float32, "hint"), stride, int(flags), _dptr(out["fitness"], torch.int64, "fitness"),
        _dptr(out["makespan"], torch.int32, "makespan"), _dptr(out["unscheduled"], torch.int32, "unscheduled"),
        _dptr(out["status"], None, "status"), _dptr(out.get("ops"), torch.uint16, "ops_out"),
        _dptr(out.get("rt_end"), torch.uint16, "rt_end_out"), _stream(stream)))
    return out


def brkga_decode_eval(S: InstanceSet, prio, hint=None, inst=None, want_ops=False, out=None, stream=None, flags=0):
    """Decode B chromosomes (see brkga_decode_eval in vrprpd.h).  prio/hint:
    [B, stride] float32 device tensors; flags 0 or DECODE_HINT_FIRST.
    Returns dict of device tensors."""
    if out is None:
        out = _decode_out(S, prio.shape[0], prio.device, inst, want_ops)
    return _decode_call(load().brkga_decode_eval, S, prio, hint, inst, out, stream, flags)


def brkga_decode_eval_noalloc(S: InstanceSet, prio, hint=None, inst=None, out=None, want_ops=False, stream=None,
                              flags=0):
    """brkga_decode_eval with the library's fixed workspace (see
    brkga_decode_eval_noalloc in vrprpd.h): the library allocates no device
    memory.  Pass `out` (the dict brkga_decode_eval returns) to allocate
    nothing here either."""
    if out is None:
        out = _decode_out(S, prio.shape[0], prio.device, inst, want_ops)
    return _decode_call(load().brkga_decode_eval_noalloc, S, prio, hint, inst, out, stream, flags)


def brkga_decode_noalloc_max_bytes():
    """Size in bytes of brkga_decode_eval_noalloc's fixed workspace."""
    return int(load().brkga_decode_noalloc_max_bytes())


def brkga_evolve(prio, hint, fitness, n_elite, n_mutant, rho_e, seed, generation, genes=None,
                 prio_out=None, hint_out=None, rank_out=None, stream=None):
    """One BRKGA generation (see brkga_evolve in vrprpd.h).  Returns
    (prio_out, hint_out, rank_out)."""
    Np, stride = prio.shape
    genes = stride if genes is None else genes
    prio_out = torch.empty_like(prio) if prio_out is None else prio_out
    if hint is not None and hint_out is None:
        hint_out = torch.empty_like(hint)
    rank_out = torch.empty(Np, dtype=torch.int32, device=prio.device) if rank_out is None else rank_out
    _check(load().brkga_evolve(
        Np, genes, stride, _dptr(prio, torch.float32, "prio"), _dptr(hint, torch.float32, "hint"),
        _dptr(fitness, torch.int64, "fitness"), n_elite, n_mutant, float(rho_e), seed & (2**64 - 1),
        generation, _dptr(prio_out, torch.float32, "prio_out"), _dptr(hint_out, torch.float32, "hint_out"),
        _dptr(rank_out, torch.int32, "rank_out"), _stream(stream)))
    return prio_out, hint_out, rank_out


def brkga_warm_start(S: InstanceSet, ops, rt_end, Np, n_warm, n_variants, seed, inst=0, stride=None,
                     stream=None):
    """Initial population seeded from a solution (see brkga_warm_start)."""
    G = 2 * S.instances[inst].n
    stride = G if stride is None else stride
    po = torch.empty((Np, stride), dtype=torch.float32, device=ops.device)
    ho = torch.empty((Np, stride), dtype=torch.float32, device=ops.device)
    _check(load().brkga_warm_start(
        S.handle, inst, _dptr(ops, torch.uint16, "ops"), _dptr(rt_end, torch.uint16, "rt_end"), Np, n_warm,
        n_variants, seed & (2**64 - 1), stride, _dptr(po, torch.float32, "prio_out"),
        _dptr(ho, torch.float32, "hint_out"), _stream(stream)))
    return po, ho


def brkga_warm_start_multi(S: InstanceSet, ops, rt_end, n_var, Np, n_warm, seed, inst=0, stride=None,
                           stream=None):
    """Initial population seeded from several solutions (see
    brkga_warm_start_multi): ops [n_src][>= 2n], rt_end [n_src][>= m] device
    uint16, n_var a list of variants per source."""
    G = 2 * S.instances[inst].n
    stride = G if stride is None else stride
    nv = (C.c_int32 * len(n_var))(*n_var)
    po = torch.empty((Np, stride), dtype=torch.float32, device=ops.device)
    ho = torch.empty((Np, stride), dtype=torch.float32, device=ops.device)
    _check(load().brkga_warm_start_multi(
        S.handle, inst, len(n_var), _dptr(ops, torch.uint16, "ops"), ops.shape[1],
        _dptr(rt_end, torch.uint16, "rt_end"), rt_end.shape[1], nv, Np, n_warm, seed & (2**64 - 1), stride,
        _dptr(po, torch.float32, "prio_out"), _dptr(ho, torch.float32, "hint_out"), _stream(stream)))
    return po, ho


def vrprpd_solution_stats(S: InstanceSet, ops, rt_end, inst=None, op_off=None, rt_off=None, stream=None):
    """Cross-vehicle and interleaved customer counts per solution (see
    vrprpd_solution_stats): ops [B][>= 2n], rt_end [B][>= m] device uint16
    (strides 2 n(0) and m(0) unless offsets are given).  Returns two [B]
    int32 device tensors (-1 where a solution has no schedule)."""
    B = ops.shape[0] if ops.dim() == 2 else 1
    cross = torch.empty(B, dtype=torch.int32, device=ops.device)
    inter = torch.empty(B, dtype=torch.int32, device=ops.device)
    _check(load().vrprpd_solution_stats(
        S.handle, B, _dptr(inst, torch.int32, "inst"), _dptr(op_off, torch.int64, "op_off"),
        _dptr(ops, torch.uint16, "ops"), _dptr(rt_off, torch.int64, "rt_off"), _dptr(rt_end, torch.uint16, "rt_end"),
        _dptr(cross, torch.int32, "cross"), _dptr(inter, torch.int32, "interleaved"), _stream(stream)))
    return cross, inter


def vrprpd_construct(S: InstanceSet, heuristic, inst=None, stream=None):
    """One solution per instance from a construction heuristic (CONS_SWEEP,
    CONS_NN, CONS_LB, CONS_SPT; see vrprpd_construct).  inst: device int32
    instance indices, or None for every instance of the set in order.
    Returns ops [B][2 n_max] and rt_end [B][m_max] (device uint16)."""
    B = S.num_inst if inst is None else int(inst.numel())
    dev = inst.device if inst is not None else torch.device("cuda", torch.cuda.current_device())
    ops = torch.zeros((B, 2 * S.n_max), dtype=torch.uint16, device=dev)
    rt = torch.zeros((B, S.m_max), dtype=torch.uint16, device=dev)
    _check(load().vrprpd_construct(S.handle, B, _dptr(inst, torch.int32, "inst"), int(heuristic), 2 * S.n_max,
                                   _dptr(ops, torch.uint16, "ops"), S.m_max, _dptr(rt, torch.uint16, "rt_end"),
                                   _stream(stream)))
    return ops, rt


def _save(fn, handle, stream):
    n = C.c_int64()
    _check(fn(handle, None, 0, C.byref(n), _stream(stream)))
    buf = C.create_string_buffer(n.value)
    _check(fn(handle, buf, n.value, C.byref(n), _stream(stream)))
    return buf.raw[:n.value]


def _load(fn, handle, blob, stream):
    buf = C.create_string_buffer(bytes(blob), len(blob))
    _check(fn(handle, buf, len(blob), _stream(stream)))


class BrkgaState:
    """Batched BRKGA over several instances (brkga_state_*)."""

    def __init__(self, S: InstanceSet, inst_ids, Np, n_elite, n_mutant, rho_e, seed, prio0=None, hint0=None,
                 stream=None, decode_flags=0):
        ids = (C.c_int32 * len(inst_ids))(*inst_ids)
        h = C.c_void_p()
        _check(load().brkga_state_create(C.byref(h), S.handle, len(inst_ids), ids, Np, n_elite, n_mutant,
                                         float(rho_e), seed & (2**64 - 1), int(decode_flags),
                                         _dptr(prio0, torch.float32, "prio0"), _dptr(hint0, torch.float32, "hint0"),
                                         _stream(stream)))
        self.handle = h
        self.P, self.Np, self.stride = len(inst_ids), Np, 2 * S.n_max

    def step(self, generations, graph=True, stream=None):
        _check(load().brkga_state_step(self.handle, generations, 1 if graph else 0, _stream(stream)))

    def best(self, stream=None):
        """(best fitness per population (numpy), best prio, best hint)."""
        f = np.zeros(self.P, np.int64)
        bp = torch.empty((self.P, self.stride), dtype=torch.float32, device="cuda")
        bh = torch.empty_like(bp)
        _check(load().brkga_state_get(self.handle, None, f.ctypes.data, _dptr(bp), _dptr(bh), None, None,
                                      _stream(stream)))
        return f, bp, bh

    def save(self, stream=None):
        """Checkpoint (bytes) of the populations, bests and generation count."""
        return _save(load().brkga_state_save, self.handle, stream)

    def load(self, blob, stream=None):
        """Continue from a checkpoint of a state with the same configuration."""
        _load(load().brkga_state_load, self.handle, blob, stream)

    def population(self, stream=None):
        p = torch.empty((self.P * self.Np, self.stride), dtype=torch.float32, device="cuda")
        h = torch.empty_like(p)
        _check(load().brkga_state_get(self.handle, None, None, None, None, _dptr(p), _dptr(h), _stream(stream)))
        return p, h

    def close(self):
        if getattr(self, "handle", None):
            load().brkga_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pop_seed(seed, p):
    """Seed of population p of a batched BRKGA run."""
    return (seed + 0x9E3779B97F4A7C15 * p) & (2**64 - 1)


class AlnsParams(C.Structure):
    """alns_params of vrprpd.h (Table 2 hyper-parameters plus the repair budget)."""
    _fields_ = [("T0", C.c_double), ("alpha", C.c_double), ("reheat", C.c_double), ("gate", C.c_double),
                ("stag_limit", C.c_int32), ("tau", C.c_int32), ("r", C.c_double),
                ("sigma1", C.c_int32), ("sigma2", C.c_int32), ("sigma3", C.c_int32),
                ("w_min", C.c_double), ("q_min", C.c_int32), ("q_max", C.c_int32),
                ("tuple_budget", C.c_int32), ("import_interval", C.c_int32), ("op_mask", C.c_uint32),
                ("ls_repos_interval", C.c_int32), ("ls_reloc_interval", C.c_int32), ("ls_budget", C.c_int32),
                ("chain_base", C.c_int32)]


def alns_params(**kw):
    d = dict(T0=0.30, alpha=0.9998, reheat=0.50, gate=0.01, stag_limit=2000, tau=100, r=0.1,
             sigma1=33, sigma2=9, sigma3=13, w_min=0.1, q_min=0, q_max=0, tuple_budget=0,
             import_interval=1000, op_mask=0x0F3F,
             ls_repos_interval=200, ls_reloc_interval=500, ls_budget=16384)
    d.update(kw)
    return AlnsParams(**d)


class AlnsState:
    """ALNS chains on the device (alns_state_create / alns_step)."""

    def __init__(self, S: InstanceSet, inst_ids, chains_per_inst, params, seed, init_ops, init_rt,
                 stream=None):
        ids = (C.c_int32 * len(inst_ids))(*inst_ids)
        h = C.c_void_p()
        _check(load().alns_state_create(C.byref(h), S.handle, len(inst_ids), ids, chains_per_inst,
                                        C.byref(params), seed & (2**64 - 1),
                                        _dptr(init_ops, torch.uint16, "init_ops"),
                                        _dptr(init_rt, torch.uint16, "init_rt"), _stream(stream)))
        self.handle = h
        self.S = S
        self.chains = len(inst_ids) * chains_per_inst
        self.n_max = max(S.instances[i].n for i in inst_ids)
        self.m_max = max(S.instances[i].m for i in inst_ids)
        self._trace = None

    def step(self, iterations, stream=None):
        _check(load().alns_step(self.handle, iterations, _stream(stream)))

    def set_trace(self, capacity):
        """Start recording per-iteration records into a new device tensor."""
        self._trace = torch.zeros((self.chains, capacity, 4), dtype=torch.int64, device="cuda")
        _check(load().alns_set_trace(self.handle, _dptr(self._trace, torch.int64, "trace"), capacity))
        return self._trace

    def best(self, chain=-1, stream=None):
        mk = C.c_int32()
        ops = torch.zeros(2 * self.n_max, dtype=torch.uint16, device="cuda")
        rt = torch.zeros(self.m_max, dtype=torch.uint16, device="cuda")
        _check(load().alns_get_best(self.handle, chain, C.byref(mk), _dptr(ops, torch.uint16, "ops"),
                                    _dptr(rt, torch.uint16, "rt"), _stream(stream)))
        return mk.value, ops, rt

    def state(self):
        it = C.c_int64()
        ev = C.c_int64()
        z = np.zeros(self.chains, np.int32)
        zb = np.zeros(self.chains, np.int32)
        T = np.zeros(self.chains, np.float64)
        wD = np.zeros((self.chains, 6), np.float64)
        wR = np.zeros((self.chains, 4), np.float64)
        _check(load().alns_get_state(self.handle, C.byref(it), C.byref(ev), z.ctypes.data, zb.ctypes.data,
                                     T.ctypes.data, wD.ctypes.data, wR.ctypes.data))
        return dict(iterations=it.value, evals=ev.value, z=z, zb=zb, T=T, wD=wD, wR=wR)

    def save(self, stream=None):
        """Checkpoint (bytes) of every chain's search state and the
        iteration counter."""
        return _save(load().alns_state_save, self.handle, stream)

    def load(self, blob, stream=None):
        """Continue from a checkpoint of a state with the same configuration."""
        _load(load().alns_state_load, self.handle, blob, stream)

    def set_graph(self, enable):
        """Replay one captured iteration (True, the default) or launch every
        kernel of every iteration (False)."""
        _check(load().alns_set_graph(self.handle, 1 if enable else 0))

    def autotune(self, iterations=2, stream=None):
        """Pick the repair rounds' scan shape (alns_autotune): returns (tuples
        per workgroup, milliseconds per iteration of the 8, 16, 32, 64
        shapes)."""
        tpb = C.c_int32()
        ms = (C.c_float * 4)()
        _check(load().alns_autotune(self.handle, iterations, C.byref(tpb), ms, _stream(stream)))
        return tpb.value, [float(x) for x in ms]

    def refine(self, max_rounds=1000, stream=None):
        """The construction's refinement rounds before the first iteration
        (alns_refine); returns the number of rounds run."""
        r = C.c_int32()
        _check(load().alns_refine(self.handle, max_rounds, C.byref(r), _stream(stream)))
        return r.value

    # ---- learned destroy proposal ------------------------------------------
    def set_learned(self, mlp, K=8, eps=0.1, stream=None):
        """Score K candidate removal sets per chain with `mlp` (None: off)."""
        self._mlp = mlp
        self.K = K if mlp is not None else 1
        _check(load().alns_set_learned(self.handle, mlp.handle if mlp is not None else None, K, float(eps),
                                       _stream(stream)))

    def record(self, capacity, stream=None):
        _check(load().alns_record(self.handle, int(capacity), _stream(stream)))

    def record_info(self):
        sets, q = C.c_int64(), C.c_int32()
        _check(load().alns_record_info(self.handle, C.byref(sets), C.byref(q)))
        return sets.value, q.value

    def record_batch(self, num_sets, seed, stream=None):
        """(x [rows, 64] uint16 bf16 bits, seg_off [num_sets + 1], target
        [num_sets]) of num_sets recorded sets; x has room for q_max rows per
        set, the filled rows are x[:seg_off[-1]]."""
        _, q = self.record_info()
        x = torch.zeros((num_sets * q, MLP_IN), dtype=torch.uint16, device="cuda")
        seg = torch.empty(num_sets + 1, dtype=torch.int64, device="cuda")
        tgt = torch.empty(num_sets, dtype=torch.float32, device="cuda")
        _check(load().alns_record_batch(self.handle, num_sets, seed & (2**64 - 1), _dptr(x), _dptr(seg),
                                        _dptr(tgt), _stream(stream)))
        return x, seg, tgt

    def learned_state(self, stream=None):
        """Device copies of the last iteration's features, candidate sets,
        counts and choices."""
        K = getattr(self, "K", 1)
        _, q = self.record_info()
        feat = torch.empty((self.chains, self.n_max, MLP_IN), dtype=torch.uint16, device="cuda")
        rem = torch.empty((self.chains, K, q), dtype=torch.int32, device="cuda")
        cnt = torch.empty((self.chains, K), dtype=torch.int32, device="cuda")
        chosen = torch.empty(self.chains, dtype=torch.int32, device="cuda")
        _check(load().alns_get_learned(self.handle, _dptr(feat), _dptr(rem), _dptr(cnt), _dptr(chosen),
                                       _stream(stream)))
        return feat, rem, cnt, chosen

    def close(self):
        if getattr(self, "handle", None):
            load().alns_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The destroy-proposal scorer network on the device (vrprpd_mlp_*).
    Features are bfloat16 bit patterns in a torch.uint16 (or torch.bfloat16)
    device tensor of shape [rows, 64]."""

    def __init__(self, max_rows, params=None, seed=0):
        h = C.c_void_p()
        host = None
        if params is not None:
            host = np.ascontiguousarray(params, dtype=np.float32)
            if host.shape != (MLP_NUM_PARAMS,):
                raise ValueError(f"params must have {MLP_NUM_PARAMS} values")
        _check(load().vrprpd_mlp_create(C.byref(h), int(max_rows),
                                        None if host is None else host.ctypes.data, seed & (2**64 - 1)))
        self.handle = h
        self.max_rows = int(max_rows)
        self.rows = 0

    @staticmethod
    def _x(x):
        if x.dtype == torch.bfloat16:
            x = x.view(torch.uint16)
        return _dptr(x, torch.uint16, "x")

    def forward(self, x, y=None, stream=None):
        rows = int(x.shape[0])
        if rows and tuple(x.shape) != (rows, MLP_IN):
            raise ValueError(f"x must be [rows, {MLP_IN}]")
        if y is None:
            y = torch.empty(rows, dtype=torch.float32, device="cuda")
        self._xkeep = x
        _check(load().vrprpd_mlp_forward(self.handle, rows, self._x(x) if rows else None,
                                         _dptr(y, torch.float32, "y"), _stream(stream)))
        self.rows = rows
        return y

    def set_scores(self, seg_off, out=None, stream=None):
        S = int(seg_off.shape[0]) - 1
        if out is None:
            out = torch.empty(S, dtype=torch.float32, device="cuda")
        _check(load().vrprpd_mlp_set_scores(self.handle, S, _dptr(seg_off, torch.int64, "seg_off"),
                                            _dptr(out, torch.float32, "set_score"), _stream(stream)))
        return out

    def loss(self, seg_off, target, sq_err=None, stream=None):
        S = int(seg_off.shape[0]) - 1
        if sq_err is None:
            sq_err = torch.empty(S, dtype=torch.float32, device="cuda")
        _check(load().vrprpd_mlp_loss(self.handle, S, _dptr(seg_off, torch.int64, "seg_off"),
                                      _dptr(target, torch.float32, "target"),
                                      _dptr(sq_err, torch.float32, "sq_err"), _stream(stream)))
        return sq_err

    def backward(self, dy=None, stream=None):
        _check(load().vrprpd_mlp_backward(self.handle, _dptr(dy, torch.float32, "dy"), _stream(stream)))

    def sgd_step(self, lr, momentum=0.0, stream=None):
        _check(load().vrprpd_mlp_sgd_step(self.handle, float(lr), float(momentum), _stream(stream)))

    def params(self, stream=None):
        p = torch.empty(MLP_NUM_PARAMS, dtype=torch.float32, device="cuda")
        _check(load().vrprpd_mlp_get_params(self.handle, _dptr(p), None, _stream(stream)))
        return p

    def grad(self, stream=None):
        g = torch.empty(MLP_NUM_PARAMS, dtype=torch.float32, device="cuda")
        _check(load().vrprpd_mlp_get_params(self.handle, None, _dptr(g), _stream(stream)))
        return g

    def set_params(self, params, stream=None):
        _check(load().vrprpd_mlp_set_params(self.handle, _dptr(params, torch.float32, "params"), _stream(stream)))

    def hidden(self, layer, stream=None):
        out = torch.empty((self.rows, MLP_HIDDEN), dtype=torch.uint16, device="cuda")
        _check(load().vrprpd_mlp_hidden(self.handle, layer, _dptr(out), _stream(stream)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            load().vrprpd_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
