"""The C-ABI library loads and exports what include/vrprpd.h declares, and its
host-side argument checks work without a GPU (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)
    return names


@pytest.fixture(scope="module")
def lib():
    import paper_2602_23685_amd as P
    return P.load()


def test_every_declared_symbol_is_exported(lib):
    import paper_2602_23685_amd as P
    names = declared_functions()
    assert "vrprpd_eval" in names and len(names) >= 5
    for name in names:
        assert hasattr(lib, name), f"{name} declared but not exported"
        assert name in P.SIGNATURES, f"{name} has no Python binding"


def test_host_argument_checks(lib):
    import paper_2602_23685_amd as P
    from paper_2602_23685_amd._lib import _Desc
    h = C.c_void_p()
    # no instances
    assert lib.vrprpd_set_create(C.byref(h), 0, None) == P._lib.EINVAL
    assert b"num_inst" in lib.vrprpd_last_error()
    # n out of range
    d = np.zeros((2, 2), np.int32)
    p = np.zeros(2, np.int32)
    desc = _Desc(0, 1, 1, 1, 0, d.ctypes.data, p.ctypes.data)
    assert lib.vrprpd_set_create(C.byref(h), 1, C.byref(desc)) == P._lib.EINVAL
    # a distance matrix whose schedules could overflow int32 times
    big = np.full((3, 3), 700_000_000, np.int32)
    np.fill_diagonal(big, 0)
    pp = np.zeros(3, np.int32)
    desc = _Desc(2, 1, 1, 1, 0, big.ctypes.data, pp.ctypes.data)
    assert lib.vrprpd_set_create(C.byref(h), 1, C.byref(desc)) == P._lib.ERANGE
    # nonzero diagonal
    dd = np.ones((2, 2), np.int32)
    desc = _Desc(1, 1, 1, 1, 0, dd.ctypes.data, p.ctypes.data)
    assert lib.vrprpd_set_create(C.byref(h), 1, C.byref(desc)) == P._lib.EINVAL
    # eval without a set
    assert lib.vrprpd_eval(None, 1, None, None, None, None, None, 0, None, None, None) == P._lib.EINVAL


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2602_23685_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, flags=re.M), f
                assert "liboracle" not in txt and "oracle/" not in txt, f


def test_host_argument_checks_of_the_newer_entry_points(lib):
    """Argument errors are reported before any device work (no GPU needed)."""
    import paper_2602_23685_amd as P
    E = P._lib.EINVAL
    h = C.c_void_p()
    # scorer network: row capacity out of range
    assert lib.vrprpd_mlp_create(C.byref(h), 0, None, 0) == E
    assert b"max_rows" in lib.vrprpd_last_error()
    assert lib.vrprpd_mlp_create(C.byref(h), (1 << 26) + 1, None, 0) == E
    assert lib.vrprpd_mlp_forward(None, 1, None, None, None) == E
    assert lib.vrprpd_mlp_backward(None, None, None) == E
    assert lib.vrprpd_mlp_sgd_step(None, C.c_float(0.1), C.c_float(0.0), None) == E
    # ALNS: learned proposal, recording, graph switch on a missing state
    assert lib.alns_set_learned(None, None, 1, C.c_double(0.0), None) == E
    assert lib.alns_record(None, 10, None) == E
    assert lib.alns_record_batch(None, 1, 0, None, None, None, None) == E
    assert lib.alns_set_graph(None, 1) == E
    # batched BRKGA without a set; autotuner without a set
    assert lib.brkga_state_create(C.byref(h), None, 1, None, 8, 1, 1, C.c_double(0.7), 0, 0, None, None, None) == E
    assert lib.brkga_state_step(None, 1, 1, None) == E
    assert lib.vrprpd_autotune_eval(None, 1, None, None, None, None, None, 0, None, None, 1, None, None, None,
                                    None) == E
    assert b"autotune" in lib.vrprpd_last_error()
    # construction heuristics, several-source warm start, refinement
    assert lib.vrprpd_construct(None, 1, None, 0, 2, None, 1, None, None) == E
    assert b"vrprpd_construct" in lib.vrprpd_last_error()
    nv = (C.c_int32 * 1)(1)
    assert lib.brkga_warm_start_multi(None, 0, 1, None, 2, None, 1, nv, 8, 1, 0, 2, None, None, None) == E
    assert lib.alns_refine(None, 5, None, None) == E
    assert lib.vrprpd_solution_stats(None, 1, None, None, None, None, None, None, None, None) == E


def test_checkpoint_argument_checks(lib):
    """Checkpoints of missing states, and loads of foreign buffers, are
    refused before any device work."""
    import paper_2602_23685_amd as P
    E = P._lib.EINVAL
    n = C.c_int64()
    assert lib.alns_state_save(None, None, 0, C.byref(n), None) == E
    assert lib.alns_state_load(None, None, 0, None) == E
    assert lib.brkga_state_save(None, None, 0, C.byref(n), None) == E
    assert lib.brkga_state_load(None, None, 0, None) == E
