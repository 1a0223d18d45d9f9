"""VRP-RPD batched exact makespan evaluation on MI355X (gfx950).

The computation lives in ``libvrprpd.so`` (hand-written HIP kernels behind the
C-ABI in ``include/vrprpd.h``); this package only marshals device tensors and
streams into it.  Importing it loads nothing; the first call loads the library
and raises if it is not built.
"""
from ._lib import (  # noqa: F401
    ALLOW_PARTIAL, FULL_START, MIN_PRELOAD, SIGNATURES, ST_BAD_COVER, ST_BAD_KEY, ST_BAD_TUPLE,
    ST_DEADLOCK, ST_LOAD, ST_RES, TUPLE_DTYPE, MLP_IN, MLP_HIDDEN, MLP_NUM_PARAMS, AlnsParams, AlnsState,
    InstanceSet, Mlp, VrpError, BrkgaState, pop_seed, alns_params, brkga_decode_eval, brkga_evolve, brkga_warm_start, load,
    vrprpd_autotune_eval, vrprpd_eval, vrprpd_insert_scan, CONS_SWEEP, CONS_NN, CONS_LB, CONS_SPT, vrprpd_construct,
    brkga_warm_start_multi, vrprpd_solution_stats, brkga_decode_eval_noalloc, brkga_decode_noalloc_max_bytes,
    DECODE_HINT_FIRST, vrprpd_gather_rate, vrprpd_eval_set_shape,
)
