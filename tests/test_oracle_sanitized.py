"""The oracle's C core under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, built with gcc).

A checked copy of the oracle library is built into a temporary folder and
loaded by child processes (VRPRPD_ORACLE_LIB) with the ASan runtime preloaded,
since the interpreter itself is not instrumented; undefined behaviour is fatal
(-fno-sanitize-recover).  The children run
  * the oracle's own test files again;
  * every C entry point once at the 1000-customer workload: evaluation (with
    cover errors and deadlocks, op times, the DAG form), insertion scan,
    decoder (special keys, both vehicle rules), a BRKGA generation and a warm
    start, the four construction heuristics, refinement, both local searches,
    solution statistics and two ALNS iterations of two chains;
and a control: a candidate whose route table claims more ops than its buffer
holds must stop the child with a heap-buffer-overflow report, which shows
that the checks are live.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECKED = ("-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all")

WORKLOAD = textwrap.dedent("""
    import sys
    sys.path[:0] = [{root!r}, {tests!r}]
    import numpy as np
    import oracle, synth
    from cases import mutate, destroy
    assert oracle.lib()._name == {lib!r}
    inst = synth.make_instance(1000, 10, 10, 100, "1R20d10", seed=3003)
    ops, rt = synth.random_candidates(inst, 6, seed=3)
    mops, mrt = mutate(inst, ops, rt, seed=4, count=6)
    oracle.eval_batch(inst, np.concatenate([ops, mops]), np.concatenate([rt, mrt]))
    oracle.eval_one(inst, ops[0], rt[0], times=True)
    oracle.eval_one(inst, ops[1], rt[1], dag=True)
    fo, off, frt = destroy(inst, ops[:1], rt[:1], seed=5, q=40)
    tuples = synth.random_tuples(fo, frt[0], 1000, 10, 300, seed=6, invalid_frac=0.05)
    oracle.insert_scan(inst, fo, frt[0], tuples, np.array([0, 120, 300], np.int64))
    prio, hint = synth.random_keys(4, 1000, seed=7, special=True)
    oracle.decode_batch(inst, prio, hint)
    oracle.decode(inst, prio[1], hint[1], want_ops=True, flags=1)
    P2, H2 = synth.random_keys(64, 1000, seed=8)
    ne, nm = oracle.brkga_sizes(64)
    oracle.brkga_evolve(P2, H2, np.arange(64, dtype=np.int64)[::-1].copy(), ne, nm,
                        oracle.rho_threshold(0.7), 9, 1)
    oracle.brkga_warm_start(inst, ops[0], rt[0], 64, 8, 4, 10)
    for h in range(4):
        c_ops, c_rt = oracle.construct(inst, h)
    oracle.refine(inst, c_ops, c_rt, budget=2048, max_rounds=1)
    for kind in (0, 1):
        oracle.alns_local_search(inst, kind, ops[0], rt[0], budget=2048, passes=1)
    oracle.solution_stats(inst, ops[0], rt[0])
    oracle.alns_run(inst, oracle.alns_params(tuple_budget=2048), 2, 2, 11, ops[0], rt[0], trace=True)
    print("workload done")
""")

CONTROL = textwrap.dedent("""
    import sys
    sys.path[:0] = [{root!r}]
    import oracle, synth
    inst = synth.make_instance(50, 3, 4, 12, seed=2)
    ops, rt = synth.random_candidates(inst, 1, seed=1)
    short = ops[0][:20].copy()          # its own 40-byte buffer; the route ends still claim 100 ops
    oracle.eval_one(inst, short, rt[0])
    print("not caught")
""")


def _runtime(name):
    try:
        out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                             timeout=60).stdout.strip()
    except (OSError, subprocess.SubprocessError):
        return None
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.fixture(scope="module")
def checked(tmp_path_factory):
    asan = _runtime("libasan.so")
    if asan is None or _runtime("libubsan.so") is None:
        pytest.skip("gcc has no ASan/UBSan runtime here")
    import oracle
    lib = str(tmp_path_factory.mktemp("oracle_checked") / "liboracle_checked.so")
    oracle.build(out=lib, opt="-O1", extra=CHECKED)
    pre = os.environ.get("LD_PRELOAD")
    env = dict(os.environ, VRPRPD_ORACLE_LIB=lib, LD_PRELOAD=asan + (":" + pre if pre else ""),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return lib, env


def _child(args, env, timeout):
    return subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=timeout)


def test_oracle_tests_under_sanitizers(checked):
    lib, env = checked
    files = sorted(f for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py") and f != os.path.basename(__file__))
    r = _child(["-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                *[os.path.join("tests", f) for f in files]], env, 900)
    assert r.returncode == 0 and " passed" in r.stdout, (r.stdout[-3000:], r.stderr[-3000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]


def test_every_entry_point_at_full_scale_under_sanitizers(checked):
    lib, env = checked
    code = WORKLOAD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    r = _child(["-c", code], env, 600)
    assert r.returncode == 0 and "workload done" in r.stdout, (r.stdout[-3000:], r.stderr[-3000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]


def test_sanitizer_control_catches_an_overread(checked):
    lib, env = checked
    r = _child(["-c", CONTROL.format(root=ROOT)], env, 120)
    assert r.returncode != 0 and "not caught" not in r.stdout
    assert "AddressSanitizer: heap-buffer-overflow" in r.stderr, r.stderr[-3000:]
