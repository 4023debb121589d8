"""Parent side of the CPU-build tests: writes a case, runs one of the child
runners in tests/simt/ in a child process under the sanitiser's runtime, and
reads the outputs back."""
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import build as B  # noqa: E402


def material_arrays(fiber, matrix):
    return (np.array([fiber["E"], fiber["nu"]]),
            np.array([matrix["E"], matrix["nu"], matrix["sigma0"], matrix["k_inf"],
                      matrix["dsigma"], matrix["b"]]))


def _child(script, lib, case, sanitizer="address", timeout=900):
    """Runs tests/simt/<script> LIB IN.npz OUT.npz on the case under the
    sanitiser's runtime; returns (outputs, the child's stderr)."""
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.npz"), os.path.join(td, "out.npz")
        np.savez(fin, **case)
        env = dict(os.environ, LD_PRELOAD=B.asan_runtime(sanitizer),
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
                   TSAN_OPTIONS="halt_on_error=1:report_signal_unsafe=0",
                   OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.join(HERE, script), lib, fin, fout],
                           env=env, capture_output=True, text=True, timeout=timeout)
        if r.returncode != 0:
            raise AssertionError(f"CPU-build run failed (exit {r.returncode}):\n"
                                 f"{r.stderr[-6000:]}")
        d = np.load(fout)
        return {k: d[k] for k in d.files}, r.stderr


STEP_KEYS = ("sigma", "C", "z", "a", "iters", "status")


def run_gp(groups, fiber, matrix, opts=(1e-10, 25, 10, 1e-4, 0, 0), prec=0, tuning=(),
           noalloc=False, defines=(B.VARIANTS,), timeout=900, sanitizer="address"):
    """groups: dicts with depth, w, E [T, P, 6] and either n or ori/p/q/lam.
    Returns (outputs per group and step, child's stderr)."""
    lib = B.build(defines, sanitizer=sanitizer)
    fib, mat = material_arrays(fiber, matrix)
    case = dict(n_groups=len(groups), opts=np.array(opts, dtype=np.float64), prec=prec,
                tuning=np.array(tuning, dtype=np.int64).reshape(-1, 3), noalloc=int(noalloc),
                fiber=fib, matrix=mat)
    for g, grp in enumerate(groups):
        for k, v in grp.items():
            case[f"g{g}_{k}"] = np.asarray(v)
    d, err = _child("run_gp.py", lib, case, sanitizer, timeout)
    T = np.asarray(groups[0]["E"]).shape[0]
    return [[{k: d[f"g{g}_s{s}_{k}"] for k in STEP_KEYS} for s in range(T)]
            for g in range(len(groups))], err


def run_f32_kernel(depth, lanes, w, n, E, fiber, matrix, timeout=900):
    """Load path through the FP32-storage kernel's CPU build (run_f32.py)."""
    lib = B.build_f32_kernel()
    fib, mat = material_arrays(fiber, matrix)
    case = dict(depth=depth, lanes=lanes, w=w, n=n, E=np.asarray(E, np.float32), fiber=fib,
                matrix=mat)
    d, _ = _child("run_f32.py", lib, case, "address", timeout)
    return [{k: d[f"s{s}_{k}"] for k in STEP_KEYS} for s in range(np.asarray(E).shape[0])]


def run_linear(depth, w, n, C1, C2, gCbar, input_grads=False, sanitizer="address", timeout=900,
               ori=None):
    """Linear map and backward through the CPU build (run_linear.py); ori =
    (code, p, q, lam) for per-sample orientations (n is then not used)."""
    lib = B.build(sanitizer=sanitizer)
    extra = {} if ori is None else dict(ori=ori[0], p=ori[1], q=ori[2], lam=ori[3])
    case = dict(depth=depth, w=w, n=n if n is not None else np.zeros(1), C1=C1, C2=C2,
                gCbar=gCbar, input_grads=int(input_grads), **extra)
    return _child("run_linear.py", lib, case, sanitizer, timeout)[0]


def run_adjoint(depth, w, n, E, g, fiber, matrix, opts=(1e-13, 50, 10, 1e-4, 0, 1),
                sanitizer="address", timeout=900):
    """Path gradient through the CPU build's forward path and step adjoint
    (run_adjoint.py)."""
    lib = B.build(sanitizer=sanitizer)
    fib, mat = material_arrays(fiber, matrix)
    case = dict(depth=depth, w=w, n=n, E=E, g=g, opts=np.array(opts, dtype=np.float64),
                fiber=fib, matrix=mat)
    return _child("run_adjoint.py", lib, case, sanitizer, timeout)[0]


def run_train(case, sanitizer="address", timeout=900):
    """Training calls through the CPU build (run_train.py): the loss for
    Cbar/target/p/q, the stiffness sampler for u/sprec, the optimiser step for
    v/alpha/beta/gw/gn/state/step/stats0/amsgrad, whichever the case holds."""
    lib = B.build(sanitizer=sanitizer)
    return _child("run_train.py", lib, case, sanitizer, timeout)[0]


def run_oriented_train(case, sanitizer="address", timeout=900):
    """One orientation-grouped training step through the CPU build
    (run_oriented_train.py)."""
    lib = B.build(sanitizer=sanitizer)
    return _child("run_oriented_train.py", lib, case, sanitizer, timeout)[0]
