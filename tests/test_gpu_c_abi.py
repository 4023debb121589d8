"""The C ABI used from a plain C++ host program (examples/gauss_point_path.cpp:
hipMalloc'd buffers, a strain path applied step by step with the state
ping-ponged), checked against the oracle's Gauss-point path."""
import os
import subprocess
import sys

import numpy as np
import pytest

import synthetic as S
from oracle.gp import DmnModel, NewtonOptions, run_path

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2103_08253_amd", "examples", "gauss_point_path")


def test_c_host_program_matches_oracle(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is missing: build the package (python -m paper_2103_08253_amd.build)")
    K, P, T = 3, 16, 5
    print(f"case: C host program K={K} P={P} T={T}", flush=True)
    rs = S.streams(120)
    net = S.random_dmn(rs["dmn"], K, 0.3)
    E = S.ramp_with_noise(rs, P, T, 0.03, 1e-3)
    fib = [S.FIBER["E"], S.FIBER["nu"]]
    mat = [S.MATRIX[k] for k in ("E", "nu", "sigma0", "k_inf", "dsigma", "b")]
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.int32(K).tobytes() + np.int64(P).tobytes() + np.int32(T).tobytes())
        f.write(np.concatenate([net.w, net.normals.ravel(), np.ascontiguousarray(E).ravel(),
                                fib, mat, [1e-10]]).astype(np.float64).tobytes())
    r = subprocess.run([EXE, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    sys.stdout.write(r.stdout + r.stderr)
    assert r.returncode == 0
    raw = open(out, "rb").read()
    step_bytes = P * 6 * 8 + P * 36 * 8 + 2 * P * 4
    assert len(raw) == T * step_bytes
    model = DmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX)
    refs = [run_path(model, E[:, p, :], NewtonOptions()) for p in range(P)]
    for t in range(T):
        b = raw[t * step_bytes:(t + 1) * step_bytes]
        sig = np.frombuffer(b[:P * 48], dtype=np.float64).reshape(P, 6)
        tan = np.frombuffer(b[P * 48:P * 336], dtype=np.float64).reshape(P, 6, 6)
        st = np.frombuffer(b[P * 336:P * 340], dtype=np.int32)
        it = np.frombuffer(b[P * 340:], dtype=np.int32)
        for p in range(P):
            ref = refs[p][t]
            if ref["margin"] < 1e-9:
                continue
            assert st[p] == ref["status"] == 0 and it[p] == ref["iters"], (t, p)
            assert np.abs(sig[p] - ref["sigma"]).max() <= 1e-10 * np.abs(ref["sigma"]).max()
            assert np.abs(tan[p] - ref["C"]).max() <= 1e-10 * np.abs(ref["C"]).max()
