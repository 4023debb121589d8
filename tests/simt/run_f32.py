"""Child process of the CPU-build tests: runs a load path through the
FP32-storage Gauss-point kernel of tests/simt/fp32_kernel.cpp.

    python run_f32.py LIB IN.npz OUT.npz

IN.npz: depth, lanes, w, n, E [T, P, 6] (float32), fiber [2], matrix [6].
OUT.npz: per step the outputs (sigma, tangent, z, a, iters, status).
"""
import ctypes
import sys

import numpy as np


def ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def main(lib_path, in_path, out_path):
    lib = ctypes.CDLL(lib_path)
    f = lib.simt_gp_update_f32
    f.restype = ctypes.c_int
    d = np.load(in_path)
    K, lanes = int(d["depth"]), int(d["lanes"])
    E = d["E"]
    T, P = E.shape[:2]
    M, L = 2 ** (K - 1), 2 ** K - 1
    w = np.ascontiguousarray(d["w"], np.float64)
    n = np.ascontiguousarray(d["n"], np.float64)
    fib = np.ascontiguousarray(d["fiber"], np.float64)
    mat = np.ascontiguousarray(d["matrix"], np.float64)
    zi, zo = np.zeros((P, M, 7), np.float32), np.zeros((P, M, 7), np.float32)
    ai, ao = np.zeros((P, L, 3), np.float32), np.zeros((P, L, 3), np.float32)
    sig, tan = np.zeros((P, 6), np.float32), np.zeros((P, 6, 6), np.float32)
    it, st = np.zeros(P, np.int32), np.zeros(P, np.int32)
    out = {}
    for s in range(T):
        Es = np.ascontiguousarray(E[s], np.float32)
        rc = f(ctypes.c_int(K), ctypes.c_int(lanes), ptr(w), ptr(n), ctypes.c_longlong(P),
               ptr(Es), ptr(zi), ptr(zo), ptr(ai), ptr(ao), ptr(sig), ptr(tan), ptr(it), ptr(st),
               ptr(fib), ptr(mat), ctypes.c_double(1e-10), ctypes.c_int(25), ctypes.c_int(10),
               ctypes.c_double(1e-4))
        if rc != 0:
            raise SystemExit(f"simt_gp_update_f32 returned {rc}")
        for k, v in (("sigma", sig), ("C", tan), ("z", zo), ("a", ao), ("iters", it),
                     ("status", st)):
            out[f"s{s}_{k}"] = v.copy()
        zi, zo = zo, zi
        ai, ao = ao, ai
    np.savez(out_path, **out)


if __name__ == "__main__":
    main(*sys.argv[1:4])
