"""Child process of the CPU-build tests: the linear map and its backward
through dmn_homogenize_linear / dmn_homogenize_backward of a sanitised CPU
library (tests/simt/build.py).

    python run_linear.py LIB IN.npz OUT.npz

IN.npz: depth, w, n, C1, C2, gCbar [B, 6, 6] (float64 or float32: the call's
precision), input_grads (1: also the phase-stiffness cotangents); for
per-sample orientations ori (1 linear, 2 tri-linear, 3 quadratic), p, q
[L, M] and lam [B, 2] instead of n (gn is then [L, 2, M]).
OUT.npz: Cbar, gw, gn (and gC1, gC2), and the two calls' device error words.
"""
import ctypes
import sys

import numpy as np

from run_gp import load_lib_module, ptr


def workspace(nbytes):
    raw = np.zeros(nbytes + 256, np.uint8)
    off = (-raw.ctypes.data) % 256
    return raw, raw[off:off + nbytes]


def main(lib_path, in_path, out_path):
    L = load_lib_module(lib_path)
    lib = L.lib()
    d = np.load(in_path)
    K = int(d["depth"])
    dt = d["C1"].dtype
    prec = L.DMN_F32 if dt == np.float32 else L.DMN_F64
    w = np.ascontiguousarray(d["w"], dt)
    C1, C2, G = (np.ascontiguousarray(d[k], dt) for k in ("C1", "C2", "gCbar"))
    B = C1.shape[0]
    ori = int(d["ori"]) if "ori" in d.files else 0
    lam = None
    if ori:
        p, q = np.ascontiguousarray(d["p"], dt), np.ascontiguousarray(d["q"], dt)
        lam = np.ascontiguousarray(d["lam"], dt)
        net = L.DmnNet(K, ptr(w), None, ori, ptr(p), ptr(q))
        gn_shape = (2 ** K - 1, 2, p.shape[1])
    else:
        n = np.ascontiguousarray(d["n"], dt)
        net = L.DmnNet(K, ptr(w), ptr(n), 0, None, None)
        gn_shape = (2 ** K - 1, 3)
    lam_p = ptr(lam) if lam is not None else None
    Cbar = np.zeros((B, 6, 6), dt)
    nb = lib.dmn_homogenize_linear_workspace_size(ctypes.byref(net), B, prec)
    keep, ws = workspace(nb)
    L.check(lib.dmn_homogenize_linear(ctypes.byref(net), B, prec, ptr(C1), ptr(C2), lam_p,
                                      ptr(Cbar), ptr(ws), nb, None), "dmn_homogenize_linear")
    err_f = int(ws[:4].view(np.int32)[0])
    gw = np.zeros(2 ** K, dt)
    gn = np.zeros(gn_shape, dt)
    ig = int(d["input_grads"])
    gC1 = np.zeros((B, 6, 6), dt) if ig else None
    gC2 = np.zeros((B, 6, 6), dt) if ig else None
    nb = lib.dmn_homogenize_backward_workspace_size(ctypes.byref(net), B, prec)
    keep2, ws2 = workspace(nb)
    L.check(lib.dmn_homogenize_backward(ctypes.byref(net), B, prec, ptr(C1), ptr(C2), lam_p,
                                        ptr(G), ptr(gw), ptr(gn), ptr(gC1) if ig else None,
                                        ptr(gC2) if ig else None, ptr(ws2), nb, None),
            "dmn_homogenize_backward")
    err_b = int(ws2[:4].view(np.int32)[0])
    out = dict(Cbar=Cbar, gw=gw, gn=gn, err=np.array([err_f, err_b]))
    if ig:
        out.update(gC1=gC1, gC2=gC2)
    np.savez(out_path, **out)


if __name__ == "__main__":
    main(*sys.argv[1:4])
