"""Child process of the CPU-build tests: the gradient of J = sum_p g_p .
sigma_p(final) along a load path, by the forward path through
dmn_update_gauss_points and the load-step adjoint dmn_update_adjoint swept
backwards over the stored steps, in a sanitised CPU library.

    python run_adjoint.py LIB IN.npz OUT.npz

IN.npz: depth, w, n, E [T, P, 6], g [P, 6], opts (as run_gp.py), fiber, matrix.
OUT.npz: sigma (final), gw, gn, and the adjoint calls' device error words.
"""
import ctypes
import sys

import numpy as np

from run_gp import load_lib_module, ptr


def aligned(nbytes):
    raw = np.zeros(nbytes + 256, np.uint8)
    off = (-raw.ctypes.data) % 256
    return raw, raw[off:off + nbytes]


def main(lib_path, in_path, out_path):
    L = load_lib_module(lib_path)
    lib = L.lib()
    d = np.load(in_path)
    K = int(d["depth"])
    E = d["E"]
    T, P = E.shape[:2]
    M, Lm = 2 ** (K - 1), 2 ** K - 1
    w = np.ascontiguousarray(d["w"], np.float64)
    n = np.ascontiguousarray(d["n"], np.float64)
    o = d["opts"]
    opts = L.DmnNewtonOpts(float(o[0]), int(o[1]), int(o[2]), float(o[3]), int(o[4]), int(o[5]))
    fib, mat = L.DmnElastic(*d["fiber"]), L.DmnJ2(*d["matrix"])
    net = L.DmnNet(K, ptr(w), ptr(n), 0, None, None)
    z, a = np.zeros((P, M, 7)), np.zeros((P, Lm, 3))
    states = []
    sigma = np.zeros((P, 6))
    for s in range(T):
        Es = np.ascontiguousarray(E[s])
        zo, ao = np.zeros_like(z), np.zeros_like(a)
        tan, it, st = np.zeros((P, 6, 6)), np.zeros(P, np.int32), np.zeros(P, np.int32)
        grp = L.DmnPointGroup(net, P, ptr(Es), ptr(z), ptr(zo), ptr(a), ptr(ao), ptr(sigma),
                              ptr(tan), ptr(it), ptr(st), None)
        arr = (L.DmnPointGroup * 1)(grp)
        nb = lib.dmn_update_gauss_points_workspace_size(arr, 1, L.DMN_F64)
        keep, ws = aligned(nb)
        L.check(lib.dmn_update_gauss_points(arr, 1, ctypes.byref(fib), ctypes.byref(mat),
                                            L.DMN_F64, ctypes.byref(opts), ptr(ws), nb, None),
                "dmn_update_gauss_points")
        if np.any(st != 0):
            raise SystemExit(f"step {s}: status {st}")
        states.append((Es, z, ao))
        z, a = zo, ao
    gw, gn = np.zeros(2 ** K), np.zeros((Lm, 3))
    g = np.ascontiguousarray(d["g"], np.float64)
    zeta = None
    errs = []
    for s in reversed(range(T)):
        Es, z_n, a_conv = states[s]
        out = np.zeros((P, M, 7))
        grp = L.DmnAdjointGroup(net, P, ptr(Es), ptr(z_n), ptr(a_conv),
                                ptr(g) if s == T - 1 else None,
                                None if zeta is None else ptr(zeta), ptr(out), ptr(gw), ptr(gn))
        arr = (L.DmnAdjointGroup * 1)(grp)
        nb = lib.dmn_update_adjoint_workspace_size(arr, 1, L.DMN_F64)
        keep, ws = aligned(nb)
        L.check(lib.dmn_update_adjoint(arr, 1, ctypes.byref(fib), ctypes.byref(mat), L.DMN_F64,
                                       ptr(ws), nb, None), "dmn_update_adjoint")
        errs.append(int(ws[:4].view(np.int32)[0]))
        zeta = out
    np.savez(out_path, sigma=sigma, gw=gw, gn=gn, err=np.array(errs))


if __name__ == "__main__":
    main(*sys.argv[1:4])
