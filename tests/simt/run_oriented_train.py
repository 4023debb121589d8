"""Child process of the CPU-build tests: one training step of an
orientation-interpolated DMN over a batch grouped by orientation, through the
calls of a sanitised CPU library (tests/simt/build.py), in the order a
training step makes them: refreshed weights, the groups' normals, the grouped
linear map, the objective, the grouped VJP, the chain to the angle
coefficients and the optimiser step.

    python run_oriented_train.py LIB IN.npz OUT.npz

IN.npz: ori (1 linear, 2 tri-linear, 3 quadratic), v [2^K], p, q [L, M],
lam [G, 2], offsets [G + 1], C1, C2, target [B, 6, 6] (float64 or float32:
the calls' precision), p_norm, q_norm, amsgrad [9].
OUT.npz: Cbar, gw, gpq, stats, v, p, q, state, step, err (the two linear
calls' error words).
"""
import ctypes
import sys

import numpy as np

from run_gp import load_lib_module, ptr
from run_linear import workspace


def main(lib_path, in_path, out_path):
    L = load_lib_module(lib_path)
    lib = L.lib()
    d = np.load(in_path)
    dt = d["C1"].dtype
    prec = L.DMN_F32 if dt == np.float32 else L.DMN_F64
    ori = int(d["ori"])
    v, p, q = (np.ascontiguousarray(d[k], dt).copy() for k in ("v", "p", "q"))
    K = int(round(np.log2(v.size)))
    NL, Lm, M = 2 ** K, 2 ** K - 1, p.shape[1]
    lam = np.ascontiguousarray(d["lam"], dt)
    G = lam.shape[0]
    off = (ctypes.c_int64 * (G + 1))(*[int(x) for x in d["offsets"]])
    C1, C2, Tt = (np.ascontiguousarray(d[k], dt) for k in ("C1", "C2", "target"))
    B = C1.shape[0]
    w = np.zeros(NL, dt)
    state = np.zeros((3, NL + 2 * Lm * M), dt)
    step = np.zeros(1, np.int64)
    P = L.DmnTrainParamsOriented(K, ori, ptr(v), ptr(p), ptr(q), ptr(w), ptr(state), ptr(step))
    L.check(lib.dmn_training_refresh_oriented(ctypes.byref(P), prec, None),
            "dmn_training_refresh_oriented")
    n_groups = np.zeros((G, Lm, 3), dt)
    L.check(lib.dmn_orientation_group_normals(K, ori, G, prec, ptr(p), ptr(q), ptr(lam),
                                              ptr(n_groups), None),
            "dmn_orientation_group_normals")
    Cbar = np.zeros((B, 6, 6), dt)
    nb = lib.dmn_homogenize_linear_groups_workspace_size(K, G, prec)
    keep1, ws1 = workspace(nb)
    L.check(lib.dmn_homogenize_linear_groups(K, G, off, prec, ptr(w), ptr(n_groups), ptr(C1),
                                             ptr(C2), ptr(Cbar), ptr(ws1), nb, None),
            "dmn_homogenize_linear_groups")
    gC = np.zeros((B, 6, 6), dt)
    stats = np.zeros(L.DMN_TRAIN_STATS, np.float64)
    nb = lib.dmn_training_loss_workspace_size(B)
    keep2, ws2 = workspace(nb)
    lo = L.DmnLossOpts(float(d["p_norm"]), float(d["q_norm"]))
    L.check(lib.dmn_training_loss(B, prec, ptr(Cbar), ptr(Tt), ctypes.byref(lo), None, ptr(gC),
                                  ptr(stats), ptr(ws2), nb, None), "dmn_training_loss")
    gw_g = np.zeros((G, NL), dt)
    gn_g = np.zeros((G, Lm, 3), dt)
    nb = lib.dmn_homogenize_backward_groups_workspace_size(K, G, off, prec)
    keep3, ws3 = workspace(nb)
    L.check(lib.dmn_homogenize_backward_groups(K, G, off, prec, ptr(w), ptr(n_groups), ptr(C1),
                                               ptr(C2), ptr(gC), ptr(gw_g), ptr(gn_g), ptr(ws3),
                                               nb, None), "dmn_homogenize_backward_groups")
    gw = np.zeros(NL, dt)
    gpq = np.zeros((Lm, 2, M), dt)
    L.check(lib.dmn_orientation_group_chain(K, ori, G, prec, ptr(p), ptr(q), ptr(lam), ptr(gw_g),
                                            ptr(gn_g), ptr(gw), ptr(gpq), None),
            "dmn_orientation_group_chain")
    a = d["amsgrad"]
    o = L.DmnAmsgradOpts(float(a[0]), float(a[1]), float(a[2]), int(a[3]), int(a[4]),
                         float(a[5]), float(a[6]), float(a[7]), float(a[8]))
    L.check(lib.dmn_training_update_oriented(ctypes.byref(P), prec, ptr(gw), ptr(gpq),
                                             ctypes.byref(o), ptr(stats), None),
            "dmn_training_update_oriented")
    err = np.array([int(ws1[:4].view(np.int32)[0]), int(ws3[:4].view(np.int32)[0])])
    np.savez(out_path, Cbar=Cbar, gw=gw, gpq=gpq, stats=stats, v=v, p=p, q=q, state=state,
             step=step, err=err)


if __name__ == "__main__":
    main(*sys.argv[1:4])
