"""Child process of the CPU-build tests: the offline-training calls
(dmn_training_loss, dmn_sample_stiffness, dmn_training_update) of a sanitised
CPU library (tests/simt/build.py).

    python run_train.py LIB IN.npz OUT.npz

IN.npz holds the inputs of whichever calls it names (float64 or float32: the
call's precision):
  loss:      Cbar, target [B, 6, 6], p, q
  stiffness: u [B, 8] (float64), sprec (0 float64, 1 float32)
  update:    v, alpha, beta, gw, gn, state [3, NP], step, stats0, amsgrad [9]
OUT.npz: e, gCbar, loss_stats; C1, C2; v, alpha, beta, w, n, state, step,
update_stats.
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
    out = {}
    if "Cbar" in d.files:
        dt = d["Cbar"].dtype
        prec = L.DMN_F32 if dt == np.float32 else L.DMN_F64
        Cb, Tt = np.ascontiguousarray(d["Cbar"]), np.ascontiguousarray(d["target"])
        B = Cb.shape[0]
        e = np.zeros(B, dt)
        g = np.zeros((B, 6, 6), dt)
        stats = np.zeros(L.DMN_TRAIN_STATS, np.float64)
        nb = lib.dmn_training_loss_workspace_size(B)
        keep, ws = workspace(nb)
        opts = L.DmnLossOpts(float(d["p"]), float(d["q"]))
        L.check(lib.dmn_training_loss(B, prec, ptr(Cb), ptr(Tt), ctypes.byref(opts), ptr(e),
                                      ptr(g), ptr(stats), ptr(ws), nb, None),
                "dmn_training_loss")
        out.update(e=e, gCbar=g, loss_stats=stats)
    if "u" in d.files:
        u = np.ascontiguousarray(d["u"], np.float64)
        sdt = np.float32 if int(d["sprec"]) else np.float64
        B = u.shape[0]
        C1, C2 = np.zeros((B, 6, 6), sdt), np.zeros((B, 6, 6), sdt)
        L.check(lib.dmn_sample_stiffness(B, L.DMN_F32 if int(d["sprec"]) else L.DMN_F64, ptr(u),
                                         ptr(C1), ptr(C2), None), "dmn_sample_stiffness")
        out.update(C1=C1, C2=C2)
    if "v" in d.files:
        dt = d["v"].dtype
        prec = L.DMN_F32 if dt == np.float32 else L.DMN_F64
        v, alpha, beta = (np.ascontiguousarray(d[k]).copy() for k in ("v", "alpha", "beta"))
        K = int(round(np.log2(v.size)))
        w = np.zeros(2 ** K, dt)
        n = np.zeros((2 ** K - 1, 3), dt)
        state = np.ascontiguousarray(d["state"]).copy()
        step = np.array([int(d["step"])], np.int64)
        P = L.DmnTrainParams(K, ptr(v), ptr(alpha), ptr(beta), ptr(w), ptr(n), ptr(state),
                             ptr(step))
        a = d["amsgrad"]
        o = L.DmnAmsgradOpts(float(a[0]), float(a[1]), float(a[2]), int(a[3]), int(a[4]),
                             float(a[5]), float(a[6]), float(a[7]), float(a[8]))
        stats = np.zeros(L.DMN_TRAIN_STATS, np.float64)
        stats[0] = float(d["stats0"])
        gw, gn = np.ascontiguousarray(d["gw"]), np.ascontiguousarray(d["gn"])
        L.check(lib.dmn_training_update(ctypes.byref(P), prec, ptr(gw), ptr(gn), ctypes.byref(o),
                                        ptr(stats), None), "dmn_training_update")
        out.update(v=v, alpha=alpha, beta=beta, w=w, n=n, state=state, step=step,
                   update_stats=stats)
    np.savez(out_path, **out)


if __name__ == "__main__":
    main(*sys.argv[1:4])
