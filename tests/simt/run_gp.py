"""Child process of the CPU-build tests: runs load paths through
dmn_update_gauss_points of the sanitised CPU library (tests/simt/build.py).

    python run_gp.py LIB IN.npz OUT.npz

IN.npz: n_groups; per group g: g{g}_depth, g{g}_w, g{g}_n (fixed normals) or
g{g}_ori (1 linear, 2 tri-linear, 3 quadratic) with g{g}_p, g{g}_q, g{g}_lam;
g{g}_E [T, P, 6]; opts [tol, max_iter, max_backtrack, armijo, local_max_iter,
polish]; prec (0 FP64, 2 FP32 state); tuning [[depth, lanes, waves], ...];
noalloc (1: the entry point without a workspace argument).
OUT.npz: per group and step the outputs (sigma, tangent, z, a, iters, status).

Runs under the ASan runtime (LD_PRELOAD): the per-point arrays are separate
host allocations, so a kernel index past any of them stops the process.
"""
import ctypes
import importlib.util
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))


def load_lib_module(path):
    spec = importlib.util.spec_from_file_location(
        "dmn_lib_simt", os.path.join(ROOT, "paper_2103_08253_amd", "_lib.py"))
    L = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(L)
    L.LIB_PATH = path
    return L


def ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def main(lib_path, in_path, out_path):
    L = load_lib_module(lib_path)
    lib = L.lib()
    d = np.load(in_path)
    ng = int(d["n_groups"])
    prec = int(d["prec"])
    st = np.float32 if prec == L.DMN_F32_STATE else np.float64
    for depth, lanes, waves in d["tuning"].reshape(-1, 3):
        L.check(lib.dmn_gp_set_tuning(int(depth), ctypes.byref(L.DmnGpTuning(int(lanes), int(waves)))),
                "dmn_gp_set_tuning")
    o = d["opts"]
    opts = L.DmnNewtonOpts(float(o[0]), int(o[1]), int(o[2]), float(o[3]), int(o[4]), int(o[5]))
    fib = L.DmnElastic(*d["fiber"])
    mat = L.DmnJ2(*d["matrix"])
    groups, keep = [], []
    for g in range(ng):
        K = int(d[f"g{g}_depth"])
        E = d[f"g{g}_E"]
        T, P = E.shape[:2]
        M, Lm = 2 ** (K - 1), 2 ** K - 1
        w = np.ascontiguousarray(d[f"g{g}_w"], dtype=np.float64)
        arr = dict(w=w, E=np.zeros((P, 6), st), z_in=np.zeros((P, M, 7), st),
                   z_out=np.zeros((P, M, 7), st), a_in=np.zeros((P, Lm, 3), st),
                   a_out=np.zeros((P, Lm, 3), st), sigma=np.zeros((P, 6), st),
                   tangent=np.zeros((P, 6, 6), st), iters=np.zeros(P, np.int32),
                   status=np.zeros(P, np.int32), path=E, steps=T)
        ori = int(d[f"g{g}_ori"]) if f"g{g}_ori" in d else 0
        if ori:
            arr["p"] = np.ascontiguousarray(d[f"g{g}_p"], dtype=np.float64)
            arr["q"] = np.ascontiguousarray(d[f"g{g}_q"], dtype=np.float64)
            arr["lam"] = np.ascontiguousarray(d[f"g{g}_lam"], dtype=np.float64)
            net = L.DmnNet(K, ptr(w), None, ori, ptr(arr["p"]), ptr(arr["q"]))
        else:
            arr["n"] = np.ascontiguousarray(d[f"g{g}_n"], dtype=np.float64)
            net = L.DmnNet(K, ptr(w), ptr(arr["n"]), 0, None, None)
        arr["net"] = net
        keep.append(arr)
    T = keep[0]["steps"]
    out = {}
    for step in range(T):
        cg = []
        for a in keep:
            a["E"][...] = a["path"][step]
            cg.append(L.DmnPointGroup(a["net"], a["E"].shape[0], ptr(a["E"]), ptr(a["z_in"]),
                                      ptr(a["z_out"]), ptr(a["a_in"]), ptr(a["a_out"]),
                                      ptr(a["sigma"]), ptr(a["tangent"]), ptr(a["iters"]),
                                      ptr(a["status"]), ptr(a.get("lam"))))
        carr = (L.DmnPointGroup * ng)(*cg)
        if int(d["noalloc"]):
            rc = lib.dmn_update_gauss_points_noalloc(carr, ng, ctypes.byref(fib),
                                                     ctypes.byref(mat), prec,
                                                     ctypes.byref(opts), None)
        else:
            nb = lib.dmn_update_gauss_points_workspace_size(carr, ng, prec)
            if nb == 0:
                raise SystemExit("workspace size rejected the groups")
            raw = np.zeros(nb + 256, np.uint8)
            off = (-raw.ctypes.data) % 256
            ws = raw[off:off + nb]
            rc = lib.dmn_update_gauss_points(carr, ng, ctypes.byref(fib), ctypes.byref(mat),
                                             prec, ctypes.byref(opts), ptr(ws), nb, None)
        L.check(rc, "dmn_update_gauss_points")
        for g, a in enumerate(keep):
            for k, src in (("sigma", "sigma"), ("C", "tangent"), ("z", "z_out"), ("a", "a_out"),
                           ("iters", "iters"), ("status", "status")):
                out[f"g{g}_s{step}_{k}"] = a[src].copy()
            a["z_in"], a["z_out"] = a["z_out"], a["z_in"]
            a["a_in"], a["a_out"] = a["a_out"], a["a_in"]
    np.savez(out_path, **out)


if __name__ == "__main__":
    main(*sys.argv[1:4])
