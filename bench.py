#!/usr/bin/env python3
"""Throughput of the DMN hot path on one MI355X.

One bench step is one pass of the whole hot path over one batch:
  * one load step of the depth-8 production workload: 65,536 Gauss points,
    FP64 (parameter prep, localisation, J2 leaves, tree Newton with
    backtracking, stress + tangent + state), taken in order along the seeded
    20-step strain path;
  * one training forward + backward of the depth-8 linear DMN map on a batch
    of 4,096 phase-stiffness pairs (FP64) with a seeded cotangent; and
  * one load-step adjoint of the depth-8 path-sensitivity workload (16,384
    points at step 25 of their 50-step path, cotangents of stress and state).

The launch of each depth is autotuned first (lanes per point, persistent
waves; cached on disk).  Reported beside the headline, outside its timed
region: the mixed-depth batch (131,072 points over 16 DMNs of depths 5-9,
the 20-step path captured as one HIP graph and replayed), the depth-8 update
with orientation-interpolated normals (every point its own fibre
orientation), the paper's six uniaxial strain hystereses with its material
constants (80 steps, one graph), and the plain one-launch-per-point and one-launch-per-sample
forms of the same library on the same GPU, for comparison with the batched
launches.

Inputs are synthetic (see synthetic/), resident on the GPU before timing.
Prints one JSON line.  `value` is Gauss-point updates per second of whole
step time; the training rate and per-component times are reported beside it,
together with the roofline of the dominant kernel and the FP64 CPU oracle
timed on a bounded sample on the host cores.

    python bench.py [--gpus 1] [--steps 20] [--warmup 2] [--no-cpu-baseline]
                    [--no-autotune] [--no-extras]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DMN Gauss-point updates/s (stress+tangent, depth 8, FP64) + train fwd+bwd samples/s"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gp_update_depth8_traffic.json")
GP_SOURCES = ["paper_2103_08253_amd/csrc/dmn_gp.hip", "paper_2103_08253_amd/csrc/dmn_algebra.hpp",
              "paper_2103_08253_amd/csrc/dmn_tree.hpp",
              "paper_2103_08253_amd/csrc/dmn_internal.hpp"]


def code_text(src: str) -> str:
    """Source without its comments and blank lines: what the compiler builds
    from (a string literal holding comment markers would be cut too, which
    only makes the digest change more often)."""
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def source_digest(paths):
    """Digest of the kernel sources' code (comments do not count), which the
    recorded HBM traffic must match."""
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from committed rocprofv3 counters, if they were taken
    on the current kernel source; None otherwise."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest(GP_SOURCES):
        return None
    return rec.get("bytes_per_launch")


# ---------------------------------------------------------------- CPU baseline

def _oracle_worker(args):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np
    import synthetic as S
    from oracle.gp import DmnModel, NewtonOptions, run_path
    points, n_steps = args
    wl = S.config1()
    net = wl.nets[0]
    model = DmnModel(net.depth, net.w, net.normals, S.FIBER, S.MATRIX)
    n = 0
    for p in points:
        outs = run_path(model, wl.E[:n_steps, p, :], NewtonOptions())
        n += len(outs)
    return n


# host cores a process on the GPU host may keep busy: the host's share for one
# GPU (os.cpu_count() there reports the whole machine)
HOST_CORE_SHARE = 16


def cpu_baseline(n_points=256, n_steps=20, workers=None):
    """The FP64 oracle (dense Newton, LAPACK Cholesky) on a sample of the same
    workload: n_points seeded points along their full 20-step path, one process
    per core of the host's share with single-threaded BLAS."""
    import multiprocessing as mp
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    workers = workers or min(HOST_CORE_SHARE, os.cpu_count() or 1, n_points)
    chunks = [list(range(i, n_points, workers)) for i in range(workers)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_worker, [([0], 1)] * workers)  # import + workload setup
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_worker, [(c, n_steps) for c in chunks]))
        dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="GP updates/s", cores=workers, kind="oracle",
                sample=f"{n_points} points x {n_steps} load steps of the depth-8 production "
                       f"workload ({done} updates, {dt:.1f} s wall on {workers} processes, "
                       f"one per core; the host reports {os.cpu_count()} logical CPUs)")


# ---------------------------------------------------------------- GPU bench

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-points", type=int, default=256)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-batch graph and the one-launch-per-point forms")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs the hot path on a single "
              "MI355X; Gauss points are independent, and sharding them over several GPUs "
              "is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synthetic as S
    from paper_2103_08253_amd import (AdjointGroup, PointGroup, dmn_homogenize_backward,
                                      dmn_homogenize_linear, dmn_update_adjoint,
                                      dmn_update_gauss_points)
    from paper_2103_08253_amd import autotune as A
    from paper_2103_08253_amd import roofline as R
    from paper_2103_08253_amd import _lib

    _lib.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    wl = S.config1()
    net = wl.nets[0]
    T, P = wl.n_steps, wl.n_points
    E_path = torch.tensor(wl.E, device=dev)           # [20, P, 6]
    w = torch.tensor(net.w, device=dev)
    n = torch.tensor(net.normals, device=dev)
    g = PointGroup.allocate(w, n, E_path[0])

    tw = S.config3()
    B = tw.C1.shape[0]
    C1 = torch.tensor(tw.C1, device=dev)
    C2 = torch.tensor(tw.C2, device=dev)
    Gc = torch.tensor(S.streams(3)["cotangent"].standard_normal((B, 6, 6)), device=dev)
    wt = torch.tensor(tw.v0, device=dev)
    nt = torch.tensor(S.angles_to_normals(tw.alpha0, tw.beta0), device=dev)

    # adjoint workload: state of the 16,384-point path at its step 25
    wa = S.config4()
    neta = wa.nets[0]
    Ea = torch.tensor(wa.E[:26], device=dev)
    wadj = torch.tensor(neta.w, device=dev)
    nadj = torch.tensor(neta.normals, device=dev)
    ga = PointGroup.allocate(wadj, nadj, Ea[0])
    ws_a = None
    for k in range(25):
        ga.E = Ea[k]
        ws_a = dmn_update_gauss_points([ga], S.FIBER, S.MATRIX, ws=ws_a)
        ga.advance()
    z25 = ga.z_in.clone()
    ga.E = Ea[25]
    dmn_update_gauss_points([ga], S.FIBER, S.MATRIX, ws=ws_a)
    Pa = wa.n_points
    rs_a = S.streams(4)
    g_sig = torch.tensor(wa.g_sigma, device=dev)
    g_znext = torch.tensor(1e3 * rs_a["cotangent"].standard_normal((Pa, 128, 7)), device=dev)
    g_zprev = torch.empty_like(g_znext)
    gw_a = torch.zeros(256, dtype=torch.float64, device=dev)
    gn_a = torch.zeros((255, 3), dtype=torch.float64, device=dev)
    adj = AdjointGroup(wadj, nadj, Ea[25], z25, ga.a_out.clone(), g_sig, g_znext, g_zprev,
                       gw_a, gn_a)
    ws_adj = None

    # one-off device copy of a known size (calibrates HBM byte counters in profiles)
    calib_src = torch.empty(256 * 2 ** 20, dtype=torch.uint8, device=dev)
    calib_dst = torch.empty_like(calib_src)
    calib_dst.copy_(calib_src)
    del calib_src, calib_dst

    ws_gp = None
    ws_lin = ws_bwd = None
    tuned = {}
    if not args.no_autotune:
        tuned = A.tune_gauss_points([g], S.FIBER, S.MATRIX)
        g.z_in.zero_()
        g.a_in.zero_()
    lanes8, waves8 = A.get_tuning(8)

    def reset_state():
        g.z_in.zero_()
        g.a_in.zero_()

    def gp_step(k):
        nonlocal ws_gp
        g.E = E_path[k % T]
        if k % T == 0 and k > 0:
            reset_state()
        ws_gp = dmn_update_gauss_points([g], S.FIBER, S.MATRIX, ws=ws_gp)
        g.advance()

    def train_step():
        nonlocal ws_lin, ws_bwd
        _, ws_lin = dmn_homogenize_linear(wt, nt, C1, C2, ws=ws_lin)
        out = dmn_homogenize_backward(wt, nt, C1, C2, Gc, ws=ws_bwd)
        ws_bwd = out[-1]

    def adjoint_step():
        nonlocal ws_adj
        ws_adj = dmn_update_adjoint([adj], S.FIBER, S.MATRIX, ws=ws_adj)

    for k in range(args.warmup):
        gp_step(k)
        train_step()
        adjoint_step()
    torch.cuda.synchronize()
    reset_state()

    K = args.steps
    iters_log = torch.empty((K, P), dtype=torch.int32, device=dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        ev[k][0].record()
        gp_step(k)
        ev[k][1].record()
        iters_log[k].copy_(g.iters)
        ev[k][2].record()
        train_step()
        ev[k][3].record()
        ev[k][4].record()
        adjoint_step()
        ev[k][5].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    gp_ms = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)])
    tr_ms = np.array([ev[k][2].elapsed_time(ev[k][3]) for k in range(K)])
    ad_ms = np.array([ev[k][4].elapsed_time(ev[k][5]) for k in range(K)])
    status_ok = bool((g.status == 0).all().item())
    it = iters_log.cpu().numpy()
    flops = np.array([sum(int(c) * R.gp_update_flops(8, int(v))
                          for v, c in zip(*np.unique(it[k], return_counts=True)))
                      for k in range(K)], dtype=np.float64)
    achieved_tf = flops.sum() / (gp_ms.sum() * 1e-3) / 1e12
    bytes_launch = P * R.gp_update_bytes(8)
    traffic = measured_traffic()
    train_flops = B * (R.linear_forward_flops(8) + R.linear_backward_flops(8))

    ms_per_step = wall * 1e3 / K
    rec = dict(
        metric=METRIC,
        value=P * K / wall,
        unit="GP updates/s",
        n_gpus=1, steps=K, warmup=args.warmup,
        ms_per_step=ms_per_step,
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload="depth8_production: 65536 Gauss points, 20-step strain path "
                             "(ramp to 1.5 % + N(0,1e-3) walk), J2 matrix + elastic fibre; "
                             "plus depth-8 linear fwd+bwd on 4096 SPD phase pairs and one "
                             "load-step adjoint on 16384 points",
                    depth=8, gauss_points=P, load_steps_in_path=T, train_batch=B,
                    newton_tol=1e-10),
        train_samples_per_s=B * K / (tr_ms.sum() * 1e-3),
        components=dict(
            gp_update=dict(tuning=[lanes8, waves8], ms_mean=float(gp_ms.mean()),
                           ms_min=float(gp_ms.min()),
                           ms_max=float(gp_ms.max()),
                           updates_per_s=float(P / (gp_ms.mean() * 1e-3)),
                           mean_newton_iters=float(it.mean()), all_converged=status_ok,
                           algorithmic_gflop_per_launch=float(flops.mean() / 1e9),
                           algorithmic_bytes_per_launch=bytes_launch),
            train_fwd_bwd=dict(ms_mean=float(tr_ms.mean()),
                               samples_per_s=float(B / (tr_ms.mean() * 1e-3)),
                               tflops=float(train_flops / (tr_ms.mean() * 1e-3) / 1e12)),
            path_adjoint_step=dict(ms_mean=float(ad_ms.mean()), points=Pa,
                                   point_steps_per_s=float(Pa / (ad_ms.mean() * 1e-3)))),
        roofline=dict(bound="alu", achieved=float(achieved_tf), peak=R.FP64_PEAK_TFLOPS,
                      unit="TFLOP/s", frac=float(achieved_tf / R.FP64_PEAK_TFLOPS),
                      traffic=traffic, kernel="gp_update_kernel<8,2> (FP64 VALU)"),
    )
    rec["roofline"]["kernel"] = (f"gp_update_kernel<8,{8 - (lanes8.bit_length() - 1)}> "
                                 f"({lanes8} lanes per point, {waves8} waves/CU; FP64 VALU)")
    if not args.no_extras:
        rec["components"].update(extras(args, dev, g, E_path, gp_step, reset_state, B, C1, C2,
                                        Gc, wt, nt, tuned))
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(args.cpu_points)
    print(json.dumps(rec), flush=True)


def _graph_of(fn):
    """Capture fn's library calls into a HIP graph (removes the host-side cost
    of issuing many small calls from the timing)."""
    import torch
    fn()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=stream):
        fn()
    torch.cuda.current_stream().wait_stream(stream)
    return graph


def _event_ms(fn, reps=1):
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b)


def extras(args, dev, g, E_path, gp_step, reset_state, B, C1, C2, Gc, wt, nt, tuned):
    """Mixed-depth batch as a replayed HIP graph, and the plain one-launch-per-
    point / per-sample forms of the same calls (timed apart from the headline)."""
    import numpy as np
    import torch
    import synthetic as S
    from paper_2103_08253_amd import (LoadStepGraph, PointGroup, dmn_homogenize_backward,
                                      dmn_homogenize_linear, dmn_update_gauss_points)
    from paper_2103_08253_amd import autotune as A
    out = {}

    # batched vs one launch per point, both at load step 10 of the production path
    reset_state()
    for k in range(10):
        gp_step(k)
    g.E = E_path[10]
    torch.cuda.synchronize()
    ws = dmn_update_gauss_points([g], S.FIBER, S.MATRIX)
    P = g.E.shape[0]
    batched_ms = _event_ms(lambda: dmn_update_gauss_points([g], S.FIBER, S.MATRIX, ws=ws), 3) / 3
    n_plain = 512
    picks = np.linspace(0, P - 1, n_plain).astype(int)
    singles = [PointGroup(g.w, g.n, g.E[p:p + 1], g.z_in[p:p + 1], g.z_out[p:p + 1],
                          g.a_in[p:p + 1], g.a_out[p:p + 1], g.sigma[p:p + 1],
                          g.tangent[p:p + 1], g.iters[p:p + 1], g.status[p:p + 1])
                for p in picks]
    ws1 = dmn_update_gauss_points([singles[0]], S.FIBER, S.MATRIX)

    def plain():
        for sg in singles:
            dmn_update_gauss_points([sg], S.FIBER, S.MATRIX, ws=ws1)
    plain_graph = _graph_of(plain)
    plain_graph.replay()
    plain_ms = _event_ms(plain_graph.replay) / n_plain
    out["gp_update_one_launch_per_point"] = dict(
        points_sampled=n_plain, load_step=10, issued_as="one library call per point, "
        "replayed from a HIP graph (device time only)", us_per_point=plain_ms * 1e3,
        updates_per_s=1e3 / plain_ms, batched_updates_per_s=P / (batched_ms * 1e-3),
        batched_speedup=(plain_ms * P) / batched_ms)

    # orientation-interpolated normals: depth 8, quadratic shape functions, every
    # point its own (l1, l2); load step 10 of the same kind of path
    from paper_2103_08253_amd import Orientation
    net_o, lam_o, E_o = S.orientation_workload()
    ori = Orientation(net_o.kind, torch.tensor(net_o.p, device=dev),
                      torch.tensor(net_o.q, device=dev), torch.tensor(lam_o, device=dev))
    E_ot = torch.tensor(E_o, device=dev)
    go = PointGroup.allocate(torch.tensor(net_o.w, device=dev), None, E_ot[0].clone(), ori=ori)
    ws_o = None
    for k in range(10):
        go.E = E_ot[k]
        ws_o = dmn_update_gauss_points([go], S.FIBER, S.MATRIX, ws=ws_o)
        go.advance()
    go.E = E_ot[10]
    ori_ms = _event_ms(lambda: dmn_update_gauss_points([go], S.FIBER, S.MATRIX, ws=ws_o), 3) / 3
    out["gp_update_orientation_interpolated"] = dict(
        points=E_o.shape[1], depth=8, shape_functions=net_o.kind, load_step=10,
        ms=ori_ms, updates_per_s=E_o.shape[1] / (ori_ms * 1e-3),
        all_converged=bool((go.status == 0).all().item()),
        fixed_normals_ms_same_step=batched_ms)

    # tree compression (Sec. 3.1): the same load step with about a third of the
    # laminates removed by zero leaf weights (the paper's compressed network keeps
    # 513 of 765 jump unknowns: 171 of 255 laminates), the dead leaves either
    # scattered (one leaf of a live pair) or whole 4-leaf subtrees (one lane's
    # subtree each); the kernel evaluates dead rows in place, so only live work
    # is credited in the rate below
    from paper_2103_08253_amd.roofline import gp_update_flops_live, live_tree_counts

    def live_tflops(counts, iters, ms):
        it = iters.double()
        tot = it.sum().item()
        per_eval = gp_update_flops_live(*counts, 0)
        desc = gp_update_flops_live(*counts, 1) - 2 * per_eval  # top-down flops per step
        return ((tot + iters.numel()) * per_eval + tot * desc) / (ms * 1e-3) / 1e12

    w_full = g.w.cpu().numpy()
    comp = dict(load_step=10, points=P, target_live_laminates=171,
                full=dict(live_laminates=255, ms=batched_ms,
                          mean_iters=g.iters.double().mean().item(),
                          live_credited_tflops=live_tflops(live_tree_counts(w_full), g.iters,
                                                           batched_ms)))
    rng_c = np.random.default_rng(11)
    for pattern in ("scattered_leaves", "dead_lane_subtrees"):
        wc = w_full.copy()
        while live_tree_counts(wc)[0] > 171:
            if pattern == "scattered_leaves":
                j = int(rng_c.integers(0, len(wc)))
                if wc[j ^ 1] > 0:
                    wc[j] = 0.0
            else:
                b = 4 * int(rng_c.integers(0, len(wc) // 4))
                wc[b:b + 4] = 0.0
        counts = live_tree_counts(wc)
        gc = PointGroup.allocate(torch.tensor(wc, device=dev), g.n, E_path[0].clone())
        ws_c = None
        for k in range(10):
            gc.E = E_path[k]
            ws_c = dmn_update_gauss_points([gc], S.FIBER, S.MATRIX, ws=ws_c)
            gc.advance()
        gc.E = E_path[10]
        ms_c = _event_ms(lambda: dmn_update_gauss_points([gc], S.FIBER, S.MATRIX, ws=ws_c), 3) / 3
        lanes_dead = int(sum(1 for b in range(0, len(wc), 4) if not (wc[b:b + 4] > 0).any()))
        comp[pattern] = dict(live_laminates=counts[0], live_matrix_leaves=counts[1],
                             live_fibre_leaves=counts[2], dead_lane_subtrees=lanes_dead,
                             ms=ms_c, mean_iters=gc.iters.double().mean().item(),
                             all_converged=bool((gc.status == 0).all().item()),
                             live_credited_tflops=live_tflops(counts, gc.iters, ms_c))
        del gc, ws_c
    out["gp_update_compressed_tree"] = comp

    # the paper's inelastic load cases: six uniaxial strain hystereses (2.5 %,
    # 80 steps, the paper's material constants) over 65,536 points, each with
    # its own fibre orientation; the 80-step path captured as one graph
    net_h, lam_h, E_h, _ = S.hysteresis_workload()
    ori_h = Orientation(net_h.kind, torch.tensor(net_h.p, device=dev),
                        torch.tensor(net_h.q, device=dev), torch.tensor(lam_h, device=dev))
    E_ht = torch.tensor(E_h, device=dev)
    gh = PointGroup.allocate(torch.tensor(net_h.w, device=dev), None, E_ht[0].clone(), ori=ori_h)
    graph_h = LoadStepGraph([gh], S.FIBER_PAPER, S.MATRIX_PAPER, [E_ht], keep_sigma=False)

    def replay_h():
        for z, a in graph_h.start_state:
            z.zero_()
            a.zero_()
        graph_h.replay()
    replay_h()
    torch.cuda.synchronize()
    hyst_ms = _event_ms(replay_h)
    out["hysteresis_paper_constants_graph"] = dict(
        points=E_h.shape[1], depth=8, shape_functions=net_h.kind, load_steps=E_h.shape[0],
        ms_per_load_step=hyst_ms / E_h.shape[0],
        updates_per_s=E_h.shape[1] * E_h.shape[0] / (hyst_ms * 1e-3),
        last_step_all_converged=bool((gh.status == 0).all().item()))
    del graph_h, gh, E_ht

    # training: one launch per sample vs the batch
    n_s = 128
    singles_t = [(C1[b:b + 1], C2[b:b + 1], Gc[b:b + 1]) for b in range(n_s)]
    _, wsf = dmn_homogenize_linear(wt, nt, C1[:1], C2[:1])
    wsb = dmn_homogenize_backward(wt, nt, C1[:1], C2[:1], Gc[:1])[-1]

    def plain_train():
        for c1, c2, gc in singles_t:
            dmn_homogenize_linear(wt, nt, c1, c2, ws=wsf)
            dmn_homogenize_backward(wt, nt, c1, c2, gc, ws=wsb)
    train_graph = _graph_of(plain_train)
    train_graph.replay()
    pt_ms = _event_ms(train_graph.replay) / n_s
    _, wsf_b = dmn_homogenize_linear(wt, nt, C1, C2)
    wsb_b = dmn_homogenize_backward(wt, nt, C1, C2, Gc)[-1]

    def batch_train():
        dmn_homogenize_linear(wt, nt, C1, C2, ws=wsf_b)
        dmn_homogenize_backward(wt, nt, C1, C2, Gc, ws=wsb_b)
    batch_train()
    bt_ms = _event_ms(batch_train, 5) / 5
    out["train_one_launch_per_sample"] = dict(
        samples_sampled=n_s, issued_as="forward + backward call per sample, replayed from a "
        "HIP graph (device time only)", us_per_sample=pt_ms * 1e3, samples_per_s=1e3 / pt_ms,
        batched_samples_per_s=B / (bt_ms * 1e-3), batched_speedup=(pt_ms * B) / bt_ms)

    # the paper's training objective end to end: forward, data term and cotangent,
    # backward, AMSGrad update as one graph per step, at the 4096-sample batch and
    # at the paper's mini-batch of 32 samples
    from paper_2103_08253_amd import (AmsgradOpts, TrainParams, TrainingStepGraph,
                                      dmn_sample_stiffness)
    tw = S.config3()
    tgt, _ = dmn_homogenize_linear(torch.tensor(tw.truth.w, device=dev),
                                   torch.tensor(tw.truth.normals, device=dev), C1, C2)
    train = {}
    for nb in (B, 32):
        Pt = TrainParams.create(torch.tensor(tw.v0, device=dev),
                                torch.tensor(tw.alpha0, device=dev),
                                torch.tensor(tw.beta0, device=dev))
        gstep = TrainingStepGraph(Pt, C1[:nb].contiguous(), C2[:nb].contiguous(),
                                  tgt[:nb].contiguous(), opts=AmsgradOpts(steps_per_epoch=10))
        gstep.replay()
        torch.cuda.synchronize()
        j0 = float(gstep.stats[3].item())
        reps = 50
        ms = _event_ms(gstep.replay, reps) / reps
        hist = {1: j0, 51: float(gstep.stats[3].item())}
        for _ in range(1950 if nb == 32 else 450):
            gstep.replay()
        hist[int(Pt.step.item())] = float(gstep.stats[3].item())
        train[nb] = dict(ms_per_step=ms, samples_per_s=nb / (ms * 1e-3),
                         objective_at_step=hist)
        # the same step in FP32 storage and arithmetic for the linear map and
        # its VJP (FP64 sums), the precision of the paper's PyTorch training
        f32 = lambda t: t.to(torch.float32)
        P32 = TrainParams.create(torch.tensor(tw.v0, device=dev, dtype=torch.float32),
                                 torch.tensor(tw.alpha0, device=dev, dtype=torch.float32),
                                 torch.tensor(tw.beta0, device=dev, dtype=torch.float32))
        g32 = TrainingStepGraph(P32, f32(C1[:nb]).contiguous(), f32(C2[:nb]).contiguous(),
                                f32(tgt[:nb]).contiguous(), opts=AmsgradOpts(steps_per_epoch=10))
        g32.replay()
        torch.cuda.synchronize()
        ms32 = _event_ms(g32.replay, reps) / reps
        train[nb]["fp32"] = dict(ms_per_step=ms32, samples_per_s=nb / (ms32 * 1e-3))
        del g32, P32
    u = torch.rand((B, 8), dtype=torch.float64, device=dev)
    dmn_sample_stiffness(u)
    torch.cuda.synchronize()
    samp_ms = _event_ms(lambda: dmn_sample_stiffness(u), 5) / 5
    # batch sweep of the captured linear forward + backward (the training step's
    # kernels) beyond the 4,096-sample workload
    from paper_2103_08253_amd import LinearStepGraph
    sweep = {}
    for nb in (4096, 16384, 65536, 262144):
        tws = S.config3(batch=nb)
        c1s = torch.tensor(tws.C1, device=dev)
        c2s = torch.tensor(tws.C2, device=dev)
        gcs = torch.tensor(S.streams(3)["cotangent"].standard_normal((nb, 6, 6)), device=dev)
        lg = LinearStepGraph(wt, nt, c1s, c2s, gcs)
        lg.replay()
        torch.cuda.synchronize()
        ms = _event_ms(lg.replay, 5) / 5
        sweep[nb] = dict(ms=ms, samples_per_s=nb / (ms * 1e-3))
        del lg
        lg32 = LinearStepGraph(wt.float(), nt.float(), c1s.float(), c2s.float(), gcs.float())
        lg32.replay()
        torch.cuda.synchronize()
        ms32 = _event_ms(lg32.replay, 5) / 5
        sweep[nb]["fp32"] = dict(ms=ms32, samples_per_s=nb / (ms32 * 1e-3))
        del lg32, c1s, c2s, gcs
    out["train_fwd_bwd_batch_sweep"] = sweep
    # training over the paper's 31 fibre orientations (linear shape functions):
    # the batch grouped by orientation, the fixed-normal maps and VJPs of all
    # groups in one grouped call each (beside: one call per group on 4 streams)
    from paper_2103_08253_amd import (OrientedTrainingStepGraph, OrientedTrainParams,
                                      dmn_homogenize_linear_groups,
                                      dmn_orientation_group_normals)
    ow = S.oriented_training_workload(batch=B)
    lam_t = torch.tensor(ow.lam, device=dev)
    truth_o = OrientedTrainParams.create(ow.truth.kind, torch.tensor(ow.truth.w, device=dev),
                                         torch.tensor(ow.truth.p, device=dev),
                                         torch.tensor(ow.truth.q, device=dev))
    n_truth = dmn_orientation_group_normals(truth_o, lam_t)
    C1o = torch.tensor(ow.C1, device=dev)
    C2o = torch.tensor(ow.C2, device=dev)
    tgt_o, _ = dmn_homogenize_linear_groups(truth_o.w, n_truth, ow.offsets, C1o, C2o)
    train_o = {}
    for nb in (B, 32):
        G = len(ow.lam)
        per = [nb // G + (1 if k < nb % G else 0) for k in range(G)]   # spread over groups
        idx = np.concatenate([ow.offsets[k] + np.arange(per[k]) for k in range(G)])
        grp = np.searchsorted(ow.offsets, idx, side="right") - 1
        offs = np.concatenate([[0], np.cumsum(np.bincount(grp, minlength=G))])
        sel = torch.tensor(idx, device=dev)
        Po = OrientedTrainParams.create(ow.truth.kind, torch.tensor(ow.v0, device=dev),
                                        torch.tensor(ow.p0, device=dev),
                                        torch.tensor(ow.q0, device=dev))
        go = OrientedTrainingStepGraph(Po, C1o[sel].contiguous(), C2o[sel].contiguous(),
                                       tgt_o[sel].contiguous(), lam_t, offs,
                                       opts=AmsgradOpts(steps_per_epoch=10))
        go.replay()
        torch.cuda.synchronize()
        j0 = float(go.stats[3].item())
        ms = _event_ms(go.replay, 20) / 20
        hist = {1: j0, 21: float(go.stats[3].item())}
        for _ in range(480):
            go.replay()
        hist[int(Po.step.item())] = float(go.stats[3].item())
        Pp = OrientedTrainParams.create(ow.truth.kind, torch.tensor(ow.v0, device=dev),
                                        torch.tensor(ow.p0, device=dev),
                                        torch.tensor(ow.q0, device=dev))
        gp = OrientedTrainingStepGraph(Pp, C1o[sel].contiguous(), C2o[sel].contiguous(),
                                       tgt_o[sel].contiguous(), lam_t, offs,
                                       opts=AmsgradOpts(steps_per_epoch=10), grouped=False)
        gp.replay()
        torch.cuda.synchronize()
        ms_pg = _event_ms(gp.replay, 20) / 20
        del gp
        train_o[nb] = dict(ms_per_step=ms, samples_per_s=nb / (ms * 1e-3),
                           per_group_calls_ms_per_step=ms_pg, objective_at_step=hist)
    out["training_oriented_step_graph"] = dict(
        depth=8, orientations=len(ow.lam), shape_functions=ow.truth.kind,
        batch_4096=train_o[B], batch_32=train_o[32])
    out["training_objective_step_graph"] = dict(
        depth=8, p=1.0, q=10.0, optimiser="AMSGrad, modulated learning rate",
        batch_4096=train[B], batch_32=train[32],
        stiffness_sampler=dict(samples=B, ms=samp_ms, samples_per_s=B / (samp_ms * 1e-3)))

    # mixed-depth batch: 16 DMNs, 131,072 points, the 20-step path as one graph
    wl = S.config2()
    groups, E_steps = [], []
    for m, net in enumerate(wl.nets):
        sel = np.nonzero(wl.dmn_id == m)[0]
        Em = torch.tensor(np.ascontiguousarray(wl.E[:, sel, :]), device=dev)
        E_steps.append(Em)
        groups.append(PointGroup.allocate(torch.tensor(net.w, device=dev),
                                          torch.tensor(net.normals, device=dev), Em[0].clone()))
    mixed_tuned = {} if args.no_autotune else A.tune_gauss_points(groups, S.FIBER, S.MATRIX)
    for gr in groups:
        gr.z_in.zero_()
        gr.a_in.zero_()
    graph = LoadStepGraph(groups, S.FIBER, S.MATRIX, E_steps, keep_sigma=False)

    def replay():
        for z, a in graph.start_state:
            z.zero_()
            a.zero_()
        graph.replay()
    replay()
    torch.cuda.synchronize()
    ok = all(bool((gr.status == 0).all().item()) for gr in groups)
    ms = _event_ms(replay, 2) / 2
    Pm = wl.n_points
    # FP32 state (per-point arrays stored in FP32, arithmetic in FP64) on the
    # same path: its last step against the FP64 run's last step just replayed
    ref64 = [(gr.sigma.clone(), gr.tangent.clone()) for gr in groups]
    groups32, E32 = [], []
    for gr, Em in zip(groups, E_steps):
        E32.append(Em.float().contiguous())
        groups32.append(PointGroup.allocate(gr.w, gr.n, E32[-1][0].clone()))
    graph32 = LoadStepGraph(groups32, S.FIBER, S.MATRIX, E32, keep_sigma=False)

    def replay32():
        for z, a in graph32.start_state:
            z.zero_()
            a.zero_()
        graph32.replay()
    replay32()
    torch.cuda.synchronize()
    ok32 = all(bool((gr.status == 0).all().item()) for gr in groups32)
    # per point: max-norm difference relative to the point's largest FP64 entry
    def per_point(a, b):
        a, b = a.double().reshape(a.shape[0], -1), b.reshape(b.shape[0], -1)
        return ((a - b).abs().max(1).values / b.abs().max(1).values).cpu().numpy()
    ds = np.concatenate([per_point(g32.sigma, s64) for g32, (s64, _) in zip(groups32, ref64)])
    dc = np.concatenate([per_point(g32.tangent, c64) for g32, (_, c64) in zip(groups32, ref64)])
    ms32 = _event_ms(replay32, 2) / 2
    fp32_state = dict(
        ms_per_load_step=ms32 / wl.n_steps, updates_per_s=Pm * wl.n_steps / (ms32 * 1e-3),
        last_step_all_converged=ok32,
        rel_diff_vs_fp64_last_step=dict(
            sigma_max=float(ds.max()), tangent_median=float(np.median(dc)),
            tangent_p999=float(np.quantile(dc, 0.999)), tangent_max=float(dc.max()),
            points_tangent_above_1e_4=int((dc > 1e-4).sum()),
            note="a point whose leaf at the yield surface takes the other branch in FP32 "
                 "keeps a continuous stress but a tangent of the other branch"))
    del graph32, groups32, E32, ref64
    # one load step (the 11th, after the first ten) called for all groups and
    # for subsets of them, to see what each depth takes of the shared launch
    for gr in groups:
        gr.z_in.zero_()
        gr.a_in.zero_()
    for step in range(10):
        for gr, Em in zip(groups, E_steps):
            gr.E = Em[step]
        dmn_update_gauss_points(groups, S.FIBER, S.MATRIX)
        for gr in groups:
            gr.advance()
    for gr, Em in zip(groups, E_steps):
        gr.E = Em[10]
    depth_of = [n.depth for n in wl.nets]

    def call_ms(sub):
        ws_sub = dmn_update_gauss_points(sub, S.FIBER, S.MATRIX)
        return _event_ms(lambda: dmn_update_gauss_points(sub, S.FIBER, S.MATRIX, ws=ws_sub),
                         5) / 5
    split = dict(load_step=11, all_groups_ms=call_ms(groups),
                 depth9_groups_ms=call_ms([gr for gr, k in zip(groups, depth_of) if k == 9]),
                 depths_5_to_8_groups_ms=call_ms([gr for gr, k in zip(groups, depth_of)
                                                  if k != 9]))
    for K in sorted(set(depth_of) - {9}):
        split[f"depth{K}_groups_alone_ms"] = call_ms(
            [gr for gr, k in zip(groups, depth_of) if k == K])
    out["mixed_batch_graph"] = dict(
        points=Pm, dmns=len(wl.nets), depths=sorted({n.depth for n in wl.nets}),
        load_steps_per_replay=wl.n_steps, ms_per_load_step=ms / wl.n_steps,
        updates_per_s=Pm * wl.n_steps / (ms * 1e-3), last_step_all_converged=ok,
        tuning={int(k): [v["lanes_per_point"], v["waves_per_cu"]]
                for k, v in mixed_tuned.items()},
        one_call_by_depth=split, fp32_state=fp32_state)
    del graph, groups, E_steps

    # what the two roofs give on this device, for context beside the published
    # peaks: an FP64 matrix product through the vendor BLAS (matrix cores) and
    # a device-to-device copy
    n = 8192
    a = torch.randn(n, n, dtype=torch.float64, device=dev)
    b = torch.randn(n, n, dtype=torch.float64, device=dev)
    c = torch.empty_like(a)
    torch.matmul(a, b, out=c)
    torch.cuda.synchronize()
    ms_mm = _event_ms(lambda: torch.matmul(a, b, out=c), 5) / 5
    del a, b, c
    nbytes = 1 << 30
    x = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    ms_cp = _event_ms(lambda: y.copy_(x), 10) / 10
    del x, y
    out["measured_peaks"] = dict(
        fp64_dgemm_n8192_tflops=2.0 * n ** 3 / (ms_mm * 1e-3) / 1e12,
        hbm_copy_1GiB_GBps=2.0 * nbytes / (ms_cp * 1e-3) / 1e9,
        published=dict(fp64_tflops=78.6, hbm_GBps=8000.0))
    return out


if __name__ == "__main__":
    main()
