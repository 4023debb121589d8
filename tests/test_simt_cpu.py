"""The Gauss-point update of the library's own HIP sources, built for the CPU
(tests/simt: lanes as host threads, cross-lane operations and barriers
emulated) under AddressSanitizer and UndefinedBehaviorSanitizer, against the
FP64 oracle.

Every global, LDS and array index the kernels take is checked on the host
here: an out-of-bounds access, a shift or overflow with undefined behaviour,
or a collective that not every lane reaches stops the child process with a
report.  The cases cover every compiled lane split of depths 1-8, including
the (8, 3) split that the device build leaves out, orientation-interpolated
normals, one call over groups of depths 1-9 (the mixed-depth launch, with
depth-9 points split over two waves), FP32 state, the entry point without a
workspace, the failure statuses, and the FP32-storage kernel instantiation
that the device build also leaves out (tests/simt/fp32_kernel.cpp); then the
linear map and its backward, the path adjoint, the training kernels
(objective, stiffness sampler, optimiser step) and a training step over a
batch grouped by orientation.  Results must match the
oracle to the GPU parity bar (FP64 relative 1e-10, equal iterations and
status; FP32 as its GPU test states)."""
import os
import shutil
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "simt"))

import synthetic as S  # noqa: E402
from oracle.gp import DmnModel, NewtonOptions, run_path  # noqa: E402
from oracle.orientation import interpolated_normals  # noqa: E402

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")

RTOL = 1e-10
MARGIN = 1e-9


def harness():
    import harness as H
    return H


@pytest.fixture(scope="module", autouse=True)
def sanitised_builds():
    """Build the three sanitised libraries side by side before the first case
    (each build's time is mostly the single compile of the Gauss-point
    source); later calls find them built."""
    import concurrent.futures as cf
    import build as B
    with cf.ThreadPoolExecutor(3) as ex:
        jobs = [ex.submit(B.build, sanitizer="address"), ex.submit(B.build, sanitizer="thread"),
                ex.submit(B.build_f32_kernel)]
        for j in jobs:
            j.result()


def rel(got, ref):
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def check_group(out, model_of, E, points, f32=False):
    """Compare the CPU-build outputs of one group with the oracle's path."""
    worst, checked = 0.0, 0
    for p in points:
        ref = run_path(model_of(p), E[:, p, :], NewtonOptions())
        if min(r["margin"] for r in ref) < MARGIN:
            continue
        checked += 1
        for s, r in enumerate(ref):
            g = out[s]
            if f32:
                worst = max(worst, rel(g["sigma"][p].astype(np.float64), r["sigma"]))
                continue
            assert g["status"][p] == r["status"] and g["iters"][p] == r["iters"], (p, s)
            es, ec = rel(g["sigma"][p], r["sigma"]), rel(g["C"][p], r["C"])
            ea = rel(g["a"][p].ravel(), r["a"]) if np.abs(r["a"]).max() > 0 else 0.0
            ez = rel(g["z"][p].ravel(), r["z"].ravel()) if np.abs(r["z"]).max() > 0 else 0.0
            worst = max(worst, es, ec, ea, ez)
    assert checked > 0
    return worst


def fixed_group(K, P, T, seed):
    rs = S.streams(seed)
    net = S.random_dmn(rs["dmn"], K, 0.25)
    E = S.ramp_with_noise(rs, P, T, 0.02, 1e-3)
    model = DmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX)
    return dict(depth=K, w=net.w, n=net.normals, E=E), (lambda p: model)


# every lane split compiled into the CPU build: (depth, lanes per point)
VARIANTS = [(1, 1), (2, 2), (2, 1), (3, 4), (3, 2), (4, 8), (4, 4), (5, 16), (5, 8),
            (6, 32), (6, 16), (7, 64), (7, 32), (8, 64), (8, 32)]


@pytest.mark.parametrize("K,lanes", VARIANTS)
def test_simt_gp_every_lane_split(K, lanes):
    ppw = 64 // lanes
    P = min(ppw + 3, 40) if ppw > 1 else 2  # a ragged last batch where a wave holds several
    grp, model = fixed_group(K, P, 2, 500 + K)
    out, _ = harness().run_gp([grp], S.FIBER, S.MATRIX, tuning=[(K, lanes, 1)])
    worst = check_group(out[0], model, grp["E"], range(P))
    assert worst <= RTOL, worst


def test_simt_gp_mixed_depths_one_call():
    """Groups of depths 9, 8, 6, 3, 2 in one call run in the mixed-depth launch
    (depth 9 split over two waves); depth 1 runs in its own launch."""
    depths = [9, 8, 6, 3, 2, 1]
    built = [fixed_group(K, 3, 2, 600 + K) for K in depths]
    out, _ = harness().run_gp([g for g, _ in built], S.FIBER, S.MATRIX)
    for i, (g, model) in enumerate(built):
        worst = check_group(out[i], model, g["E"], range(3))
        assert worst <= RTOL, (depths[i], worst)


@pytest.mark.parametrize("K,kind", [(1, "quadratic"), (3, "trilinear"), (6, "linear")])
def test_simt_gp_orientation(K, kind):
    rs = S.streams(300 + K)
    net = S.interpolated_dmn(rs["dmn"], K, 0.25, kind)
    P = 9
    lam = S.triangle_points(rs["assignment"], P)
    E = S.ramp_with_noise(rs, P, 2, 0.02, 1e-3)
    code = {"linear": 1, "trilinear": 2, "quadratic": 3}[kind]
    out, _ = harness().run_gp([dict(depth=K, w=net.w, ori=code, p=net.p, q=net.q, lam=lam,
                                    E=E)], S.FIBER, S.MATRIX)

    def model(p):
        nrm = interpolated_normals(net.p, net.q, lam[p, 0], lam[p, 1], net.kind)
        return DmnModel(K, net.w, nrm, S.FIBER, S.MATRIX)
    worst = check_group(out[0], model, E, range(P))
    assert worst <= RTOL, worst


def test_simt_gp_fp32_state_and_noalloc():
    """FP32 state (FP64 arithmetic on widened copies) within 1e-4 of the
    oracle; the entry point without a workspace gives the workspace call's
    results bit for bit."""
    H = harness()
    built = [fixed_group(K, P, 2, 700 + K) for K, P in ((6, 5), (3, 7))]
    groups = [g for g, _ in built]
    g32 = [dict(g, E=g["E"].astype(np.float32)) for g in groups]
    out32, _ = H.run_gp(g32, S.FIBER, S.MATRIX, prec=2)
    for i, (g, model) in enumerate(built):
        assert check_group(out32[i], model, g["E"].astype(np.float32).astype(np.float64),
                           range(g["E"].shape[1]), f32=True) <= 1e-4
    ref, _ = H.run_gp(groups, S.FIBER, S.MATRIX)
    na, _ = H.run_gp(groups, S.FIBER, S.MATRIX, noalloc=True)
    for i in range(len(groups)):
        for s in range(2):
            for k in ref[i][s]:
                assert np.array_equal(ref[i][s][k], na[i][s][k]), (i, s, k)


def test_simt_gp_failure_statuses():
    """A non-finite strain fails its point alone (status 2, state passed
    through); invalid DMN parameters (a negative weight) fail every point of
    their group (status 5) in a call shared with a valid group."""
    H = harness()
    g1, _ = fixed_group(4, 6, 1, 801)
    g1["E"] = g1["E"].copy()
    g1["E"][0, 2, 3] = np.nan
    g2, _ = fixed_group(9, 2, 1, 802)
    g2["w"] = g2["w"].copy()
    g2["w"][5] = -1.0
    out, _ = H.run_gp([g1, g2], S.FIBER, S.MATRIX)
    st1, st2 = out[0][0]["status"], out[1][0]["status"]
    assert st1[2] == 2 and all(st1[p] == 0 for p in range(6) if p != 2)
    assert np.all(out[0][0]["z"][2] == 0) and np.all(out[0][0]["a"][2] == 0)
    assert np.all(st2 == 5)


@pytest.mark.parametrize("K,lanes", [(1, 1), (3, 2), (5, 16), (8, 64)])
def test_simt_fp32_storage_kernel(K, lanes):
    """The FP32-storage instantiation gp_update_kernel<K, D, float>, which the
    device build leaves out after a device fault: bounds-checked on the CPU and
    within 1e-4 of the oracle on the FP32-rounded strains, with the oracle's
    iteration counts."""
    rs = S.streams(900 + K)
    net = S.random_dmn(rs["dmn"], K, 0.25)
    P = min(64 // lanes + 3, 40) if lanes < 64 else 2
    E = S.ramp_with_noise(rs, P, 3, 0.02, 1e-3).astype(np.float32)
    out = harness().run_f32_kernel(K, lanes, net.w, net.normals, E, S.FIBER, S.MATRIX)
    model = DmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX)
    for p in range(P):
        ref = run_path(model, E[:, p, :].astype(np.float64), NewtonOptions())
        for s, r in enumerate(ref):
            assert out[s]["status"][p] == r["status"] == 0
            assert out[s]["iters"][p] == r["iters"], (p, s)
            assert rel(out[s]["sigma"][p].astype(np.float64), r["sigma"]) <= 1e-4
            assert rel(out[s]["C"][p].astype(np.float64), r["C"]) <= 1e-4


def test_simt_gp_no_race_between_lanes():
    """The same sources under ThreadSanitizer: LDS and global data that one
    GPU thread writes and another reads are ordered by a wave or workgroup
    barrier in the one-wave kernel (depth 8) and in the mixed-depth launch
    (depth-9 points split over two waves, depths 6 and 3 by batches), so the
    run reports no data race; results as in the sanitised build."""
    built = [fixed_group(K, 2, 2, 1000 + K) for K in (9, 6, 3)]
    out, _ = harness().run_gp([g for g, _ in built], S.FIBER, S.MATRIX, sanitizer="thread")
    for i, (g, model) in enumerate(built):
        assert check_group(out[i], model, g["E"], range(2)) <= RTOL
    single, model8 = fixed_group(8, 2, 2, 1008)
    out8, _ = harness().run_gp([single], S.FIBER, S.MATRIX, sanitizer="thread")
    assert check_group(out8[0], model8, single["E"], range(2)) <= RTOL


def linear_case(K, B, seed):
    tw = S.config3(batch=B, depth=K)
    G = S.streams(seed)["cotangent"].standard_normal((B, 6, 6))
    return tw, G


def check_linear(K, tw, G, out, tol):
    from oracle.grad import linear_gradients
    from oracle.linear import dmn_linear
    net = tw.truth
    B = tw.C1.shape[0]
    assert list(out["err"]) == [0, 0]
    ref = dmn_linear(K, net.w, net.normals, tw.C1, tw.C2)
    assert max(rel(out["Cbar"][b].astype(np.float64), ref[b]) for b in range(B)) <= tol
    alpha, beta = S.normals_to_angles(net.normals)
    gn = out["gn"].astype(np.float64)
    da = np.stack([np.cos(alpha) * np.cos(beta), np.cos(alpha) * np.sin(beta), -np.sin(alpha)], -1)
    db = np.stack([-np.sin(alpha) * np.sin(beta), np.sin(alpha) * np.cos(beta),
                   np.zeros_like(alpha)], -1)
    ga, gb = (gn * da).sum(-1), (gn * db).sum(-1)
    w_idx = np.arange(0, 2 ** K, max(1, 2 ** K // 8))
    a_idx = np.arange(0, 2 ** K - 1, max(1, (2 ** K - 1) // 6))
    r = linear_gradients(K, net.w, alpha, beta, tw.C1, tw.C2, G, w_idx, a_idx)
    assert rel(out["gw"][w_idx].astype(np.float64), r["gw"][w_idx]) <= tol
    ref_a = np.concatenate([r["galpha"][a_idx], r["gbeta"][a_idx]])
    assert rel(np.concatenate([ga[a_idx], gb[a_idx]]), ref_a) <= tol


@pytest.mark.parametrize("K,B,dtype", [(3, 37, np.float64), (5, 70, np.float64),
                                       (8, 4, np.float64), (8, 19, np.float64),
                                       (7, 17, np.float64), (3, 37, np.float32),
                                       (8, 17, np.float32)])
def test_simt_linear_map_and_backward(K, B, dtype):
    """The linear map and its backward (dmn_homogenize_linear / _backward) in
    the sanitised build against the oracle's map and complex-step gradients:
    ragged batches, depths 7 and 8 with two samples sharing a wave's upper
    levels in the forward once a batch has more than 8 samples per CU (two
    emulated CUs here; odd batches leave the last wave one sample) and in the
    backward at depths 7 and 8, and
    at depth 5 with 70 samples 72 partial-sum slots, so the batch sum runs
    through the workgroup tree reduction; FP32 storage and arithmetic within
    1e-4."""
    tw, G = linear_case(K, B, 3)
    f = (lambda x: np.asarray(x, dtype))
    out = harness().run_linear(K, f(tw.truth.w), f(tw.truth.normals), f(tw.C1), f(tw.C2), f(G),
                               input_grads=(K == 3))
    check_linear(K, tw, G, out, 1e-10 if dtype == np.float64 else 1e-4)


def test_simt_linear_fp64_depth8_pair_backward(monkeypatch):
    """The FP64 depth-8 backward with two samples per wave over many pair
    steps per wave: 71 samples on one emulated CU, against the oracle's map
    and complex-step gradients."""
    monkeypatch.setenv("SIMT_CUS", "1")
    tw, G = linear_case(8, 71, 3)
    out = harness().run_linear(8, tw.truth.w, tw.truth.normals, tw.C1, tw.C2, G)
    check_linear(8, tw, G, out, 1e-10)


@pytest.mark.parametrize("K,B", [(8, 19), (7, 37)])
def test_simt_linear_backward_more_samples_than_waves(monkeypatch, K, B):
    """The backward's persistent waves are capped at what the device holds at
    once; with one emulated CU holding 4 waves, each wave accumulates several
    samples (depth 8: one per wave-step; depth 7: two per wave-step, an odd
    batch leaving a last half pair), against the oracle's map and
    complex-step gradients."""
    monkeypatch.setenv("SIMT_CUS", "1")
    monkeypatch.setenv("SIMT_BLOCKS_PER_CU", "4")
    tw, G = linear_case(K, B, 6)
    out = harness().run_linear(K, tw.truth.w, tw.truth.normals, tw.C1, tw.C2, G)
    check_linear(K, tw, G, out, 1e-10)


def test_simt_linear_no_race_between_lanes():
    """The linear map, its backward and the reductions of the batch sum (the
    workgroup tree at depth 5 with 72 slots), the depth-8 forward with two
    samples per wave (an odd batch) and the depth-7 backward with two samples
    per wave, under ThreadSanitizer."""
    for K, B in ((5, 70), (8, 17), (7, 17)):
        tw, G = linear_case(K, B, 4)
        out = harness().run_linear(K, tw.truth.w, tw.truth.normals, tw.C1, tw.C2, G,
                                   sanitizer="thread")
        check_linear(K, tw, G, out, 1e-10)


@pytest.mark.parametrize("K,P,T,every,sanitizer,blocks", [(3, 3, 4, True, "address", None),
                                                          (5, 4, 3, False, "address", None),
                                                          (5, 9, 3, False, "address", "1"),
                                                          (3, 2, 3, False, "thread", None)])
def test_simt_path_adjoint(monkeypatch, K, P, T, every, sanitizer, blocks):
    """The path gradient of J = sum_p g_p . sigma_p(final): forward path with
    the tight tolerance and one polishing step, then dmn_update_adjoint swept
    backwards over the steps, in the sanitised build, against the oracle's
    complex-step path derivative along unit directions (every parameter at
    depth 3; weights and both angles of a few laminates at depth 5); under
    ThreadSanitizer too (the per-wave partial sums and their reduction).  With
    one emulated CU holding one wave, the adjoint's single persistent wave
    takes the 9 points of depth 5 in three turns of 4."""
    if blocks:
        monkeypatch.setenv("SIMT_CUS", "1")
        monkeypatch.setenv("SIMT_BLOCKS_PER_CU", blocks)
    from oracle.adjoint import path_directional_derivative
    rs = S.streams(400 + K)
    net = S.random_dmn(rs["dmn"], K, 0.25)
    E = S.ramp_with_noise(rs, P, T, 0.02, 1e-3)
    g = S.unit_directions(rs["cotangent"], P)
    out = harness().run_adjoint(K, net.w, net.normals, E, g, S.FIBER, S.MATRIX,
                                sanitizer=sanitizer)
    assert not np.any(out["err"])
    alpha, beta = S.normals_to_angles(net.normals)
    gn = out["gn"]
    da = np.stack([np.cos(alpha) * np.cos(beta), np.cos(alpha) * np.sin(beta), -np.sin(alpha)], -1)
    db = np.stack([-np.sin(alpha) * np.sin(beta), np.sin(alpha) * np.cos(beta),
                   np.zeros_like(alpha)], -1)
    ga, gb = (gn * da).sum(-1), (gn * db).sum(-1)
    nl, L = 2 ** K, 2 ** K - 1
    picks = range(nl + 2 * L) if every else [0, 5, nl - 1, nl, nl + L // 2, nl + L, nl + 2 * L - 1]
    scale = max(np.abs(out["gw"]).max(), np.abs(ga).max(), np.abs(gb).max())
    for k in picks:
        vw, va, vb = np.zeros(nl), np.zeros(L), np.zeros(L)
        if k < nl:
            vw[k], got = 1.0, out["gw"][k]
        elif k < nl + L:
            va[k - nl], got = 1.0, ga[k - nl]
        else:
            vb[k - nl - L], got = 1.0, gb[k - nl - L]
        ref = path_directional_derivative(K, net.w, alpha, beta, S.FIBER, S.MATRIX, E, g,
                                          vw, va, vb)
        assert abs(got - ref) <= RTOL * scale, (k, got, ref)


@pytest.mark.parametrize("K,B,kind,dtype,tol", [(3, 37, "trilinear", np.float64, 1e-10),
                                                (6, 6, "quadratic", np.float64, 1e-10),
                                                (5, 17, "linear", np.float32, 2e-3)])
def test_simt_oriented_linear_map_and_backward(K, B, kind, dtype, tol):
    """Per-sample orientation in the linear map and its backward (each
    sample's normals from its own (l1, l2)) in the sanitised build: the map
    against the oracle, the cotangents of (w, p, q) along random directions
    against the oracle's complex-step derivative."""
    from oracle.orientation import oriented_directional_derivative, oriented_linear
    rs = S.streams(700 + K)
    net = S.interpolated_dmn(rs["dmn"], K, 0.3, kind)
    lam = S.triangle_points(rs["assignment"], B)
    C1, C2 = S.random_spd(rs["stiffness"], B), S.random_spd(rs["stiffness"], B)
    G = rs["cotangent"].standard_normal((B, 6, 6))
    code = {"linear": 1, "trilinear": 2, "quadratic": 3}[kind]
    f = (lambda x: np.asarray(x, dtype))
    out = harness().run_linear(K, f(net.w), None, f(C1), f(C2), f(G),
                               ori=(code, f(net.p), f(net.q), f(lam)))
    assert list(out["err"]) == [0, 0]
    ref = oriented_linear(K, net.w, net.p, net.q, kind, lam, C1, C2)
    assert rel(out["Cbar"].astype(np.float64), ref) <= (tol if dtype == np.float32 else 1e-10)
    gw, gpq = out["gw"].astype(np.float64), out["gn"].astype(np.float64)
    L, M = net.p.shape
    rng = np.random.default_rng(3)
    for _ in range(2):
        vw, vp, vq = (rng.standard_normal(L + 1), rng.standard_normal((L, M)),
                      rng.standard_normal((L, M)))
        got = gw @ vw + np.sum(gpq[:, 0, :] * vp) + np.sum(gpq[:, 1, :] * vq)
        r = oriented_directional_derivative(K, net.w, net.p, net.q, kind, lam, C1, C2, G,
                                            vw, vp, vq)
        assert abs(got - r) <= tol * abs(r), (got, r)


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-10), (np.float32, 1e-4)])
def test_simt_training_loss(dtype, tol):
    """The objective's data term, per-sample errors and cotangent (the loss's
    three kernels: per-sample norms, the one-workgroup reduction, the
    cotangent) in the sanitised build against the oracle, for B = 37 over two
    64-sample workgroups and p, q pairs away from 1."""
    from oracle import training as T
    from training_cases import loss_case
    Cb, Tt = loss_case(37, 41)
    Cb, Tt = Cb.astype(dtype), Tt.astype(dtype)
    C64, T64 = Cb.astype(np.float64), Tt.astype(np.float64)
    for p, q in [(1.0, 10.0), (1.5, 1.0)]:
        out = harness().run_train(dict(Cbar=Cb, target=Tt, p=p, q=q))
        e_ref = T.sample_errors(C64, T64, p)
        assert rel(out["e"].astype(np.float64), e_ref) < tol
        st = out["loss_stats"]
        assert abs(st[0] - T.data_term(e_ref, q)) <= tol * T.data_term(e_ref, q)
        assert abs(st[1] - e_ref.max()) <= tol * e_ref.max()
        assert rel(out["gCbar"].astype(np.float64), T.data_cotangent(C64, T64, p, q)) < tol
        assert np.all(out["gCbar"][0] == 0.0)


def test_simt_sample_stiffness():
    """The stiffness sampler in the sanitised build, both output precisions,
    against the oracle at scrambled Sobol points and the corner cases."""
    from oracle import training as T
    from training_cases import special_points
    u = special_points(64, 13)
    for sprec, tol in [(0, 1e-12), (1, 1e-5)]:
        out = harness().run_train(dict(u=u, sprec=sprec))
        for b, x in enumerate(u):
            r1, r2 = T.sample_stiffness(x)
            assert rel(out["C1"][b].astype(np.float64), r1) < tol, b
            assert rel(out["C2"][b].astype(np.float64), r2) < tol, b


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
def test_simt_training_update(dtype, tol):
    """One optimiser step (gradient chain through the Macaulay weights, the
    normal angles and the mixing penalty; AMSGrad; the learning-rate
    schedule; refreshed weights and normals) in the sanitised build against
    the oracle."""
    from oracle import training as T
    from oracle.grad import normals_from_angles
    from training_cases import update_case, update_reference
    K = 4
    NL, L = 2 ** K, 2 ** K - 1
    c = update_case(17, K)
    for k in ("v", "alpha", "beta", "gw", "gn", "m1", "m2", "mx"):
        c[k] = np.asarray(c[k], dtype).astype(np.float64)
    o = c["opts"]
    f = (lambda x: np.ascontiguousarray(x, dtype))
    case = dict(v=f(c["v"]), alpha=f(c["alpha"]), beta=f(c["beta"]), gw=f(c["gw"]),
                gn=f(c["gn"]), state=f(np.stack([c["m1"], c["m2"], c["mx"]])), step=c["t0"],
                stats0=c["data"],
                amsgrad=np.array([o["lr_min"], o["lr_max"], o["lr_decay"], o["half_period"],
                                  o["steps_per_epoch"], o["beta1"], o["beta2"], o["eps"],
                                  o["penalty"]]))
    out = harness().run_train(case)
    ref = update_reference(c)
    th = ref["theta"]
    got = np.concatenate([out[k].astype(np.float64) for k in ("v", "alpha", "beta")])
    assert rel(got, th) < tol
    assert rel(out["state"].astype(np.float64), ref["state"]) < tol
    assert int(out["step"][0]) == c["t0"] + 1
    assert rel(out["w"].astype(np.float64), T.macaulay(th[:NL])) < tol
    assert rel(out["n"].astype(np.float64),
               normals_from_angles(th[NL:NL + L], th[NL + L:])) < tol
    st = out["update_stats"]
    assert abs(st[4] - ref["penalty"]) <= 1e-12 * max(ref["penalty"], 1.0)
    assert abs(st[3] - (c["data"] + ref["penalty"])) <= 1e-12 * (c["data"] + ref["penalty"])
    assert abs(st[5] - ref["lr"]) <= 1e-14 * ref["lr"]


def test_simt_training_no_race_between_lanes():
    """The objective (per-sample norms, the one-workgroup reduction, the
    cotangent), the stiffness sampler and the optimiser step (its workgroup
    reductions of the penalty and the weight sum) in one run under
    ThreadSanitizer; results as in the sanitised build."""
    from oracle import training as T
    from training_cases import loss_case, special_points, update_case, update_reference
    Cb, Tt = loss_case(37, 41)
    u = special_points(16, 13)
    c = update_case(17, 4)
    o = c["opts"]
    case = dict(Cbar=Cb, target=Tt, p=1.5, q=3.0, u=u, sprec=0, v=c["v"], alpha=c["alpha"],
                beta=c["beta"], gw=c["gw"], gn=c["gn"],
                state=np.stack([c["m1"], c["m2"], c["mx"]]), step=c["t0"], stats0=c["data"],
                amsgrad=np.array([o["lr_min"], o["lr_max"], o["lr_decay"], o["half_period"],
                                  o["steps_per_epoch"], o["beta1"], o["beta2"], o["eps"],
                                  o["penalty"]]))
    out = harness().run_train(case, sanitizer="thread")
    assert rel(out["gCbar"], T.data_cotangent(Cb, Tt, 1.5, 3.0)) < 1e-10
    assert abs(out["loss_stats"][0] - T.data_term(T.sample_errors(Cb, Tt, 1.5), 3.0)) <= \
        1e-10 * out["loss_stats"][0]
    for b, x in enumerate(u):
        r1, r2 = T.sample_stiffness(x)
        assert rel(out["C1"][b], r1) < 1e-12 and rel(out["C2"][b], r2) < 1e-12, b
    ref = update_reference(c)
    got = np.concatenate([out[k] for k in ("v", "alpha", "beta")])
    assert rel(got, ref["theta"]) < 1e-12
    assert rel(out["state"], ref["state"]) < 1e-12


@pytest.mark.parametrize("kind,dead,dtype", [("trilinear", False, np.float64),
                                             ("quadratic", True, np.float64),
                                             ("linear", False, np.float32)])
def test_simt_oriented_training_step(kind, dead, dtype):
    """One training step of an orientation-interpolated DMN over a batch
    grouped by orientation (the groups' normals, the grouped linear map and
    VJP, the chain to the angle coefficients, the optimiser step) in the
    sanitised build: the batch gradient, chained through the oracle's Macaulay
    bracket and penalty, against the oracle's complex-step objective gradient,
    and the objective; FP32 at its bar."""
    from oracle import training as T
    from training_cases import oriented_case, weight_chain
    K, B, lam_pen = 3, 16, 10.0
    C1, C2, Tt, lam_g, lam_s, offsets, v, p, q = oriented_case(K, B, kind, 92)
    if dead:
        v[2], v[3] = -0.01, -0.02
    f = (lambda x: np.ascontiguousarray(x, dtype))
    r = (lambda x: np.asarray(x, dtype).astype(np.float64))
    v, p, q, C1, C2, Tt, lam_g = map(r, (v, p, q, C1, C2, Tt, lam_g))
    lam_s = lam_g[np.repeat(np.arange(len(lam_g)), np.diff(offsets))]
    code = {"linear": 1, "trilinear": 2, "quadratic": 3}[kind]
    case = dict(ori=code, v=f(v), p=f(p), q=f(q), lam=f(lam_g), offsets=offsets, C1=f(C1),
                C2=f(C2), target=f(Tt), p_norm=1.0, q_norm=10.0,
                amsgrad=np.array([1e-3, 1e-2, 0.999, 50, 1, 0.9, 0.999, 1e-8, lam_pen]))
    out = harness().run_oriented_train(case)
    assert list(out["err"]) == [0, 0]
    ref = T.objective_oriented_gradient(K, v, p, q, kind, lam_s, C1, C2, Tt, 1.0, 10.0, lam_pen)
    g_ref = np.concatenate([ref["gv"], ref["gP"].ravel(), ref["gQ"].ravel()])
    gpq = out["gpq"].astype(np.float64)
    g = np.concatenate([weight_chain(v, out["gw"].astype(np.float64), lam_pen),
                        gpq[:, 0, :].ravel(), gpq[:, 1, :].ravel()])
    tol = 1e-10 if dtype == np.float64 else 1e-4
    assert rel(g, g_ref) < tol
    J = T.objective_oriented(K, v, p, q, kind, lam_s, C1, C2, Tt, 1.0, 10.0, lam_pen)
    assert abs(out["stats"][3] - J) <= tol * J
    assert int(out["step"][0]) == 1
    # the update: the oracle's AMSGrad step (first step, zero state) on its gradient
    lr = T.learning_rate(0, 1e-3, 1e-2, 50, 0.999)
    th, *_ = T.amsgrad(np.concatenate([v, p.ravel(), q.ravel()]), g_ref, *([np.zeros(len(g_ref))]
                                                                           * 3), 1, lr)
    got = np.concatenate([out[k].astype(np.float64).ravel() for k in ("v", "p", "q")])
    assert rel(got, th) < tol


def test_simt_linear_pair_forward_is_bit_identical(monkeypatch):
    """In the CPU build the forward with two samples per wave (used once a
    launch has more than 8 samples per CU) gives every sample the same bits as
    one sample per wave (the gfx950 build contracts some operations
    differently, within rounding):
    17 depth-8 samples with two emulated CUs take the pair kernel, with three
    the one-sample kernel."""
    tw, G = linear_case(8, 17, 5)
    outs = []
    for cus in ("2", "3"):
        monkeypatch.setenv("SIMT_CUS", cus)
        outs.append(harness().run_linear(8, tw.truth.w, tw.truth.normals, tw.C1, tw.C2, G))
    assert np.array_equal(outs[0]["Cbar"].view(np.int64), outs[1]["Cbar"].view(np.int64))
    assert list(outs[0]["err"]) == [0, 0] and list(outs[1]["err"]) == [0, 0]
