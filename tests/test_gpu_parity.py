"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars: FP64 results within a relative 1e-10 (max-norm, relative to the
largest entry of the reference), iteration counts and status codes equal,
FP32 linear map within 1e-4.  Points whose oracle history contains a leaf
trial state within 1e-9 (relative) of the yield surface are reported and
excluded, because there the elastic/plastic decision flips with roundoff.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthetic as S
from oracle.gp import DmnModel, NewtonOptions, gp_update, run_path
from oracle.grad import linear_gradients
from oracle.linear import dmn_linear

pytestmark = pytest.mark.gpu

RTOL = 1e-10
MARGIN = 1e-9


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(got, ref):
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def close_state(got, ref, rtol=RTOL):
    scale = max(np.abs(ref).max(), 1e-300)
    return np.abs(got - ref).max() <= rtol * scale + 1e-18


def gpu_path(net, E_path, opts=None):
    """Run a load path through dmn_update_gauss_points; returns per-step host copies."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    d = dev()
    w = torch.tensor(net.w, device=d)
    n = torch.tensor(net.normals, device=d)
    T, P = E_path.shape[:2]
    g = PointGroup.allocate(w, n, torch.tensor(E_path[0], device=d))
    out = []
    ws = None
    for step in range(T):
        g.E.copy_(torch.tensor(E_path[step], device=d))
        ws = dmn_update_gauss_points([g], S.FIBER, S.MATRIX, ws=ws, **(opts or {}))
        torch.cuda.synchronize()
        out.append(dict(sigma=g.sigma.cpu().numpy(), C=g.tangent.cpu().numpy(),
                        z=g.z_out.cpu().numpy(), a=g.a_out.cpu().numpy(),
                        iters=g.iters.cpu().numpy(), status=g.status.cpu().numpy()))
        g.advance()
    return out


def compare_paths(net, E_path, points, gpu, opts=NewtonOptions()):
    model = DmnModel(net.depth, net.w, net.normals, S.FIBER, S.MATRIX)
    worst = dict(sigma=0.0, C=0.0)
    skipped = []
    for p in points:
        ref = run_path(model, E_path[:, p, :], opts)
        if min(r["margin"] for r in ref) < MARGIN:
            skipped.append(p)
            continue
        for step, r in enumerate(ref):
            g = gpu[step]
            assert g["status"][p] == r["status"], (p, step, g["status"][p], r["status"])
            assert g["iters"][p] == r["iters"], (p, step, g["iters"][p], r["iters"])
            es = rel(g["sigma"][p], r["sigma"])
            ec = rel(g["C"][p], r["C"])
            worst["sigma"] = max(worst["sigma"], es)
            worst["C"] = max(worst["C"], ec)
            assert es <= RTOL, (p, step, es)
            assert ec <= RTOL, (p, step, ec)
            assert close_state(g["z"][p], r["z"]), (p, step)
            assert close_state(g["a"][p].ravel(), r["a"]), (p, step)
    say(f"  depth {net.depth}: checked {len(points) - len(skipped)} points, "
        f"near-yield skipped {skipped}, worst rel sigma {worst['sigma']:.2e} C {worst['C']:.2e}")
    return worst


def test_gp_depth2_full_path_all_points():
    """Depth-2 DMN, 64 points, 10-step ramp to 2 %: every point, every step."""
    say("case: gp depth 2, 64 points x 10 steps")
    wl = S.config0()
    gpu = gpu_path(wl.nets[0], wl.E)
    compare_paths(wl.nets[0], wl.E, range(wl.n_points), gpu)


@pytest.mark.parametrize("K", [1, 3, 4, 5, 6, 7])
def test_gp_small_depths_ragged(K):
    """Depths 1..7 (several points per wave), a ragged point count, 6 steps."""
    say(f"case: gp depth {K}, 37 points x 6 steps")
    rs = S.streams(100 + K)
    net = S.random_dmn(rs["dmn"], K, 0.25)
    E = S.ramp_with_noise(rs, 37, 6, 0.02, 1e-3)
    gpu = gpu_path(net, E)
    compare_paths(net, E, range(37), gpu)


def test_gp_depth8_production_size_sampled():
    """Depth 8 at the full production size (65,536 points, 20 steps); the oracle
    follows 6 sampled points along their whole path."""
    say("case: gp depth 8, 65536 points x 20 steps, 6 sampled")
    wl = S.config1()
    gpu = gpu_path(wl.nets[0], wl.E)
    picks = S.streams(1)["picks"].choice(wl.n_points, 6, replace=False)
    compare_paths(wl.nets[0], wl.E, picks, gpu)
    st = np.stack([g["status"] for g in gpu])
    assert np.all(st == 0), np.unique(st, return_counts=True)
    plastic = np.mean(gpu[-1]["z"][:, :, 6] > 0)
    say(f"  plastic matrix-leaf fraction at the last step: {plastic:.3f}")


def test_gp_depth8_state_offsets_beyond_32_bits():
    """Maximum size: depth 8 with 2,818,048 points (43 copies of the
    production workload's 65,536), so the element offsets of the last
    points' internal variables and jumps pass 2^31 (about 75 GB of state in
    HBM).  A large first increment (the path's tenth strain from the initial
    state), then its eleventh: every copy's outputs equal the first copy's
    bit for bit, and points of the last copy match the oracle."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    d = dev()
    wl = S.config1()
    net = wl.nets[0]
    P0, reps = wl.n_points, 43
    P = P0 * reps
    M, L = 2 ** (net.depth - 1), 2 ** net.depth - 1
    assert (P - 1) * M * 7 >= 2 ** 31 and (P - 1) * L * 3 >= 2 ** 31
    torch.cuda.empty_cache()
    need = P * (2 * M * 7 + 2 * L * 3 + 6 + 6 + 36) * 8
    if torch.cuda.mem_get_info()[0] < need + (4 << 30):
        pytest.skip(f"needs {need / 2 ** 30:.0f} GiB of free device memory")
    say(f"case: gp depth 8, {P} points ({reps} copies of {P0}) x 2 steps, "
        f"{need / 2 ** 30:.0f} GiB")
    E2 = wl.E[[9, 10]]
    picks = S.streams(1)["picks"].choice(P0, 3, replace=False)
    last = (reps - 1) * P0 + picks
    g = PointGroup.allocate(torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d),
                            torch.tensor(E2[0], device=d).repeat(reps, 1))
    gpu, ws = [], None
    for step in range(2):
        g.E.copy_(torch.tensor(E2[step], device=d).repeat(reps, 1))
        ws = dmn_update_gauss_points([g], S.FIBER, S.MATRIX, ws=ws)
        torch.cuda.synchronize()
        for name in ("sigma", "tangent", "z_out", "a_out", "iters", "status"):
            t = getattr(g, name)
            if t.dtype == torch.float64:
                t = t.view(torch.int64)  # bit patterns: a failed point's NaN tangent too
            t = t.view(reps, P0, -1)
            assert torch.equal(t, t[:1].expand_as(t)), (step, name)
        st = g.status.cpu().numpy()
        say(f"  step {step}: copies equal; status counts {np.unique(st, return_counts=True)}, "
            f"mean iterations {g.iters.double().mean().item():.2f}")
        gpu.append(dict(sigma=g.sigma[last].cpu().numpy(), C=g.tangent[last].cpu().numpy(),
                        z=g.z_out[last].cpu().numpy(), a=g.a_out[last].cpu().numpy(),
                        iters=g.iters[last].cpu().numpy(), status=st[last]))
        g.advance()
    del g, ws
    torch.cuda.empty_cache()
    compare_paths(net, E2[:, picks, :], range(len(picks)), gpu)


def test_gp_mixed_launch_offsets_beyond_32_bits():
    """Maximum size for the mixed-depth launch: a depth-9 group of 1,441,792
    points (44 copies of 32,768; each point split over the two waves of a
    workgroup) with a depth-5 group in the same call, so the element offsets
    of the last depth-9 points' internal variables and jumps pass 2^31
    (about 77 GB).  Two steps; every copy's outputs equal those of the same
    call with one copy, bit for bit (that call's points are held to the
    oracle by the mixed-launch parity tests)."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    d = dev()
    P0, reps = 32768, 44
    P = P0 * reps
    M, L = 2 ** 8, 2 ** 9 - 1
    assert (P - 1) * M * 7 >= 2 ** 31 and (P - 1) * L * 3 >= 2 ** 31
    torch.cuda.empty_cache()
    need = P * (2 * M * 7 + 2 * L * 3 + 6 + 6 + 36) * 8
    if torch.cuda.mem_get_info()[0] < need + (4 << 30):
        pytest.skip(f"needs {need / 2 ** 30:.0f} GiB of free device memory")
    say(f"case: mixed launch, depth 9 with {P} points ({reps} copies of {P0}) + depth 5, "
        f"x 2 steps, {need / 2 ** 30:.0f} GiB")
    rs = S.streams(63)
    net9, net5 = S.random_dmn(rs["dmn"], 9, 0.25), S.random_dmn(rs["dmn"], 5, 0.3)
    E9 = torch.tensor(S.ramp_with_noise(rs, P0, 11, 0.015, 1e-3)[[9, 10]], device=d)
    E5 = torch.tensor(S.ramp_with_noise(rs, 333, 2, 0.02, 1e-3), device=d)

    def run(copies):
        g9 = PointGroup.allocate(torch.tensor(net9.w, device=d),
                                 torch.tensor(net9.normals, device=d), E9[0].repeat(copies, 1))
        g5 = PointGroup.allocate(torch.tensor(net5.w, device=d),
                                 torch.tensor(net5.normals, device=d), E5[0].clone())
        for step in range(2):
            g9.E.copy_(E9[step].repeat(copies, 1))
            g5.E.copy_(E5[step])
            dmn_update_gauss_points([g9, g5], S.FIBER, S.MATRIX)
            torch.cuda.synchronize()
            yield g9, g5
            g9.advance()
            g5.advance()

    one = []
    for g9, g5 in run(1):
        one.append({k: getattr(g9, k).clone() for k in
                    ("sigma", "tangent", "z_out", "a_out", "iters", "status")})
        one[-1]["g5"] = {k: getattr(g5, k).clone() for k in ("sigma", "tangent", "z_out")}
    for step, (g9, g5) in enumerate(run(reps)):
        for name in ("sigma", "tangent", "z_out", "a_out", "iters", "status"):
            t, r = getattr(g9, name), one[step][name]
            if t.dtype == torch.float64:
                t, r = t.view(torch.int64), r.view(torch.int64)
            t = t.view(reps, P0, -1)
            assert torch.equal(t, r.view(1, P0, -1).expand_as(t)), (step, name)
        for name in ("sigma", "tangent", "z_out"):
            assert torch.equal(getattr(g5, name).view(torch.int64),
                               one[step]["g5"][name].view(torch.int64)), (step, name)
        st = g9.status.cpu().numpy()
        say(f"  step {step}: every copy equals the one-copy call; status counts "
            f"{np.unique(st, return_counts=True)}, mean iterations "
            f"{g9.iters.double().mean().item():.2f}")
    del one
    torch.cuda.empty_cache()


def test_gp_mixed_batch_full_size_sampled(tmp_path):
    """The mixed-depth batch at its full size (131,072 points over 16 DMNs of
    depths 5-9, 20 steps) in the launch configuration the bench times: tuned
    per depth, all 16 groups in one call per step.  The oracle follows two
    sampled points of every DMN along their whole path; every point of the
    batch converges at every step."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    from paper_2103_08253_amd import autotune as A
    say("case: gp mixed batch, 131072 points over 16 DMNs x 20 steps, 2 sampled per DMN")
    d = dev()
    wl = S.config2()
    rs = S.streams(2)["picks"]
    idx = [np.nonzero(wl.dmn_id == m)[0] for m in range(len(wl.nets))]
    picks = [rs.choice(sel, 2, replace=False) for sel in idx]
    groups = [PointGroup.allocate(torch.tensor(net.w, device=d),
                                  torch.tensor(net.normals, device=d),
                                  torch.tensor(wl.E[0, sel], device=d))
              for net, sel in zip(wl.nets, idx)]
    try:
        A.tune_gauss_points(groups, S.FIBER, S.MATRIX, cache_path=str(tmp_path / "tune.json"))
        for g in groups:
            g.z_in.zero_()
            g.a_in.zero_()
        outs = [[] for _ in groups]
        ws = None
        for step in range(wl.n_steps):
            for g, sel in zip(groups, idx):
                g.E.copy_(torch.tensor(wl.E[step, sel], device=d))
            ws = dmn_update_gauss_points(groups, S.FIBER, S.MATRIX, ws=ws)
            torch.cuda.synchronize()
            for m, (g, sel, pk) in enumerate(zip(groups, idx, picks)):
                assert bool((g.status == 0).all().item()), (m, step)
                rows = torch.tensor(np.searchsorted(sel, pk), device=d)
                outs[m].append(dict(sigma=g.sigma[rows].cpu().numpy(),
                                    C=g.tangent[rows].cpu().numpy(),
                                    z=g.z_out[rows].cpu().numpy(), a=g.a_out[rows].cpu().numpy(),
                                    iters=g.iters[rows].cpu().numpy(),
                                    status=g.status[rows].cpu().numpy()))
                g.advance()
    finally:
        A.reset_tuning()
    for m, net in enumerate(wl.nets):
        compare_paths(net, wl.E[:, picks[m], :], range(2), outs[m])


def test_gp_depth9_small():
    say("case: gp depth 9, 5 points x 4 steps")
    rs = S.streams(109)
    net = S.random_dmn(rs["dmn"], 9, 0.2)
    E = S.ramp_with_noise(rs, 5, 4, 0.015, 1e-3)
    gpu = gpu_path(net, E)
    compare_paths(net, E, range(5), gpu)


def test_gp_mixed_depth_groups_one_call():
    """16 DMNs of depths 5..9 in one call, a few points each, 30 % near-elastic."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    say("case: gp 16 mixed-depth groups, 4 steps")
    d = dev()
    wl = S.config2(n_points=64, n_steps=4)
    groups, idx = [], []
    for m, net in enumerate(wl.nets):
        sel = np.nonzero(wl.dmn_id == m)[0]
        idx.append(sel)
        groups.append(PointGroup.allocate(torch.tensor(net.w, device=d),
                                          torch.tensor(net.normals, device=d),
                                          torch.tensor(wl.E[0, sel], device=d)))
    outs = []
    for step in range(wl.n_steps):
        for m, g in enumerate(groups):
            g.E.copy_(torch.tensor(wl.E[step, idx[m]], device=d))
        dmn_update_gauss_points(groups, S.FIBER, S.MATRIX)
        torch.cuda.synchronize()
        outs.append([dict(sigma=g.sigma.cpu().numpy(), C=g.tangent.cpu().numpy(),
                          z=g.z_out.cpu().numpy(), a=g.a_out.cpu().numpy(),
                          iters=g.iters.cpu().numpy(), status=g.status.cpu().numpy())
                     for g in groups])
        for g in groups:
            g.advance()
    for m, net in enumerate(wl.nets):
        sel = idx[m]
        if len(sel) == 0:
            continue
        gpu = [o[m] for o in outs]
        Em = wl.E[:, sel, :]
        compare_paths(net, Em, range(min(len(sel), 2)), gpu)


def test_gp_mixed_launch_all_depths():
    """One call over groups of depths 1-4, 7 and 9 (ragged point counts): depths
    2-9 share one launch (depth 9 split over two waves, the others with the
    depth of each batch at run time), depth 1 runs on its own; every point of
    every group against the oracle along 3 steps."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    say("case: gp mixed launch, depths 1, 2, 3, 4, 7, 9")
    d = dev()
    rs = S.streams(140)
    depths, counts = (9, 1, 2, 3, 4, 7, 9), (3, 70, 129, 37, 21, 11, 2)
    nets = [S.random_dmn(rs["dmn"], K, 0.25) for K in depths]
    paths = [S.ramp_with_noise(rs, P, 3, 0.02, 1e-3) for P in counts]
    groups = [PointGroup.allocate(torch.tensor(n.w, device=d), torch.tensor(n.normals, device=d),
                                  torch.tensor(E[0], device=d)) for n, E in zip(nets, paths)]
    outs = [[] for _ in groups]
    for step in range(3):
        for g, E in zip(groups, paths):
            g.E.copy_(torch.tensor(E[step], device=d))
        dmn_update_gauss_points(groups, S.FIBER, S.MATRIX)
        torch.cuda.synchronize()
        for m, g in enumerate(groups):
            outs[m].append(dict(sigma=g.sigma.cpu().numpy(), C=g.tangent.cpu().numpy(),
                                z=g.z_out.cpu().numpy(), a=g.a_out.cpu().numpy(),
                                iters=g.iters.cpu().numpy(), status=g.status.cpu().numpy()))
            g.advance()
    for m, (net, E) in enumerate(zip(nets, paths)):
        compare_paths(net, E, range(E.shape[1]), outs[m])


F32_STATE_RTOL = 1e-4


def gpu_groups_path(nets, E_path, idx, dtype):
    """Run one call per step over several groups; per-step, per-group host copies."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    d = dev()
    groups = [PointGroup.allocate(torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d),
                                  torch.tensor(E_path[0, sel], device=d, dtype=dtype))
              for net, sel in zip(nets, idx)]
    outs = []
    for step in range(E_path.shape[0]):
        for g, sel in zip(groups, idx):
            g.E.copy_(torch.tensor(E_path[step, sel], device=d, dtype=dtype))
        dmn_update_gauss_points(groups, S.FIBER, S.MATRIX)
        torch.cuda.synchronize()
        outs.append([dict(sigma=g.sigma.double().cpu().numpy(), C=g.tangent.double().cpu().numpy(),
                          z=g.z_out.double().cpu().numpy(), status=g.status.cpu().numpy())
                     for g in groups])
        for g in groups:
            g.advance()
    return outs


def test_gp_f32_state_mixed_groups():
    """FP32-stored state (DMN_F32_STATE) over 16 mixed-depth groups, 6 steps.

    Against the FP64 oracle on the FP32-rounded strains (2 points per group) and
    against the GPU FP64 path on every point: sigma within 1e-4 everywhere, the
    tangent within 1e-4 wherever both paths take the same elastic/plastic
    decision at every matrix leaf (a decision within FP32 rounding of the
    yield surface may flip, and the tangent jumps there)."""
    say("case: gp FP32 state, 16 mixed-depth groups, 256 points x 6 steps")
    wl = S.config2(n_points=256, n_steps=6)
    E32 = wl.E.astype(np.float32).astype(np.float64)
    idx = [np.nonzero(wl.dmn_id == m)[0] for m in range(len(wl.nets))]
    f32 = gpu_groups_path(wl.nets, E32, idx, torch.float32)
    f64 = gpu_groups_path(wl.nets, E32, idx, torch.float64)
    worst_o, worst_s, worst_c, flips = 0.0, 0.0, 0.0, 0
    for m, net in enumerate(wl.nets):
        sel = idx[m]
        if len(sel) == 0:
            continue
        model = DmnModel(net.depth, net.w, net.normals, S.FIBER, S.MATRIX)
        for p in range(min(len(sel), 2)):
            ref = run_path(model, E32[:, sel[p], :], NewtonOptions())
            if min(r["margin"] for r in ref) < 1e-5:
                continue
            for step, r in enumerate(ref):
                g = f32[step][m]
                assert g["status"][p] == 0 and r["status"] == 0
                e = max(rel(g["sigma"][p], r["sigma"]), rel(g["C"][p], r["C"]))
                worst_o = max(worst_o, e)
                assert e <= F32_STATE_RTOL, (m, p, step, e)
        same = np.ones(len(sel), bool)
        for step in range(wl.n_steps):
            a, b = f32[step][m], f64[step][m]
            assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
            zin_a = f32[step - 1][m]["z"][..., 6] if step else 0.0
            zin_b = f64[step - 1][m]["z"][..., 6] if step else 0.0
            same &= np.all((a["z"][..., 6] > zin_a) == (b["z"][..., 6] > zin_b), axis=1)
            for p in range(len(sel)):
                es = rel(a["sigma"][p], b["sigma"][p])
                worst_s = max(worst_s, es)
                assert es <= F32_STATE_RTOL, (m, p, step, es)
                if same[p]:
                    ec = rel(a["C"][p], b["C"][p])
                    worst_c = max(worst_c, ec)
                    assert ec <= F32_STATE_RTOL, (m, p, step, ec)
        flips += int((~same).sum())
    say(f"  worst rel vs oracle {worst_o:.2e}; vs GPU FP64 sigma {worst_s:.2e} C {worst_c:.2e}; "
        f"{flips} points with a flipped leaf decision")
    assert flips <= 8


def test_gp_f32_state_depth8_production_size_sampled():
    """FP32 state at the production size (depth 8, 65,536 points, 20 steps);
    the FP64 oracle follows 4 sampled points on the FP32-rounded strains."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    say("case: gp FP32 state, depth 8, 65536 points x 20 steps, 4 sampled")
    d = dev()
    wl = S.config1()
    net = wl.nets[0]
    E32 = torch.tensor(wl.E, device=d, dtype=torch.float32)
    picks = S.streams(1)["picks"].choice(wl.n_points, 4, replace=False)
    g = PointGroup.allocate(torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d),
                            E32[0].clone())
    sig, tan = [], []
    pk = torch.tensor(picks, device=d)
    ws = None
    for step in range(wl.n_steps):
        g.E.copy_(E32[step])
        ws = dmn_update_gauss_points([g], S.FIBER, S.MATRIX, ws=ws)
        assert bool((g.status == 0).all())
        sig.append(g.sigma[pk].double().cpu().numpy())
        tan.append(g.tangent[pk].double().cpu().numpy())
        g.advance()
    model = DmnModel(net.depth, net.w, net.normals, S.FIBER, S.MATRIX)
    E_ref = E32.double().cpu().numpy()
    worst = 0.0
    for i, p in enumerate(picks):
        ref = run_path(model, E_ref[:, p, :], NewtonOptions())
        if min(r["margin"] for r in ref) < 1e-5:
            continue
        for step, r in enumerate(ref):
            e = max(rel(sig[step][i], r["sigma"]), rel(tan[step][i], r["C"]))
            worst = max(worst, e)
            assert e <= F32_STATE_RTOL, (p, step, e)
    say(f"  worst rel vs oracle {worst:.2e}")


def test_gp_f32_state_offsets_beyond_32_bits():
    """Maximum size with FP32 state: depth 8, 2,818,048 points (43 copies of
    the production points), so the widening and rounding of the per-point
    arrays run over more than 2^31 elements (2.5e9 internal variables) and
    the FP64 working copies sit past 2^31-element offsets (about 110 GB with
    the workspace).  Two steps; every copy's outputs equal the first copy's
    bit for bit, and points of the last copy match the FP64 oracle on the
    FP32-rounded strains."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    d = dev()
    wl = S.config1()
    net = wl.nets[0]
    P0, reps = wl.n_points, 43
    P = P0 * reps
    M, L = 2 ** (net.depth - 1), 2 ** net.depth - 1
    assert P * M * 7 >= 2 ** 31 and (P - 1) * L * 3 >= 2 ** 31
    torch.cuda.empty_cache()
    per_point = 2 * M * 7 + 2 * L * 3 + 6 + 6 + 36
    need = P * per_point * (4 + 8)   # FP32 arrays and their FP64 working copies
    if torch.cuda.mem_get_info()[0] < need + (8 << 30):
        pytest.skip(f"needs {need / 2 ** 30:.0f} GiB of free device memory")
    say(f"case: gp FP32 state, depth 8, {P} points ({reps} copies of {P0}) x 2 steps, "
        f"{need / 2 ** 30:.0f} GiB")
    E2 = torch.tensor(wl.E[[9, 10]], device=d, dtype=torch.float32)
    picks = S.streams(1)["picks"].choice(P0, 3, replace=False)
    last = (reps - 1) * P0 + picks
    g = PointGroup.allocate(torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d),
                            E2[0].repeat(reps, 1))
    sig, tan, ws = [], [], None
    for step in range(2):
        g.E.copy_(E2[step].repeat(reps, 1))
        ws = dmn_update_gauss_points([g], S.FIBER, S.MATRIX, ws=ws)
        torch.cuda.synchronize()
        for name in ("sigma", "tangent", "z_out", "a_out", "iters", "status"):
            t = getattr(g, name)
            t = t.view(torch.int32).view(reps, P0, -1)   # float32 bit patterns too
            assert torch.equal(t, t[:1].expand_as(t)), (step, name)
        assert bool((g.status == 0).all())
        sig.append(g.sigma[last].double().cpu().numpy())
        tan.append(g.tangent[last].double().cpu().numpy())
        g.advance()
    del g, ws
    torch.cuda.empty_cache()
    model = DmnModel(net.depth, net.w, net.normals, S.FIBER, S.MATRIX)
    E_ref = E2.double().cpu().numpy()
    worst = 0.0
    for i, p in enumerate(picks):
        ref = run_path(model, E_ref[:, p, :], NewtonOptions())
        if min(r["margin"] for r in ref) < 1e-5:
            continue
        for step, r in enumerate(ref):
            e = max(rel(sig[step][i], r["sigma"]), rel(tan[step][i], r["C"]))
            worst = max(worst, e)
            assert e <= F32_STATE_RTOL, (p, step, e)
    say(f"  every copy equal; worst rel vs oracle {worst:.2e}")


def test_gp_status_codes_and_failure_state():
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    say("case: gp status codes")
    d = dev()
    rs = S.streams(200)
    net = S.random_dmn(rs["dmn"], 3, 0.25)
    w = torch.tensor(net.w, device=d)
    n = torch.tensor(net.normals, device=d)
    E_host = 0.03 * S.unit_directions(rs["direction"], 6)
    E_host[1, 2] = np.nan
    E = torch.tensor(E_host, device=d)
    z0 = 1e-3 * rs["noise"].standard_normal((6, 4, 7))
    z0[:, :, 6] = np.abs(z0[:, :, 6])
    g = PointGroup.allocate(w, n, E, z_in=torch.tensor(z0, device=d))
    dmn_update_gauss_points([g], S.FIBER, S.MATRIX, max_iter=1)
    torch.cuda.synchronize()
    st = g.status.cpu().numpy()
    assert st[1] == 2
    assert torch.equal(g.z_out[1], g.z_in[1]) and torch.equal(g.a_out[1], g.a_in[1])
    model = DmnModel(3, net.w, net.normals, S.FIBER, S.MATRIX)
    for p in (0, 2, 3, 4, 5):
        ref = gp_update(model, E_host[p], z0[p], np.zeros(21), NewtonOptions(max_iter=1))
        assert st[p] == ref["status"], (p, st[p], ref["status"])
        if st[p] != 0:
            assert torch.equal(g.z_out[p], g.z_in[p])
            assert torch.isnan(g.tangent[p]).all()
    # invalid weights: every point reports a bad parameter, state passes through
    wb = w.clone()
    wb[0] = -0.1
    gb = PointGroup.allocate(wb, n, E)
    dmn_update_gauss_points([gb], S.FIBER, S.MATRIX)
    torch.cuda.synchronize()
    assert (gb.status == 5).all()
    assert torch.equal(gb.a_out, gb.a_in)
    # an empty group next to a populated one
    ge = PointGroup.allocate(w, n, E[:0])
    g2 = PointGroup.allocate(w, n, E[:1])
    dmn_update_gauss_points([ge, g2], S.FIBER, S.MATRIX)
    torch.cuda.synchronize()
    assert int(g2.status[0]) == 0


def test_empty_inputs_every_call():
    """No points or samples: the linear map (FP64 and FP32) returns with its
    error word clear; its backward overwrites gw, gn with zeros; the adjoint
    of an empty group leaves the accumulated gradients as they were; the
    Gauss-point update and its no-workspace form with only an empty group,
    and the stiffness sampler, launch nothing and report success."""
    from paper_2103_08253_amd import (AdjointGroup, PointGroup, dmn_homogenize_backward,
                                      dmn_homogenize_linear, dmn_sample_stiffness,
                                      dmn_update_adjoint, dmn_update_gauss_points,
                                      dmn_update_gauss_points_noalloc, error_word)
    say("case: empty inputs through every call")
    d = dev()
    K = 5
    net = S.random_dmn(S.streams(64)["dmn"], K, 0.3)
    M, L = 2 ** (K - 1), 2 ** K - 1
    for dt in (torch.float64, torch.float32):
        w, n = torch.tensor(net.w, device=d, dtype=dt), torch.tensor(net.normals, device=d,
                                                                      dtype=dt)
        empty = torch.empty((0, 6, 6), device=d, dtype=dt)
        Cbar, ws = dmn_homogenize_linear(w, n, empty, empty)
        assert Cbar.shape == (0, 6, 6) and error_word(ws) == 0
        gw = torch.full((2 ** K,), float("nan"), device=d, dtype=dt)
        gn = torch.full((L, 3), float("nan"), device=d, dtype=dt)
        dmn_homogenize_backward(w, n, empty, empty, empty, gw=gw, gn=gn)
        torch.cuda.synchronize()
        assert bool((gw == 0).all()) and bool((gn == 0).all()), dt
    w, n = torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d)
    f64 = dict(device=d, dtype=torch.float64)
    gw, gn = torch.full((2 ** K,), 3.0, **f64), torch.full((L, 3), 3.0, **f64)
    ag = AdjointGroup(w, n, torch.empty((0, 6), **f64), torch.empty((0, M, 7), **f64),
                      torch.empty((0, L, 3), **f64), torch.empty((0, 6), **f64), None,
                      torch.empty((0, M, 7), **f64), gw, gn)
    dmn_update_adjoint([ag], S.FIBER, S.MATRIX)
    ge = PointGroup.allocate(w, n, torch.empty((0, 6), **f64))
    dmn_update_gauss_points([ge], S.FIBER, S.MATRIX)
    dmn_update_gauss_points_noalloc([ge], S.FIBER, S.MATRIX)
    C1, C2 = dmn_sample_stiffness(torch.empty((0, 8), **f64))
    torch.cuda.synchronize()
    assert bool((gw == 3.0).all()) and bool((gn == 3.0).all())
    assert C1.shape == (0, 6, 6) and C2.shape == (0, 6, 6)


def test_calls_on_two_streams_run_concurrently():
    """Calls on different streams with their own workspaces may overlap: a
    depth-7 Gauss-point update of 20,000 points on one stream and a depth-8
    linear map with its backward on 4,096 samples on another (both default
    priority), enqueued back to back, give bit for bit the results of the
    same calls made one after the other."""
    from paper_2103_08253_amd import (PointGroup, dmn_homogenize_backward,
                                      dmn_homogenize_linear, dmn_update_gauss_points)
    say("case: Gauss-point update and linear map + backward on two streams")
    d = dev()
    rs = S.streams(65)
    net = S.random_dmn(rs["dmn"], 7, 0.25)
    E = torch.tensor(S.ramp_with_noise(rs, 20000, 3, 0.02, 1e-3)[2], device=d)
    tw = S.config3(batch=4096, depth=8)
    w8, n8 = torch.tensor(tw.truth.w, device=d), torch.tensor(tw.truth.normals, device=d)
    C1, C2 = torch.tensor(tw.C1, device=d), torch.tensor(tw.C2, device=d)
    G = torch.tensor(rs["cotangent"].standard_normal((4096, 6, 6)), device=d)
    w7, n7 = torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d)

    def run(streams):
        g = PointGroup.allocate(w7, n7, E.clone())
        ws_g = dmn_update_gauss_points([g], S.FIBER, S.MATRIX)     # sizes the workspace
        Cb, ws_f = dmn_homogenize_linear(w8, n8, C1, C2)
        gw, gn, _, _, ws_b = dmn_homogenize_backward(w8, n8, C1, C2, G)
        torch.cuda.synchronize()
        g.sigma.fill_(0.0)
        Cb.fill_(0.0)
        gw.fill_(0.0)
        main = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(main)
        with torch.cuda.stream(streams[0]):
            dmn_update_gauss_points([g], S.FIBER, S.MATRIX, ws=ws_g)
        with torch.cuda.stream(streams[-1]):
            dmn_homogenize_linear(w8, n8, C1, C2, Cbar=Cb, ws=ws_f)
            dmn_homogenize_backward(w8, n8, C1, C2, G, ws=ws_b, gw=gw, gn=gn)
        for st in streams:
            main.wait_stream(st)
        torch.cuda.synchronize()
        return [t.clone() for t in (g.sigma, g.tangent, g.z_out, g.a_out, g.iters, g.status,
                                    Cb, gw, gn)]

    one = run([torch.cuda.Stream(device=d)])
    two = run([torch.cuda.Stream(device=d), torch.cuda.Stream(device=d)])
    for a, b in zip(one, two):
        if a.dtype == torch.float64:
            a, b = a.view(torch.int64), b.view(torch.int64)
        assert torch.equal(a, b)


# ---------------------------------------------------------------- linear map

@pytest.mark.parametrize("K,B", [(1, 5), (3, 37), (5, 70), (8, 33), (9, 3)])
def test_linear_forward_f64(K, B):
    from paper_2103_08253_amd import dmn_homogenize_linear, error_word
    say(f"case: linear forward f64 depth {K} batch {B}")
    d = dev()
    tw = S.config3(batch=B, depth=K)
    Cbar, ws = dmn_homogenize_linear(torch.tensor(tw.truth.w, device=d),
                                     torch.tensor(tw.truth.normals, device=d),
                                     torch.tensor(tw.C1, device=d), torch.tensor(tw.C2, device=d))
    ref = dmn_linear(K, tw.truth.w, tw.truth.normals, tw.C1, tw.C2)
    got = Cbar.cpu().numpy()
    assert error_word(ws) == 0
    errs = [rel(got[b], ref[b]) for b in range(B)]
    say(f"  worst rel err {max(errs):.2e}")
    assert max(errs) <= RTOL


@pytest.mark.parametrize("K,B", [(3, 37), (8, 64)])
def test_linear_forward_f32(K, B):
    from paper_2103_08253_amd import dmn_homogenize_linear
    say(f"case: linear forward f32 depth {K} batch {B}")
    d = dev()
    tw = S.config3(batch=B, depth=K)
    f = lambda x: torch.tensor(x, device=d, dtype=torch.float32)
    Cbar, _ = dmn_homogenize_linear(f(tw.truth.w), f(tw.truth.normals), f(tw.C1), f(tw.C2))
    ref = dmn_linear(K, tw.truth.w, tw.truth.normals, tw.C1, tw.C2)
    got = Cbar.double().cpu().numpy()
    errs = [rel(got[b], ref[b]) for b in range(B)]
    say(f"  worst rel err {max(errs):.2e}")
    assert max(errs) <= 1e-4


def chain_angles(gn, alpha, beta):
    da = np.stack([np.cos(alpha) * np.cos(beta), np.cos(alpha) * np.sin(beta), -np.sin(alpha)], -1)
    db = np.stack([-np.sin(alpha) * np.sin(beta), np.sin(alpha) * np.cos(beta),
                   np.zeros_like(alpha)], -1)
    return np.sum(gn * da, -1), np.sum(gn * db, -1)


@pytest.mark.parametrize("K,B,subset", [(3, 5, None), (5, 9, None), (7, 9, 24), (8, 2, 24)])
def test_linear_backward_f64_vs_complex_step(K, B, subset):
    from paper_2103_08253_amd import dmn_homogenize_backward
    say(f"case: linear backward f64 depth {K} batch {B}")
    d = dev()
    tw = S.config3(batch=B, depth=K)
    net = tw.truth
    alpha, beta = S.normals_to_angles(net.normals)
    G = S.streams(3)["cotangent"].standard_normal((B, 6, 6))
    gw, gn, gC1, gC2, _ = dmn_homogenize_backward(
        torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d),
        torch.tensor(tw.C1, device=d), torch.tensor(tw.C2, device=d), torch.tensor(G, device=d),
        want_input_grads=True)
    gw, gn = gw.cpu().numpy(), gn.cpu().numpy()
    ga, gb = chain_angles(gn, alpha, beta)
    rng = np.random.default_rng(7)
    w_idx = None if subset is None else rng.choice(2 ** K, subset, replace=False)
    a_idx = None if subset is None else rng.choice(2 ** K - 1, subset, replace=False)
    ref = linear_gradients(K, net.w, alpha, beta, tw.C1, tw.C2, G, w_idx, a_idx)
    mw = ~np.isnan(ref["gw"])
    ma = ~np.isnan(ref["galpha"])
    scale_w = np.abs(ref["gw"][mw]).max()
    scale_a = max(np.abs(ref["galpha"][ma]).max(), np.abs(ref["gbeta"][ma]).max())
    ew = np.abs(gw[mw] - ref["gw"][mw]).max() / scale_w
    ea = max(np.abs(ga[ma] - ref["galpha"][ma]).max(), np.abs(gb[ma] - ref["gbeta"][ma]).max()) / scale_a
    say(f"  rel err gw {ew:.2e}, angles {ea:.2e}")
    assert ew <= RTOL and ea <= RTOL
    # Euler identity of the scale-invariant map, and tangency of gn
    assert abs(net.w @ gw) <= 1e-10 * np.abs(gw).max() * np.abs(net.w).sum()
    assert np.abs(np.sum(gn * net.normals, -1)).max() <= 1e-9 * np.abs(gn).max()
    # input cotangent: one entry of C1 and of C2 by complex step on a symmetric perturbation
    h = 1e-30
    for which, gC, (i, j) in (("C1", gC1, (0, 4)), ("C2", gC2, (2, 2))):
        E_ij = np.zeros((6, 6), complex)
        E_ij[i, j] += 1j * h
        E_ij[j, i] += 1j * h if i != j else 0
        C1c = tw.C1.astype(complex) + (E_ij if which == "C1" else 0)
        C2c = tw.C2.astype(complex) + (E_ij if which == "C2" else 0)
        cs = np.imag(np.sum(G * dmn_linear(K, net.w, net.normals, C1c, C2c))) / h
        gpu_val = gC[:, i, j].sum().item() * (2 if i != j else 1)
        assert abs(gpu_val - cs) <= 1e-9 * max(abs(cs), 1e-12), (which, gpu_val, cs)


def test_linear_backward_tree_reduction_vs_complex_step():
    """Depth 8, B = 256: 256 partial-sum slots per parameter row, more than the
    64 that one thread sums in slot order, so the batch sum runs through the
    workgroup tree reduction.  12 weights and 8 laminates' angle gradients
    against the oracle's complex-step derivatives at 1e-10."""
    from paper_2103_08253_amd import dmn_homogenize_backward
    K, B = 8, 256
    say(f"case: linear backward f64 depth {K} batch {B} (tree reduction of the batch sum)")
    d = dev()
    tw = S.config3(batch=B, depth=K)
    net = tw.truth
    alpha, beta = S.normals_to_angles(net.normals)
    G = S.streams(4)["cotangent"].standard_normal((B, 6, 6))
    gw, gn, _, _, _ = dmn_homogenize_backward(
        torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d),
        torch.tensor(tw.C1, device=d), torch.tensor(tw.C2, device=d), torch.tensor(G, device=d))
    gw, gn = gw.cpu().numpy(), gn.cpu().numpy()
    ga, gb = chain_angles(gn, alpha, beta)
    rng = np.random.default_rng(17)
    w_idx = rng.choice(2 ** K, 12, replace=False)
    a_idx = np.concatenate([[0, 127, 254], rng.choice(np.arange(1, 254), 5, replace=False)])
    ref = linear_gradients(K, net.w, alpha, beta, tw.C1, tw.C2, G, w_idx, a_idx)
    ew = np.abs(gw[w_idx] - ref["gw"][w_idx]).max() / np.abs(ref["gw"][w_idx]).max()
    ra = np.concatenate([ref["galpha"][a_idx], ref["gbeta"][a_idx]])
    ea = np.abs(np.concatenate([ga[a_idx], gb[a_idx]]) - ra).max() / np.abs(ra).max()
    say(f"  rel err gw {ew:.2e}, angles {ea:.2e} (element-wise over the selected entries)")
    assert ew <= RTOL and ea <= RTOL


def test_linear_offsets_beyond_32_bits():
    """Maximum size: the depth-8 linear map and its backward over 59,801,600
    samples (14,600 copies of a 4,096-sample batch, 69 GB), so the element
    offsets of the last samples' stiffnesses pass 2^31.  Every copy's Cbar
    equals the first copy's bit for bit, sampled outputs of the last copy
    match the oracle, and the batch gradient equals 14,600 times the single
    batch's within rounding of the sum."""
    from paper_2103_08253_amd import dmn_homogenize_backward, dmn_homogenize_linear
    d = dev()
    K, B0, reps = 8, 4096, 14600
    B = B0 * reps
    assert (B - 1) * 36 >= 2 ** 31
    torch.cuda.empty_cache()
    need = 4 * B * 36 * 8
    if torch.cuda.mem_get_info()[0] < need + (4 << 30):
        pytest.skip(f"needs {need / 2 ** 30:.0f} GiB of free device memory")
    say(f"case: linear map and backward depth {K}, {B} samples ({reps} copies of {B0}), "
        f"{need / 2 ** 30:.0f} GiB")
    rs = S.streams(61)
    net = S.random_dmn(rs["dmn"], K, 0.25)
    C1s, C2s = S.random_spd(rs["stiffness"], B0), S.random_spd(rs["stiffness"], B0)
    Gs = rs["cotangent"].standard_normal((B0, 6, 6))
    w, n = torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d)
    small = [torch.tensor(x, device=d) for x in (C1s, C2s, Gs)]
    gw0, gn0, _, _, _ = dmn_homogenize_backward(w, n, *small)
    C1, C2, G = (x.repeat(reps, 1, 1) for x in small)
    del small
    Cbar, ws = dmn_homogenize_linear(w, n, C1, C2)
    torch.cuda.synchronize()
    from paper_2103_08253_amd import error_word
    assert error_word(ws) == 0
    bits = Cbar.view(torch.int64).view(reps, B0, -1)
    assert torch.equal(bits, bits[:1].expand_as(bits))
    picks = np.array([0, 1777, B0 - 1])
    got = Cbar[(reps - 1) * B0 + picks].cpu().numpy()
    del Cbar, ws, bits
    ref = dmn_linear(K, net.w, net.normals, C1s[picks], C2s[picks])
    e_map = rel(got, ref)
    gw, gn, _, _, wsb = dmn_homogenize_backward(w, n, C1, C2, G)
    torch.cuda.synchronize()
    assert error_word(wsb) == 0
    del C1, C2, G, wsb
    torch.cuda.empty_cache()
    e_w = rel(gw.cpu().numpy(), reps * gw0.cpu().numpy())
    e_n = rel(gn.cpu().numpy(), reps * gn0.cpu().numpy())
    say(f"  map rel err {e_map:.2e}; batch gradient vs {reps} x one batch: gw {e_w:.2e}, "
        f"gn {e_n:.2e}")
    assert e_map <= RTOL
    assert e_w <= 1e-12 and e_n <= 1e-12


def test_linear_backward_finite_differences_and_f32():
    from paper_2103_08253_amd import dmn_homogenize_backward, dmn_homogenize_linear
    say("case: linear backward depth 8 batch 4096: FD h=1e-6 and FP32")
    d = dev()
    tw = S.config3()
    net = tw.truth
    t = lambda x, dt=torch.float64: torch.tensor(x, device=d, dtype=dt)
    G = S.streams(3)["cotangent"].standard_normal((4096, 6, 6))
    gw, gn, _, _, _ = dmn_homogenize_backward(t(net.w), t(net.normals), t(tw.C1), t(tw.C2), t(G))
    J = lambda w, n: float(torch.sum(t(G) * dmn_homogenize_linear(w, n, t(tw.C1), t(tw.C2))[0]))
    h = 1e-6
    for j in (0, 77, 255):
        wp, wm = t(net.w), t(net.w)
        wp[j] += h
        wm[j] -= h
        fd = (J(wp, t(net.normals)) - J(wm, t(net.normals))) / (2 * h)
        assert abs(fd - gw[j].item()) <= 1e-5 * abs(gw).max().item(), (j, fd, gw[j].item())
    for p in (3, 200, 254):
        for c in range(3):
            npl, nmi = t(net.normals), t(net.normals)
            npl[p, c] += h
            nmi[p, c] -= h
            fd = (J(t(net.w), npl) - J(t(net.w), nmi)) / (2 * h)
            assert abs(fd - gn[p, c].item()) <= 1e-5 * abs(gn).max().item(), (p, c, fd)
    f = torch.float32
    gw32, gn32, _, _, _ = dmn_homogenize_backward(t(net.w, f), t(net.normals, f), t(tw.C1, f),
                                                  t(tw.C2, f), t(G, f))
    ew = (gw32.double() - gw).abs().max().item() / gw.abs().max().item()
    en = (gn32.double() - gn).abs().max().item() / gn.abs().max().item()
    say(f"  FP32 vs FP64 gradient rel err: w {ew:.2e}, n {en:.2e}")
    assert ew <= 1e-4 and en <= 1e-4


@pytest.mark.parametrize("K,dtype", [(7, "f64"), (7, "f32"), (8, "f64"), (8, "f32")])
def test_linear_two_samples_per_wave_match_one_sample_calls(K, dtype):
    """Above 8 samples per CU in a launch, the linear map at depths 7 and 8 and
    its backward run two samples per wave that share the upper tree levels.
    On a batch 37 samples above that size, compare with calls on chunks at
    or below it, which run one sample per wave:
    * Cbar agrees per sample within rounding (each sample sees the same
      laminate operations, Sec. 3.1, in the same order, but the compiler may
      contract them into FMAs differently in the two kernels);
    * the batch gradient equals the sum of the chunks' gradients within
      rounding.
    The gradient is also checked against an independent reference:
    * FP64 at depth 7: two weights and the root laminate's angles against the
      oracle's complex-step derivative;
    * FP32: the whole gradient against the FP64 call (1e-4 of its largest
      entry)."""
    from paper_2103_08253_amd import dmn_homogenize_backward, dmn_homogenize_linear
    d = dev()
    cus = torch.cuda.get_device_properties(d).multi_processor_count
    fwd_cut = 8 * cus
    bwd_cut = 8 * cus
    B = bwd_cut + 37
    chunks = lambda n: [(a, min(a + n, B)) for a in range(0, B, n)]
    say(f"case: linear map and backward, depth {K}, {dtype}, batch {B} ({cus} CUs)")
    tw = S.config3(batch=B, depth=K)
    net = tw.truth
    G = S.streams(3)["cotangent"].standard_normal((B, 6, 6))
    f = torch.float64 if dtype == "f64" else torch.float32
    t = lambda x, dt=f: torch.tensor(x, device=d, dtype=dt)
    w, n, C1, C2, Gt = t(net.w), t(net.normals), t(tw.C1), t(tw.C2), t(G)
    Cb, _ = dmn_homogenize_linear(w, n, C1, C2)
    gw, gn, _, _, _ = dmn_homogenize_backward(w, n, C1, C2, Gt)
    Cc = torch.cat([dmn_homogenize_linear(w, n, C1[a:b], C2[a:b])[0]
                    for a, b in chunks(fwd_cut)])
    gparts = [dmn_homogenize_backward(w, n, C1[a:b], C2[a:b], Gt[a:b])[:2]
              for a, b in chunks(bwd_cut)]
    torch.cuda.synchronize()
    Cb_np, Cc_np = Cb.double().cpu().numpy(), Cc.double().cpu().numpy()
    diff = np.abs(Cb_np - Cc_np).max(axis=(1, 2)) / np.abs(Cc_np).max(axis=(1, 2))
    say(f"  Cbar batch vs chunks: {int((diff > 0).sum())} of {B} samples differ, "
        f"worst {diff.max():.2e}")
    assert diff.max() <= (1e-13 if dtype == "f64" else 1e-5)
    gw_np, gn_np = gw.double().cpu().numpy(), gn.double().cpu().numpy()
    gw_c = sum(g[0].double().cpu().numpy() for g in gparts)
    gn_c = sum(g[1].double().cpu().numpy() for g in gparts)
    ew, en = rel(gw_np, gw_c), rel(gn_np, gn_c)
    say(f"  batch vs chunks: gw {ew:.2e}, gn {en:.2e}")
    bar = 1e-12 if dtype == "f64" else 1e-5
    assert ew <= bar and en <= bar
    if dtype == "f32":
        t64 = lambda x: t(x, torch.float64)
        gw64, gn64, _, _, _ = dmn_homogenize_backward(t64(net.w), t64(net.normals), t64(tw.C1),
                                                      t64(tw.C2), t64(G))
        ew = rel(gw_np, gw64.cpu().numpy())
        en = rel(gn_np, gn64.cpu().numpy())
        say(f"  FP32 vs FP64: gw {ew:.2e}, gn {en:.2e}")
        assert ew <= 1e-4 and en <= 1e-4
    elif K == 7:
        alpha, beta = S.normals_to_angles(net.normals)
        iw = [int(np.argmax(net.w)), 5]
        root = 2 ** K - 2
        ref = linear_gradients(K, net.w, alpha, beta, tw.C1, tw.C2, G, iw, [root])
        ga, gb = chain_angles(gn_np, alpha, beta)
        e_w = rel(gw_np[iw], ref["gw"][iw])
        got_a = np.array([ga[root], gb[root]])
        ref_a = np.array([ref["galpha"][root], ref["gbeta"][root]])
        e_a = rel(got_a, ref_a)
        say(f"  vs oracle complex step: gw {e_w:.2e}, root angles {e_a:.2e}")
        assert e_w <= RTOL and e_a <= RTOL
