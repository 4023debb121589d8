"""HIP-graph capture of the library calls: every replay against eager calls.

The kernels compute each point (and each reduction) in a fixed order, so a
replayed graph and the eager calls give bit-identical results.  Each test
replays several times with eager work (library calls on other buffers,
torch kernels, host synchronisation) between the replays, and checks every
replay.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthetic as S

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_groups(d, n_points, n_steps, pick):
    wl = S.config2(n_points=n_points, n_steps=n_steps)
    out = []
    for m in pick:
        sel = np.nonzero(wl.dmn_id == m)[0]
        net = wl.nets[m]
        out.append((torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d),
                    torch.tensor(np.ascontiguousarray(wl.E[:, sel, :]), device=d)))
    return out


def eager_path(specs, E_list, z0=None, a0=None):
    """Eager steps over the groups; returns per-step sigma and the final records."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    groups = [PointGroup.allocate(w, n, E[0].clone()) for (w, n, _), E in zip(specs, E_list)]
    if z0 is not None:
        for g, z, a in zip(groups, z0, a0):
            g.z_in.copy_(z)
            g.a_in.copy_(a)
    sig = [[] for _ in groups]
    ws = None
    for t in range(E_list[0].shape[0]):
        for g, E in zip(groups, E_list):
            g.E.copy_(E[t])
        ws = dmn_update_gauss_points(groups, S.FIBER, S.MATRIX, ws=ws)
        for m, g in enumerate(groups):
            sig[m].append(g.sigma.clone())
            g.advance()
    torch.cuda.synchronize()
    return groups, [torch.stack(s) for s in sig]


def busy_work(d):
    """Eager work between replays: a library call on unrelated buffers and torch kernels."""
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    rs = S.streams(77)
    net = S.random_dmn(rs["dmn"], 4, 0.3)
    E = torch.tensor(S.ramp_with_noise(rs, 50, 1, 0.01, 1e-3)[0], device=d)
    g = PointGroup.allocate(torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d), E)
    dmn_update_gauss_points([g], S.FIBER, S.MATRIX)
    x = torch.randn(1 << 20, device=d, dtype=torch.float64)
    (x * x).sum().item()
    torch.cuda.synchronize()


def test_load_step_graph_replays_match_eager():
    """Three mixed-depth groups, 4 steps in one graph, replayed 3 times from the
    same initial state; stresses of every step and the final records bit-exact."""
    from paper_2103_08253_amd import LoadStepGraph, PointGroup
    say("case: load-step graph, groups of depth 5, 7, 8, 4 steps, 3 replays")
    d = dev()
    specs = mixed_groups(d, 384, 4, [0, 2, 3])
    E_list = [E for _, _, E in specs]
    ref_groups, ref_sig = eager_path(specs, E_list)
    groups = [PointGroup.allocate(w, n, E[0].clone()) for w, n, E in specs]
    E_static = [E.clone() for E in E_list]
    graph = LoadStepGraph(groups, S.FIBER, S.MATRIX, E_static)
    starts = graph.start_state
    for r in range(3):
        for z, a in starts:
            z.zero_()
            a.zero_()
        graph.replay()
        torch.cuda.synchronize()
        for m, (g, rg) in enumerate(zip(groups, ref_groups)):
            assert torch.equal(graph.sigma_steps[m], ref_sig[m]), (r, m)
            assert torch.equal(g.z_in, rg.z_in) and torch.equal(g.a_in, rg.a_in), (r, m)
            assert torch.equal(g.tangent, rg.tangent), (r, m)
            assert torch.equal(g.iters, rg.iters) and torch.equal(g.status, rg.status), (r, m)
        say(f"  replay {r}: bit-exact")
        busy_work(d)


def test_load_step_graph_chains_along_the_path():
    """A 2-step graph replayed 4 times, its strain tensor refilled in place before
    each replay, continues the path: equals 8 eager steps bit for bit."""
    from paper_2103_08253_amd import LoadStepGraph, PointGroup
    say("case: 2-step graph chained over an 8-step path, depth 8 and 6")
    d = dev()
    specs = mixed_groups(d, 512, 8, [3, 1])
    E_list = [E for _, _, E in specs]
    ref_groups, ref_sig = eager_path(specs, E_list)
    groups = [PointGroup.allocate(w, n, E[0].clone()) for w, n, E in specs]
    E_static = [E[:2].clone() for E in E_list]
    graph = LoadStepGraph(groups, S.FIBER, S.MATRIX, E_static)
    for r in range(4):
        for Es, E in zip(E_static, E_list):
            Es.copy_(E[2 * r:2 * r + 2])
        graph.replay()
        torch.cuda.synchronize()
        for m in range(len(groups)):
            assert torch.equal(graph.sigma_steps[m], ref_sig[m][2 * r:2 * r + 2]), (r, m)
        if r == 1:
            busy_work(d)
    for g, rg in zip(groups, ref_groups):
        assert torch.equal(g.z_in, rg.z_in) and torch.equal(g.a_in, rg.a_in)
        assert torch.equal(g.tangent, rg.tangent)
    say("  8 chained steps bit-exact")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_linear_step_graph_replays_match_eager(dtype):
    """Forward + backward of the depth-8 linear map captured once; inputs refilled
    in place between 3 replays; every replay equals the eager calls."""
    from paper_2103_08253_amd import (LinearStepGraph, dmn_homogenize_backward,
                                      dmn_homogenize_linear)
    say(f"case: linear step graph, depth 8, B 1024, {dtype}")
    d = dev()
    tw = S.config3(batch=1024)
    w = torch.tensor(tw.v0, device=d, dtype=dtype)
    n = torch.tensor(S.angles_to_normals(tw.alpha0, tw.beta0), device=d, dtype=dtype)
    C1 = torch.tensor(tw.C1, device=d, dtype=dtype)
    C2 = torch.tensor(tw.C2, device=d, dtype=dtype)
    rng = np.random.default_rng(9)
    G = torch.tensor(rng.standard_normal((1024, 6, 6)), device=d, dtype=dtype)
    graph = LinearStepGraph(w, n, C1, C2, G, want_input_grads=True)
    for r in range(3):
        C1.copy_(torch.tensor(tw.C1 * (1.0 + 0.1 * r), device=d, dtype=dtype))
        G.copy_(torch.tensor(rng.standard_normal((1024, 6, 6)), device=d, dtype=dtype))
        graph.replay()
        torch.cuda.synchronize()
        Cb, _ = dmn_homogenize_linear(w, n, C1, C2)
        gw, gn, gC1, gC2, _ = dmn_homogenize_backward(w, n, C1, C2, G, want_input_grads=True)
        torch.cuda.synchronize()
        assert torch.equal(graph.Cbar, Cb), r
        assert torch.equal(graph.gw, gw) and torch.equal(graph.gn, gn), r
        assert torch.equal(graph.gC1, gC1) and torch.equal(graph.gC2, gC2), r
        say(f"  replay {r}: bit-exact")
        busy_work(d)
