"""GPU parity of the Newton control paths that the standard workloads never take.

* Backtracking (reading R5): with a strict sufficient-decrease factor the full
  Newton step is rejected and halved; with max_backtrack = 1 a half step is
  taken whatever its residual.  The oracle's trials are counted, so the test
  asserts that backtracking did happen, and the GPU must take the same
  iterations (equal counts) to the same converged state (1e-10).
* Status 3 (pivot not positive definite), forced from the host by a zero
  lamination normal: that laminate's block of the Newton Hessian vanishes.
* Status 4 (J2 return not converged), forced from the host by capping the
  scalar Newton iterations of the return (local_max_iter).
On failure the input state is passed through and the tangent is NaN.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthetic as S
from oracle.gp import LOCALFAIL, NOTSPD, DmnModel, NewtonOptions, gp_update
from test_gpu_parity import compare_paths, dev, gpu_path, say

pytestmark = pytest.mark.gpu


def count_trials(model):
    """Wrap the oracle model's evaluation to log every residual norm it computes
    (one per Newton trial, plus the initial evaluation)."""
    log = []
    orig = model.evaluate

    def ev(*args):
        out = orig(*args)
        log.append(np.linalg.norm(out["r"]))
        return out

    model.evaluate = ev
    return log


@pytest.mark.parametrize("K,armijo,max_bt", [(3, 0.99, 10), (5, 0.99, 10), (3, 0.9999, 1),
                                             (8, 0.999, 3)])
def test_gp_backtracking_matches_oracle(K, armijo, max_bt):
    say(f"case: gp backtracking, depth {K}, armijo {armijo}, max_backtrack {max_bt}")
    rs = S.streams(300 + K)
    n_pts = 12 if K < 8 else 3
    net = S.random_dmn(rs["dmn"], K, 0.25)
    E = S.ramp_with_noise(rs, n_pts, 3, 0.02, 1e-3)
    opts = NewtonOptions(armijo=armijo, max_backtrack=max_bt)
    gpu = gpu_path(net, E, dict(armijo=armijo, max_backtrack=max_bt))
    compare_paths(net, E, range(n_pts), gpu, opts)
    # the oracle did backtrack on these inputs (counted on its own run)
    model = DmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX)
    log = count_trials(model)
    rejected = 0
    for p in range(n_pts):
        z, a = np.zeros((2 ** (K - 1), 7)), np.zeros(3 * (2 ** K - 1))
        for step in range(E.shape[0]):
            log.clear()
            out = gp_update(model, E[step, p], z, a, opts)
            assert out["status"] == 0
            rejected += len(log) - 1 - out["iters"]
            z, a = out["z"], out["a"]
    say(f"  oracle rejected {rejected} trial steps over {n_pts} points x {E.shape[0]} steps")
    assert rejected > 0
    # GPU iteration counts are above the no-backtracking ones somewhere
    plain = gpu_path(net, E)
    more = sum(int((g["iters"] > h["iters"]).sum()) for g, h in zip(gpu, plain))
    assert more > 0


@pytest.mark.parametrize("K", [3, 8])
def test_gp_polish_matches_oracle(K):
    """polish = 1: one full Newton step after the stop test, not counted in the
    iterations and taken without the backtracking test, as the oracle's polish."""
    say(f"case: gp polish step, depth {K}")
    rs = S.streams(320 + K)
    n_pts = 8 if K < 8 else 3
    net = S.random_dmn(rs["dmn"], K, 0.25)
    E = S.ramp_with_noise(rs, n_pts, 4, 0.02, 1e-3)
    gpu = gpu_path(net, E, dict(polish=1))
    compare_paths(net, E, range(n_pts), gpu, NewtonOptions(polish=1))
    plain = gpu_path(net, E)
    for g, h in zip(gpu, plain):
        assert np.array_equal(g["iters"], h["iters"])  # polish steps are not counted


def failure_case(K, zero_pos=None, seed=210):
    rs = S.streams(seed + K)
    net = S.random_dmn(rs["dmn"], K, 0.25)
    if zero_pos is not None:
        net.normals = net.normals.copy()
        net.normals[zero_pos] = 0.0
    P = 6
    E = 0.02 * S.unit_directions(rs["direction"], P)
    E[:2] *= 1e-4  # two points stay elastic
    M = 2 ** (K - 1)
    z0 = 1e-4 * rs["noise"].standard_normal((P, M, 7))
    z0[:, :, :6] -= (z0[:, :, :3].sum(-1) / 3.0)[..., None] * np.array([1, 1, 1, 0, 0, 0])
    z0[:, :, 6] = np.abs(z0[:, :, 6])
    a0 = 1e-4 * rs["noise"].standard_normal((P, 2 ** K - 1, 3))
    return net, E, z0, a0


def run_failure(net, E, z0, a0, **opts):
    from paper_2103_08253_amd import PointGroup, dmn_update_gauss_points
    d = dev()
    g = PointGroup.allocate(torch.tensor(net.w, device=d), torch.tensor(net.normals, device=d),
                            torch.tensor(E, device=d), z_in=torch.tensor(z0, device=d),
                            a_in=torch.tensor(a0, device=d))
    dmn_update_gauss_points([g], S.FIBER, S.MATRIX, **opts)
    torch.cuda.synchronize()
    return g


def check_against_oracle(net, E, z0, a0, g, opts, expect):
    model = DmnModel(net.depth, net.w, net.normals, S.FIBER, S.MATRIX)
    seen = set()
    for p in range(E.shape[0]):
        ref = gp_update(model, E[p], z0[p], a0[p].ravel(), opts)
        st, it = int(g.status[p]), int(g.iters[p])
        assert st == ref["status"] and it == ref["iters"], (p, st, it, ref["status"], ref["iters"])
        seen.add(st)
        sig = g.sigma[p].cpu().numpy()
        assert np.abs(sig - ref["sigma"]).max() <= 1e-10 * np.abs(ref["sigma"]).max(), p
        if st != 0:
            assert torch.equal(g.z_out[p], g.z_in[p]) and torch.equal(g.a_out[p], g.a_in[p])
            assert torch.isnan(g.tangent[p]).all()
        else:
            C = g.tangent[p].cpu().numpy()
            assert np.abs(C - ref["C"]).max() <= 1e-10 * np.abs(ref["C"]).max(), p
    assert expect in seen, seen
    return seen


@pytest.mark.parametrize("K,zero_pos", [(3, 2), (3, 6), (8, 17), (8, 254)])
def test_gp_status_not_spd_from_zero_normal(K, zero_pos):
    """A zero normal (a lane-subtree laminate or the root) gives status 3 at
    the first Newton step, iteration count 0, input state passed through."""
    say(f"case: gp status 3 (zero normal at laminate {zero_pos}), depth {K}")
    net, E, z0, a0 = failure_case(K, zero_pos)
    g = run_failure(net, E, z0, a0)
    seen = check_against_oracle(net, E, z0, a0, g, NewtonOptions(), NOTSPD)
    say(f"  statuses {sorted(seen)}")


@pytest.mark.parametrize("K,cap", [(3, 1), (5, 2), (8, 1)])
def test_gp_status_local_from_capped_return(K, cap):
    """The J2 return capped at `cap` scalar iterations: plastic points fail with
    status 4 (input state passed through), elastic points converge."""
    say(f"case: gp status 4 (local_max_iter {cap}), depth {K}")
    net, E, z0, a0 = failure_case(K)
    g = run_failure(net, E, z0, a0, local_max_iter=cap)
    seen = check_against_oracle(net, E, z0, a0, g, NewtonOptions(local_max_iter=cap), LOCALFAIL)
    assert 0 in seen
    say(f"  statuses {sorted(seen)}")
