"""Load paths through the DMN Gauss-point update and their adjoint.

`run_path` applies a strain path with dmn_update_gauss_points.
`forward_checkpointed` does the same and keeps the state (z, a) at the start
of every `checkpoint_every`-step segment; `adjoint_sweep` then returns the
gradient of J = sum_p g_p . sigma_p(final) with respect to the DMN's leaf
weights and normals by the load-step adjoint (dmn_update_adjoint) swept
backwards over the steps, recomputing one segment of states at a time.
Orchestration only: every step runs in the HIP kernels.
"""
import torch

from .api import AdjointGroup, PointGroup, dmn_update_adjoint, dmn_update_gauss_points


class PathFailed(RuntimeError):
    pass


def _check(g: PointGroup, step: int):
    bad = (g.status != 0).nonzero()
    if bad.numel():
        p = int(bad[0, 0])
        raise PathFailed(f"step {step}: point {p} ended with status {int(g.status[p])}")


def run_path(w, n, E_path, fiber, matrix, z0=None, a0=None, check=True, **newton):
    """Apply E_path [T, P, 6]; returns the PointGroup of the last step (outputs in
    sigma, tangent, z_out, a_out)."""
    g = PointGroup.allocate(w, n, E_path[0], z0, a0)
    ws = None
    for step in range(E_path.shape[0]):
        g.E = E_path[step]
        ws = dmn_update_gauss_points([g], fiber, matrix, ws=ws, **newton)
        if check:
            _check(g, step)
        if step + 1 < E_path.shape[0]:
            g.advance()
    return g


def forward_checkpointed(w, n, E_path, fiber, matrix, checkpoint_every=10, check=True,
                         **newton):
    """(sigma_final [P, 6], {step: (z, a)} at the start of every segment)."""
    T = E_path.shape[0]
    ck = max(1, int(checkpoint_every))
    g = PointGroup.allocate(w, n, E_path[0])
    checkpoints = {0: (g.z_in.clone(), g.a_in.clone())}
    ws = None
    for step in range(T):
        g.E = E_path[step]
        ws = dmn_update_gauss_points([g], fiber, matrix, ws=ws, **newton)
        if check:
            _check(g, step)
        g.advance()
        if (step + 1) % ck == 0 and step + 1 < T:
            checkpoints[step + 1] = (g.z_in.clone(), g.a_in.clone())
    return g.sigma.clone(), checkpoints


def adjoint_sweep(w, n, E_path, checkpoints, g_sigma, fiber, matrix, checkpoint_every=10,
                  **newton):
    """(dJ/dw, dJ/dn) of J = sum_p g_sigma[p] . sigma_p(final)."""
    T, P = E_path.shape[0], E_path.shape[1]
    dev = E_path.device
    K = int(w.numel()).bit_length() - 1
    M, Lm = 2 ** (K - 1), 2 ** K - 1
    ck = max(1, int(checkpoint_every))
    gw = torch.zeros(2 ** K, dtype=torch.float64, device=dev)
    gn = torch.zeros((Lm, 3), dtype=torch.float64, device=dev)
    zeta = None
    zeta_buf = [torch.empty((P, M, 7), dtype=torch.float64, device=dev) for _ in range(2)]
    ws = ws_adj = None
    for start in sorted(checkpoints, reverse=True):
        stop = min(start + ck, T)
        z, a = checkpoints[start]
        seg = PointGroup.allocate(w, n, E_path[start], z.clone(), a.clone())
        states = []  # (z^n, a^{n+1}) of every step of the segment
        for step in range(start, stop):
            seg.E = E_path[step]
            ws = dmn_update_gauss_points([seg], fiber, matrix, ws=ws, **newton)
            states.append((seg.z_in.clone(), seg.a_out.clone()))
            seg.advance()
        for i in reversed(range(len(states))):
            step = start + i
            z_n, a_conv = states[i]
            out = zeta_buf[step % 2]
            grp = AdjointGroup(w, n, E_path[step], z_n, a_conv,
                               g_sigma if step == T - 1 else None, zeta, out, gw, gn)
            ws_adj = dmn_update_adjoint([grp], fiber, matrix, ws=ws_adj)
            zeta = out
        del states
    return gw, gn


def path_gradient(w, n, E_path, g_sigma, fiber, matrix, checkpoint_every=10, **newton):
    """(sigma_final, dJ/dw, dJ/dn) for J = sum_p g_sigma[p] . sigma_p(final)."""
    sigma, cks = forward_checkpointed(w, n, E_path, fiber, matrix, checkpoint_every, **newton)
    gw, gn = adjoint_sweep(w, n, E_path, cks, g_sigma, fiber, matrix, checkpoint_every, **newton)
    return sigma, gw, gn
