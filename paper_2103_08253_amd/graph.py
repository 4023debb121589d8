"""HIP-graph capture of load steps and of the linear training step.

Every libdmn call enqueues kernels only: it allocates nothing, never
synchronises, reads no device data on the host and clears its work counters
with a kernel rather than a memset node.  A sequence of calls can therefore
be captured once into a HIP graph (``torch.cuda.CUDAGraph``) and replayed,
which removes the per-call host overhead (argument validation, ctypes
marshalling, up to a few launches per call) from loops of many short steps.

A graph replays the device pointers it was captured with: inputs are read
from, and outputs written to, the same tensors on every replay, so a caller
refills the input tensors in place (``copy_``) between replays.
"""
from typing import List, Sequence

import torch

from . import _lib as L
from .api import (PointGroup, dmn_homogenize_backward, dmn_homogenize_linear,
                  dmn_update_gauss_points, workspace)


def _gp_workspace(groups: Sequence[PointGroup]):
    arr = (L.DmnPointGroup * len(groups))(*[g.to_c() for g in groups])
    nbytes = L.lib().dmn_update_gauss_points_workspace_size(arr, len(groups), groups[0].prec)
    if nbytes == 0:
        raise L.DmnError("dmn_update_gauss_points_workspace_size rejected the groups")
    return workspace(nbytes, groups[0].E.device)


class LoadStepGraph:
    """T consecutive load steps of ``dmn_update_gauss_points`` as one graph.

    At capture time each group's ``z_in``/``a_in`` hold the state entering the
    first step.  The captured steps ping-pong between (z_in, a_in) and
    (z_out, a_out) exactly as the eager loop ``update; advance()`` does.  The
    macro strain of step t is read from ``E_steps[m][t]`` ([T, P, 6], one
    tensor per group) when the graph replays.  With ``keep_sigma`` the stress
    of step t goes to ``sigma_steps[m][t]``; the tangent, iteration counts and
    statuses are those of the last step.  Capturing runs no kernel; the
    groups' Python-side buffers are left as after T eager steps, so after a
    replay ``groups[m].z_in`` / ``a_in`` hold the final state.  For even T
    these are the buffers the replay starts from, and consecutive replays
    continue the path.
    """

    def __init__(self, groups: List[PointGroup], fiber: dict, matrix: dict,
                 E_steps: List[torch.Tensor], keep_sigma: bool = True, **newton):
        if len(groups) != len(E_steps) or not groups:
            raise ValueError("one [T, P, 6] strain tensor per group is required")
        T = int(E_steps[0].shape[0])
        for g, E in zip(groups, E_steps):
            if E.dim() != 3 or E.shape[0] != T or tuple(E.shape[1:]) != tuple(g.E.shape):
                raise ValueError("E_steps[m] must be [T, P_m, 6] with a common T")
            if E.dtype != g.E.dtype or not E.is_contiguous() or E.device != g.E.device:
                raise ValueError("E_steps[m] must be contiguous, on the group's device, "
                                 "in the group's dtype")
        self.groups = groups
        self.T = T
        self.E_steps = E_steps
        self.sigma_steps = ([torch.empty((T,) + tuple(g.sigma.shape), dtype=g.sigma.dtype,
                                         device=g.sigma.device) for g in groups]
                            if keep_sigma else None)
        self.ws = _gp_workspace(groups)
        self.start_state = [(g.z_in, g.a_in) for g in groups]
        self.graph = torch.cuda.CUDAGraph()
        stream = torch.cuda.Stream(device=groups[0].E.device)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=stream):
            for t in range(T):
                for m, g in enumerate(groups):
                    g.E = E_steps[m][t]
                    if self.sigma_steps is not None:
                        g.sigma = self.sigma_steps[m][t]
                dmn_update_gauss_points(groups, fiber, matrix, ws=self.ws, **newton)
                for g in groups:
                    g.advance()
        torch.cuda.current_stream().wait_stream(stream)

    def replay(self):
        """Enqueue the T steps on the current stream."""
        self.graph.replay()


class LinearStepGraph:
    """Forward and backward of the linear map (one training step) as one graph.

    ``w``, ``n``, ``C1``, ``C2`` and ``gCbar`` are read at replay time from the
    tensors given here; ``Cbar``, ``gw`` and ``gn`` are written on every replay.
    """

    def __init__(self, w, n, C1, C2, gCbar, want_input_grads: bool = False):
        self.w, self.n, self.C1, self.C2, self.gCbar = w, n, C1, C2, gCbar
        self.Cbar = torch.empty((C1.shape[0], 6, 6), dtype=C1.dtype, device=C1.device)
        _, self.ws_fwd = dmn_homogenize_linear(w, n, C1, C2, Cbar=self.Cbar, ws=None)
        out = dmn_homogenize_backward(w, n, C1, C2, gCbar, want_input_grads)
        self.ws_bwd = out[-1]
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        stream = torch.cuda.Stream(device=C1.device)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=stream):
            dmn_homogenize_linear(w, n, C1, C2, Cbar=self.Cbar, ws=self.ws_fwd)
            self.gw, self.gn, self.gC1, self.gC2, _ = dmn_homogenize_backward(
                w, n, C1, C2, gCbar, want_input_grads, ws=self.ws_bwd)
        torch.cuda.current_stream().wait_stream(stream)

    def replay(self):
        """Enqueue forward + backward on the current stream."""
        self.graph.replay()
