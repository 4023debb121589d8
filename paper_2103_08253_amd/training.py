"""Offline training of a DMN with fixed normals on the GPU (Sec. 3.1 objective
and parameterisation, Sec. 4.4 stiffness sampling, Sec. 4.5 optimiser).

A step is the linear map, the objective's data term and cotangent, the
linear map's VJP and the AMSGrad update; ``TrainingStepGraph`` captures the
four calls as one HIP graph, so a training loop is one replay per step with
no host synchronisation (the objective stays on the device in ``stats``).
"""
import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib as L
from .api import (_PREC, _need, _ptr, _stream, dmn_homogenize_backward,
                  dmn_homogenize_backward_groups, dmn_homogenize_linear,
                  dmn_homogenize_linear_groups, workspace)

STATS_NAMES = ("data", "max_error", "scaled_sum", "objective", "penalty", "lr", "weight_sum")


@dataclass
class AmsgradOpts:
    """Optimiser settings; defaults are the paper's (Sec. 4.5) and Adam's
    customary moments."""
    lr_min: float = 1.5e-3
    lr_max: float = 1.5e-2
    lr_decay: float = 0.999
    half_period: int = 50
    steps_per_epoch: int = 1
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    penalty: float = 1e3

    def to_c(self):
        return L.DmnAmsgradOpts(self.lr_min, self.lr_max, self.lr_decay, self.half_period,
                                self.steps_per_epoch, self.beta1, self.beta2, self.eps,
                                self.penalty)


@dataclass
class TrainParams:
    """Device tensors of the trainable parameters and the optimiser state."""
    v: torch.Tensor
    alpha: torch.Tensor
    beta: torch.Tensor
    w: torch.Tensor
    n: torch.Tensor
    state: torch.Tensor
    step: torch.Tensor

    @classmethod
    def create(cls, v, alpha, beta):
        """Copies of v [2^K], alpha, beta [L] (one dtype, one device) with zero
        optimiser state; w and n are refreshed from them."""
        dev, dt = v.device, v.dtype
        K = int(round(torch.log2(torch.tensor(float(v.numel()))).item()))
        L_ = 2 ** K - 1
        p = cls(v.detach().clone().contiguous(), alpha.detach().clone().contiguous(),
                beta.detach().clone().contiguous(),
                torch.empty(2 ** K, dtype=dt, device=dev), torch.empty((L_, 3), dtype=dt,
                                                                       device=dev),
                torch.zeros((3, 2 ** K + 2 * L_), dtype=dt, device=dev),
                torch.zeros(1, dtype=torch.int64, device=dev))
        dmn_training_refresh(p)
        return p

    @property
    def depth(self):
        return int(round(torch.log2(torch.tensor(float(self.v.numel()))).item()))

    def to_c(self):
        K = self.depth
        if 2 ** K != self.v.numel() or not 1 <= K <= 10:
            raise ValueError("v must hold 2^K weights with 1 <= K <= 10")
        dt, L_ = self.v.dtype, 2 ** K - 1
        _need(self.v, "v", dt, (2 ** K,))
        _need(self.alpha, "alpha", dt, (L_,))
        _need(self.beta, "beta", dt, (L_,))
        _need(self.w, "w", dt, (2 ** K,))
        _need(self.n, "n", dt, (L_, 3))
        _need(self.state, "state", dt, (3, 2 ** K + 2 * L_))
        _need(self.step, "step", torch.int64, (1,))
        return L.DmnTrainParams(K, self.v.data_ptr(), self.alpha.data_ptr(),
                                self.beta.data_ptr(), self.w.data_ptr(), self.n.data_ptr(),
                                self.state.data_ptr(), self.step.data_ptr())


def new_stats(device) -> torch.Tensor:
    return torch.zeros(L.DMN_TRAIN_STATS, dtype=torch.float64, device=device)


def stats_dict(stats: torch.Tensor) -> dict:
    vals = stats.cpu().tolist()
    return {k: vals[i] for i, k in enumerate(STATS_NAMES)}


def dmn_training_loss(Cbar, target, p: float = 1.0, q: float = 10.0, gCbar=None, stats=None,
                      e=None, ws=None):
    """Data term of the objective (into stats[0..2]) and its cotangent gCbar."""
    dtype = Cbar.dtype
    if dtype not in _PREC:
        raise TypeError("float64 or float32 expected")
    B = Cbar.shape[0]
    _need(Cbar, "Cbar", dtype)
    _need(target, "target", dtype)
    if Cbar.numel() != 36 * B or target.numel() != 36 * B:
        raise ValueError("Cbar, target must be [B, 6, 6]")
    if gCbar is None:
        gCbar = torch.empty((B, 6, 6), dtype=dtype, device=Cbar.device)
    _need(gCbar, "gCbar", dtype)
    if stats is None:
        stats = new_stats(Cbar.device)
    _need(stats, "stats", torch.float64, (L.DMN_TRAIN_STATS,))
    if e is not None:
        _need(e, "e", dtype, (B,))
    lib = L.lib()
    nbytes = lib.dmn_training_loss_workspace_size(B)
    if ws is None or ws.numel() < nbytes:
        ws = workspace(nbytes, Cbar.device)
    opts = L.DmnLossOpts(float(p), float(q))
    rc = lib.dmn_training_loss(B, _PREC[dtype], _ptr(Cbar), _ptr(target), ctypes.byref(opts),
                               _ptr(e), _ptr(gCbar), _ptr(stats), _ptr(ws), ws.numel(),
                               _stream())
    L.check(rc, "dmn_training_loss")
    return gCbar, stats, ws


def dmn_training_update(params: TrainParams, gw, gn, opts: Optional[AmsgradOpts] = None,
                        stats=None):
    """One AMSGrad step on params from the linear map's VJP (gw, gn)."""
    dt = params.v.dtype
    K = params.depth
    _need(gw, "gw", dt, (2 ** K,))
    _need(gn, "gn", dt, (2 ** K - 1, 3))
    if stats is None:
        stats = new_stats(params.v.device)
    _need(stats, "stats", torch.float64, (L.DMN_TRAIN_STATS,))
    o = (opts or AmsgradOpts()).to_c()
    rc = L.lib().dmn_training_update(ctypes.byref(params.to_c()), _PREC[dt], _ptr(gw), _ptr(gn),
                                     ctypes.byref(o), _ptr(stats), _stream())
    L.check(rc, "dmn_training_update")
    return stats


def dmn_training_refresh(params: TrainParams):
    """w = <v>_+ and n(alpha, beta) without a step."""
    rc = L.lib().dmn_training_refresh(ctypes.byref(params.to_c()), _PREC[params.v.dtype],
                                      _stream())
    L.check(rc, "dmn_training_refresh")


def dmn_sample_stiffness(u, dtype=torch.float64):
    """Phase stiffness pairs (C1, C2) [B, 6, 6] from unit-cube points u [B, 8]
    (float64, device)."""
    _need(u, "u", torch.float64)
    if u.dim() != 2 or u.shape[1] != 8:
        raise ValueError("u must be [B, 8]")
    if dtype not in _PREC:
        raise TypeError("float64 or float32 expected")
    B = u.shape[0]
    C1 = torch.empty((B, 6, 6), dtype=dtype, device=u.device)
    C2 = torch.empty((B, 6, 6), dtype=dtype, device=u.device)
    rc = L.lib().dmn_sample_stiffness(B, _PREC[dtype], _ptr(u), _ptr(C1), _ptr(C2), _stream())
    L.check(rc, "dmn_sample_stiffness")
    return C1, C2


class TrainingStepGraph:
    """One training step (forward, objective, backward, update) as a HIP graph.

    ``C1``, ``C2`` and ``target`` are read at replay time from the tensors
    given here (refill them in place to change the batch); ``params`` are
    updated in place on every replay and ``stats`` receives the objective of
    the parameters the step started from."""

    def __init__(self, params: TrainParams, C1, C2, target, p: float = 1.0, q: float = 10.0,
                 opts: Optional[AmsgradOpts] = None):
        self.params, self.C1, self.C2, self.target = params, C1, C2, target
        self.p, self.q, self.opts = p, q, opts or AmsgradOpts()
        dev, dt = C1.device, C1.dtype
        B = C1.shape[0]
        self.Cbar = torch.empty((B, 6, 6), dtype=dt, device=dev)
        self.gCbar = torch.empty((B, 6, 6), dtype=dt, device=dev)
        self.stats = new_stats(dev)
        # workspaces sized outside the capture
        _, self.ws_fwd = dmn_homogenize_linear(params.w, params.n, C1, C2, Cbar=self.Cbar)
        _, _, self.ws_loss = dmn_training_loss(self.Cbar, target, p, q, gCbar=self.gCbar,
                                               stats=self.stats)
        self.ws_bwd = dmn_homogenize_backward(params.w, params.n, C1, C2, self.gCbar)[-1]
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        stream = torch.cuda.Stream(device=dev)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=stream):
            self._enqueue()
        torch.cuda.current_stream().wait_stream(stream)

    def _enqueue(self):
        P = self.params
        dmn_homogenize_linear(P.w, P.n, self.C1, self.C2, Cbar=self.Cbar, ws=self.ws_fwd)
        dmn_training_loss(self.Cbar, self.target, self.p, self.q, gCbar=self.gCbar,
                          stats=self.stats, ws=self.ws_loss)
        self.gw, self.gn, _, _, _ = dmn_homogenize_backward(P.w, P.n, self.C1, self.C2,
                                                            self.gCbar, ws=self.ws_bwd)
        dmn_training_update(P, self.gw, self.gn, self.opts, self.stats)

    def replay(self):
        """Enqueue one training step on the current stream."""
        self.graph.replay()

    def step_eager(self):
        """The same step without the graph (for comparisons)."""
        self._enqueue()


# ---------------------------------------------------------------- orientation groups

@dataclass
class OrientedTrainParams:
    """Device tensors of an orientation-interpolated DMN's trainable parameters
    (weights v, angle coefficients p, q [L, M]) and optimiser state."""
    kind: str
    v: torch.Tensor
    p: torch.Tensor
    q: torch.Tensor
    w: torch.Tensor
    state: torch.Tensor
    step: torch.Tensor

    @classmethod
    def create(cls, kind, v, p, q):
        if kind not in L.ORI_COUNT:
            raise ValueError(f"unknown shape functions {kind!r}")
        dev, dt = v.device, v.dtype
        NL = v.numel()
        LM = p.numel()
        prm = cls(kind, v.detach().clone().contiguous(), p.detach().clone().contiguous(),
                  q.detach().clone().contiguous(), torch.empty(NL, dtype=dt, device=dev),
                  torch.zeros((3, NL + 2 * LM), dtype=dt, device=dev),
                  torch.zeros(1, dtype=torch.int64, device=dev))
        rc = L.lib().dmn_training_refresh_oriented(ctypes.byref(prm.to_c()), _PREC[dt], _stream())
        L.check(rc, "dmn_training_refresh_oriented")
        return prm

    @property
    def depth(self):
        return int(round(torch.log2(torch.tensor(float(self.v.numel()))).item()))

    @property
    def m(self):
        return L.ORI_COUNT[self.kind]

    def to_c(self):
        K, dt = self.depth, self.v.dtype
        if 2 ** K != self.v.numel() or not 1 <= K <= 10:
            raise ValueError("v must hold 2^K weights with 1 <= K <= 10")
        Lm, M = 2 ** K - 1, self.m
        _need(self.v, "v", dt, (2 ** K,))
        _need(self.p, "p", dt, (Lm, M))
        _need(self.q, "q", dt, (Lm, M))
        _need(self.w, "w", dt, (2 ** K,))
        _need(self.state, "state", dt, (3, 2 ** K + 2 * Lm * M))
        _need(self.step, "step", torch.int64, (1,))
        return L.DmnTrainParamsOriented(K, L.DMN_ORI[self.kind], self.v.data_ptr(),
                                        self.p.data_ptr(), self.q.data_ptr(), self.w.data_ptr(),
                                        self.state.data_ptr(), self.step.data_ptr())


def dmn_orientation_group_normals(params: OrientedTrainParams, lam, n=None):
    """Normals [G, L, 3] of the orientations lam [G, 2]."""
    dt, K = params.v.dtype, params.depth
    G = lam.shape[0]
    _need(lam, "lam", dt, (G, 2))
    if n is None:
        n = torch.empty((G, 2 ** K - 1, 3), dtype=dt, device=lam.device)
    _need(n, "n", dt, (G, 2 ** K - 1, 3))
    rc = L.lib().dmn_orientation_group_normals(K, L.DMN_ORI[params.kind], G, _PREC[dt],
                                               _ptr(params.p), _ptr(params.q), _ptr(lam),
                                               _ptr(n), _stream())
    L.check(rc, "dmn_orientation_group_normals")
    return n


def dmn_orientation_group_chain(params: OrientedTrainParams, lam, gw_groups, gn_groups,
                                gw=None, gpq=None):
    """(gw [2^K], gpq [L, 2, M]) from the groups' VJPs [G, 2^K], [G, L, 3]."""
    dt, K, M = params.v.dtype, params.depth, params.m
    G = lam.shape[0]
    _need(gw_groups, "gw_groups", dt, (G, 2 ** K))
    _need(gn_groups, "gn_groups", dt, (G, 2 ** K - 1, 3))
    if gw is None:
        gw = torch.empty(2 ** K, dtype=dt, device=lam.device)
    if gpq is None:
        gpq = torch.empty((2 ** K - 1, 2, M), dtype=dt, device=lam.device)
    rc = L.lib().dmn_orientation_group_chain(K, L.DMN_ORI[params.kind], G, _PREC[dt],
                                             _ptr(params.p), _ptr(params.q), _ptr(lam),
                                             _ptr(gw_groups), _ptr(gn_groups), _ptr(gw),
                                             _ptr(gpq), _stream())
    L.check(rc, "dmn_orientation_group_chain")
    return gw, gpq


def dmn_training_update_oriented(params: OrientedTrainParams, gw, gpq,
                                 opts: Optional[AmsgradOpts] = None, stats=None):
    dt, K = params.v.dtype, params.depth
    _need(gw, "gw", dt, (2 ** K,))
    _need(gpq, "gpq", dt, (2 ** K - 1, 2, params.m))
    if stats is None:
        stats = new_stats(params.v.device)
    o = (opts or AmsgradOpts()).to_c()
    rc = L.lib().dmn_training_update_oriented(ctypes.byref(params.to_c()), _PREC[dt], _ptr(gw),
                                              _ptr(gpq), ctypes.byref(o), _ptr(stats), _stream())
    L.check(rc, "dmn_training_update_oriented")
    return stats


class OrientedTrainingStepGraph:
    """One training step of an orientation-interpolated DMN over a batch
    grouped by orientation (samples offsets[k]:offsets[k+1] have orientation
    lam[k]) as a HIP graph: group normals, the fixed-normal linear map of
    every group, the objective over the whole batch, the VJP of every group,
    the chain to (p, q) and the AMSGrad update.

    ``grouped``: all groups in one call each for the map and its VJP
    (dmn_homogenize_linear_groups / dmn_homogenize_backward_groups);
    otherwise one call per group, spread over ``streams`` streams."""

    def __init__(self, params: OrientedTrainParams, C1, C2, target, lam, offsets,
                 p: float = 1.0, q: float = 10.0, opts: Optional[AmsgradOpts] = None,
                 streams: int = 4, grouped: bool = True):
        self.params, self.C1, self.C2, self.target, self.lam = params, C1, C2, target, lam
        self.grouped = grouped
        # per-group calls are independent: spread them over a few streams
        # (default priority) that fork from and join the main stream
        self.side = [] if grouped else [torch.cuda.Stream(device=C1.device)
                                        for _ in range(max(0, streams - 1))]
        self.offsets = [int(x) for x in offsets]
        self.p, self.q, self.opts = p, q, opts or AmsgradOpts()
        dev, dt = C1.device, C1.dtype
        B, G, K = C1.shape[0], lam.shape[0], params.depth
        if len(self.offsets) != G + 1 or self.offsets[0] != 0 or self.offsets[-1] != B:
            raise ValueError("offsets must split the batch into one range per orientation")
        self.Cbar = torch.empty((B, 6, 6), dtype=dt, device=dev)
        self.gCbar = torch.empty((B, 6, 6), dtype=dt, device=dev)
        self.stats = new_stats(dev)
        self.n_groups = torch.empty((G, 2 ** K - 1, 3), dtype=dt, device=dev)
        self.gw_groups = torch.empty((G, 2 ** K), dtype=dt, device=dev)
        self.gn_groups = torch.empty((G, 2 ** K - 1, 3), dtype=dt, device=dev)
        self.gw = torch.empty(2 ** K, dtype=dt, device=dev)
        self.gpq = torch.empty((2 ** K - 1, 2, params.m), dtype=dt, device=dev)
        self.ws_fwd, self.ws_bwd = [None] * G, [None] * G
        self.ws_gfwd = self.ws_gbwd = None
        self._enqueue(sizing=True)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        stream = torch.cuda.Stream(device=dev)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=stream):
            self._enqueue()
        torch.cuda.current_stream().wait_stream(stream)

    def _fan_out(self, fn):
        """Run fn(k) for every group, group k on stream k mod (1 + side streams)."""
        main = torch.cuda.current_stream()
        lanes = [main] + self.side
        for st in self.side:
            st.wait_stream(main)
        for k in range(len(self.offsets) - 1):
            with torch.cuda.stream(lanes[k % len(lanes)]):
                fn(k)
        for st in self.side:
            main.wait_stream(st)

    def _enqueue(self, sizing=False):
        P, o = self.params, self.offsets
        dmn_orientation_group_normals(P, self.lam, n=self.n_groups)

        def fwd(k):
            a, b = o[k], o[k + 1]
            _, self.ws_fwd[k] = dmn_homogenize_linear(P.w, self.n_groups[k], self.C1[a:b],
                                                      self.C2[a:b], Cbar=self.Cbar[a:b],
                                                      ws=self.ws_fwd[k])

        def bwd(k):
            a, b = o[k], o[k + 1]
            self.ws_bwd[k] = dmn_homogenize_backward(
                P.w, self.n_groups[k], self.C1[a:b], self.C2[a:b], self.gCbar[a:b],
                ws=self.ws_bwd[k], gw=self.gw_groups[k], gn=self.gn_groups[k])[-1]

        if self.grouped:
            _, self.ws_gfwd = dmn_homogenize_linear_groups(P.w, self.n_groups, o, self.C1,
                                                           self.C2, Cbar=self.Cbar,
                                                           ws=self.ws_gfwd)
        else:
            self._fan_out(fwd)
        _, _, ws = dmn_training_loss(self.Cbar, self.target, self.p, self.q, gCbar=self.gCbar,
                                     stats=self.stats, ws=None if sizing else self.ws_loss)
        self.ws_loss = ws
        if self.grouped:
            self.ws_gbwd = dmn_homogenize_backward_groups(
                P.w, self.n_groups, o, self.C1, self.C2, self.gCbar, gw_groups=self.gw_groups,
                gn_groups=self.gn_groups, ws=self.ws_gbwd)[-1]
        else:
            self._fan_out(bwd)
        dmn_orientation_group_chain(P, self.lam, self.gw_groups, self.gn_groups, gw=self.gw,
                                    gpq=self.gpq)
        if not sizing:
            dmn_training_update_oriented(P, self.gw, self.gpq, self.opts, self.stats)

    def replay(self):
        """Enqueue one training step on the current stream."""
        self.graph.replay()

    def step_eager(self):
        self._enqueue()

    def error_words(self):
        """Device error words of the linear maps and VJPs (synchronises)."""
        from .api import error_word
        if self.grouped:
            return [error_word(self.ws_gfwd), error_word(self.ws_gbwd)]
        return [error_word(w) for w in self.ws_fwd + self.ws_bwd]
