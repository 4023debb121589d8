"""Python binding of libdmn with the C ABI's names (argument marshalling only).

Every function takes torch tensors that already live on the GPU, checks
their dtypes, shapes and contiguity, and enqueues the library call on the
current HIP stream.  No computation happens here.
"""
import ctypes
from dataclasses import dataclass
from typing import List, Optional

import torch

from . import _lib as L

_PREC = {torch.float64: L.DMN_F64, torch.float32: L.DMN_F32}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t: torch.Tensor, name: str, dtype, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _net(w: torch.Tensor, n: torch.Tensor, dtype):
    K = int(round(torch.log2(torch.tensor(float(w.numel()))).item()))
    if 2 ** K != w.numel() or not 1 <= K <= 10:
        raise ValueError("w must hold 2^K leaf weights with 1 <= K <= 10")
    _need(w, "w", dtype, (2 ** K,))
    _need(n, "n", dtype, (2 ** K - 1, 3))
    return L.DmnNet(K, w.data_ptr(), n.data_ptr()), K


def _net_ori(w: torch.Tensor, ori: "Orientation", dtype=torch.float64):
    """dmn_net with orientation-interpolated normals (arrays in dtype)."""
    K = int(round(torch.log2(torch.tensor(float(w.numel()))).item()))
    if 2 ** K != w.numel() or not 1 <= K <= 10:
        raise ValueError("w must hold 2^K leaf weights with 1 <= K <= 10")
    if ori.kind not in L.ORI_COUNT:
        raise ValueError(f"unknown shape functions {ori.kind!r}")
    M = L.ORI_COUNT[ori.kind]
    _need(w, "w", dtype, (2 ** K,))
    _need(ori.p, "p", dtype, (2 ** K - 1, M))
    _need(ori.q, "q", dtype, (2 ** K - 1, M))
    return L.DmnNet(K, w.data_ptr(), None, L.DMN_ORI[ori.kind], ori.p.data_ptr(),
                    ori.q.data_ptr()), K


def workspace(nbytes: int, device) -> torch.Tensor:
    """Device workspace (torch's allocator returns 512-byte aligned blocks)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def error_word(ws: torch.Tensor) -> int:
    """Device error word of a linear / backward call (synchronises on read)."""
    return int(ws[:4].view(torch.int32).item())


def _linear_net(w, n, ori, dtype, B):
    """dmn_net and lam pointer of a linear call (fixed or per-sample normals)."""
    if ori is None:
        net, K = _net(w, n, dtype)
        return net, K, None
    net, K = _net_ori(w, ori, dtype)
    _need(ori.lam, "lam", dtype, (B, 2))
    return net, K, _ptr(ori.lam)


def dmn_homogenize_linear(w, n, C1, C2, Cbar=None, ws=None, ori=None):
    """Cbar[b] = DMN^L(C1[b], C2[b]) for a batch [B, 6, 6] (or [B, 36]).

    With ``ori`` (an Orientation whose lam is [B, 2]) every sample has its own
    fibre orientation and n is not read."""
    dtype = C1.dtype
    if dtype not in _PREC:
        raise TypeError("float64 or float32 expected")
    B = C1.shape[0]
    net, K, lam = _linear_net(w, n, ori, dtype, B)
    _need(C1, "C1", dtype)
    _need(C2, "C2", dtype)
    if C1.numel() != 36 * B or C2.numel() != 36 * B:
        raise ValueError("C1, C2 must be [B, 6, 6]")
    if Cbar is None:
        Cbar = torch.empty((B, 6, 6), dtype=dtype, device=C1.device)
    _need(Cbar, "Cbar", dtype)
    prec = _PREC[dtype]
    lib = L.lib()
    nbytes = lib.dmn_homogenize_linear_workspace_size(ctypes.byref(net), B, prec)
    if ws is None or ws.numel() < nbytes:
        ws = workspace(nbytes, C1.device)
    rc = lib.dmn_homogenize_linear(ctypes.byref(net), B, prec, _ptr(C1), _ptr(C2), lam,
                                   _ptr(Cbar), _ptr(ws), ws.numel(), _stream())
    L.check(rc, "dmn_homogenize_linear")
    return Cbar, ws


def dmn_homogenize_backward(w, n, C1, C2, gCbar, want_input_grads=False, ws=None, ori=None,
                            gw=None, gn=None):
    """(gw, gn, gC1, gC2) of sum_b <gCbar[b], Cbar[b]>; gC1/gC2 None unless requested.

    With ``ori`` gn is [L, 2, M]: the cotangents of the angle coefficients p
    (first) and q of every laminate, summed over the samples.  ``gw``, ``gn``
    may be given as output tensors (e.g. rows of a per-group stack)."""
    dtype = C1.dtype
    B = C1.shape[0]
    net, K, lam = _linear_net(w, n, ori, dtype, B)
    for t, nm in ((C1, "C1"), (C2, "C2"), (gCbar, "gCbar")):
        _need(t, nm, dtype)
        if t.numel() != 36 * B:
            raise ValueError(f"{nm} must be [B, 6, 6]")
    gn_shape = (2 ** K - 1, 3) if ori is None else (2 ** K - 1, 2, L.ORI_COUNT[ori.kind])
    if gw is None:
        gw = torch.empty(2 ** K, dtype=dtype, device=C1.device)
    if gn is None:
        gn = torch.empty(gn_shape, dtype=dtype, device=C1.device)
    _need(gw, "gw", dtype, (2 ** K,))
    _need(gn, "gn", dtype, gn_shape)
    gC1 = gC2 = None
    if want_input_grads:
        gC1 = torch.empty((B, 6, 6), dtype=dtype, device=C1.device)
        gC2 = torch.empty((B, 6, 6), dtype=dtype, device=C1.device)
    prec = _PREC[dtype]
    lib = L.lib()
    nbytes = lib.dmn_homogenize_backward_workspace_size(ctypes.byref(net), B, prec)
    if ws is None or ws.numel() < nbytes:
        ws = workspace(nbytes, C1.device)
    rc = lib.dmn_homogenize_backward(ctypes.byref(net), B, prec, _ptr(C1), _ptr(C2), lam,
                                     _ptr(gCbar), _ptr(gw), _ptr(gn), _ptr(gC1), _ptr(gC2),
                                     _ptr(ws), ws.numel(), _stream())
    L.check(rc, "dmn_homogenize_backward")
    return gw, gn, gC1, gC2, ws


def _group_offsets(offsets, G: int, B: int):
    """Host int64 array of the G + 1 sample offsets of a grouped call."""
    off = [int(x) for x in offsets]
    if len(off) != G + 1 or off[0] != 0 or off[-1] != B or any(
            b < a for a, b in zip(off, off[1:])):
        raise ValueError("offsets must split the batch into one range per group")
    return (ctypes.c_int64 * (G + 1))(*off)


def _groups_args(w, n_groups, offsets, C1, tensors):
    dtype = C1.dtype
    if dtype not in _PREC:
        raise TypeError("float64 or float32 expected")
    K = int(round(torch.log2(torch.tensor(float(w.numel()))).item()))
    if 2 ** K != w.numel() or not 1 <= K <= 10:
        raise ValueError("w must hold 2^K leaf weights with 1 <= K <= 10")
    if n_groups.dim() != 3 or n_groups.shape[1:] != (2 ** K - 1, 3) or n_groups.shape[0] < 1:
        raise ValueError("n_groups must be [G, 2^K - 1, 3]")
    G, B = n_groups.shape[0], C1.shape[0]
    _need(w, "w", dtype, (2 ** K,))
    _need(n_groups, "n_groups", dtype)
    for t, nm in tensors:
        _need(t, nm, dtype)
        if t.numel() != 36 * B:
            raise ValueError(f"{nm} must be [B, 6, 6]")
    return K, G, B, _group_offsets(offsets, G, B), _PREC[dtype]


def dmn_homogenize_linear_groups(w, n_groups, offsets, C1, C2, Cbar=None, ws=None):
    """Linear map of G DMNs sharing w with normals n_groups [G, L, 3]; samples
    offsets[k]:offsets[k+1] of the batch belong to group k."""
    if Cbar is None:
        Cbar = torch.empty((C1.shape[0], 6, 6), dtype=C1.dtype, device=C1.device)
    K, G, B, off, prec = _groups_args(w, n_groups, offsets, C1,
                                      ((C1, "C1"), (C2, "C2"), (Cbar, "Cbar")))
    lib = L.lib()
    nbytes = lib.dmn_homogenize_linear_groups_workspace_size(K, G, prec)
    if ws is None or ws.numel() < nbytes:
        ws = workspace(nbytes, C1.device)
    rc = lib.dmn_homogenize_linear_groups(K, G, off, prec, _ptr(w), _ptr(n_groups), _ptr(C1),
                                          _ptr(C2), _ptr(Cbar), _ptr(ws), ws.numel(), _stream())
    L.check(rc, "dmn_homogenize_linear_groups")
    return Cbar, ws


def dmn_homogenize_backward_groups(w, n_groups, offsets, C1, C2, gCbar, gw_groups=None,
                                   gn_groups=None, ws=None):
    """(gw_groups [G, 2^K], gn_groups [G, L, 3], ws): group k's rows are the
    VJP of its samples at normals n_groups[k]."""
    K, G, B, off, prec = _groups_args(w, n_groups, offsets, C1,
                                      ((C1, "C1"), (C2, "C2"), (gCbar, "gCbar")))
    if gw_groups is None:
        gw_groups = torch.empty((G, 2 ** K), dtype=C1.dtype, device=C1.device)
    if gn_groups is None:
        gn_groups = torch.empty((G, 2 ** K - 1, 3), dtype=C1.dtype, device=C1.device)
    _need(gw_groups, "gw_groups", C1.dtype, (G, 2 ** K))
    _need(gn_groups, "gn_groups", C1.dtype, (G, 2 ** K - 1, 3))
    lib = L.lib()
    nbytes = lib.dmn_homogenize_backward_groups_workspace_size(K, G, off, prec)
    if ws is None or ws.numel() < nbytes:
        ws = workspace(nbytes, C1.device)
    rc = lib.dmn_homogenize_backward_groups(K, G, off, prec, _ptr(w), _ptr(n_groups), _ptr(C1),
                                            _ptr(C2), _ptr(gCbar), _ptr(gw_groups),
                                            _ptr(gn_groups), _ptr(ws), ws.numel(), _stream())
    L.check(rc, "dmn_homogenize_backward_groups")
    return gw_groups, gn_groups, ws


@dataclass
class Orientation:
    """Normals interpolated over the fibre orientation triangle: shape-function
    family ("linear", "trilinear", "quadratic"), angle coefficients p, q
    [L, M] (float64, device) and per-point (l1, l2) lam [P, 2]."""
    kind: str
    p: torch.Tensor
    q: torch.Tensor
    lam: torch.Tensor


@dataclass
class PointGroup:
    """Device arrays of one batch of Gauss points sharing a DMN (see include/dmn.h).

    With ``ori`` set the normals follow each point's fibre orientation and
    ``n`` is not read (it may be None)."""
    w: torch.Tensor
    n: Optional[torch.Tensor]
    E: torch.Tensor
    z_in: torch.Tensor
    z_out: torch.Tensor
    a_in: torch.Tensor
    a_out: torch.Tensor
    sigma: torch.Tensor
    tangent: torch.Tensor
    iters: torch.Tensor
    status: torch.Tensor
    ori: Optional[Orientation] = None

    @staticmethod
    def allocate(w, n, E, z_in=None, a_in=None, ori=None):
        """Outputs (and zero initial state if not given) for the points of E [P, 6].

        The per-point arrays take E's dtype (float64; float32 maps to
        DMN_F32_STATE: FP32 state, FP64 arithmetic); w and n are float64."""
        K = int(round(torch.log2(torch.tensor(float(w.numel()))).item()))
        P = E.shape[0]
        dev, dt = E.device, E.dtype
        M, Lm = 2 ** (K - 1), 2 ** K - 1
        if z_in is None:
            z_in = torch.zeros((P, M, 7), dtype=dt, device=dev)
        if a_in is None:
            a_in = torch.zeros((P, Lm, 3), dtype=dt, device=dev)
        return PointGroup(w, n, E, z_in, torch.empty_like(z_in), a_in, torch.empty_like(a_in),
                          torch.empty((P, 6), dtype=dt, device=dev),
                          torch.empty((P, 6, 6), dtype=dt, device=dev),
                          torch.empty(P, dtype=torch.int32, device=dev),
                          torch.empty(P, dtype=torch.int32, device=dev), ori)

    def advance(self):
        """Make the outputs the next step's inputs (swap the state buffers)."""
        self.z_in, self.z_out = self.z_out, self.z_in
        self.a_in, self.a_out = self.a_out, self.a_in

    @property
    def prec(self):
        """DMN_F64 for float64 per-point arrays, DMN_F32_STATE for float32."""
        if self.E.dtype == torch.float64:
            return L.DMN_F64
        if self.E.dtype == torch.float32:
            return L.DMN_F32_STATE
        raise TypeError(f"E must be float64 or float32, got {self.E.dtype}")

    def to_c(self):
        if self.ori is None:
            net, K = _net(self.w, self.n, torch.float64)
        else:
            net, K = _net_ori(self.w, self.ori)
        P = self.E.shape[0]
        M, Lm = 2 ** (K - 1), 2 ** K - 1
        dt = self.E.dtype
        self.prec  # dtype check
        _need(self.E, "E", dt, (P, 6))
        for t, nm in ((self.z_in, "z_in"), (self.z_out, "z_out")):
            _need(t, nm, dt, (P, M, 7))
        for t, nm in ((self.a_in, "a_in"), (self.a_out, "a_out")):
            _need(t, nm, dt, (P, Lm, 3))
        _need(self.sigma, "sigma", dt, (P, 6))
        _need(self.tangent, "tangent", dt)
        if self.tangent.numel() != 36 * P:
            raise ValueError("tangent must be [P, 6, 6]")
        _need(self.iters, "iters", torch.int32, (P,))
        _need(self.status, "status", torch.int32, (P,))
        lam = None
        if self.ori is not None:
            _need(self.ori.lam, "lam", torch.float64, (P, 2))
            lam = self.ori.lam.data_ptr()
        return L.DmnPointGroup(net, P, self.E.data_ptr(), self.z_in.data_ptr(),
                               self.z_out.data_ptr(), self.a_in.data_ptr(), self.a_out.data_ptr(),
                               self.sigma.data_ptr(), self.tangent.data_ptr(),
                               self.iters.data_ptr(), self.status.data_ptr(), lam)


def _materials(fiber: dict, matrix: dict):
    return (L.DmnElastic(fiber["E"], fiber["nu"]),
            L.DmnJ2(matrix["E"], matrix["nu"], matrix["sigma0"], matrix["k_inf"],
                    matrix["dsigma"], matrix["b"]))


def dmn_update_gauss_points(groups: List[PointGroup], fiber: dict, matrix: dict, tol=1e-10,
                            max_iter=25, max_backtrack=10, armijo=1e-4, ws=None,
                            local_max_iter=0, polish=0):
    """One load step at every point of every group (outputs written in place).

    All groups hold their per-point arrays in one dtype: float64 (DMN_F64);
    float32 maps to DMN_F32_STATE (FP32 storage of the per-point arrays, FP64
    arithmetic on FP64 copies in the workspace)."""
    precs = {g.prec for g in groups}
    if len(precs) != 1:
        raise TypeError("all groups of one call must use the same per-point dtype")
    prec = precs.pop()
    arr = (L.DmnPointGroup * len(groups))(*[g.to_c() for g in groups])
    fib, mat = _materials(fiber, matrix)
    opts = L.DmnNewtonOpts(tol, max_iter, max_backtrack, armijo, local_max_iter, polish)
    lib = L.lib()
    nbytes = lib.dmn_update_gauss_points_workspace_size(arr, len(groups), prec)
    if nbytes == 0:
        raise L.DmnError("dmn_update_gauss_points_workspace_size rejected the groups")
    if ws is None or ws.numel() < nbytes:
        ws = workspace(nbytes, groups[0].E.device)
    rc = lib.dmn_update_gauss_points(arr, len(groups), ctypes.byref(fib), ctypes.byref(mat),
                                     prec, ctypes.byref(opts), _ptr(ws), ws.numel(),
                                     _stream())
    L.check(rc, "dmn_update_gauss_points")
    return ws


def dmn_update_gauss_points_noalloc(groups: List[PointGroup], fiber: dict, matrix: dict,
                                    tol=1e-10, max_iter=25, max_backtrack=10, armijo=1e-4,
                                    local_max_iter=0, polish=0):
    """dmn_update_gauss_points without a workspace argument: the library's
    static per-device array serves as workspace (include/dmn.h); no device
    memory is allocated by the call."""
    precs = {g.prec for g in groups}
    if len(precs) != 1:
        raise TypeError("all groups of one call must use the same per-point dtype")
    arr = (L.DmnPointGroup * len(groups))(*[g.to_c() for g in groups])
    fib, mat = _materials(fiber, matrix)
    opts = L.DmnNewtonOpts(tol, max_iter, max_backtrack, armijo, local_max_iter, polish)
    rc = L.lib().dmn_update_gauss_points_noalloc(arr, len(groups), ctypes.byref(fib),
                                                  ctypes.byref(mat), precs.pop(),
                                                  ctypes.byref(opts), _stream())
    L.check(rc, "dmn_update_gauss_points_noalloc")


@dataclass
class AdjointGroup:
    """Device arrays of one batch of points for dmn_update_adjoint (include/dmn.h)."""
    w: torch.Tensor
    n: torch.Tensor
    E: torch.Tensor
    z_in: torch.Tensor
    a_conv: torch.Tensor
    g_sigma: Optional[torch.Tensor]
    g_z_next: Optional[torch.Tensor]
    g_z_prev: torch.Tensor
    gw: torch.Tensor
    gn: torch.Tensor

    def to_c(self):
        net, K = _net(self.w, self.n, torch.float64)
        P = self.E.shape[0]
        M, Lm = 2 ** (K - 1), 2 ** K - 1
        _need(self.E, "E", torch.float64, (P, 6))
        _need(self.z_in, "z_in", torch.float64, (P, M, 7))
        _need(self.a_conv, "a_conv", torch.float64, (P, Lm, 3))
        _need(self.g_z_prev, "g_z_prev", torch.float64, (P, M, 7))
        if self.g_sigma is not None:
            _need(self.g_sigma, "g_sigma", torch.float64, (P, 6))
        if self.g_z_next is not None:
            _need(self.g_z_next, "g_z_next", torch.float64, (P, M, 7))
        _need(self.gw, "gw", torch.float64, (2 ** K,))
        _need(self.gn, "gn", torch.float64, (Lm, 3))
        ptr = lambda t: None if t is None else t.data_ptr()
        return L.DmnAdjointGroup(net, P, self.E.data_ptr(), self.z_in.data_ptr(),
                                 self.a_conv.data_ptr(), ptr(self.g_sigma), ptr(self.g_z_next),
                                 self.g_z_prev.data_ptr(), self.gw.data_ptr(), self.gn.data_ptr())


def dmn_update_adjoint(groups: List[AdjointGroup], fiber: dict, matrix: dict, ws=None):
    """Adjoint of one converged load step for every group; gw, gn accumulate (+=)."""
    arr = (L.DmnAdjointGroup * len(groups))(*[g.to_c() for g in groups])
    fib, mat = _materials(fiber, matrix)
    lib = L.lib()
    nbytes = lib.dmn_update_adjoint_workspace_size(arr, len(groups), L.DMN_F64)
    if nbytes == 0:
        raise L.DmnError("dmn_update_adjoint_workspace_size rejected the groups")
    if ws is None or ws.numel() < nbytes:
        ws = workspace(nbytes, groups[0].E.device)
    rc = lib.dmn_update_adjoint(arr, len(groups), ctypes.byref(fib), ctypes.byref(mat),
                                L.DMN_F64, _ptr(ws), ws.numel(), _stream())
    L.check(rc, "dmn_update_adjoint")
    return ws
