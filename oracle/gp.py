"""Online evaluation of a direct DMN at one Gauss point (Sec. 3.2, Sec. 4.6).

Given the macro strain E of the new step, the internal variables z^n of the
last converged step and the stored jumps a^n (the initial guess, Sec. 6), the
Euler-Lagrange equation  A^T W sigma(E + A a, z^n) = 0  is solved for the
jumps a by Newton's method with the explicit Hessian H = A^T W D A and a
dense Cholesky factorisation (LAPACK), followed by the effective stress
sigma = sum_j w~_j sigma_j and the algorithmic tangent
C = [I..I]^T W (D_E + D A dA/dE) with H dA/dE = -A^T W D B.

Readings of what the paper leaves open:
* weights are normalised, w~ = w / sum(w), both in W and in the averages;
* stopping test of Sec. 4.6 with norms in Mandel l2 (Frobenius):
  |A^T W sigma| <= tol (2^K - 1) |sigma_bar|; a zero residual counts as
  converged;
* backtracking (Sec. 3.2 only says a step below one may arise): start with
  s = 1, halve while the trial residual is non-finite or
  |r(a + s da)| > (1 - armijo s) |r(a)|, at most max_backtrack halvings; after
  the last halving a finite trial is accepted as it is;
* the tangent uses D and H at the converged jumps;
* on any failure the returned state is the input state (z^n, a^n) so a
  caller can retry the increment.

Status codes: 0 converged, 1 iteration limit, 2 non-finite residual,
3 Hessian not positive definite, 4 J2 return did not converge,
5 invalid DMN parameter (negative weight or a laminate whose children carry
zero total weight).
"""
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .j2 import LOCAL_MAXIT, J2Material, j2_update
from .mandel import iso_from_E_nu
from .tree import gradient_operator, lam_leaves, laminates

OK, MAXITER, NONFINITE, NOTSPD, LOCALFAIL, BADPARAM = 0, 1, 2, 3, 4, 5


@dataclass
class NewtonOptions:
    tol: float = 1e-10
    max_iter: int = 25
    max_backtrack: int = 10
    armijo: float = 1e-4
    # extra full Newton steps after the stop test is met (complex-step runs: the
    # imaginary part of an iterate is the derivative at the previous iterate, so
    # one more step makes it the derivative at the converged jumps)
    polish: int = 0
    # cap of the scalar Newton iterations of the J2 return at each matrix leaf
    local_max_iter: int = LOCAL_MAXIT


class DmnModel:
    """A depth-K DMN with its phase laws, holding the explicit gradient operator.

    Weights and normals may be complex (complex-step differentiation): every
    decision is then taken on real parts and linear systems are solved without
    conjugation."""

    def __init__(self, K, w, normals, fiber, matrix):
        self.K = K
        self.nL = 2 ** K
        self.L = 2 ** K - 1
        self.w = np.asarray(w)
        self.normals = np.asarray(normals)
        self.dtype = np.result_type(self.w, self.normals, 1.0)
        self.valid = bool(np.all(np.real(self.w) >= 0.0))
        for (k, i) in laminates(K):
            lo, hi = lam_leaves(K, k, i)
            if not np.real(self.w[lo:hi].sum()) > 0.0:
                self.valid = False
        self.wt = self.w / self.w.sum() if self.valid else None
        self.A = gradient_operator(K, self.w, self.normals) if self.valid else None
        self.Cf = iso_from_E_nu(fiber["E"], fiber["nu"])
        self.mat = J2Material(**matrix)
        self.B = np.tile(np.eye(6), (self.nL, 1))

    def evaluate(self, E, z_n, a, local_max_iter=LOCAL_MAXIT):
        """Leaf strains, stresses, tangents and the residual at jumps a."""
        eps = E[None, :] + (self.A @ a).reshape(self.nL, 6)
        dt = np.result_type(self.dtype, eps, z_n)
        sig = np.zeros((self.nL, 6), dtype=dt)
        D = np.zeros((self.nL, 6, 6), dtype=dt)
        z = np.array(z_n, dtype=dt, copy=True)
        margin = np.inf
        local_ok = True
        for j in range(self.nL):
            if j % 2 == 0:
                sig[j] = self.Cf @ eps[j]
                D[j] = self.Cf
            else:
                m = j // 2
                out = j2_update(self.mat, eps[j], z_n[m, :6], z_n[m, 6], local_max_iter)
                sig[j], D[j] = out["sigma"], out["D"]
                z[m, :6], z[m, 6] = out["ep"], out["p"]
                margin = min(margin, abs(out["margin"]))
                local_ok &= out["ok"]
        wsig = self.wt[:, None] * sig
        r = self.A.T @ wsig.ravel()
        sbar = wsig.sum(axis=0)
        return dict(eps=eps, sig=sig, D=D, z=z, r=r, sbar=sbar, margin=margin,
                    local_ok=local_ok)

    def hessian(self, D):
        WD = sp.block_diag([self.wt[j] * D[j] for j in range(self.nL)], format="csr")
        H = (self.A.T @ (WD @ self.A)).toarray()
        return H, WD

    def solve(self, H, rhs):
        """H^-1 rhs with a Cholesky factorisation of (the real part of) H; raises
        LinAlgError when H is not positive definite.  Complex H (complex step) is
        solved by LU without conjugation."""
        cho = sla.cho_factor(np.real(H), lower=True)
        if np.iscomplexobj(H) or np.iscomplexobj(rhs):
            return np.linalg.solve(H, rhs)
        return sla.cho_solve(cho, rhs)

    def tangent(self, D):
        """Algorithmic tangent of Sec. 3.2 at the given leaf tangents."""
        H, WD = self.hessian(D)
        rhs = -(self.A.T @ (WD @ self.B))
        X = self.solve(H, rhs)
        return self.B.T @ (WD @ (self.B + self.A @ X))


def _finite(ev):
    return bool(np.all(np.isfinite(ev["r"])) and np.all(np.isfinite(ev["sbar"])))


def gp_update(model: DmnModel, E, z_n, a_n, opts: NewtonOptions = NewtonOptions()):
    """Newton solve of the DMN Euler-Lagrange equation at one Gauss point.

    E: [6] macro strain; z_n: [M, 7] internal variables of the M = 2^(K-1)
    matrix leaves (plastic strain in Mandel, then p); a_n: [3L] jumps in
    paper order.  Returns dict(sigma, C, z, a, iters, status, margin).
    """
    E = np.asarray(E)
    z_n = np.asarray(z_n)
    a_n = np.asarray(a_n)
    fail = dict(sigma=np.full(6, np.nan), C=np.full((6, 6), np.nan), z=z_n.copy(),
                a=a_n.copy(), iters=0, margin=np.inf)
    if not model.valid:
        return dict(fail, status=BADPARAM)
    if not (np.all(np.isfinite(E)) and np.all(np.isfinite(z_n)) and np.all(np.isfinite(a_n))):
        return dict(fail, status=NONFINITE)
    scale = opts.tol * model.L
    a = a_n.copy()
    ev = model.evaluate(E, z_n, a, opts.local_max_iter)
    margin = ev["margin"]
    iters = 0
    status = OK
    polish = opts.polish
    while True:
        if not ev["local_ok"]:
            status = LOCALFAIL
            break
        if not _finite(ev):
            status = NONFINITE
            break
        rn = np.linalg.norm(ev["r"])
        if rn == 0.0 or rn <= scale * np.linalg.norm(ev["sbar"]):
            if polish == 0:
                break
            polish -= 1
            H, _ = model.hessian(ev["D"])
            a = a - model.solve(H, ev["r"])
            ev = model.evaluate(E, z_n, a, opts.local_max_iter)
            continue
        if iters == opts.max_iter:
            status = MAXITER
            break
        H, _ = model.hessian(ev["D"])
        try:
            da = -model.solve(H, ev["r"])
        except np.linalg.LinAlgError:
            status = NOTSPD
            break
        s = 1.0
        for bt in range(opts.max_backtrack + 1):
            trial = model.evaluate(E, z_n, a + s * da, opts.local_max_iter)
            margin = min(margin, trial["margin"])
            good = _finite(trial) and trial["local_ok"]
            if good and np.linalg.norm(trial["r"]) <= (1.0 - opts.armijo * s) * rn:
                break
            if bt < opts.max_backtrack:
                s *= 0.5
        a = a + s * da
        ev = trial
        iters += 1
    if status != OK:
        return dict(fail, sigma=ev["sbar"], iters=iters, status=status, margin=margin)
    try:
        C = model.tangent(ev["D"])
    except np.linalg.LinAlgError:
        return dict(fail, sigma=ev["sbar"], iters=iters, status=NOTSPD, margin=margin)
    return dict(sigma=ev["sbar"], C=C, z=ev["z"], a=a, iters=iters, status=OK,
                margin=margin, eps=ev["eps"], sig_leaf=ev["sig"])


def run_path(model, E_path, opts=NewtonOptions(), z0=None, a0=None):
    """Apply a macro strain path E_path [T, 6] from the initial state z = 0, a = 0."""
    M = model.nL // 2
    z = np.zeros((M, 7), dtype=model.dtype) if z0 is None else z0
    a = np.zeros(3 * model.L, dtype=model.dtype) if a0 is None else a0
    outs = []
    for E in E_path:
        out = gp_update(model, E, z, a, opts)
        outs.append(out)
        if out["status"] != OK:
            break
        z, a = out["z"], out["a"]
    return outs
