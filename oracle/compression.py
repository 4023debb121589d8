"""Tree compression of a direct DMN (Sec. 3.1).  Test infrastructure like the
rest of the oracle.

During training some leaf weights reach zero and stay there; the paper then
removes such subtrees from the binary tree: a leaf without weight is deleted,
a laminate left with a single child is replaced by that child, and a subtree
without any weight disappears.  The linear map of the compressed tree is
evaluated here with the same laminate formula (Milton's, Sec. 3.1) over the
laminates that remain, with volume fractions from the remaining weights.
"""
import numpy as np
import scipy.sparse as sp

from .j2 import LOCAL_MAXIT
from .linear import laminate_milton
from .tree import lam_pos


def compressed_tree(K, w):
    """The compressed tree as nested tuples: ("leaf", j) or
    ("laminate", pos, left, right), with pos the laminate's paper position;
    None when no leaf carries weight.  A weight counts as zero when its real
    part is zero (complex steps keep the structure)."""
    def build(k, i):
        # subtree of laminate (k, i); its children are (k+1, 2i-1), (k+1, 2i),
        # or leaves 2i-2, 2i-1 at level K
        if k > K:
            j = i - 1
            return ("leaf", j) if np.real(w[j]) != 0 else None
        left, right = build(k + 1, 2 * i - 1), build(k + 1, 2 * i)
        if left is None:
            return right
        if right is None:
            return left
        return ("laminate", lam_pos(K, k, i), left, right)
    return build(1, 1)


def subtree_weight(node, w):
    if node[0] == "leaf":
        return w[node[1]]
    return subtree_weight(node[2], w) + subtree_weight(node[3], w)


def dmn_linear_compressed(K, w, normals, C1, C2, alpha=None):
    """DMN^L of the compressed tree: leaves carry C1 (even index) or C2 (odd
    index); every remaining laminate mixes its children with fractions
    W_left / (W_left + W_right) of the remaining weights.  Complex-safe."""
    root = compressed_tree(K, w)
    if root is None:
        raise ValueError("no leaf carries weight")

    def evaluate(node):
        if node[0] == "leaf":
            return C1 if node[1] % 2 == 0 else C2
        _, pos, left, right = node
        WL, WR = subtree_weight(left, w), subtree_weight(right, w)
        return laminate_milton(evaluate(left), evaluate(right), WL / (WL + WR),
                               WR / (WL + WR), normals[pos], alpha)
    return evaluate(root)


# ---------------------------------------------------------------- online evaluation

class CompressedDmnModel:
    """Gauss-point model (Sec. 3.2) of the compressed tree: only leaves with
    weight carry strains and stresses, only laminates whose two children both
    carry weight carry jumps; for a live leaf the strain is
    E + sum over those of its ancestors of -c2 N(n) a (left subtree) or
    +c1 N(n) a (right subtree), with fractions from the live weights.  (An
    ancestor with one dead child does not move its live child, whose fraction
    in it is zero, so it leaves the strain unchanged: that is the merge of
    the laminate into its surviving child.)  Interface of ``oracle.gp``'s
    model, with the jump vector reduced to the live laminates: use
    ``expand_jumps`` / ``reduce_jumps`` for full 3 (2^K - 1) vectors.

    Reading: the stop test keeps the factor 2^K - 1 of the uncompressed depth."""

    def __init__(self, K, w, normals, fiber, matrix):
        from .gp import DmnModel
        from .mandel import N_matrix, iso_from_E_nu
        from .j2 import J2Material
        from .tree import lam_leaves, lam_pos, laminates
        self.K, self.nL, self.L = K, 2 ** K, 2 ** K - 1
        self.w = np.asarray(w)
        self.normals = np.asarray(normals)
        self.dtype = np.result_type(self.w, self.normals, 1.0)
        wr = np.real(self.w)
        self.valid = bool(np.all(wr >= 0.0) and wr.sum() > 0.0)
        self.live_leaves = [j for j in range(self.nL) if wr[j] > 0.0]
        self.live_lams = []
        for (k, i) in laminates(K):
            lo, hi = lam_leaves(K, k, i)
            mid = (lo + hi) // 2
            if wr[lo:mid].sum() > 0.0 and wr[mid:hi].sum() > 0.0:
                self.live_lams.append((k, i))
        self.live_lams.sort(key=lambda ki: lam_pos(K, *ki))
        self.pos = [lam_pos(K, k, i) for (k, i) in self.live_lams]
        self.wt = (self.w / self.w.sum())[self.live_leaves] if self.valid else None
        row = {j: r for r, j in enumerate(self.live_leaves)}
        A = np.zeros((6 * len(self.live_leaves), 3 * len(self.pos)), dtype=self.dtype)
        for c, (k, i) in enumerate(self.live_lams):
            lo, hi = lam_leaves(K, k, i)
            mid = (lo + hi) // 2
            WL, WR = self.w[lo:mid].sum(), self.w[mid:hi].sum()
            c1, c2 = WL / (WL + WR), WR / (WL + WR)
            Nm = N_matrix(self.normals[lam_pos(K, k, i)])
            for j in range(lo, hi):
                if j in row:
                    A[6 * row[j]:6 * row[j] + 6, 3 * c:3 * c + 3] = -c2 * Nm if j < mid else c1 * Nm
        self.A = A
        self.Cf = iso_from_E_nu(fiber["E"], fiber["nu"])
        self.mat = J2Material(**matrix)
        self.B = np.tile(np.eye(6), (len(self.live_leaves), 1))
        self._solve = DmnModel.solve

    def reduce_jumps(self, a_full):
        a = np.asarray(a_full).reshape(-1, 3)
        return a[self.pos].ravel()

    def expand_jumps(self, a_red, a_full):
        out = np.array(a_full, dtype=np.result_type(a_red, a_full), copy=True).reshape(-1, 3)
        out[self.pos] = np.asarray(a_red).reshape(-1, 3)
        return out.ravel()

    def evaluate(self, E, z_n, a, local_max_iter=LOCAL_MAXIT):
        from .j2 import j2_update
        n = len(self.live_leaves)
        eps = E[None, :] + (self.A @ a).reshape(n, 6)
        dt = np.result_type(self.dtype, eps, z_n)
        sig = np.zeros((n, 6), dtype=dt)
        D = np.zeros((n, 6, 6), dtype=dt)
        z = np.array(z_n, dtype=dt, copy=True)
        margin, local_ok = np.inf, True
        for r, j in enumerate(self.live_leaves):
            if j % 2 == 0:
                sig[r] = self.Cf @ eps[r]
                D[r] = self.Cf
            else:
                m = j // 2
                out = j2_update(self.mat, eps[r], z_n[m, :6], z_n[m, 6], local_max_iter)
                sig[r], D[r] = out["sigma"], out["D"]
                z[m, :6], z[m, 6] = out["ep"], out["p"]
                margin = min(margin, abs(out["margin"]))
                local_ok &= out["ok"]
        wsig = self.wt[:, None] * sig
        return dict(eps=eps, sig=sig, D=D, z=z, r=self.A.T @ wsig.ravel(),
                    sbar=wsig.sum(axis=0), margin=margin, local_ok=local_ok)

    def hessian(self, D):
        WD = sp.block_diag([self.wt[r] * D[r] for r in range(len(self.live_leaves))],
                           format="csr")
        return self.A.T @ (WD @ self.A), WD

    def solve(self, H, rhs):
        return self._solve(self, H, rhs)

    def tangent(self, D):
        H, WD = self.hessian(D)
        X = self.solve(H, -(self.A.T @ (WD @ self.B)))
        return self.B.T @ (WD @ (self.B + self.A @ X))


def compressed_path(model, E_path, opts=None):
    """A strain path from z = 0, a = 0 on the compressed model; the jumps are
    returned as full 3 (2^K - 1) vectors (entries of removed laminates zero)."""
    from .gp import NewtonOptions, OK, gp_update
    opts = opts or NewtonOptions()
    z = np.zeros((model.nL // 2, 7), dtype=model.dtype)
    a_full = np.zeros(3 * model.L, dtype=model.dtype)
    outs = []
    for E in E_path:
        out = gp_update(model, E, z, model.reduce_jumps(a_full), opts)
        out = dict(out, a=model.expand_jumps(out["a"], a_full))
        outs.append(out)
        if out["status"] != OK:
            break
        z, a_full = out["z"], out["a"]
    return outs
