"""Linear elastic homogenisation of a direct DMN (Sec. 3.1, Sec. 3.2).

Two independent evaluations:

* ``dmn_linear``: bottom-up propagation of stiffnesses from level K to the
  root, each laminate homogenised with Milton's formula in terms of the
  projector P(n) and a reference parameter alpha (Sec. 3.1).
* ``dmn_linear_dense``: the algorithmic-tangent form of Sec. 3.2 with the
  explicit gradient operator, C = [I..I]^T W D (B + A X) with
  (A^T W D A) X = -A^T W D B, where D holds the leaf stiffnesses.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .mandel import projector_P
from .tree import fractions, gradient_operator, lam_pos


def milton_alpha(CL, CR):
    """Reading: alpha = half the smallest eigenvalue of both children (the paper only
    asks for alpha 'sufficiently large or suitably small'); the laminate result does
    not depend on the admissible alpha chosen.  Works on stacks [..., 6, 6] and
    returns [..., 1, 1]."""
    sym = lambda C: np.real(0.5 * (C + np.swapaxes(C, -1, -2)))
    lo = np.minimum(np.linalg.eigvalsh(sym(CL)).min(axis=-1),
                    np.linalg.eigvalsh(sym(CR)).min(axis=-1))
    return (0.5 * lo)[..., None, None]


def laminate_milton(CL, CR, c1, c2, n, alpha=None):
    """Effective stiffness of a rank-one laminate from Milton's formula (Sec. 3.1).

    (P + alpha [C - alpha I]^-1)^-1 = c1 (P + alpha [CL - alpha I]^-1)^-1
                                    + c2 (P + alpha [CR - alpha I]^-1)^-1,
    solved for C.  CL, CR may be stacks [..., 6, 6] sharing the laminate.
    Complex-safe for complex-step differentiation.
    """
    P = projector_P(n)
    I = np.eye(6)
    if alpha is None:
        alpha = milton_alpha(CL, CR)
    inv = np.linalg.inv
    YL = inv(P + alpha * inv(CL - alpha * I))
    YR = inv(P + alpha * inv(CR - alpha * I))
    Y = c1 * YL + c2 * YR
    return alpha * I + alpha * inv(inv(Y) - P)


def dmn_linear(K, w, normals, C1, C2, alpha=None, return_nodes=False):
    """DMN^L: effective stiffness of a depth-K DMN (Sec. 3.1, stiffness propagation).

    Phase-1 stiffness C1 sits on even 0-based leaves, C2 on odd leaves; level K
    laminates are homogenised first, then their results feed level K-1, up to
    the root.  Weights need not be normalised (fractions are weight ratios).
    """
    c1, c2 = fractions(K, w)
    level = [C1 if j % 2 == 0 else C2 for j in range(2 ** K)]
    nodes = {}
    for k in range(K, 0, -1):
        nxt = []
        for i in range(1, 2 ** (k - 1) + 1):
            p = lam_pos(K, k, i)
            C = laminate_milton(level[2 * i - 2], level[2 * i - 1], c1[p], c2[p],
                                normals[p], alpha)
            nodes[p] = C
            nxt.append(C)
        level = nxt
    return (level[0], nodes) if return_nodes else level[0]


def dmn_linear_dense(K, w, normals, leaf_stiffness):
    """Effective stiffness from the explicit operators of Sec. 3.2.

    leaf_stiffness: [2^K, 6, 6] stiffness of every leaf.  With W = diag(w~_j I),
    w~ = w / sum(w), H = A^T W D A, solve H X = -A^T W D B with B = [I; ...; I]
    and return B^T W D (B + A X).
    """
    nL = 2 ** K
    wt = np.asarray(w) / np.sum(w)
    A = gradient_operator(K, w, normals)
    WD = sp.block_diag([wt[j] * leaf_stiffness[j] for j in range(nL)], format="csr")
    B = np.tile(np.eye(6), (nL, 1))
    H = (A.T @ (WD @ A))
    H = H.toarray() if sp.issparse(H) else H
    rhs = -(A.T @ (WD @ B))
    X = sla.solve(H, rhs, assume_a="pos") if H.size else np.zeros((0, 6))
    return B.T @ (WD @ (B + A @ X))


def voigt_reuss(w, C1, C2):
    """Voigt (arithmetic) and Reuss (harmonic) averages of the two phases, weighted by
    the summed leaf weights of each phase."""
    w = np.asarray(w)
    f1 = w[0::2].sum() / w.sum()
    f2 = 1.0 - f1
    V = f1 * C1 + f2 * C2
    R = np.linalg.inv(f1 * np.linalg.inv(C1) + f2 * np.linalg.inv(C2))
    return V, R
