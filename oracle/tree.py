"""Topology of a perfect two-phase direct DMN of depth K (Sec. 2.1, Sec. 3.2).

Levels k = 1 (root) ... K (laminates whose children are leaves); laminate
(k, i) has 1-based horizontal index i = 1 ... 2^(k-1) and children (k+1, 2i-1)
(left) and (k+1, 2i) (right).  Leaves are numbered 0 ... 2^K - 1 here; the
paper's odd leaves (1-based) carry phase 1, i.e. even 0-based leaves are
phase 1 (the fibre).

Paper ordering of laminate parameters, normals and jumps: level K first, then
K-1, ..., root last (ordering equation in Sec. 3.1 and 3.2).  The 0-based
position of (k, i) in that order is 2^K - 2^k + (i - 1).
"""
import numpy as np
import scipy.sparse as sp

from .mandel import N_matrix


def n_laminates(K):
    return 2 ** K - 1


def lam_pos(K, k, i):
    """0-based paper position of laminate (k, i), i 1-based."""
    return 2 ** K - 2 ** k + (i - 1)


def lam_leaves(K, k, i):
    """Half-open 0-based leaf range [lo, hi) covered by laminate (k, i)."""
    span = 2 ** (K - k + 1)
    return (i - 1) * span, i * span


def laminates(K):
    """All laminates as (k, i) pairs in paper order."""
    return [(k, i) for k in range(K, 0, -1) for i in range(1, 2 ** (k - 1) + 1)]


def fractions(K, w):
    """Volume fractions (c1, c2) of every laminate, in paper order (Sec. 2.1).

    Subtree weights are sums of the leaf weights below a node (weight
    propagation); c1 = W_left / (W_left + W_right), c2 = 1 - c1.
    """
    L = n_laminates(K)
    c1 = np.zeros(L, dtype=np.result_type(w, 1.0))
    for (k, i) in laminates(K):
        lo, hi = lam_leaves(K, k, i)
        mid = (lo + hi) // 2
        WL = w[lo:mid].sum()
        WR = w[mid:hi].sum()
        c1[lam_pos(K, k, i)] = WL / (WL + WR)
    return c1, 1.0 - c1


def gradient_operator(K, w, normals, sparse=True):
    """Gradient operator A: jumps (3 per laminate, paper order) -> leaf strains (6 per leaf).

    For laminate (k, i) and leaf j below it, block (j, pos(k, i)) is -c2 N(n)
    when j lies in the left subtree and +c1 N(n) when it lies in the right
    subtree (the depth-3 example of Sec. 3.2 fixes these signs and fractions).
    """
    L = n_laminates(K)
    c1, c2 = fractions(K, w)
    dtype = np.result_type(w, normals, 1.0)
    rows, cols, vals = [], [], []
    for (k, i) in laminates(K):
        p = lam_pos(K, k, i)
        Nm = N_matrix(normals[p])
        lo, hi = lam_leaves(K, k, i)
        mid = (lo + hi) // 2
        for j in range(lo, hi):
            blk = -c2[p] * Nm if j < mid else c1[p] * Nm
            for a in range(6):
                for b in range(3):
                    rows.append(6 * j + a)
                    cols.append(3 * p + b)
                    vals.append(blk[a, b])
    A = sp.csr_matrix((np.array(vals, dtype=dtype), (rows, cols)),
                      shape=(6 * 2 ** K, 3 * L))
    return A if sparse else A.toarray()


def leaf_phase(j):
    """1 for the fibre phase (even 0-based leaf), 2 for the matrix phase."""
    return 1 if j % 2 == 0 else 2
