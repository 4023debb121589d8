"""Mandel notation for symmetric second- and fourth-order tensors.

Ordering of the 6-vector: [11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12].  The
Mandel dot product equals the Frobenius product of the tensors, so Mandel
l2-norms are Frobenius norms.  All functions are complex-safe (no conjugation)
so that complex-step derivatives pass through them.
"""
import numpy as np

SQ2 = np.sqrt(2.0)
PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
FAC = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])
DELTA6 = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])  # Mandel image of the identity


def sym_to_mandel(S):
    """3x3 symmetric tensor -> Mandel 6-vector."""
    return np.array([S[i, j] * f for (i, j), f in zip(PAIRS, FAC)])


def mandel_to_sym(v):
    S = np.zeros((3, 3), dtype=np.result_type(v, 1.0))
    for I, (i, j) in enumerate(PAIRS):
        S[i, j] = v[I] / FAC[I]
        S[j, i] = v[I] / FAC[I]
    return S


def tensor4_to_mandel(T):
    """Fourth-order tensor with minor symmetries -> 6x6 Mandel matrix."""
    M = np.zeros((6, 6), dtype=np.result_type(T, 1.0))
    for I, (i, j) in enumerate(PAIRS):
        for J, (k, l) in enumerate(PAIRS):
            M[I, J] = FAC[I] * FAC[J] * T[i, j, k, l]
    return M


def projector_P(n):
    """Laminate projector P(n) from its Cartesian components (Sec. 3.1, Milton's formula).

    P_mnop = 1/2 (n_m d_no n_p + n_n d_mo n_p + n_m d_np n_o + n_n d_mp n_o) - n_m n_n n_o n_p
    """
    d = np.eye(3)
    T = 0.5 * (np.einsum("m,no,p->mnop", n, d, n) + np.einsum("n,mo,p->mnop", n, d, n)
               + np.einsum("m,np,o->mnop", n, d, n) + np.einsum("n,mp,o->mnop", n, d, n)) \
        - np.einsum("m,n,o,p->mnop", n, n, n, n)
    return tensor4_to_mandel(T)


def N_matrix(n):
    """Symmetrisation operator N(n): a -> 1/2 (a (x) n + n (x) a) as a 6x3 Mandel matrix (Sec. 3.2)."""
    cols = []
    for c in range(3):
        e = np.zeros(3)
        e[c] = 1.0
        cols.append(sym_to_mandel(0.5 * (np.outer(e, n) + np.outer(n, e))))
    return np.stack(cols, axis=1)


P1 = np.outer(DELTA6, DELTA6) / 3.0   # spherical projector
P2 = np.eye(6) - P1                    # deviatoric projector


def bulk_shear(E, nu):
    """Compression and shear modulus from Young's modulus and Poisson's ratio."""
    return E / (3.0 * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def iso_stiffness(K, G):
    """Isotropic stiffness 3K P1 + 2G P2 (Sec. 4.4)."""
    return 3.0 * K * P1 + 2.0 * G * P2


def iso_from_E_nu(E, nu):
    return iso_stiffness(*bulk_shear(E, nu))


def rotation_mandel(R):
    """6x6 Mandel matrix of the map S -> R S R^T on symmetric tensors."""
    Q = np.zeros((6, 6))
    for J in range(6):
        e = np.zeros(6)
        e[J] = 1.0
        Q[:, J] = sym_to_mandel(R @ mandel_to_sym(e) @ R.T)
    return Q
