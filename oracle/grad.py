"""Gradients of the linear DMN map by complex-step differentiation.

For a real-analytic f, Im f(x + i h e_k) / h equals df/dx_k up to O(h^2)
with no subtractive cancellation, so h = 1e-30 gives derivatives to machine
precision.  The map differentiated here is the oracle's Milton-form DMN^L
(Sec. 3.1) with normals from spherical angles (Sec. 2.3); the functional is
J = sum_s <G_s, C_s> for given cotangents G_s.

Derivatives are taken with respect to the leaf weights w and the angles
(alpha, beta) of every normal: the angles span exactly the directions in which
a unit normal can move.
"""
import numpy as np

from .linear import dmn_linear

H = 1e-30


def normals_from_angles(alpha, beta):
    """n = (sin a cos b, sin a sin b, cos a), Sec. 2.3; complex-safe."""
    return np.stack([np.sin(alpha) * np.cos(beta), np.sin(alpha) * np.sin(beta),
                     np.cos(alpha)], axis=-1)


def functional(K, w, alpha, beta, C1, C2, G):
    C = dmn_linear(K, w, normals_from_angles(alpha, beta), C1, C2)
    return np.sum(G * C)


def linear_gradients(K, w, alpha, beta, C1, C2, G, w_idx=None, ang_idx=None):
    """Complex-step gradients of J = sum_s <G_s, DMN^L(C1_s, C2_s)>.

    C1, C2, G: [B, 6, 6].  w_idx / ang_idx select the parameters to
    differentiate (default: all).  Returns dict(gw, galpha, gbeta) with NaN
    for parameters not selected.
    """
    nl, L = 2 ** K, 2 ** K - 1
    w_idx = range(nl) if w_idx is None else w_idx
    ang_idx = range(L) if ang_idx is None else ang_idx
    gw = np.full(nl, np.nan)
    ga = np.full(L, np.nan)
    gb = np.full(L, np.nan)
    for j in w_idx:
        wc = w.astype(complex)
        wc[j] += 1j * H
        gw[j] = np.imag(functional(K, wc, alpha, beta, C1, C2, G)) / H
    for p in ang_idx:
        ac = alpha.astype(complex)
        ac[p] += 1j * H
        ga[p] = np.imag(functional(K, w, ac, beta, C1, C2, G)) / H
        bc = beta.astype(complex)
        bc[p] += 1j * H
        gb[p] = np.imag(functional(K, w, alpha, bc, C1, C2, G)) / H
    return dict(gw=gw, galpha=ga, gbeta=gb)
