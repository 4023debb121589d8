"""Sensitivity of the final effective stress of a load path with respect to the
DMN parameters, by complex-step differentiation through the whole path.

The functional is J = sum_p g_p . sigma_p^(T), the macro stress of each point
after the last load step contracted with a given vector g_p.  Perturbing the
leaf weights and the normal angles by i h v (h = 1e-30) and running the
oracle's Newton path (Sec. 3.2) in complex arithmetic gives
Im J / h = (dJ/dtheta) . v to machine precision: no subtractive cancellation,
and the elastic/plastic decisions are taken on real parts, so no branch flips.
Each step is polished with one extra Newton step after convergence so that
the imaginary part is the derivative at the converged jumps.

This route shares nothing with a reverse-mode adjoint: it differentiates the
forward computation directly.
"""
import numpy as np

from .gp import DmnModel, NewtonOptions, run_path
from .grad import normals_from_angles

H = 1e-30
TIGHT = NewtonOptions(tol=1e-13, max_iter=50, polish=1)


def path_functional(K, w, normals, fiber, matrix, E_paths, g, opts=TIGHT, compressed=False):
    """J = sum_p g_p . sigma_p after the last step.  E_paths: [T, P, 6]; g: [P, 6].
    With ``compressed`` the path runs on the compressed tree (zero-weight
    subtrees removed, Sec. 3.1)."""
    if compressed:
        from .compression import CompressedDmnModel, compressed_path
        model = CompressedDmnModel(K, w, normals, fiber, matrix)
        run = lambda E: compressed_path(model, E, opts)
    else:
        model = DmnModel(K, w, normals, fiber, matrix)
        run = lambda E: run_path(model, E, opts)
    J = 0.0
    for p in range(E_paths.shape[1]):
        outs = run(E_paths[:, p, :])
        if len(outs) != E_paths.shape[0] or outs[-1]["status"] != 0:
            raise RuntimeError(f"oracle path failed at point {p}")
        J = J + g[p] @ outs[-1]["sigma"]
    return J


def path_directional_derivative(K, w, alpha, beta, fiber, matrix, E_paths, g, v_w, v_alpha,
                                v_beta, opts=TIGHT, compressed=False):
    """(dJ/dw, dJ/dalpha, dJ/dbeta) . (v_w, v_alpha, v_beta) by complex step."""
    wc = np.asarray(w, dtype=complex) + 1j * H * np.asarray(v_w)
    ac = np.asarray(alpha, dtype=complex) + 1j * H * np.asarray(v_alpha)
    bc = np.asarray(beta, dtype=complex) + 1j * H * np.asarray(v_beta)
    J = path_functional(K, wc, normals_from_angles(ac, bc), fiber, matrix, E_paths, g, opts,
                        compressed)
    return np.imag(J) / H
