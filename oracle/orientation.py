"""Fibre-orientation interpolation of the lamination directions (FE-DMN
paper, Sec. 2.3).  Test infrastructure like the rest of the oracle.

A fibre-orientation state enters through the two largest eigenvalues
(l1, l2) of the second-order fibre orientation tensor, a point of the
orientation triangle 1/3 <= l1 <= 1, 1 - 2 l1 <= l2 <= l1.  Its barycentric
coordinates phi = (phi1, phi2, phi3) with respect to the triangle's vertices
(unidirectional (1, 0), isotropic (1/3, 1/3), planar isotropic (1/2, 1/2))
solve the 3x3 linear system of Sec. 2.3.  The shape functions of the
orientation-interpolation table (linear: 3, tri-linear: 4, quadratic: 6) are
polynomials in phi; every laminate carries coefficient vectors p, q of that
length, its spherical angles are alpha = p . shape, beta = q . shape, and its
normal follows from the angles as in Sec. 2.3.  The leaf weights do not
depend on the orientation.
"""
import numpy as np

from .grad import normals_from_angles

SHAPES = {"linear": 3, "trilinear": 4, "quadratic": 6}

# vertices of the orientation triangle as columns, with the row of ones
# that fixes sum(phi) = 1 (Sec. 2.3)
_TRIANGLE = np.array([[1.0, 1.0 / 3.0, 0.5],
                      [0.0, 1.0 / 3.0, 0.5],
                      [1.0, 1.0, 1.0]])


def in_triangle(l1, l2, tol=0.0):
    """The orientation-triangle inequalities of Sec. 2.3."""
    return (l1 >= 1.0 / 3.0 - tol) and (l1 <= 1.0 + tol) and \
        (l2 >= 1.0 - 2.0 * l1 - tol) and (l2 <= l1 + tol)


def barycentric(l1, l2):
    """phi solving the Sec. 2.3 system [vertices; ones] phi = (l1, l2, 1)."""
    return np.linalg.solve(_TRIANGLE, np.array([l1, l2, 1.0]))


def shape_functions(phi, kind):
    """Shape functions of the orientation-interpolation table at barycentric phi."""
    f1, f2, f3 = phi
    if kind == "linear":
        return np.array([f1, f2, f3])
    if kind == "trilinear":
        b = f1 * f2 * f3
        return np.array([f1 - 9.0 * b, f2 - 9.0 * b, f3 - 9.0 * b, 27.0 * b])
    if kind == "quadratic":
        return np.array([f1 * (2.0 * f1 - 1.0), f2 * (2.0 * f2 - 1.0), f3 * (2.0 * f3 - 1.0),
                         4.0 * f1 * f2, 4.0 * f1 * f3, 4.0 * f2 * f3])
    raise ValueError(f"unknown shape functions {kind!r}")


def interpolated_angles(p, q, l1, l2, kind):
    """alpha = p . shape(l1, l2), beta = q . shape(l1, l2) for every laminate.

    p, q: [L, M] coefficient vectors of the laminates (paper order)."""
    s = shape_functions(barycentric(l1, l2), kind)
    return np.asarray(p) @ s, np.asarray(q) @ s


def interpolated_normals(p, q, l1, l2, kind):
    """Lamination normals [L, 3] of the DMN at orientation (l1, l2)."""
    a, b = interpolated_angles(p, q, l1, l2, kind)
    return normals_from_angles(a, b)


def oriented_linear(K, w, p, q, kind, lam, C1, C2):
    """DMN^L (Sec. 3.1) of every sample with the normals of its own orientation
    lam[b] = (l1, l2): [B, 6, 6].  Complex-safe in w, p, q."""
    from .linear import dmn_linear
    out = []
    for b in range(len(lam)):
        n = interpolated_normals(p, q, lam[b][0], lam[b][1], kind)
        out.append(dmn_linear(K, w, n, C1[b:b + 1], C2[b:b + 1])[0])
    return np.stack(out)


def oriented_functional(K, w, p, q, kind, lam, C1, C2, G):
    """J = sum_b <G_b, DMN^L_b>."""
    return np.sum(G * oriented_linear(K, w, p, q, kind, lam, C1, C2))


def oriented_directional_derivative(K, w, p, q, kind, lam, C1, C2, G, vw, vp, vq, h=1e-30):
    """dJ/d(w, p, q) . (vw, vp, vq) by one complex step of size h."""
    J = oriented_functional(K, np.asarray(w) + 1j * h * np.asarray(vw),
                            np.asarray(p) + 1j * h * np.asarray(vp),
                            np.asarray(q) + 1j * h * np.asarray(vq), kind, lam, C1, C2, G)
    return J.imag / h
