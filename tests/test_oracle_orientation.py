"""Pins of the oracle's fibre-orientation interpolation (Sec. 2.3 and the
orientation-interpolation table): triangle vertices, inversion of the
barycentric map, partition of unity, Kronecker and reproduction properties of
each shape-function family, unit normals."""
import os

import numpy as np
import pytest

from oracle.grad import normals_from_angles
from oracle.orientation import (SHAPES, barycentric, in_triangle, interpolated_angles,
                                interpolated_normals, shape_functions)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "orientation_triangle.txt")


def vertices():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return {r[0]: (float(r[1]), float(r[2]), np.array([float(x) for x in r[3:6]])) for r in rows}


def random_points(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        l1, l2 = rng.uniform(1 / 3, 1.0), rng.uniform(0.0, 1.0)
        if in_triangle(l1, l2):
            out.append((l1, l2))
    return out


def test_vertices_have_unit_barycentric_coordinates():
    for name, (l1, l2, phi) in vertices().items():
        assert in_triangle(l1, l2, 1e-15), name
        assert np.allclose(barycentric(l1, l2), phi, atol=1e-14), name


def test_barycentric_map_inverts_the_vertex_combination():
    """l = sum_j phi_j vertex_j for random phi on the simplex; solving must return phi."""
    v = vertices()
    verts = np.array([[v[k][0], v[k][1]] for k in ("unidirectional", "isotropic",
                                                   "planar_isotropic")])
    rng = np.random.default_rng(3)
    for phi in rng.dirichlet([1.0, 1.0, 1.0], 50):
        l1, l2 = phi @ verts
        assert in_triangle(l1, l2, 1e-12)
        assert np.allclose(barycentric(l1, l2), phi, atol=1e-13)


@pytest.mark.parametrize("kind", list(SHAPES))
def test_partition_of_unity(kind):
    for l1, l2 in random_points(40):
        s = shape_functions(barycentric(l1, l2), kind)
        assert len(s) == SHAPES[kind]
        assert abs(s.sum() - 1.0) < 1e-13


def test_linear_and_quadratic_kronecker_property():
    e = np.eye(3)
    for j in range(3):
        assert np.allclose(shape_functions(e[j], "linear"), e[j])
        sq = shape_functions(e[j], "quadratic")
        assert np.allclose(sq[:3], e[j]) and np.allclose(sq[3:], 0.0)
    # quadratic edge functions: 4 phi_a phi_b is one at the midpoint of edge (a, b)
    for (a, b), k in (((0, 1), 3), ((0, 2), 4), ((1, 2), 5)):
        phi = np.zeros(3)
        phi[a] = phi[b] = 0.5
        s = shape_functions(phi, "quadratic")
        assert abs(s[k] - 1.0) < 1e-15 and np.allclose(np.delete(s, k), 0.0)


def test_trilinear_bubble_at_vertices_and_centroid():
    e = np.eye(3)
    for j in range(3):
        s = shape_functions(e[j], "trilinear")
        assert np.allclose(s[:3], e[j]) and abs(s[3]) < 1e-15
    s = shape_functions(np.full(3, 1.0 / 3.0), "trilinear")
    assert np.allclose(s[:3], 0.0, atol=1e-15) and abs(s[3] - 1.0) < 1e-14


def test_reproduction_of_polynomials():
    """Linear and tri-linear shapes reproduce linear functions of (l1, l2), the
    quadratic shapes quadratic ones, given the function's values at the nodes."""
    v = vertices()
    V = [np.array(v[k][:2]) for k in ("unidirectional", "isotropic", "planar_isotropic")]
    lin = lambda x: 0.3 + 1.7 * x[0] - 2.2 * x[1]
    quad = lambda x: 0.1 - 0.4 * x[0] + 0.9 * x[1] + 1.3 * x[0] ** 2 - 0.7 * x[0] * x[1] + 2.1 * x[1] ** 2
    c = (V[0] + V[1] + V[2]) / 3
    p_lin = np.array([[lin(V[0]), lin(V[1]), lin(V[2])]])
    p_tri = np.array([[lin(V[0]), lin(V[1]), lin(V[2]), lin(c)]])
    mids = [(V[0] + V[1]) / 2, (V[0] + V[2]) / 2, (V[1] + V[2]) / 2]
    p_quad = np.array([[quad(V[0]), quad(V[1]), quad(V[2])] + [quad(m) for m in mids]])
    zero = np.zeros_like
    for l1, l2 in random_points(30, seed=5):
        x = np.array([l1, l2])
        assert abs(interpolated_angles(p_lin, zero(p_lin), l1, l2, "linear")[0][0] - lin(x)) < 1e-13
        assert abs(interpolated_angles(p_tri, zero(p_tri), l1, l2, "trilinear")[0][0] - lin(x)) < 1e-13
        assert abs(interpolated_angles(p_quad, zero(p_quad), l1, l2, "quadratic")[0][0] - quad(x)) < 1e-12


@pytest.mark.parametrize("kind", list(SHAPES))
def test_normals_are_unit_and_constant_angles_give_fixed_normals(kind):
    rng = np.random.default_rng(7)
    M = SHAPES[kind]
    a0, b0 = rng.uniform(0, np.pi, 15), rng.uniform(0, 2 * np.pi, 15)
    p = np.repeat(a0[:, None], M, axis=1)
    q = np.repeat(b0[:, None], M, axis=1)
    for l1, l2 in random_points(5, seed=9):
        n = interpolated_normals(p, q, l1, l2, kind)
        assert np.allclose(np.linalg.norm(n, axis=1), 1.0)
        assert np.allclose(n, normals_from_angles(a0, b0), atol=1e-13)
    pr, qr = rng.normal(size=(15, M)), rng.normal(size=(15, M))
    n = interpolated_normals(pr, qr, 0.6, 0.3, kind)
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0)


def _training_case(K=2, B=3, kind="quadratic", seed=11):
    import synthetic as S
    rs = S.streams(seed)
    net = S.interpolated_dmn(rs["dmn"], K, 0.3, kind)
    lam = S.triangle_points(rs["assignment"], B)
    C1 = S.random_spd(rs["stiffness"], B)
    C2 = S.random_spd(rs["stiffness"], B)
    G = rs["cotangent"].standard_normal((B, 6, 6))
    return net, lam, C1, C2, G


def test_oriented_linear_with_constant_coefficients_is_the_fixed_map():
    """Equal shape coefficients give orientation-independent normals (partition
    of unity), so every sample sees the fixed-normal map."""
    from oracle.linear import dmn_linear
    net, lam, C1, C2, _ = _training_case(K=3, B=4)
    a0, b0 = net.p[:, 0], net.q[:, 0]
    M = net.p.shape[1]
    p = np.repeat(a0[:, None], M, 1)
    q = np.repeat(b0[:, None], M, 1)
    from oracle.orientation import oriented_linear
    got = oriented_linear(3, net.w, p, q, net.kind, lam, C1, C2)
    ref = dmn_linear(3, net.w, normals_from_angles(a0, b0), C1, C2)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("kind", list(SHAPES))
def test_oriented_directional_derivative_matches_central_differences(kind):
    from oracle.orientation import oriented_directional_derivative, oriented_functional
    net, lam, C1, C2, G = _training_case(K=2, B=3, kind=kind)
    rng = np.random.default_rng(2)
    vw, vp, vq = rng.standard_normal(4), rng.standard_normal(net.p.shape), rng.standard_normal(net.q.shape)
    d = oriented_directional_derivative(2, net.w, net.p, net.q, kind, lam, C1, C2, G, vw, vp, vq)
    def central(h):
        Jp = oriented_functional(2, net.w + h * vw, net.p + h * vp, net.q + h * vq, kind, lam,
                                 C1, C2, G)
        Jm = oriented_functional(2, net.w - h * vw, net.p - h * vp, net.q - h * vq, kind, lam,
                                 C1, C2, G)
        return (Jp - Jm) / (2 * h)
    h = 1e-4
    fd = (4.0 * central(h / 2) - central(h)) / 3.0   # Richardson: O(h^4)
    assert abs(d - fd) <= 1e-8 * max(abs(d), 1.0)


def test_coefficient_gradients_sum_to_the_angle_gradient():
    """Partition of unity: at fixed orientation, the derivative along v_p = 1 for
    every shape coefficient of one laminate equals the derivative along its angle."""
    from oracle.grad import linear_gradients
    from oracle.orientation import interpolated_angles, oriented_directional_derivative
    net, lam, C1, C2, G = _training_case(K=2, B=1, kind="trilinear")
    L, M = net.p.shape
    a, b = interpolated_angles(net.p, net.q, lam[0, 0], lam[0, 1], net.kind)
    ref = linear_gradients(2, net.w, a, b, C1, C2, G)
    for i in range(L):
        vp = np.zeros((L, M))
        vp[i] = 1.0
        d = oriented_directional_derivative(2, net.w, net.p, net.q, net.kind, lam, C1, C2, G,
                                            np.zeros(4), vp, np.zeros((L, M)))
        assert abs(d - ref["galpha"][i]) <= 1e-10 * max(1.0, abs(ref["galpha"][i]))
