"""Pins of the oracle's path sensitivity (complex step through the whole path).

* it matches central finite differences (h = 1e-6) on a plastic depth-2 path
  whose leaves stay away from the yield surface under the perturbation;
* on an elastic path it equals the derivative of the linear DMN map (a
  different code path: Milton's formula) contracted with the macro strain;
* the outputs depend on the weights only through w / sum(w) (Sec. 3.2), so on
  a plastic path the derivative along v_w = w vanishes (a dropped
  normalisation anywhere in the path breaks this).
"""
import numpy as np

import synthetic as S
from oracle.adjoint import TIGHT, path_directional_derivative, path_functional
from oracle.gp import DmnModel, run_path
from oracle.grad import linear_gradients, normals_from_angles
from oracle.mandel import iso_from_E_nu


def setup(K, seed, n_points=2, steps=4, mag=0.02):
    rs = S.streams(seed)
    net = S.random_dmn(rs["dmn"], K, 0.25)
    alpha, beta = S.normals_to_angles(net.normals)
    E = S.ramp_with_noise(rs, n_points, steps, mag, 1e-3)
    g = S.unit_directions(rs["cotangent"], n_points)
    return net, alpha, beta, E, g


def test_complex_step_path_matches_finite_differences():
    K = 2
    net, alpha, beta, E, g = setup(K, 300)
    model = DmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX)
    margins = [min(o["margin"] for o in run_path(model, E[:, p, :], TIGHT)) for p in range(2)]
    assert min(margins) > 1e-4, margins
    rng = np.random.default_rng(1)
    for _ in range(3):
        vw, va, vb = rng.standard_normal(4), rng.standard_normal(3), rng.standard_normal(3)
        cs = path_directional_derivative(K, net.w, alpha, beta, S.FIBER, S.MATRIX, E, g, vw, va, vb)
        h = 1e-6
        f = lambda s: path_functional(K, net.w + s * vw,
                                      normals_from_angles(alpha + s * va, beta + s * vb),
                                      S.FIBER, S.MATRIX, E, g)
        fd = (f(h) - f(-h)) / (2 * h)
        assert abs(cs - fd) <= 1e-5 * max(abs(cs), 1.0), (cs, fd)


def test_elastic_path_equals_linear_map_derivative():
    K = 3
    net, alpha, beta, E, g = setup(K, 301, n_points=2, steps=2, mag=2e-4)
    Cf = iso_from_E_nu(S.FIBER["E"], S.FIBER["nu"])
    Cm = iso_from_E_nu(S.MATRIX["E"], S.MATRIX["nu"])
    # J = sum_p g_p . Cbar E_p = <sum_p g_p E_p^T, Cbar>
    G = np.einsum("pi,pj->ij", g, E[-1])[None]
    lin = linear_gradients(K, net.w, alpha, beta, Cf[None], Cm[None], G)
    rng = np.random.default_rng(2)
    vw, va, vb = rng.standard_normal(8), rng.standard_normal(7), rng.standard_normal(7)
    cs = path_directional_derivative(K, net.w, alpha, beta, S.FIBER, S.MATRIX, E, g, vw, va, vb)
    ref = lin["gw"] @ vw + lin["galpha"] @ va + lin["gbeta"] @ vb
    assert abs(cs - ref) <= 1e-9 * max(abs(ref), 1e-12), (cs, ref)


def test_path_derivative_vanishes_along_weight_scaling():
    K = 3
    net, alpha, beta, E, g = setup(K, 302, n_points=2, steps=4, mag=0.02)
    model = DmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX)
    plastic = any(o["z"][:, 6].max() > 0 for p in range(2) for o in run_path(model, E[:, p, :], TIGHT))
    assert plastic
    za, zb = np.zeros(7), np.zeros(7)
    along = path_directional_derivative(K, net.w, alpha, beta, S.FIBER, S.MATRIX, E, g, net.w,
                                        za, zb)
    rng = np.random.default_rng(3)
    scale = abs(path_directional_derivative(K, net.w, alpha, beta, S.FIBER, S.MATRIX, E, g,
                                            rng.standard_normal(8), za, zb))
    assert scale > 1e-3
    assert abs(along) <= 1e-12 * scale, (along, scale)
