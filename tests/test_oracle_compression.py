"""Pins of the oracle's tree compression (Sec. 3.1): without zero weights it
is the full tree; with zero weights it is the limit of the uncompressed DMN
as those weights go to zero; a dead half reduces a depth-2 DMN to its live
laminate; a single live leaf returns its phase."""
import numpy as np

import synthetic as S
from oracle.compression import compressed_tree, dmn_linear_compressed
from oracle.linear import dmn_linear, laminate_milton
from oracle.tree import lam_pos


def case(K, B=3, seed=61):
    rs = S.streams(seed)
    net = S.random_dmn(rs["dmn"], K, 0.3)
    return net, S.random_spd(rs["stiffness"], B), S.random_spd(rs["stiffness"], B)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_positive_weights_keep_the_full_tree():
    for K in (1, 3, 5):
        net, C1, C2 = case(K)
        tree = compressed_tree(K, net.w)
        count = lambda n: 0 if n[0] == "leaf" else 1 + count(n[2]) + count(n[3])
        assert count(tree) == 2 ** K - 1
        assert rel(dmn_linear_compressed(K, net.w, net.normals, C1, C2),
                   dmn_linear(K, net.w, net.normals, C1, C2)) < 1e-11  # rounding of the fractions


def test_compression_is_the_zero_weight_limit():
    """Leaves 3 (alone: its sibling 2 stays), 8-11 (a whole depth-2 subtree)
    and 14 go to zero; the uncompressed DMN with weights eps there approaches
    the compressed one linearly in eps."""
    K = 4
    net, C1, C2 = case(K)
    dead = [3, 8, 9, 10, 11, 14]
    w0 = net.w.copy()
    w0[dead] = 0.0
    Cc = dmn_linear_compressed(K, w0, net.normals, C1, C2)
    errs = []
    for eps in (1e-6, 1e-8):
        we = w0.copy()
        we[dead] = eps
        errs.append(rel(dmn_linear(K, we, net.normals, C1, C2), Cc))
    assert errs[1] < 1e-6 and errs[1] < 0.05 * errs[0]


def test_dead_half_reduces_to_the_live_laminate():
    K = 2
    net, C1, C2 = case(K)
    w = net.w.copy()
    w[2:] = 0.0
    p = lam_pos(K, 2, 1)    # laminate over leaves 0, 1
    ref = laminate_milton(C1, C2, w[0] / (w[0] + w[1]), w[1] / (w[0] + w[1]), net.normals[p])
    assert rel(dmn_linear_compressed(K, w, net.normals, C1, C2), ref) < 1e-14


def test_single_live_leaf_returns_its_phase():
    K = 3
    net, C1, C2 = case(K)
    for j in (0, 5):
        w = np.zeros(2 ** K)
        w[j] = 0.7
        ref = C1 if j % 2 == 0 else C2
        assert np.array_equal(dmn_linear_compressed(K, w, net.normals, C1, C2), ref)
    assert compressed_tree(K, np.zeros(2 ** K)) is None


# ---------------------------------------------------------------- online evaluation

def gp_case(K, seed, T=4, mag=0.05):
    rs = S.streams(seed)
    net = S.random_dmn(rs["dmn"], K, 0.3)
    E = S.ramp_with_noise(rs, 1, T, mag, 1e-3)[:, 0, :]
    return net, E


def test_compressed_gp_without_dead_leaves_is_the_full_model():
    from oracle.compression import CompressedDmnModel, compressed_path
    from oracle.gp import DmnModel, run_path
    K = 3
    net, E = gp_case(K, 101)
    full = run_path(DmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX), E)
    comp = compressed_path(CompressedDmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX), E)
    for f, c in zip(full, comp):
        assert f["status"] == c["status"] == 0 and f["iters"] == c["iters"]
        assert rel(c["sigma"], f["sigma"]) < 1e-12 and rel(c["C"], f["C"]) < 1e-11
        assert rel(c["a"], f["a"]) < 1e-10 and rel(c["z"], f["z"]) < 1e-10


def test_compressed_gp_is_the_zero_weight_limit():
    """The dense model with weights eps on the removed leaves approaches the
    compressed model as eps -> 0 (stress, tangent, live internal variables)."""
    from oracle.compression import CompressedDmnModel, compressed_path
    from oracle.gp import DmnModel, run_path
    K = 3
    net, E = gp_case(K, 102, T=3)
    dead = [2, 3, 5]          # a dead sibling pair and a zero leaf beside a live one
    w0 = net.w.copy()
    w0[dead] = 0.0
    model = CompressedDmnModel(K, w0, net.normals, S.FIBER, S.MATRIX)
    comp = compressed_path(model, E)
    live_m = [m for m in range(2 ** (K - 1)) if 2 * m + 1 in model.live_leaves]
    errs = []
    for eps in (1e-5, 1e-7, 1e-9):
        we = w0.copy()
        we[dead] = eps
        full = run_path(DmnModel(K, we, net.normals, S.FIBER, S.MATRIX), E)
        e = 0.0
        for f, c in zip(full, comp):
            assert f["status"] == c["status"] == 0
            e = max(e, rel(f["sigma"], c["sigma"]), rel(f["C"], c["C"]),
                    rel(f["z"][live_m], c["z"][live_m]))
        errs.append(e)
    # first-order convergence in eps (a dilute inclusion perturbs at O(eps))
    assert errs[2] < 1e-4 and errs[1] < 0.05 * errs[0] and errs[2] < 0.05 * errs[1], errs


def test_compressed_gp_dead_half_is_the_live_laminate():
    from oracle.compression import CompressedDmnModel, compressed_path
    from oracle.gp import DmnModel, run_path
    K = 2
    net, E = gp_case(K, 103, T=3)
    w = net.w.copy()
    w[2:] = 0.0
    p = lam_pos(K, 2, 1)
    ref = run_path(DmnModel(1, w[:2], net.normals[p:p + 1], S.FIBER, S.MATRIX), E)
    comp = compressed_path(CompressedDmnModel(K, w, net.normals, S.FIBER, S.MATRIX), E)
    for f, c in zip(ref, comp):
        assert f["status"] == c["status"] == 0 and f["iters"] == c["iters"]
        assert rel(c["sigma"], f["sigma"]) < 1e-13 and rel(c["C"], f["C"]) < 1e-12
        assert rel(c["z"][:1], f["z"]) < 1e-12
        assert rel(c["a"][3 * p:3 * p + 3], f["a"]) < 1e-12


def test_compressed_path_derivative_matches_differences():
    """Complex-step derivative of the compressed path (a dead sibling pair)
    along a direction over the live weights and all angles, against central
    differences of the same functional."""
    from oracle.adjoint import TIGHT, path_directional_derivative, path_functional
    from oracle.grad import normals_from_angles
    K = 2
    net, E = gp_case(K, 104, T=3)
    w = net.w.copy()
    w[2:] = 0.0
    alpha, beta = S.normals_to_angles(net.normals)
    rs = S.streams(105)
    g = S.unit_directions(rs["cotangent"], 1)
    E3 = E[:, None, :]
    vw = np.array([0.3, -0.7, 0.0, 0.0])
    va, vb = rs["noise"].standard_normal(3), rs["noise"].standard_normal(3)
    d = path_directional_derivative(K, w, alpha, beta, S.FIBER, S.MATRIX, E3, g, vw, va, vb,
                                    compressed=True)
    f = lambda h: path_functional(K, w + h * vw, normals_from_angles(alpha + h * va, beta + h * vb),
                                  S.FIBER, S.MATRIX, E3, g, TIGHT, compressed=True)
    h = 1e-6
    fd = (f(h) - f(-h)) / (2 * h)
    assert abs(d - fd) <= 1e-6 * max(abs(d), 1.0)
