"""Pins of the oracle's linear DMN map (CPU only).

* single laminate vs the textbook closed form of a rank-one laminate
  (Backus averaging in the frame where the normal is e3);
* Milton's formula is independent of the admissible reference alpha;
* an independent Schur-complement laminate written here agrees with Milton's;
* equal normals collapse a deep DMN to one laminate; identical phases return
  the phase; SPD with Reuss <= C <= Voigt; scale invariance in the weights;
  rotational covariance;
* the dense algorithmic-tangent form of Sec. 3.2 equals the tree for K = 1..3.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import mandel as M
from oracle.linear import dmn_linear, dmn_linear_dense, laminate_milton, voigt_reuss


def rand_unit(rng):
    g = rng.standard_normal(3)
    return g / np.linalg.norm(g)


def rand_spd(rng, lo=1.0, hi=1e3):
    q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    lam = 10 ** rng.uniform(np.log10(lo), np.log10(hi), 6)
    C = q @ np.diag(lam) @ q.T
    return 0.5 * (C + C.T)


def rotation_to_e3(n):
    """Rotation R with R n = e3."""
    e3 = np.array([0.0, 0.0, 1.0])
    v = np.cross(n, e3)
    s, c = np.linalg.norm(v), n @ e3
    if s < 1e-14:
        return np.eye(3) if c > 0 else np.diag([1.0, -1.0, -1.0])
    vx = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
    return np.eye(3) + vx + vx @ vx * ((1 - c) / s ** 2)


def backus_laminate_e3(CL, CR, c1, c2):
    """Textbook rank-one laminate with normal e3: strains continuous in the plane
    components t = {11, 22, 12}, tractions continuous in nu = {33, 23, 13}.

    C_nn = <C_nn^-1>^-1, C_tn = <C_tn C_nn^-1> C_nn,
    C_tt = <C_tt - C_tn C_nn^-1 C_nt> + <C_tn C_nn^-1> C_nn <C_nn^-1 C_nt>.
    """
    t, nu = [0, 1, 5], [2, 3, 4]
    parts = []
    for C in (CL, CR):
        Cnn_inv = np.linalg.inv(C[np.ix_(nu, nu)])
        Ctn = C[np.ix_(t, nu)]
        Ctt = C[np.ix_(t, t)]
        parts.append((Cnn_inv, Ctn @ Cnn_inv, Ctt - Ctn @ Cnn_inv @ Ctn.T))
    avg = lambda idx: c1 * parts[0][idx] + c2 * parts[1][idx]
    Cnn = np.linalg.inv(avg(0))
    Ctn = avg(1) @ Cnn
    Ctt = avg(2) + avg(1) @ Cnn @ avg(1).T
    out = np.zeros((6, 6))
    out[np.ix_(nu, nu)] = Cnn
    out[np.ix_(t, nu)] = Ctn
    out[np.ix_(nu, t)] = Ctn.T
    out[np.ix_(t, t)] = Ctt
    return out


def test_single_laminate_matches_backus_closed_form():
    rng = np.random.default_rng(10)
    for _ in range(6):
        CL, CR = rand_spd(rng), rand_spd(rng)
        c1 = rng.uniform(0.05, 0.95)
        n = rand_unit(rng)
        R = rotation_to_e3(n)
        Q = M.rotation_mandel(R)          # rotates the frame so that n -> e3
        ref_e3 = backus_laminate_e3(Q @ CL @ Q.T, Q @ CR @ Q.T, c1, 1 - c1)
        ref = Q.T @ ref_e3 @ Q
        got = laminate_milton(CL, CR, c1, 1 - c1, n)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_milton_alpha_independence():
    rng = np.random.default_rng(11)
    CL, CR = rand_spd(rng), rand_spd(rng)
    n = rand_unit(rng)
    lo = min(np.linalg.eigvalsh(CL).min(), np.linalg.eigvalsh(CR).min())
    a = laminate_milton(CL, CR, 0.3, 0.7, n, alpha=0.3 * lo)
    b = laminate_milton(CL, CR, 0.3, 0.7, n, alpha=0.9 * lo)
    c = laminate_milton(CL, CR, 0.3, 0.7, n, alpha=-5.0)
    scale = np.abs(a).max()
    assert np.abs(a - b).max() <= 1e-11 * scale
    assert np.abs(a - c).max() <= 1e-11 * scale


def schur_laminate(CL, CR, c1, c2, n):
    """Independent laminate via the interface condition: jump a solves
    N^T (c2 CL + c1 CR) N a = -N^T (CR - CL) e; C e = average stress."""
    N = M.N_matrix(n)
    Kmat = N.T @ (c2 * CL + c1 * CR) @ N
    U = (CR - CL) @ N
    return c1 * CL + c2 * CR - c1 * c2 * U @ np.linalg.solve(Kmat, U.T)


def test_schur_form_matches_milton():
    rng = np.random.default_rng(12)
    for _ in range(6):
        CL, CR = rand_spd(rng), rand_spd(rng)
        c1 = rng.uniform(0.05, 0.95)
        n = rand_unit(rng)
        a = laminate_milton(CL, CR, c1, 1 - c1, n)
        b = schur_laminate(CL, CR, c1, 1 - c1, n)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("K", [3, 8])
def test_equal_normals_collapse_to_one_laminate(K):
    rng = np.random.default_rng(13)
    net = S.random_dmn(rng, K, 0.25)
    n = rand_unit(rng)
    normals = np.tile(n, (2 ** K - 1, 1))
    C1, C2 = rand_spd(rng), rand_spd(rng)
    f1 = net.w[0::2].sum() / net.w.sum()
    ref = laminate_milton(C1, C2, f1, 1 - f1, n)
    got = dmn_linear(K, net.w, normals, C1, C2)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_identical_phases_return_phase():
    rng = np.random.default_rng(14)
    net = S.random_dmn(rng, 4, 0.3)
    C = rand_spd(rng)
    got = dmn_linear(4, net.w, net.normals, C, C)
    assert np.abs(got - C).max() <= 1e-11 * np.abs(C).max()


def test_spd_between_reuss_and_voigt():
    rng = np.random.default_rng(15)
    for K in (1, 3, 6):
        net = S.random_dmn(rng, K, 0.25)
        C1, C2 = rand_spd(rng), rand_spd(rng)
        C = dmn_linear(K, net.w, net.normals, C1, C2)
        V, R = voigt_reuss(net.w, C1, C2)
        scale = np.abs(C).max()
        # Milton's nested inverses keep symmetry only to roundoff (~1e-12 here)
        assert np.abs(C - C.T).max() <= 1e-10 * scale
        C = 0.5 * (C + C.T)
        assert np.linalg.eigvalsh(C).min() > 0
        # a laminate meets both bounds in some directions, so equality holds up to
        # the roundoff of Milton's formula
        assert np.linalg.eigvalsh(V - C).min() >= -1e-10 * scale
        assert np.linalg.eigvalsh(C - R).min() >= -1e-10 * scale


def test_weight_scale_invariance():
    rng = np.random.default_rng(16)
    net = S.random_dmn(rng, 5, 0.25)
    C1, C2 = rand_spd(rng), rand_spd(rng)
    a = dmn_linear(5, net.w, net.normals, C1, C2)
    b = dmn_linear(5, 7.3 * net.w, net.normals, C1, C2)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_rotational_covariance():
    rng = np.random.default_rng(17)
    net = S.random_dmn(rng, 4, 0.25)
    C1, C2 = rand_spd(rng), rand_spd(rng)
    R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    Q = M.rotation_mandel(R)
    base = dmn_linear(4, net.w, net.normals, C1, C2)
    rot = dmn_linear(4, net.w, net.normals @ R.T, Q @ C1 @ Q.T, Q @ C2 @ Q.T)
    assert np.abs(rot - Q @ base @ Q.T).max() <= 1e-11 * np.abs(base).max()


@pytest.mark.parametrize("K", [1, 2, 3])
def test_dense_operator_form_equals_tree(K):
    rng = np.random.default_rng(18 + K)
    net = S.random_dmn(rng, K, 0.25)
    C1, C2 = rand_spd(rng), rand_spd(rng)
    leaf = np.array([C1 if j % 2 == 0 else C2 for j in range(2 ** K)])
    a = dmn_linear(K, net.w, net.normals, C1, C2)
    b = dmn_linear_dense(K, net.w, net.normals, leaf)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
