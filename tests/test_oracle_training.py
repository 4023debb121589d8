"""Pins of the oracle's training objective, optimiser and stiffness sampler
(Sec. 3.1 objective, Sec. 4.4 sampling, Sec. 4.5 optimiser): closed-form
norms of isotropic stiffnesses, limits of the q-norm, the exact zero of the
objective at the generating parameters, complex-step gradients against
Richardson-extrapolated differences, the scale invariance of the DMN in its
weights, first-step and constant-gradient properties of AMSGrad, special
values of the learning-rate modulation, and the spectra and rotation
properties of the sampled stiffnesses (checked against scipy's rotation
vectors)."""
import numpy as np
import pytest

import synthetic as S
from oracle import training as T
from oracle.linear import dmn_linear
from oracle.mandel import P1, iso_stiffness, sym_to_mandel


def lame(K, G):
    return K - 2.0 * G / 3.0, G


@pytest.mark.parametrize("K,G", [(1.0, 0.3), (40.0, 30.0), (5.0, 20.0)])
def test_voigt_norms_of_isotropic_stiffness(K, G):
    """Voigt matrix of an isotropic stiffness: lambda + 2 mu on three diagonal
    entries, lambda on the six normal off-diagonals, mu on the three shear
    diagonals (not 2 mu as in Mandel storage)."""
    lam, mu = lame(K, G)
    C = iso_stiffness(K, G)
    n1 = 3 * abs(lam + 2 * mu) + 6 * abs(lam) + 3 * abs(mu)
    n2 = np.sqrt(3 * (lam + 2 * mu) ** 2 + 6 * lam ** 2 + 3 * mu ** 2)
    assert abs(T.stiffness_norm(C, 1.0) - n1) <= 1e-14 * n1
    assert abs(T.stiffness_norm(C, 2.0) - n2) <= 1e-14 * n2


def test_sample_errors_scale_and_zero():
    rs = S.streams(31)
    Tt = S.random_spd(rs["stiffness"], 5)
    for p in (1.0, 2.0):
        assert np.allclose(T.sample_errors(Tt, Tt, p), 0.0, atol=0.0)
        assert np.allclose(T.sample_errors(np.zeros_like(Tt), Tt, p), 1.0, rtol=1e-15)
        assert np.allclose(T.sample_errors(3.0 * Tt, Tt, p), 2.0, rtol=1e-14)
        assert np.allclose(T.sample_errors(0.75 * Tt, Tt, p), 0.25, rtol=1e-14)


def test_q_norm_limits():
    """q = 1 gives the mean error; for any q the value lies between max/N_b and
    N_b^(1/q) max/N_b, and tends to max/N_b as q grows."""
    e = np.random.default_rng(4).uniform(0.01, 0.5, 32)
    B = len(e)
    assert abs(T.data_term(e, 1.0) - e.sum() / B) <= 1e-15
    for q in (2.0, 10.0, 40.0):
        v = T.data_term(e, q)
        assert e.max() / B - 1e-16 <= v <= B ** (1 / q) * e.max() / B + 1e-16
    assert abs(T.data_term(e, 400.0) * B / e.max() - 1.0) < 1e-2


def _case(K=2, B=4, seed=5):
    rs = S.streams(seed)
    C1 = S.random_spd(rs["stiffness"], B)
    C2 = S.random_spd(rs["stiffness"], B)
    truth = S.random_dmn(rs["ground_truth"], K, 0.3)
    a_t, b_t = S.normals_to_angles(truth.normals)
    v = rs["init"].uniform(0.2, 1.0, 2 ** K)
    v = 1.1 * v / v.sum()
    alpha = rs["init"].uniform(0.0, 2 * np.pi, 2 ** K - 1)
    beta = rs["init"].uniform(0.0, 2 * np.pi, 2 ** K - 1)
    return C1, C2, truth, a_t, b_t, v, alpha, beta


def test_objective_vanishes_at_the_generating_dmn():
    K = 3
    C1, C2, truth, a_t, b_t, _, _, _ = _case(K=K, B=6)
    Tt = dmn_linear(K, truth.w, truth.normals, C1, C2)
    assert abs(truth.w.sum() - 1.0) < 1e-14
    for p, q in ((1.0, 10.0), (2.0, 1.0)):
        J = T.objective(K, truth.w, a_t, b_t, C1, C2, Tt, p, q, 1e3)
        assert abs(J) < 1e-11  # angles round-trip the normals to rounding
    # a weight-only rescaling leaves the data term at zero and costs the penalty
    J = T.objective(K, 1.5 * truth.w, a_t, b_t, C1, C2, Tt, 1.0, 10.0, 1e3)
    assert abs(J - 1e3 * 0.25) < 1e-9


def _richardson(f, x, i, h):
    def central(hh):
        xp, xm = x.copy(), x.copy()
        xp[i] += hh
        xm[i] -= hh
        return (f(xp) - f(xm)) / (2 * hh)
    return (4.0 * central(h / 2) - central(h)) / 3.0


@pytest.mark.parametrize("p,q", [(1.0, 10.0), (2.0, 3.0)])
def test_objective_gradient_matches_differences(p, q):
    K = 2
    C1, C2, truth, _, _, v, alpha, beta = _case(K=K, B=4)
    Tt = dmn_linear(K, truth.w, truth.normals, C1, C2)
    g = T.objective_gradient(K, v, alpha, beta, C1, C2, Tt, p, q, 10.0)
    fv = lambda x: T.objective(K, x, alpha, beta, C1, C2, Tt, p, q, 10.0)
    fa = lambda x: T.objective(K, v, x, beta, C1, C2, Tt, p, q, 10.0)
    fb = lambda x: T.objective(K, v, alpha, x, C1, C2, Tt, p, q, 10.0)
    for key, f, x in (("gv", fv, v), ("galpha", fa, alpha), ("gbeta", fb, beta)):
        for i in range(len(x)):
            fd = _richardson(f, x, i, 1e-4)
            assert abs(g[key][i] - fd) <= 1e-7 * max(1.0, abs(fd)), (key, i)


def test_weight_gradient_scale_identity_and_macaulay_cutoff():
    """C-bar is invariant under w -> s w, so sum_i v_i dJ/dv_i over the positive
    v_i equals the penalty's 2 lambda (sum v - 1) sum v; negative v_i get no
    gradient."""
    K = 2
    C1, C2, truth, _, _, v, alpha, beta = _case(K=K, B=3)
    Tt = dmn_linear(K, truth.w, truth.normals, C1, C2)
    lam = 7.0
    g = T.objective_gradient(K, v, alpha, beta, C1, C2, Tt, 1.0, 10.0, lam)
    s = v.sum()
    assert abs(np.dot(v, g["gv"]) - 2 * lam * (s - 1) * s) <= 1e-10 * max(1.0, abs(g["gv"]).max())
    v2 = v.copy()
    v2[1] = -0.3
    g2 = T.objective_gradient(K, v2, alpha, beta, C1, C2, Tt, 1.0, 10.0, lam)
    assert g2["gv"][1] == 0.0


def test_data_cotangent_matches_differences():
    rs = S.streams(33)
    Tt = S.random_spd(rs["stiffness"], 3)
    Cb = Tt * (1.0 + 0.2 * rs["noise"].standard_normal(Tt.shape))
    G = T.data_cotangent(Cb, Tt, 1.0, 10.0)
    f = lambda x: T.data_term(T.sample_errors(x.reshape(Cb.shape), Tt, 1.0), 10.0)
    x = Cb.reshape(-1).copy()
    for i in range(0, x.size, 7):
        fd = _richardson(f, x, i, 1e-6 * abs(x[i]))
        assert abs(G.reshape(-1)[i] - fd) <= 1e-5 * abs(fd) + 1e-9 * abs(G).max(), i


def test_amsgrad_first_step_and_constant_gradient():
    """With bias correction the first step is lr g / (|g| + eps); a constant
    gradient keeps that step size; the running maximum never decreases."""
    rng = np.random.default_rng(8)
    g = rng.normal(0.0, 3.0, 10)
    th = rng.normal(0.0, 1.0, 10)
    z = np.zeros(10)
    th1, m1, m2, mx = T.amsgrad(th, g, z, z, z, 1, 0.01)
    assert np.allclose(th - th1, 0.01 * g / (np.abs(g) + T.EPS), rtol=1e-12, atol=0)
    th_t, state = th1, (m1, m2, mx)
    for t in range(2, 8):
        prev = th_t
        th_t, *state = T.amsgrad(th_t, g, *state, t, 0.01)
        assert np.allclose(prev - th_t, 0.01 * g / (np.abs(g) + T.EPS), rtol=1e-10, atol=0)
    mx_prev = state[2]
    th_t, *state = T.amsgrad(th_t, 0.1 * g, *state, 8, 0.01)
    assert np.all(state[2] >= mx_prev)


def test_learning_rate_modulation_special_values():
    lo, hi, M, gm = 1.5e-3, 1.5e-2, 50, 0.999
    assert T.learning_rate(0, lo, hi, M, gm) == hi
    assert abs(T.learning_rate(M, lo, hi, M, gm) - gm ** M * lo) < 1e-18
    assert abs(T.learning_rate(2 * M, lo, hi, M, gm) - gm ** (2 * M) * hi) < 1e-17
    assert abs(T.learning_rate(M // 2, lo, hi, M, gm) - gm ** (M // 2) * 0.5 * (lo + hi)) < 1e-17


def test_deviatoric_direction_is_trace_free_unit_and_matches_the_closed_form():
    """Everywhere trace-free and unit, including the two angles where the
    printed closed form is 0/0; equal to the closed form up to sign elsewhere."""
    betas = np.concatenate([np.linspace(0.0, 2 * np.pi, 97), [0.75 * np.pi, 1.75 * np.pi]])
    for beta in betas:
        d = T.deviatoric_direction(beta)
        assert abs(d.sum()) < 1e-15 and abs(np.dot(d, d) - 1.0) < 1e-15
        if abs(np.cos(beta) + np.sin(beta)) > 0.1:
            c = T.deviatoric_direction_closed_form(beta)
            sgn = np.sign(np.dot(c, d))
            assert np.allclose(sgn * c, d, atol=1e-13), beta


def test_rotation_matches_rotation_vector():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(9)
    for _ in range(20):
        th, psi, phi = rng.uniform(0, np.pi), rng.uniform(0, np.pi), rng.uniform(0, 2 * np.pi)
        n = np.array([np.sin(psi) * np.cos(phi), np.sin(psi) * np.sin(phi), np.cos(psi)])
        R = T.axis_angle_rotation(th, psi, phi)
        assert np.allclose(R, Rotation.from_rotvec(th * n).as_matrix(), atol=1e-14)


def test_theta_inversion():
    for u in (0.0, 1e-9, 0.1, 0.37, 0.5, 0.999, 1.0):
        th = T.theta_from_unit(u)
        assert 0.0 <= th <= np.pi
        assert abs(th - np.sin(th) - np.pi * u) < 1e-14


def test_sampled_stiffness_spectra():
    """C1 has eigenvalues 3 K1 (once) and 2 G1 (five times); C2 has 3 K2, 2 G2
    four times and 2 G2 (1 - a) along the rotated direction N'."""
    from scipy.stats import qmc
    u = qmc.Sobol(d=8, scramble=True, seed=12).random(64)
    for x in u:
        a, e1, e2, e3, beta, th, psi, phi = T.sample_parameters(x)
        C1, C2 = T.sample_stiffness(x)
        G1, K2, G2 = 10.0 ** e1, 10.0 ** e2, 10.0 ** e3
        ev1 = np.sort(np.linalg.eigvalsh(C1))
        assert np.allclose(ev1, np.sort([3.0] + [2 * G1] * 5), rtol=1e-12)
        ev2 = np.sort(np.linalg.eigvalsh(C2))
        assert np.allclose(ev2, np.sort([3 * K2] + [2 * G2] * 4 + [2 * G2 * (1 - a)]),
                           rtol=1e-11)
        Q = T.axis_angle_rotation(th, psi, phi)
        nv = sym_to_mandel(Q @ np.diag(T.deviatoric_direction(beta)) @ Q.T)
        assert abs(np.dot(nv, nv) - 1.0) < 1e-12 and abs(nv[:3].sum()) < 1e-12
        assert np.allclose(C2 @ nv, 2 * G2 * (1 - a) * nv, rtol=1e-11, atol=1e-11 * G2)
        assert np.allclose(C2 @ P1 @ np.ones(6), 3 * K2 * P1 @ np.ones(6), rtol=1e-12)


def test_sampler_domains_at_cube_corners():
    lo = T.sample_parameters(np.zeros(8))
    hi = T.sample_parameters(np.ones(8))
    assert np.allclose(lo, (0.0, -3.0, -3.0, -3.0, 0.0, 0.0, 0.0, 0.0), rtol=0, atol=1e-14)
    assert np.allclose(hi, (1.0, 3.0, 3.0, 3.0, 2 * np.pi, np.pi, np.pi, 2 * np.pi), atol=1e-14)


def test_zero_differences_have_zero_derivative():
    """Reading T2: entries where target and prediction agree contribute no
    gradient, and neither does a sample without error."""
    rs = S.streams(34)
    Tt = S.random_spd(rs["stiffness"], 3)
    Cb = Tt * (1.0 + 0.1 * rs["noise"].standard_normal(Tt.shape))
    Cb[0] = Tt[0]
    Cb[1, 2, 2] = Tt[1, 2, 2]
    for p, q in ((1.0, 1.0), (1.0, 10.0), (2.0, 1.0)):
        G = T.data_cotangent(Cb, Tt, p, q)
        assert np.all(G[0] == 0.0) and G[1, 2, 2] == 0.0
        assert np.all(G[2] != 0.0)


def test_objective_with_a_dead_subtree_matches_differences():
    """Leaves 2 and 3 (a whole sibling pair) cut off by the Macaulay bracket:
    the objective is that of the compressed tree; its complex-step gradient
    matches differences in every parameter, and the dead weights and the
    normal of the dead laminate and of its parent get none."""
    K = 2
    C1, C2, truth, _, _, v, alpha, beta = _case(K=K, B=4)
    Tt = dmn_linear(K, truth.w, truth.normals, C1, C2)
    v = v.copy()
    v[2], v[3] = -0.05, -0.02
    g = T.objective_gradient(K, v, alpha, beta, C1, C2, Tt, 1.0, 10.0, 10.0)
    fv = lambda x: T.objective(K, x, alpha, beta, C1, C2, Tt, 1.0, 10.0, 10.0)
    fa = lambda x: T.objective(K, v, x, beta, C1, C2, Tt, 1.0, 10.0, 10.0)
    fb = lambda x: T.objective(K, v, alpha, x, C1, C2, Tt, 1.0, 10.0, 10.0)
    for key, f, x in (("gv", fv, v), ("galpha", fa, alpha), ("gbeta", fb, beta)):
        for i in range(len(x)):
            fd = _richardson(f, x, i, 1e-4)
            assert abs(g[key][i] - fd) <= 1e-7 * max(1.0, abs(fd)), (key, i)
    # laminate over leaves 2, 3 is dead; the root then has a single child
    from oracle.tree import lam_pos
    for k, i in ((2, 2), (1, 1)):
        p = lam_pos(K, k, i)
        assert g["galpha"][p] == 0.0 and g["gbeta"][p] == 0.0
    assert g["gv"][2] == 0.0 and g["gv"][3] == 0.0


def test_orientation_discretization_counts_and_hierarchy():
    """Four, ten and 31 sampling points after 0, 1, 2 subdivisions (Sec. 4.3),
    each level containing the previous one, all inside the triangle."""
    from oracle.orientation import in_triangle
    prev = None
    for level, n in ((0, 4), (1, 10), (2, 31)):
        pts = S.orientation_discretization(level)
        assert len(pts) == n
        assert all(in_triangle(l1, l2, 1e-12) for l1, l2 in pts)
        if prev is not None:
            for p in prev:
                assert np.min(np.abs(pts - p).sum(axis=1)) < 1e-12
        prev = pts


def _oriented_case(K=2, B=4, kind="trilinear", seed=81):
    rs = S.streams(seed)
    C1 = S.random_spd(rs["stiffness"], B)
    C2 = S.random_spd(rs["stiffness"], B)
    truth = S.interpolated_dmn(rs["ground_truth"], K, 0.3, kind)
    lam = S.orientation_discretization(1)[[0, 4, 7, 9][:B]]
    v = rs["init"].uniform(0.2, 1.0, 2 ** K)
    v = 1.1 * v / v.sum()
    M = S.SHAPE_COUNTS[kind]
    P = rs["init"].uniform(0.0, 2 * np.pi, (2 ** K - 1, M))
    Q = rs["init"].uniform(0.0, 2 * np.pi, (2 ** K - 1, M))
    from oracle.orientation import oriented_linear
    Tt = oriented_linear(K, truth.w, truth.p, truth.q, kind, lam, C1, C2)
    return C1, C2, lam, v, P, Q, Tt


def test_oriented_objective_reduces_to_fixed_normals():
    """Equal coefficients across the shape functions give every orientation
    the same angles (partition of unity): the oriented objective and its
    coefficient gradients reduce to the fixed-normal ones (summed over j)."""
    K, kind = 2, "quadratic"
    C1, C2, lam, v, P, Q, Tt = _oriented_case(K=K, kind=kind)
    M = S.SHAPE_COUNTS[kind]
    a, b = P[:, 0], Q[:, 0]
    Pc, Qc = np.repeat(a[:, None], M, 1), np.repeat(b[:, None], M, 1)
    J1 = T.objective_oriented(K, v, Pc, Qc, kind, lam, C1, C2, Tt, 1.0, 10.0, 10.0)
    J0 = T.objective(K, v, a, b, C1, C2, Tt, 1.0, 10.0, 10.0)
    assert abs(J1 - J0) <= 1e-12 * abs(J0)
    g1 = T.objective_oriented_gradient(K, v, Pc, Qc, kind, lam, C1, C2, Tt, 1.0, 10.0, 10.0)
    g0 = T.objective_gradient(K, v, a, b, C1, C2, Tt, 1.0, 10.0, 10.0)
    assert np.allclose(g1["gv"], g0["gv"], rtol=1e-10, atol=1e-12)
    assert np.allclose(g1["gP"].sum(axis=1), g0["galpha"], rtol=1e-10, atol=1e-12)
    assert np.allclose(g1["gQ"].sum(axis=1), g0["gbeta"], rtol=1e-10, atol=1e-12)


def test_oriented_objective_gradient_matches_differences():
    K, kind = 2, "linear"
    C1, C2, lam, v, P, Q, Tt = _oriented_case(K=K, kind=kind, seed=82)
    g = T.objective_oriented_gradient(K, v, P, Q, kind, lam, C1, C2, Tt, 1.0, 10.0, 10.0)
    f = lambda vv, PP, QQ: T.objective_oriented(K, vv, PP, QQ, kind, lam, C1, C2, Tt, 1.0,
                                                10.0, 10.0)
    for i in range(len(v)):
        fd = _richardson(lambda x: f(x, P, Q), v, i, 1e-4)
        assert abs(g["gv"][i] - fd) <= 1e-7 * max(1.0, abs(fd)), i
    for idx in np.ndindex(*P.shape):
        flat = np.ravel_multi_index(idx, P.shape)
        fdp = _richardson(lambda x: f(v, x.reshape(P.shape), Q), P.ravel(), flat, 1e-4)
        fdq = _richardson(lambda x: f(v, P, x.reshape(Q.shape)), Q.ravel(), flat, 1e-4)
        assert abs(g["gP"][idx] - fdp) <= 1e-7 * max(1.0, abs(fdp)), idx
        assert abs(g["gQ"][idx] - fdq) <= 1e-7 * max(1.0, abs(fdq)), idx


def _training_setup():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "training_setup.txt")
    disc, const = [], {}
    for line in open(path):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "discretization":
            disc.append(tuple(int(x) for x in f[1:]))
        else:
            const[f[0]] = float(f[1])
    return disc, const


def test_sample_table_of_the_paper():
    """The table of sample counts: 4, 10, 31 sampling points; cyclic
    assignment of the samples gives the printed samples per microstructure;
    the 90 / 10 split gives the printed set sizes."""
    disc, _ = _training_setup()
    for level, points, total, per, train, val in disc:
        lam = S.orientation_discretization(level)
        assert len(lam) == points
        counts = np.bincount(np.arange(total) % points, minlength=points)
        assert np.all(counts == per)
        assert round(0.9 * total) == train and total - train == val


def test_optimiser_defaults_are_the_papers():
    from paper_2103_08253_amd.training import AmsgradOpts
    _, c = _training_setup()
    o = AmsgradOpts()
    assert (o.lr_max, o.lr_min, o.lr_decay, o.half_period, o.penalty) == \
        (c["lr_max"], c["lr_min"], c["lr_decay"], int(c["half_period"]), c["penalty"])
    assert T.learning_rate(0) == c["lr_max"]
    assert abs(T.learning_rate(int(c["half_period"])) -
               c["lr_decay"] ** c["half_period"] * c["lr_min"]) < 1e-18
