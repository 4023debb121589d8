"""Pins of the oracle's Gauss-point update (CPU only).

* an elastic step reproduces the linear DMN: sigma = C_lin E, C_algo = C_lin
  (C_lin from Milton's formula, an independent route);
* at convergence the leaf strains average to E and the Hill-Mandel identity
  E . sigma = sum_j w~_j eps_j . sigma_j holds;
* the algorithmic tangent equals central finite differences of sigma(E);
* depth 1 agrees with a general-purpose root finder on the interface
  condition written out by hand;
* equal normals collapse a nonlinear depth-4 DMN to a single laminate;
* identical elastic phases leave the jumps at zero;
* the status codes of the failure modes;
* rotating the load path and the normals rotates the outputs (isotropic phases);
* exchanging the two subtrees of the root leaves the outputs unchanged and
  negates the root jump.
"""
import numpy as np
import scipy.optimize as so

import synthetic as S
from oracle import gp as G
from oracle.j2 import J2Material, j2_update
from oracle.linear import dmn_linear
from oracle.mandel import N_matrix, iso_from_E_nu


def model_for(net, fiber=S.FIBER, matrix=S.MATRIX):
    return G.DmnModel(net.depth, net.w, net.normals, fiber, matrix)


def test_elastic_step_equals_linear_dmn():
    rng = np.random.default_rng(30)
    net = S.random_dmn(rng, 3, 0.25)
    m = model_for(net)
    E = 1e-4 * S.unit_directions(rng, 1)[0]
    out = G.gp_update(m, E, np.zeros((4, 7)), np.zeros(21))
    assert out["status"] == 0 and out["iters"] == 1
    Cf = iso_from_E_nu(S.FIBER["E"], S.FIBER["nu"])
    Cm = iso_from_E_nu(S.MATRIX["E"], S.MATRIX["nu"])
    Clin = dmn_linear(3, net.w, net.normals, Cf, Cm)
    assert np.abs(out["C"] - Clin).max() <= 1e-11 * np.abs(Clin).max()
    assert np.abs(out["sigma"] - Clin @ E).max() <= 1e-11 * np.abs(out["sigma"]).max()
    assert np.all(out["z"] == 0.0)


def plastic_state(K, seed, steps=6, mag=0.02):
    rng = np.random.default_rng(seed)
    net = S.random_dmn(rng, K, 0.25)
    m = model_for(net)
    d = S.unit_directions(rng, 1)[0]
    path = [(n / steps) * mag * d for n in range(1, steps + 1)]
    outs = G.run_path(m, path)
    assert all(o["status"] == 0 for o in outs)
    return m, path, outs


def test_equilibrium_strain_average_and_hill_mandel():
    m, path, outs = plastic_state(4, 31)
    last = outs[-1]
    assert np.any(last["z"][:, 6] > 0)
    eps, sig = last["eps"], last["sig_leaf"]
    wt = m.w / m.w.sum()
    assert np.allclose(wt @ eps, path[-1], atol=1e-15)
    lhs = path[-1] @ last["sigma"]
    rhs = np.sum(wt * np.einsum("ja,ja->j", eps, sig))
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs)


def test_algorithmic_tangent_matches_finite_differences():
    m, path, outs = plastic_state(3, 32)
    z_n, a_n = outs[-2]["z"], outs[-2]["a"]
    E = path[-1]
    tight = G.NewtonOptions(tol=1e-14, max_iter=50)
    C = G.gp_update(m, E, z_n, a_n, tight)["C"]
    h = 1e-7
    fd = np.zeros((6, 6))
    for c in range(6):
        d = np.zeros(6)
        d[c] = h
        fd[:, c] = (G.gp_update(m, E + d, z_n, a_n, tight)["sigma"]
                    - G.gp_update(m, E - d, z_n, a_n, tight)["sigma"]) / (2 * h)
    assert np.abs(fd - C).max() <= 1e-5 * np.abs(C).max()
    assert np.abs(C - C.T).max() <= 1e-10 * np.abs(C).max()


def test_depth1_matches_generic_root_finder():
    rng = np.random.default_rng(33)
    net = S.random_dmn(rng, 1, 0.3)
    m = model_for(net)
    mat = J2Material(**S.MATRIX)
    Cf = iso_from_E_nu(S.FIBER["E"], S.FIBER["nu"])
    c1 = net.w[0] / net.w.sum()
    c2 = 1 - c1
    N = N_matrix(net.normals[0])
    d = S.unit_directions(rng, 1)[0]
    z, a = np.zeros((1, 7)), np.zeros(3)
    for n in range(1, 6):
        E = n * 0.005 * d
        out = G.gp_update(m, E, z, a, G.NewtonOptions(tol=1e-14, max_iter=50))

        def interface(x):
            sf = Cf @ (E - c2 * N @ x)
            sm = j2_update(mat, E + c1 * N @ x, z[0, :6], z[0, 6])["sigma"]
            return N.T @ (sm - sf)

        sol = so.root(interface, a, method="hybr", options=dict(xtol=1e-14))
        x = sol.x
        sf = Cf @ (E - c2 * N @ x)
        mo = j2_update(mat, E + c1 * N @ x, z[0, :6], z[0, 6])
        sbar = c1 * sf + c2 * mo["sigma"]
        assert np.abs(out["sigma"] - sbar).max() <= 1e-9 * np.abs(sbar).max()
        z, a = out["z"], out["a"]


def test_equal_normals_collapse_nonlinear():
    rng = np.random.default_rng(34)
    net = S.random_dmn(rng, 4, 0.25)
    n = net.normals[0]
    deep = G.DmnModel(4, net.w, np.tile(n, (15, 1)), S.FIBER, S.MATRIX)
    f = net.w[0::2].sum()
    one = G.DmnModel(1, np.array([f, 1 - f]), n[None, :], S.FIBER, S.MATRIX)
    d = S.unit_directions(rng, 1)[0]
    path = [k * 0.004 * d for k in range(1, 7)]
    tight = G.NewtonOptions(tol=1e-14, max_iter=50)
    a_deep = G.run_path(deep, path, tight)
    a_one = G.run_path(one, path, tight)
    for x, y in zip(a_deep, a_one):
        assert np.abs(x["sigma"] - y["sigma"]).max() <= 1e-9 * np.abs(y["sigma"]).max()
        assert np.abs(x["C"] - y["C"]).max() <= 1e-8 * np.abs(y["C"]).max()


def test_identical_elastic_phases_keep_zero_jumps():
    rng = np.random.default_rng(35)
    net = S.random_dmn(rng, 3, 0.25)
    soft = dict(S.MATRIX)
    m = G.DmnModel(3, net.w, net.normals, dict(E=soft["E"], nu=soft["nu"]), soft)
    E = 1e-4 * S.unit_directions(rng, 1)[0]
    out = G.gp_update(m, E, np.zeros((4, 7)), np.zeros(21))
    assert out["status"] == 0
    assert np.abs(out["a"]).max() <= 1e-15
    C = iso_from_E_nu(soft["E"], soft["nu"])
    assert np.allclose(out["sigma"], C @ E, rtol=1e-13)


def test_status_codes():
    rng = np.random.default_rng(36)
    net = S.random_dmn(rng, 2, 0.25)
    z, a = np.zeros((2, 7)), np.zeros(9)
    E = 0.02 * S.unit_directions(rng, 1)[0]
    bad = G.DmnModel(2, np.array([0.5, -0.1, 0.3, 0.3]), net.normals, S.FIBER, S.MATRIX)
    assert G.gp_update(bad, E, z, a)["status"] == G.BADPARAM
    zero_pair = G.DmnModel(2, np.array([0.0, 0.0, 0.5, 0.5]), net.normals, S.FIBER, S.MATRIX)
    assert G.gp_update(zero_pair, E, z, a)["status"] == G.BADPARAM
    m = model_for(net)
    out = G.gp_update(m, E * np.nan, z, a)
    assert out["status"] == G.NONFINITE and np.all(out["z"] == z)
    out = G.gp_update(m, E, z, a, G.NewtonOptions(max_iter=0))
    assert out["status"] == G.MAXITER and out["iters"] == 0
    # zero strain from the virgin state: zero residual, converged without a step
    out = G.gp_update(m, np.zeros(6), z, a)
    assert out["status"] == 0 and out["iters"] == 0
    # a zero normal makes its laminate's block of the Hessian vanish: not positive definite
    nz = net.normals.copy()
    nz[1] = 0.0
    out = G.gp_update(G.DmnModel(2, net.w, nz, S.FIBER, S.MATRIX), E, z, a)
    assert out["status"] == G.NOTSPD and out["iters"] == 0 and np.all(out["a"] == a)
    # the J2 return capped at one scalar iteration cannot meet its test on a plastic leaf
    out = G.gp_update(m, E, z, a, G.NewtonOptions(local_max_iter=1))
    assert out["status"] == G.LOCALFAIL and np.all(out["z"] == z)
    assert G.gp_update(m, E, z, a, G.NewtonOptions(local_max_iter=50))["status"] == 0
    # an elastic step never enters the scalar iteration
    out = G.gp_update(m, 1e-5 * E, z, a, G.NewtonOptions(local_max_iter=1))
    assert out["status"] == 0


def test_backtracking_rule():
    """With a strict sufficient-decrease factor (armijo close to 1) the full
    Newton step is rejected and halved (reading R5); the converged answer is
    the same as without backtracking, only the iteration count changes.  With
    max_backtrack = 1 a half step is accepted whatever its residual."""
    rng = np.random.default_rng(41)
    net = S.random_dmn(rng, 3, 0.25)
    m = model_for(net)
    E = 0.02 * S.unit_directions(rng, 1)[0]
    z, a = np.zeros((4, 7)), np.zeros(21)
    trials = []
    orig = m.evaluate

    def counting(*args):
        ev = orig(*args)
        trials.append(np.linalg.norm(ev["r"]))
        return ev

    m.evaluate = counting
    ref = G.gp_update(m, E, z, a)
    n_ref = len(trials)
    assert n_ref == ref["iters"] + 1  # no backtracking with the default rule
    for opts in (G.NewtonOptions(armijo=0.99), G.NewtonOptions(armijo=0.9999, max_backtrack=1)):
        trials.clear()
        out = G.gp_update(m, E, z, a, opts)
        assert out["status"] == 0
        assert len(trials) > out["iters"] + 1          # some trials were rejected
        assert np.allclose(out["sigma"], ref["sigma"], rtol=1e-9, atol=1e-9)
        assert np.allclose(out["C"], ref["C"], rtol=1e-7, atol=1e-6)


def test_rotational_covariance_of_the_nonlinear_update():
    """Isotropic phases: rotating the macro strain path and every normal by R
    rotates the stress, the tangent and the plastic strains, and leaves the
    accumulated plastic strains, the iteration counts and the jump lengths
    unchanged."""
    from oracle.mandel import rotation_mandel
    rng = np.random.default_rng(19)
    K = 3
    net = S.random_dmn(rng, K, 0.3)
    R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    Q = rotation_mandel(R)
    d = rng.standard_normal(6)
    E_path = np.outer(np.linspace(0.25, 1.0, 4), 0.04 * d / np.linalg.norm(d))
    base = G.run_path(G.DmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX), E_path)
    rot = G.run_path(G.DmnModel(K, net.w, net.normals @ R.T, S.FIBER, S.MATRIX),
                     E_path @ Q.T)
    assert any(np.abs(o["z"][:, 6]).max() > 0 for o in base)   # the path yields
    for b, r in zip(base, rot):
        assert b["status"] == r["status"] == 0 and b["iters"] == r["iters"]
        assert np.abs(r["sigma"] - Q @ b["sigma"]).max() <= 1e-10 * np.abs(b["sigma"]).max()
        assert np.abs(r["C"] - Q @ b["C"] @ Q.T).max() <= 1e-10 * np.abs(b["C"]).max()
        assert np.allclose(r["z"][:, :6], b["z"][:, :6] @ Q.T, atol=1e-12)
        assert np.allclose(r["z"][:, 6], b["z"][:, 6], atol=1e-14)
        ja = np.linalg.norm(b["a"].reshape(-1, 3), axis=1)
        jr = np.linalg.norm(r["a"].reshape(-1, 3), axis=1)
        assert np.allclose(ja, jr, rtol=1e-9, atol=1e-14)


def test_swapping_the_root_subtrees():
    """The laminate law is symmetric in its two children: exchanging the two
    subtrees of the root (their weights, normals and states) leaves stress,
    tangent and iteration counts unchanged, negates the root jump (the left
    child moves by -c2 N a, the right one by +c1 N a, Sec. 3.2) and permutes
    the other jumps and the internal variables.  A wrong fraction or sign in
    the localisation breaks the symmetry."""
    from oracle.tree import lam_pos, laminates
    rng = np.random.default_rng(20)
    K = 3
    net = S.random_dmn(rng, K, 0.3)
    half = 2 ** (K - 1)
    # laminate (k, i) below the root maps to (k, i -/+ 2^(k-2)) in the other subtree
    perm = np.arange(2 ** K - 1)
    for (k, i) in laminates(K):
        if k > 1:
            shift = 2 ** (k - 2)
            perm[lam_pos(K, k, i)] = lam_pos(K, k, i + shift if i <= shift else i - shift)
    w_sw = np.concatenate([net.w[half:], net.w[:half]])
    n_sw = net.normals[perm]
    d = rng.standard_normal(6)
    E_path = np.outer(np.linspace(0.25, 1.0, 4), 0.04 * d / np.linalg.norm(d))
    base = G.run_path(G.DmnModel(K, net.w, net.normals, S.FIBER, S.MATRIX), E_path)
    sw = G.run_path(G.DmnModel(K, w_sw, n_sw, S.FIBER, S.MATRIX), E_path)
    assert any(np.abs(o["z"][:, 6]).max() > 0 for o in base)   # the path yields
    root = lam_pos(K, 1, 1)
    mhalf = half // 2
    for b, s in zip(base, sw):
        assert b["status"] == s["status"] == 0 and b["iters"] == s["iters"]
        assert np.abs(s["sigma"] - b["sigma"]).max() <= 1e-10 * np.abs(b["sigma"]).max()
        assert np.abs(s["C"] - b["C"]).max() <= 1e-10 * np.abs(b["C"]).max()
        zb = np.concatenate([b["z"][mhalf:], b["z"][:mhalf]])
        assert np.allclose(s["z"], zb, rtol=1e-9, atol=1e-14)
        ab, as_ = b["a"].reshape(-1, 3), s["a"].reshape(-1, 3)
        assert np.allclose(as_[root], -ab[root], rtol=1e-9, atol=1e-14)
        others = [p for p in range(2 ** K - 1) if p != root]
        assert np.allclose(as_[perm[others]], ab[others], rtol=1e-9, atol=1e-14)
