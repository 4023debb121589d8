"""Pins of the oracle's J2 leaf law (CPU only).

* linear hardening (dsigma = 0) has the textbook closed-form radial return;
* after a plastic return the von Mises stress equals the current yield stress,
  the plastic strain stays traceless and flows along the stress deviator;
* the consistent tangent equals central finite differences of the stress;
* a uniaxial-stress path follows sigma_11 = sigma_Y(p) while loading
  plastically and unloads with slope E.
"""
import numpy as np
import pytest

import synthetic as S
from oracle.j2 import J2Material, j2_update
from oracle.mandel import DELTA6, iso_from_E_nu

SQ23 = np.sqrt(2.0 / 3.0)


def dev(v):
    return v - (v[0] + v[1] + v[2]) / 3.0 * DELTA6


def von_mises(sig):
    s = dev(sig)
    return np.sqrt(1.5 * s @ s)


def test_elastic_branch_is_linear_elastic():
    mat = J2Material(**S.MATRIX)
    eps = np.array([1e-3, -2e-4, 3e-4, 1e-4, 0.0, -2e-4])
    out = j2_update(mat, eps, np.zeros(6), 0.0)
    assert not out["plastic"]
    C = iso_from_E_nu(S.MATRIX["E"], S.MATRIX["nu"])
    assert np.allclose(out["sigma"], C @ eps, rtol=1e-14, atol=1e-12)
    assert np.allclose(out["D"], C)


def test_linear_hardening_closed_form():
    prm = dict(S.MATRIX, dsigma=0.0)
    mat = J2Material(**prm)
    rng = np.random.default_rng(20)
    for _ in range(5):
        eps = rng.standard_normal(6) * 0.02
        ep_n = dev(rng.standard_normal(6)) * 1e-3
        p_n = 0.01
        out = j2_update(mat, eps, ep_n, p_n)
        e = eps - ep_n
        s_tr = 2 * mat.G * dev(e)
        q = np.linalg.norm(s_tr)
        f = q - SQ23 * (prm["sigma0"] + prm["k_inf"] * p_n)
        assert f > 0 and out["plastic"]
        dgam = f / (2 * mat.G + 2.0 / 3.0 * prm["k_inf"])
        assert np.isclose(out["p"], p_n + SQ23 * dgam, rtol=1e-13)
        assert np.allclose(out["ep"], ep_n + dgam * s_tr / q, rtol=1e-12, atol=1e-16)
        sig = mat.K * (e[0] + e[1] + e[2]) * DELTA6 + s_tr - 2 * mat.G * dgam * s_tr / q
        assert np.allclose(out["sigma"], sig, rtol=1e-12, atol=1e-9)


def test_plastic_return_consistency_and_flow():
    mat = J2Material(**S.MATRIX)
    rng = np.random.default_rng(21)
    for _ in range(20):
        eps = rng.standard_normal(6) * 0.03
        ep_n = dev(rng.standard_normal(6)) * 2e-3
        p_n = rng.uniform(0, 0.05)
        out = j2_update(mat, eps, ep_n, p_n)
        if not out["plastic"]:
            continue
        assert out["ok"]
        assert np.isclose(von_mises(out["sigma"]), mat.sigma_y(out["p"]), rtol=1e-12)
        dep = out["ep"] - ep_n
        assert abs(dep[0] + dep[1] + dep[2]) <= 1e-15
        s = dev(out["sigma"])
        assert np.allclose(dep / np.linalg.norm(dep), s / np.linalg.norm(s), atol=1e-12)
        assert np.isclose(out["p"] - p_n, SQ23 * np.linalg.norm(dep), rtol=1e-12)


@pytest.mark.parametrize("seed", [22, 23, 24])
def test_consistent_tangent_matches_finite_differences(seed):
    mat = J2Material(**S.MATRIX)
    rng = np.random.default_rng(seed)
    eps = rng.standard_normal(6) * 0.02
    ep_n = dev(rng.standard_normal(6)) * 1e-3
    p_n = 0.004
    out = j2_update(mat, eps, ep_n, p_n)
    assert out["plastic"]
    h = 1e-7
    fd = np.zeros((6, 6))
    for c in range(6):
        d = np.zeros(6)
        d[c] = h
        fd[:, c] = (j2_update(mat, eps + d, ep_n, p_n)["sigma"]
                    - j2_update(mat, eps - d, ep_n, p_n)["sigma"]) / (2 * h)
    D = out["D"]
    assert np.allclose(D, D.T, atol=1e-9)
    assert np.abs(fd - D).max() <= 1e-6 * np.abs(D).max()


def test_uniaxial_stress_path_and_unloading():
    """Drive eps_11, keep all other stresses zero (lateral strains from Newton)."""
    mat = J2Material(**S.MATRIX)
    E_young = S.MATRIX["E"]
    ep, p = np.zeros(6), 0.0
    eps = np.zeros(6)
    history = []
    for e11 in list(np.linspace(0.0, 0.04, 41)[1:]) + list(np.linspace(0.04, 0.035, 6)[1:]):
        eps[0] = e11
        for _ in range(30):
            out = j2_update(mat, eps, ep, p)
            r = out["sigma"][1:]
            if np.abs(r).max() < 1e-10:
                break
            eps[1:] -= np.linalg.solve(out["D"][1:, 1:], r)
        history.append((e11, out["sigma"][0], out["p"], out["plastic"]))
        ep, p = out["ep"], out["p"]
    for e11, s11, pp, plastic in history:
        if plastic:
            assert np.isclose(s11, mat.sigma_y(pp), rtol=1e-10)
    # unloading steps are elastic with slope E
    unl = history[-5:]
    assert not any(h[3] for h in unl)
    slope = (unl[-1][1] - unl[0][1]) / (unl[-1][0] - unl[0][0])
    assert np.isclose(slope, E_young, rtol=1e-10)
