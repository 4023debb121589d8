"""Pins of the exponential-linear hardening law of the matrix (Sec. 4.1, CPU only).

The paper writes the yield stress in terms of four table constants,

    sigma_Y(p) = sigma0 + k_inf p + (sigma_inf - sigma0)(1 - exp(-(k0 - k_inf)/(sigma_inf - sigma0) p)),

so the initial yield stress is sigma0, the initial hardening modulus is k0,
the late hardening modulus is k_inf and the saturation stress of the
exponential part is sigma_inf.  The oracle (and the kernels) use the
equivalent form sigma0 + k_inf p + dsigma (1 - exp(-b p)).  These tests pin
that form through the four properties that define the table constants, not by
retyping a formula: a sign or factor slip in the exponential term (exponent,
rate, amplitude) changes at least one of them.  The constants come from the
golden fixture of the material table (tests/golden/material_parameters.txt).
"""
import os

import numpy as np
import pytest

import synthetic as S
from oracle.j2 import J2Material, j2_update
from oracle.mandel import DELTA6

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "material_parameters.txt")


def table():
    """{phase: {name: value}} from the golden material table (MPa)."""
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            phase, name, value = line.split()
            out.setdefault(phase, {})[name] = float(value)
    return out


def yield_derivative(mat, p, h=1e-20):
    """dsigma_Y/dp by complex step (no cancellation; not the oracle's dsigma_y)."""
    return np.imag(mat.sigma_y(p + 1j * h)) / h


def check_table_properties(mat, sigma0, sigma_inf, k0, k_inf):
    """The four defining properties of the table constants; returns worst errors."""
    err = {}
    err["sigma_Y(0) = sigma0"] = abs(mat.sigma_y(0.0) - sigma0) / sigma0
    err["dsigma_Y/dp(0) = k0"] = abs(yield_derivative(mat, 0.0) - k0) / k0
    # late slope and saturation: at p far beyond the decay length (sigma_inf - sigma0)/(k0 - k_inf)
    p_far = 200.0 * (sigma_inf - sigma0) / (k0 - k_inf)
    err["dsigma_Y/dp(inf) = k_inf"] = abs(yield_derivative(mat, p_far) - k_inf) / k_inf
    err["sigma_Y(p) - k_inf p -> sigma_inf"] = abs(mat.sigma_y(p_far) - k_inf * p_far - sigma_inf) / sigma_inf
    # the oracle's own derivative (used in the return and its tangent) agrees
    for p in (0.0, 1e-4, 3e-3, 0.05):
        d = abs(mat.dsigma_y(p) - yield_derivative(mat, p)) / k0
        err["dsigma_y = d sigma_y / dp"] = max(err.get("dsigma_y = d sigma_y / dp", 0.0), d)
    return err


def test_golden_table_values():
    """The fixture holds the paper's table (Sec. 4.1) in MPa."""
    t = table()
    assert t["matrix"] == dict(E=2100.0, nu=0.3, sigma0=29.0, sigma_inf=61.7, k0=10600.0,
                               k_inf=139.0)
    assert t["fiber"] == dict(E=72000.0, nu=0.22)


def test_paper_constants_derive_from_the_table():
    """synthetic.MATRIX_PAPER (the kernels' form) follows from the table:
    dsigma = sigma_inf - sigma0, b = (k0 - k_inf) / (sigma_inf - sigma0)."""
    t = table()
    m = t["matrix"]
    P = S.MATRIX_PAPER
    assert P["E"] == m["E"] and P["nu"] == m["nu"]
    assert P["sigma0"] == m["sigma0"] and P["k_inf"] == m["k_inf"]
    assert np.isclose(P["dsigma"], m["sigma_inf"] - m["sigma0"], rtol=1e-15)
    assert np.isclose(P["b"], (m["k0"] - m["k_inf"]) / (m["sigma_inf"] - m["sigma0"]), rtol=1e-15)
    assert S.FIBER_PAPER == t["fiber"]


def test_paper_hardening_law_has_the_table_properties():
    m = table()["matrix"]
    mat = J2Material(**S.MATRIX_PAPER)
    err = check_table_properties(mat, m["sigma0"], m["sigma_inf"], m["k0"], m["k_inf"])
    for name, e in err.items():
        assert e <= 1e-12, (name, e)


def test_workload_hardening_law_has_its_table_properties():
    """The workload's law 50 + 200 p + 30 (1 - e^{-60 p}) in table form:
    sigma0 = 50, k_inf = 200, sigma_inf = 80, k0 = 200 + 30 * 60 = 2000."""
    mat = J2Material(**S.MATRIX)
    err = check_table_properties(mat, 50.0, 80.0, 2000.0, 200.0)
    for name, e in err.items():
        assert e <= 1e-12, (name, e)


def test_curvature_at_zero():
    """sigma_Y''(0) = -(k0 - k_inf)^2 / (sigma_inf - sigma0): the exponential part is
    concave with that curvature (second derivative by complex step of the slope)."""
    m = table()["matrix"]
    mat = J2Material(**S.MATRIX_PAPER)
    h = 1e-20
    curv = np.imag(mat.dsigma_y(0.0 + 1j * h)) / h
    ref = -(m["k0"] - m["k_inf"]) ** 2 / (m["sigma_inf"] - m["sigma0"])
    assert abs(curv - ref) <= 1e-12 * abs(ref)


def test_plastic_return_reaches_the_table_yield_stress():
    """After a plastic return with the paper's constants, the von Mises stress
    equals the table-form yield stress at the new p (uniaxial-like strain,
    several sizes reaching into the exponential and the linear regime)."""
    m = table()["matrix"]
    s0, si, k0, ki = m["sigma0"], m["sigma_inf"], m["k0"], m["k_inf"]

    def table_yield(p):
        return s0 + ki * p + (si - s0) * (1.0 - np.exp(-(k0 - ki) / (si - s0) * p))

    mat = J2Material(**S.MATRIX_PAPER)
    for amp in (0.02, 0.03, 0.06, 0.2):
        eps = amp * np.array([1.0, -0.3, -0.3, 0.0, 0.0, 0.0])
        out = j2_update(mat, eps, np.zeros(6), 0.0)
        assert out["plastic"] and out["ok"]
        s = out["sigma"] - (out["sigma"][:3].sum() / 3.0) * DELTA6
        vm = np.sqrt(1.5 * s @ s)
        assert abs(vm - table_yield(out["p"])) <= 1e-10 * vm


@pytest.mark.parametrize("mutation", ["exponent_sign", "rate_factor", "amplitude_sign"])
def test_pins_detect_a_planted_mistake(monkeypatch, mutation):
    """A slip planted in the oracle's exponential term (on the CPU) fails the pins."""
    def wrong(self, p):
        if mutation == "exponent_sign":
            return self.sigma0 + self.k_inf * p + self.dsigma * (1.0 - np.exp(self.b * p))
        if mutation == "rate_factor":
            return self.sigma0 + self.k_inf * p + self.dsigma * (1.0 - np.exp(-0.5 * self.b * p))
        return self.sigma0 + self.k_inf * p - self.dsigma * (1.0 - np.exp(-self.b * p))

    monkeypatch.setattr(J2Material, "sigma_y", wrong)
    m = table()["matrix"]
    mat = J2Material(**S.MATRIX_PAPER)
    with np.errstate(over="ignore", invalid="ignore"):
        err = check_table_properties(mat, m["sigma0"], m["sigma_inf"], m["k0"], m["k_inf"])
    assert any(not (e <= 1e-12) for e in err.values()), err
