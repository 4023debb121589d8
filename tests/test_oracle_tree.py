"""Pins of the oracle's Mandel algebra and tree topology (CPU only).

The laminate projector and the symmetrisation operator are built by two
independent routes (the paper's component formula for P(n), the definition
of N(n)) and checked against each other and against their algebraic
properties.  The gradient operator is checked against the depth-3 example
printed in Sec. 3.2 (golden fixture) and against the strain-average identity.
"""
import os
import re

import numpy as np

from oracle import mandel as M
from oracle import tree as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_unit(rng):
    g = rng.standard_normal(3)
    return g / np.linalg.norm(g)


def test_mandel_roundtrip_and_inner_product():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 3)); A = A + A.T
    B = rng.standard_normal((3, 3)); B = B + B.T
    a, b = M.sym_to_mandel(A), M.sym_to_mandel(B)
    assert np.allclose(M.mandel_to_sym(a), A)
    assert np.isclose(a @ b, np.sum(A * B))  # Mandel dot = Frobenius product


def test_N_gram_matrix():
    rng = np.random.default_rng(1)
    for _ in range(5):
        n = rand_unit(rng)
        N = M.N_matrix(n)
        assert np.allclose(N.T @ N, 0.5 * (np.eye(3) + np.outer(n, n)), atol=1e-15)
        a = rng.standard_normal(3)
        S = 0.5 * (np.outer(a, n) + np.outer(n, a))
        assert np.allclose(N @ a, M.sym_to_mandel(S))


def test_projector_matches_symmetrisation_range():
    """P(n) from the paper's component formula = orthogonal projector onto {sym(a (x) n)}."""
    rng = np.random.default_rng(2)
    for _ in range(5):
        n = rand_unit(rng)
        P = M.projector_P(n)
        N = M.N_matrix(n)
        assert np.allclose(P, P.T, atol=1e-15)
        assert np.allclose(P @ P, P, atol=1e-14)
        assert np.isclose(np.trace(P), 3.0)
        assert np.allclose(P @ N, N, atol=1e-14)
        assert np.allclose(P, N @ np.linalg.solve(N.T @ N, N.T), atol=1e-14)


def test_isotropic_stiffness_is_lame_law():
    E, nu = 2800.0, 0.35
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    C = M.iso_from_E_nu(E, nu)
    rng = np.random.default_rng(3)
    eps = rng.standard_normal((3, 3)); eps = eps + eps.T
    sig = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
    assert np.allclose(C @ M.sym_to_mandel(eps), M.sym_to_mandel(sig))


def test_laminate_positions_follow_paper_order():
    K = 3
    order = [(3, 1), (3, 2), (3, 3), (3, 4), (2, 1), (2, 2), (1, 1)]
    assert T.laminates(K) == order
    assert [T.lam_pos(K, k, i) for (k, i) in order] == list(range(7))
    assert T.lam_leaves(3, 1, 1) == (0, 8)
    assert T.lam_leaves(3, 2, 2) == (4, 8)
    assert T.lam_leaves(3, 3, 4) == (6, 8)


def test_fractions_from_weight_propagation():
    w = np.array([0.1, 0.3, 0.2, 0.4])
    c1, c2 = T.fractions(2, w)
    # level 2: (0.1 | 0.3), (0.2 | 0.4); root: (0.4 | 0.6)
    assert np.allclose(c1, [0.25, 1 / 3, 0.4])
    assert np.allclose(c1 + c2, 1.0)


def _parse_printed_operator():
    rows = []
    with open(os.path.join(GOLDEN, "gradient_operator_depth3.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([e.strip() for e in line.split("|")])
    return rows


def test_gradient_operator_matches_printed_depth3_example():
    """Sec. 3.2, displayed depth-3 operator: block pattern, signs, fractions, order."""
    rows = _parse_printed_operator()
    assert len(rows) == 8 and all(len(r) == 7 for r in rows)
    rng = np.random.default_rng(4)
    K = 3
    w = rng.uniform(0.2, 1.0, 8)
    normals = np.array([rand_unit(rng) for _ in range(7)])
    A = T.gradient_operator(K, w, normals, sparse=False)
    c1, c2 = T.fractions(K, w)
    pat = re.compile(r"([+-])c\^(\d+)_(\d+) N\^(\d+)_(\d+)")
    for r, row in enumerate(rows):
        for col, entry in enumerate(row):
            blk = A[6 * r:6 * r + 6, 3 * col:3 * col + 3]
            if entry == "0":
                assert np.all(blk == 0.0)
                continue
            m = pat.fullmatch(entry)
            assert m, entry
            sign = 1.0 if m.group(1) == "+" else -1.0
            j, kc, i, kn = (int(m.group(g)) for g in (2, 3, 4, 5))
            assert kc == kn
            assert T.lam_pos(K, kn, i) == col  # column order of the printed example
            assert j in (2 * i - 1, 2 * i)
            c = c1[col] if j == 2 * i - 1 else c2[col]
            expect = sign * c * M.N_matrix(normals[col])
            assert np.allclose(blk, expect, atol=1e-15)


def test_strain_average_identity():
    """sum_j w~_j (A a)_j = 0 for every a: the jumps never change the mean strain."""
    rng = np.random.default_rng(5)
    for K in (1, 2, 4, 6):
        w = rng.uniform(0.1, 1.0, 2 ** K)
        normals = np.array([rand_unit(rng) for _ in range(2 ** K - 1)])
        A = T.gradient_operator(K, w, normals)
        a = rng.standard_normal(3 * (2 ** K - 1))
        eps = (A @ a).reshape(-1, 6)
        assert np.allclose((w / w.sum()) @ eps, 0.0, atol=1e-14)


def test_state_counts_of_paper():
    """Sec. 6: a depth-8 DMN stores 128 x (1+5) = 768 internal variables and 765 jumps."""
    vals = {}
    with open(os.path.join(GOLDEN, "state_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = int(v)
    K = vals["depth"]
    assert 2 ** K // 2 == vals["matrix_leaves"]
    assert vals["matrix_leaves"] * vals["internal_per_leaf_paper"] == vals["internal_total_paper"]
    assert 3 * T.n_laminates(K) == vals["jumps"]
    assert vals["internal_total_paper"] + vals["jumps"] == vals["total_paper"]
