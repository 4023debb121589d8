"""Seeded synthetic workloads for the DMN Gauss-point engine.

This module only draws random numbers and lays them out as inputs: DMN
parameters (leaf weights, lamination normals), phase constants, macro strain
paths and training stiffness pairs.  It holds none of the method's arithmetic
(no laminate homogenisation, no material law, no Newton step), so both the
CPU oracle and the GPU path can consume it without sharing any computation.

Workload shapes follow the paper's application: depth-8 direct DMNs
(Sec. 4.5), an isotropic elastic glass fibre and a J2 elasto-plastic matrix
(Sec. 4.1, table of material parameters), a fibre fraction around 25 %, and
macro strain increments of a few percent (Sec. 4.6).  The paper's own data
(FFT training tuples, trained DMN parameters, FE strain histories) is not
available; every input here is synthetic.

Random streams: ``numpy.random.default_rng`` seeded from
``SeedSequence(1000 + config_index).spawn(10)``; sub-stream roles are fixed by
``STREAMS`` so adding a draw to one role never shifts another.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

STREAMS = ("dmn", "direction", "noise", "elastic_mask", "assignment",
           "stiffness", "ground_truth", "init", "cotangent", "picks")

# Phase constants in MPa.  Fibre: E-glass (Sec. 4.1).  Matrix: the J2 law of
# Sec. 4.1 with the workload's constants sigma_y(p) = 50 + 200 p + 30 (1 - e^{-60 p}).
FIBER = dict(E=72000.0, nu=0.22)
MATRIX = dict(E=2800.0, nu=0.35, sigma0=50.0, k_inf=200.0, dsigma=30.0, b=60.0)
# The paper's own matrix constants (table of material parameters, Sec. 4.1):
# sigma0 = 29 MPa, sigma_inf = 61.7 MPa, k0 = 10.6 GPa, k_inf = 139 MPa, so
# dsigma = sigma_inf - sigma0 and b = (k0 - k_inf) / (sigma_inf - sigma0).
MATRIX_PAPER = dict(E=2100.0, nu=0.3, sigma0=29.0, k_inf=139.0,
                    dsigma=61.7 - 29.0, b=(10600.0 - 139.0) / (61.7 - 29.0))
FIBER_PAPER = dict(E=72000.0, nu=0.22)


def streams(config_index: int) -> dict:
    """Independent generators, one per role, for a configuration index."""
    ss = np.random.SeedSequence(1000 + int(config_index)).spawn(len(STREAMS))
    return {name: np.random.default_rng(s) for name, s in zip(STREAMS, ss)}


@dataclass
class DmnParams:
    """Parameters of one direct DMN of depth K.

    w: [2^K] non-negative leaf weights (leaf j even = fibre, odd = matrix).
    normals: [2^K - 1, 3] unit lamination normals in the paper's order
             (deepest level first, root last).
    """
    depth: int
    w: np.ndarray
    normals: np.ndarray

    @property
    def n_laminates(self) -> int:
        return 2 ** self.depth - 1


def unit_normals(rng: np.random.Generator, count: int) -> np.ndarray:
    g = rng.standard_normal((count, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def normals_to_angles(normals: np.ndarray):
    """Spherical angles (alpha, beta) with n = (sin a cos b, sin a sin b, cos a)."""
    alpha = np.arccos(np.clip(normals[:, 2], -1.0, 1.0))
    beta = np.arctan2(normals[:, 1], normals[:, 0])
    return alpha, beta


def rescale_to_fiber_fraction(w_raw: np.ndarray, fiber_fraction: float) -> np.ndarray:
    """Scale even (fibre) and odd (matrix) leaf weights to the given split; sum 1."""
    w = np.array(w_raw, dtype=np.float64)
    w[0::2] *= fiber_fraction / w[0::2].sum()
    w[1::2] *= (1.0 - fiber_fraction) / w[1::2].sum()
    return w


def random_dmn(rng: np.random.Generator, depth: int, fiber_fraction: float,
               weights: str = "lognormal") -> DmnParams:
    n_leaves = 2 ** depth
    if weights == "lognormal":
        w_raw = np.exp(rng.normal(0.0, 0.5, n_leaves))
    elif weights == "abs_normal":
        w_raw = np.abs(rng.normal(1.0, 0.3, n_leaves))
    else:
        raise ValueError(weights)
    w = rescale_to_fiber_fraction(w_raw, fiber_fraction)
    return DmnParams(depth, w, unit_normals(rng, n_leaves - 1))


def unit_directions(rng: np.random.Generator, count: int, dim: int = 6) -> np.ndarray:
    g = rng.standard_normal((count, dim))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


@dataclass
class GaussPointWorkload:
    """Macro strain paths at P Gauss points over T load steps.

    E: [T, P, 6] total macro strain (Mandel) at the end of each step.
    dmn_id: [P] index of the DMN of each point (all zero for one DMN).
    """
    nets: List[DmnParams]
    E: np.ndarray
    dmn_id: np.ndarray
    elastic_mask: Optional[np.ndarray] = None
    g_sigma: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def n_points(self) -> int:
        return self.E.shape[1]

    @property
    def n_steps(self) -> int:
        return self.E.shape[0]


def ramp_with_noise(rs: dict, n_points: int, n_steps: int, magnitude: float,
                    noise_std: float) -> np.ndarray:
    """E^n = (n/T) * magnitude * d_p + sum_{m<=n} xi_m, xi ~ N(0, noise_std^2 I6)."""
    d = unit_directions(rs["direction"], n_points)
    steps = np.arange(1, n_steps + 1, dtype=np.float64) / n_steps
    E = steps[:, None, None] * magnitude * d[None, :, :]
    if noise_std > 0.0:
        xi = rs["noise"].normal(0.0, noise_std, (n_steps, n_points, 6))
        E = E + np.cumsum(xi, axis=0)
    return E


def config0(n_points: int = 64, n_steps: int = 10) -> GaussPointWorkload:
    """Tiny: depth 2, |N(1,0.3)| weights at 25 % fibre, 10-step ramp to 2 %."""
    rs = streams(0)
    net = random_dmn(rs["dmn"], 2, 0.25, weights="abs_normal")
    E = ramp_with_noise(rs, n_points, n_steps, 0.02, 0.0)
    return GaussPointWorkload([net], E, np.zeros(n_points, np.int32),
                              meta=dict(name="depth2_tiny", config=0))


def config1(n_points: int = 65536, n_steps: int = 20) -> GaussPointWorkload:
    """Production depth: depth 8, log-normal weights, ramp to 1.5 % + N(0,1e-3) walk."""
    rs = streams(1)
    net = random_dmn(rs["dmn"], 8, 0.25, weights="lognormal")
    E = ramp_with_noise(rs, n_points, n_steps, 0.015, 1e-3)
    return GaussPointWorkload([net], E, np.zeros(n_points, np.int32),
                              meta=dict(name="depth8_production", config=1))


def config2(n_points: int = 131072, n_steps: int = 20) -> GaussPointWorkload:
    """Batching: 16 DMNs of depths 5..9, 30 % of points held nearly elastic."""
    rs = streams(2)
    depths = [5, 6, 7, 8, 9]
    nets = []
    for m in range(16):
        f = rs["dmn"].uniform(0.15, 0.35)
        nets.append(random_dmn(rs["dmn"], depths[m % 5], f, weights="lognormal"))
    dmn_id = rs["assignment"].integers(0, 16, n_points).astype(np.int32)
    E = ramp_with_noise(rs, n_points, n_steps, 0.015, 1e-3)
    perm = rs["elastic_mask"].permutation(n_points)
    mask = np.zeros(n_points, bool)
    mask[perm[: int(round(0.3 * n_points))]] = True
    E[:, mask, :] *= 0.05
    return GaussPointWorkload(nets, E, dmn_id, elastic_mask=mask,
                              meta=dict(name="mixed_depth_batch", config=2))


def config4(n_points: int = 16384, n_steps: int = 50) -> GaussPointWorkload:
    """Adjoint path: depth 8, ramp to 1.5 % over 50 steps + N(0,1e-3) walk."""
    rs = streams(4)
    net = random_dmn(rs["dmn"], 8, 0.25, weights="lognormal")
    E = ramp_with_noise(rs, n_points, n_steps, 0.015, 1e-3)
    g = unit_directions(rs["cotangent"], n_points)
    return GaussPointWorkload([net], E, np.zeros(n_points, np.int32), g_sigma=g,
                              meta=dict(name="depth8_adjoint_path", config=4))


def haar_orthogonal(rng: np.random.Generator, count: int, dim: int = 6) -> np.ndarray:
    """Haar-distributed O(dim) matrices: QR of a Gaussian, columns sign-fixed by diag(R)."""
    g = rng.standard_normal((count, dim, dim))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diagonal(r, axis1=1, axis2=2))
    s[s == 0] = 1.0
    return q * s[:, None, :]


def random_spd(rng: np.random.Generator, count: int, lo_exp: float = 0.0,
               hi_exp: float = 3.0) -> np.ndarray:
    """Q diag(lambda) Q^T with Q Haar and lambda = 10^U(lo,hi) (GPa-scaled)."""
    q = haar_orthogonal(rng, count)
    lam = 10.0 ** rng.uniform(lo_exp, hi_exp, (count, 6))
    c = np.einsum("bij,bj,bkj->bik", q, lam, q)
    return 0.5 * (c + np.transpose(c, (0, 2, 1)))


@dataclass
class TrainingWorkload:
    """Training batch: phase stiffness pairs, a ground-truth DMN and an init DMN.

    C1, C2: [B, 6, 6] Mandel stiffnesses (phase 1 on even leaves).
    truth: the DMN whose linear map produces the targets.
    v0, alpha0, beta0: initial unconstrained weights and normal angles.
    """
    C1: np.ndarray
    C2: np.ndarray
    truth: DmnParams
    v0: np.ndarray
    alpha0: np.ndarray
    beta0: np.ndarray
    meta: dict = field(default_factory=dict)


def config3(batch: int = 4096, depth: int = 8) -> TrainingWorkload:
    """Training: anisotropic SPD phase pairs, a seeded ground-truth depth-8 DMN."""
    rs = streams(3)
    C1 = random_spd(rs["stiffness"], batch)
    C2 = random_spd(rs["stiffness"], batch)
    truth = random_dmn(rs["ground_truth"], depth, 0.25, weights="lognormal")
    n_leaves = 2 ** depth
    v0 = rs["init"].uniform(0.0, 1.0, n_leaves)
    v0 = v0 / v0.sum()
    alpha0 = rs["init"].uniform(0.0, 2.0 * np.pi, n_leaves - 1)
    beta0 = rs["init"].uniform(0.0, 2.0 * np.pi, n_leaves - 1)
    return TrainingWorkload(C1, C2, truth, v0, alpha0, beta0,
                            meta=dict(name="depth8_training", config=3))


def angles_to_normals(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """n = (sin a cos b, sin a sin b, cos a): the spherical parameterisation of Sec. 2.3."""
    return np.stack([np.sin(alpha) * np.cos(beta), np.sin(alpha) * np.sin(beta),
                     np.cos(alpha)], axis=-1)


# ---------------------------------------------------------------- orientation

SHAPE_COUNTS = {"linear": 3, "trilinear": 4, "quadratic": 6}


@dataclass
class InterpolatedDmn:
    """A DMN whose normals depend on the fibre orientation (l1, l2): shared
    leaf weights w [2^K] and, per laminate (paper order), coefficient vectors
    p, q [2^K - 1, M] of the spherical angles over M shape functions."""
    depth: int
    w: np.ndarray
    p: np.ndarray
    q: np.ndarray
    kind: str


def interpolated_dmn(rng: np.random.Generator, depth: int, fiber_fraction: float, kind: str,
                     spread: float = 0.3) -> InterpolatedDmn:
    """Weights and base angles as random_dmn; each shape-function coefficient is
    the base angle plus N(0, spread^2), so the normals vary with orientation."""
    net = random_dmn(rng, depth, fiber_fraction)
    alpha, beta = normals_to_angles(net.normals)
    M = SHAPE_COUNTS[kind]
    L = net.n_laminates
    p = alpha[:, None] + spread * rng.standard_normal((L, M))
    q = beta[:, None] + spread * rng.standard_normal((L, M))
    return InterpolatedDmn(depth, net.w, p, q, kind)


def triangle_points(rng: np.random.Generator, count: int) -> np.ndarray:
    """[count, 2] points (l1, l2) uniform in the fibre orientation triangle
    1/3 <= l1 <= 1, 1 - 2 l1 <= l2 <= l1 (rejection from the bounding box)."""
    out = np.empty((0, 2))
    while out.shape[0] < count:
        c = np.column_stack([rng.uniform(1.0 / 3.0, 1.0, 4 * count),
                             rng.uniform(0.0, 1.0, 4 * count)])
        ok = (c[:, 1] >= 1.0 - 2.0 * c[:, 0]) & (c[:, 1] <= c[:, 0])
        out = np.vstack([out, c[ok]])
    return out[:count].copy()


def orientation_workload(n_points: int = 65536, n_steps: int = 20, kind: str = "quadratic",
                         depth: int = 8):
    """Depth-8 orientation-interpolated DMN, every point with its own (l1, l2);
    strain paths as the production workload.  Returns (net, lam [P, 2], E)."""
    rs = streams(5)
    net = interpolated_dmn(rs["dmn"], depth, 0.25, kind)
    lam = triangle_points(rs["assignment"], n_points)
    E = ramp_with_noise(rs, n_points, n_steps, 0.015, 1e-3)
    return net, lam, E


# ---------------------------------------------------------------- hysteresis

# Mandel components of the six uniaxial strain directions e_i (x) e_j
# (i, j) = 11, 22, 33, 23, 13, 12: the symmetric part of e_i (x) e_j, whose
# Mandel entry is sqrt(2) * 1/2 for i != j.
UNIAXIAL_DIRECTIONS = np.array([
    [1.0, 0.0, 0.0, 0.0, 0.0, 0.0],
    [0.0, 1.0, 0.0, 0.0, 0.0, 0.0],
    [0.0, 0.0, 1.0, 0.0, 0.0, 0.0],
    [0.0, 0.0, 0.0, np.sqrt(0.5), 0.0, 0.0],
    [0.0, 0.0, 0.0, 0.0, np.sqrt(0.5), 0.0],
    [0.0, 0.0, 0.0, 0.0, 0.0, np.sqrt(0.5)],
])


def hysteresis_factor(n_steps: int = 80) -> np.ndarray:
    """Scalar load factor of a full cycle in n_steps equidistant steps:
    0 -> +1 in a quarter, +1 -> -1 in a half, -1 -> 0 in the last quarter."""
    t = np.arange(1, n_steps + 1, dtype=np.float64) / n_steps
    return np.where(t <= 0.25, 4.0 * t, np.where(t <= 0.75, 2.0 - 4.0 * t, 4.0 * t - 4.0))


def hysteresis_workload(n_points: int = 65536, n_steps: int = 80, amplitude: float = 0.025,
                        kind: str = "linear", depth: int = 8, fiber_fraction: float = 0.16):
    """The paper's inelastic load cases on an orientation-interpolated DMN:
    point p runs the uniaxial strain hysteresis of direction p mod 6 with the
    given amplitude and has its own fibre orientation (l1, l2).  Use with
    FIBER_PAPER and MATRIX_PAPER.  Returns (net, lam [P, 2], E [T, P, 6],
    case [P])."""
    rs = streams(6)
    net = interpolated_dmn(rs["dmn"], depth, fiber_fraction, kind)
    lam = triangle_points(rs["assignment"], n_points)
    case = np.arange(n_points) % 6
    E = (amplitude * hysteresis_factor(n_steps))[:, None, None] * UNIAXIAL_DIRECTIONS[case][None]
    return net, lam, E, case


# ---------------------------------------------------------------- training on orientations

TRIANGLE_VERTICES = ((1.0, 0.0), (1.0 / 3.0, 1.0 / 3.0), (0.5, 0.5))


def orientation_discretization(level: int) -> np.ndarray:
    """Sampling points of the fibre-orientation triangle after `level`
    subdivisions into four self-similar triangles each (Sec. 4.3): the
    vertices of all sub-triangles plus their centres, [n, 2] as (l1, l2)."""
    tris = [tuple(np.array(v) for v in TRIANGLE_VERTICES)]
    for _ in range(level):
        nxt = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        tris = nxt
    pts = {}
    for t in tris:
        for p in list(t) + [(t[0] + t[1] + t[2]) / 3]:
            pts[tuple(np.round(p, 12))] = p
    return np.array(sorted(pts.values(), key=lambda p: (p[0], p[1])))


@dataclass
class OrientedTrainingWorkload:
    """Training batch over a discrete set of fibre orientations: samples are
    assigned to the orientations cyclically (Sec. 4.5) and stored grouped by
    orientation; `offsets[k]:offsets[k+1]` are the samples of orientation k."""
    C1: np.ndarray
    C2: np.ndarray
    lam: np.ndarray          # [G, 2] orientations
    offsets: np.ndarray      # [G + 1]
    truth: InterpolatedDmn
    v0: np.ndarray
    p0: np.ndarray
    q0: np.ndarray


def oriented_training_workload(batch: int = 4096, depth: int = 8, level: int = 2,
                               kind: str = "linear") -> OrientedTrainingWorkload:
    rs = streams(7)
    C1 = random_spd(rs["stiffness"], batch)
    C2 = random_spd(rs["stiffness"], batch)
    lam = orientation_discretization(level)
    G = len(lam)
    group = np.arange(batch) % G                      # cyclic assignment
    order = np.argsort(group, kind="stable")
    counts = np.bincount(group, minlength=G)
    offsets = np.concatenate([[0], np.cumsum(counts)])
    truth = interpolated_dmn(rs["ground_truth"], depth, 0.25, kind)
    n_leaves, M = 2 ** depth, SHAPE_COUNTS[kind]
    v0 = rs["init"].uniform(0.0, 1.0, n_leaves)
    v0 = v0 / v0.sum()
    p0 = rs["init"].uniform(0.0, 2.0 * np.pi, (n_leaves - 1, M))
    q0 = rs["init"].uniform(0.0, 2.0 * np.pi, (n_leaves - 1, M))
    return OrientedTrainingWorkload(C1[order], C2[order], lam, offsets, truth, v0, p0, q0)
