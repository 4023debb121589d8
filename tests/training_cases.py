"""Seeded cases of the offline-training calls shared by their GPU tests and
their CPU-build tests (no torch): objective inputs, stiffness-sampler points
and the gradient chain of the optimiser step."""
import numpy as np

import synthetic as S
from oracle import training as T
from oracle.grad import normals_from_angles


def loss_case(B, seed):
    """Predicted and target stiffness pairs [B, 6, 6] with a sample without
    error and a sample with zero differences on some components."""
    rs = S.streams(seed)
    Tt = S.random_spd(rs["stiffness"], B)
    Cb = Tt * (1.0 + 0.2 * rs["noise"].standard_normal(Tt.shape))
    Cb[0] = Tt[0]                      # a sample without error
    Cb[1, :3, :3] = Tt[1, :3, :3]      # zero differences on some components
    return Cb, Tt


def special_points(n, seed):
    """n scrambled Sobol points of the unit 8-cube and five corner and edge
    points (u5 = 0 and u5 near 0 make theta = 0 and theta small)."""
    from scipy.stats import qmc
    u = qmc.Sobol(d=8, scramble=True, seed=seed).random(n)
    extra = np.array([[0.0] * 8, [1.0] * 8, [0.5, 0.5, 0.5, 0.5, 0.375, 0.0, 0.25, 0.1],
                      [0.9, 0.1, 0.9, 0.2, 0.875, 1.0, 1.0, 0.9],
                      [0.3, 0.7, 0.2, 0.6, 0.125, 1e-9, 0.5, 0.5]])
    return np.concatenate([u, extra])


def weight_chain(v, gw, lam):
    """dJ/dv from the weight cotangent gw: Macaulay cut-off and mixing penalty
    by complex steps of the oracle's functions."""
    h = 1e-30
    gv = np.zeros_like(v)
    for i in range(len(v)):
        vc = v.astype(complex)
        vc[i] += 1j * h
        gv[i] = np.imag(np.dot(gw, T.macaulay(vc)) + T.penalty(vc, lam)) / h
    return gv


def chain_gradient(v, alpha, beta, gw, gn, lam):
    """dJ/d(v, alpha, beta) from gw, gn: the weight chain (weight_chain) and
    the angle chain by complex steps of the oracle's normals."""
    h = 1e-30
    gv = weight_chain(v, gw, lam)
    ga = np.imag(np.sum(gn * normals_from_angles(alpha + 1j * h, beta), axis=1)) / h
    gb = np.imag(np.sum(gn * normals_from_angles(alpha, beta + 1j * h), axis=1)) / h
    return gv, ga, gb


def update_case(seed=17, K=4):
    """Parameters, gradients and optimiser state of one AMSGrad step at depth K
    (step counter 7, a data term of 0.125) and the optimiser settings."""
    NL, L = 2 ** K, 2 ** K - 1
    NP = NL + 2 * L
    rng = np.random.default_rng(seed)
    v = rng.uniform(-0.05, 0.15, NL)
    alpha, beta = rng.uniform(0, 2 * np.pi, L), rng.uniform(0, 2 * np.pi, L)
    gw, gn = rng.normal(0, 1e-2, NL), rng.normal(0, 1e-2, (L, 3))
    m1 = rng.normal(0, 1e-3, (NP,))
    m2 = rng.uniform(0, 1e-5, NP)
    mx = m2 + rng.uniform(0, 1e-5, NP)
    opts = dict(lr_min=1e-3, lr_max=2e-2, lr_decay=0.99, half_period=5, steps_per_epoch=3,
                beta1=0.9, beta2=0.999, eps=1e-8, penalty=10.0)
    return dict(v=v, alpha=alpha, beta=beta, gw=gw, gn=gn, m1=m1, m2=m2, mx=mx, t0=7,
                data=0.125, opts=opts)


def update_reference(c):
    """The oracle's AMSGrad step of an update_case (inputs as rounded for the
    call): parameters, moments, learning rate and penalty."""
    o = c["opts"]
    gv, ga, gb = chain_gradient(c["v"], c["alpha"], c["beta"], c["gw"], c["gn"], o["penalty"])
    lr = T.learning_rate(c["t0"] // o["steps_per_epoch"], o["lr_min"], o["lr_max"],
                         o["half_period"], o["lr_decay"])
    th, n1, n2, nx = T.amsgrad(np.concatenate([c["v"], c["alpha"], c["beta"]]),
                               np.concatenate([gv, ga, gb]), c["m1"], c["m2"], c["mx"],
                               c["t0"] + 1, lr, o["beta1"], o["beta2"], o["eps"])
    return dict(theta=th, state=np.stack([n1, n2, nx]), lr=lr,
                penalty=T.penalty(c["v"], o["penalty"]))


def oriented_case(K, B, kind, seed, level=0):
    """A batch of B samples grouped by orientation (level of the orientation
    discretization), targets from a ground-truth interpolated DMN, and an
    initial (v, p, q)."""
    from oracle.orientation import oriented_linear
    rs = S.streams(seed)
    lam_g = S.orientation_discretization(level)
    G = len(lam_g)
    group = np.arange(B) % G
    order = np.argsort(group, kind="stable")
    offsets = np.concatenate([[0], np.cumsum(np.bincount(group, minlength=G))])
    C1 = S.random_spd(rs["stiffness"], B)[order]
    C2 = S.random_spd(rs["stiffness"], B)[order]
    lam_s = lam_g[group[order]]
    truth = S.interpolated_dmn(rs["ground_truth"], K, 0.25, kind)
    Tt = oriented_linear(K, truth.w, truth.p, truth.q, kind, lam_s, C1, C2)
    M = S.SHAPE_COUNTS[kind]
    v = rs["init"].uniform(0.0, 1.0, 2 ** K)
    v = v / v.sum()
    p = rs["init"].uniform(0.0, 2 * np.pi, (2 ** K - 1, M))
    q = rs["init"].uniform(0.0, 2 * np.pi, (2 ** K - 1, M))
    return C1, C2, Tt, lam_g, lam_s, offsets, v, p, q
