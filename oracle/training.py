"""Offline training of a DMN: objective, gradient, optimiser and stiffness
sampler.  Test infrastructure like the rest of the oracle.

* Objective (Sec. 3.1): leaf weights w = <v>_+ (Macaulay bracket of
  unconstrained weights v), the per-sample relative error of the effective
  stiffness in a p-norm, combined over a mini-batch of N_b samples by a
  q-norm and divided by N_b, plus the quadratic penalty
  lambda (sum <v>_+ - 1)^2 of the mixing constraint.  Exponents p = 1,
  q = 10 and lambda = 1e3 in the paper's training (Sec. 4.5).
* Gradient: complex-step derivative of the objective through the oracle's
  Milton-form linear map of the compressed tree (complex-safe throughout).
* Optimiser (Sec. 4.5): AMSGrad with the learning rate modulated between a
  minimum and a maximum by a cosine of half period M and damped
  geometrically by gamma per epoch.
* Sampler (Sec. 4.4): isotropic phase-1 stiffness and an isotropic minus
  rank-one phase-2 stiffness from eight parameters
  (a, e1, e2, e3, beta, theta, psi, phi) taken from points of the unit cube.

Readings (where the paper leaves a choice open):

* T1  The p-norm of a stiffness is the l^p norm of its 36 components in
      Voigt notation (the paper defines the p = 1 case that way); with the
      Mandel storage used here the Voigt components are C_IJ / (s_I s_J),
      s = (1, 1, 1, sqrt 2, sqrt 2, sqrt 2).
* T2  Derivatives of |x| and <x>_+ at x = 0 are taken as 0; a batch whose
      errors are all zero has zero data gradient.
* T3  AMSGrad as Adam with the running maximum of the second moment; Adam's
      bias corrections are applied to the first moment and to the running
      maximum; beta1 = 0.9, beta2 = 0.999, eps = 1e-8 (the paper gives no
      values).  One learning-rate schedule for all three parameter groups
      (the paper finds the three rates almost identical).
* T4  The learning rate of epoch m (0-based) is the printed modulation
      gamma^m (a_min + (a_max - a_min)(1 + cos(pi m / M)) / 2), period 2M.
* T5  Sampler domains: a in [0, 1), e_i in [-3, 3], beta, phi in [0, 2 pi],
      psi in [0, pi], and theta from the stated condition on
      theta - sin(theta) in [0, pi]: each of these is the image of one
      unit-cube coordinate under the affine map onto its interval (theta
      by inverting theta - sin theta).  Moduli in GPa with K1 = 1.
"""
import numpy as np

from .compression import dmn_linear_compressed
from .grad import normals_from_angles
from .mandel import FAC, P1, P2, sym_to_mandel

H = 1e-30


# ---------------------------------------------------------------- objective

def cabs(x):
    """|x| for real x, continued analytically from the sign of the real part
    (complex-step safe); at x = 0 the continuation is 0, so the derivative
    there is 0 (reading T2)."""
    r = np.real(x)
    return np.where(r > 0, x, np.where(r < 0, -x, 0.0 * x))


def macaulay(v):
    """<v>_+ = max(0, v) (Sec. 3.1), complex-step safe."""
    return np.where(np.real(v) > 0, v, 0.0 * v)


def voigt(C):
    """Voigt components of Mandel stiffnesses [..., 6, 6] (reading T1)."""
    return C / np.outer(FAC, FAC)


def stiffness_norm(C, p):
    """l^p norm of the Voigt components of each stiffness [..., 6, 6]."""
    V = cabs(voigt(C)).reshape(*np.shape(C)[:-2], 36)
    return np.sum(V ** p, axis=-1) ** (1.0 / p)


def sample_errors(Cbar, T, p):
    """e_s = ||T_s - Cbar_s||_p / ||T_s||_p for a batch [B, 6, 6]."""
    return stiffness_norm(T - Cbar, p) / stiffness_norm(T, p)


def data_term(e, q):
    """(1/N_b) (sum_s e_s^q)^(1/q) (Sec. 3.1)."""
    return np.sum(e ** q) ** (1.0 / q) / len(e)


def penalty(v, lam):
    """lambda (sum_i <v_i>_+ - 1)^2, the mixing constraint's penalty (Sec. 3.1)."""
    return lam * (np.sum(macaulay(v)) - 1.0) ** 2


def objective(K, v, alpha, beta, C1, C2, T, p=1.0, q=10.0, lam=1e3):
    """J(v, alpha, beta) for fixed lamination normals n(alpha, beta); leaves
    whose weight <v>_+ is zero are removed by tree compression (Sec. 3.1)."""
    Cbar = dmn_linear_compressed(K, macaulay(v), normals_from_angles(alpha, beta), C1, C2)
    return data_term(sample_errors(Cbar, T, p), q) + penalty(v, lam)


def objective_gradient(K, v, alpha, beta, C1, C2, T, p=1.0, q=10.0, lam=1e3):
    """Complex-step gradient of ``objective``: dict(gv, galpha, gbeta)."""
    def grad_of(x, put):
        g = np.zeros(len(x))
        for i in range(len(x)):
            xc = np.asarray(x, dtype=complex).copy()
            xc[i] += 1j * H
            g[i] = np.imag(put(xc)) / H
        return g
    gv = grad_of(v, lambda vc: objective(K, vc, alpha, beta, C1, C2, T, p, q, lam))
    ga = grad_of(alpha, lambda ac: objective(K, v, ac, beta, C1, C2, T, p, q, lam))
    gb = grad_of(beta, lambda bc: objective(K, v, alpha, bc, C1, C2, T, p, q, lam))
    return dict(gv=gv, galpha=ga, gbeta=gb)


def objective_oriented(K, v, P, Q, kind, lam, C1, C2, T, p=1.0, q=10.0, penalty_lam=1e3):
    """J(v, P, Q) with orientation-interpolated normals (Sec. 2.3): sample s
    sees the normals of its own orientation lam[s] = (l1, l2), from the angle
    coefficients P, Q [L, M]; the compressed tree as in ``objective``."""
    from .orientation import interpolated_normals
    w = macaulay(v)
    Cbar = np.stack([dmn_linear_compressed(K, w, interpolated_normals(P, Q, l[0], l[1], kind),
                                           C1[s:s + 1], C2[s:s + 1])[0]
                     for s, l in enumerate(lam)])
    return data_term(sample_errors(Cbar, T, p), q) + penalty(v, penalty_lam)


def objective_oriented_gradient(K, v, P, Q, kind, lam, C1, C2, T, p=1.0, q=10.0,
                                penalty_lam=1e3):
    """Complex-step gradient of ``objective_oriented``: dict(gv, gP, gQ)."""
    f = lambda vv, PP, QQ: objective_oriented(K, vv, PP, QQ, kind, lam, C1, C2, T, p, q,
                                              penalty_lam)
    gv = np.zeros(len(v))
    for i in range(len(v)):
        vc = np.asarray(v, dtype=complex).copy()
        vc[i] += 1j * H
        gv[i] = np.imag(f(vc, P, Q)) / H
    gP, gQ = np.zeros(np.shape(P)), np.zeros(np.shape(Q))
    for idx in np.ndindex(*np.shape(P)):
        Pc = np.asarray(P, dtype=complex).copy()
        Pc[idx] += 1j * H
        gP[idx] = np.imag(f(v, Pc, Q)) / H
        Qc = np.asarray(Q, dtype=complex).copy()
        Qc[idx] += 1j * H
        gQ[idx] = np.imag(f(v, P, Qc)) / H
    return dict(gv=gv, gP=gP, gQ=gQ)


def data_cotangent(Cbar, T, p=1.0, q=10.0):
    """d(data term)/d(Cbar) entry by entry [B, 6, 6], by complex steps."""
    B = len(Cbar)
    G = np.zeros((B, 6, 6))
    for b in range(B):
        for i in range(6):
            for j in range(6):
                Cc = np.asarray(Cbar, dtype=complex).copy()
                Cc[b, i, j] += 1j * H
                G[b, i, j] = np.imag(data_term(sample_errors(Cc, T, p), q)) / H
    return G


# ---------------------------------------------------------------- optimiser

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def learning_rate(m, lr_min=1.5e-3, lr_max=1.5e-2, M=50, gamma=0.999):
    """Learning rate of epoch m (Sec. 4.5, reading T4)."""
    return gamma ** m * (lr_min + 0.5 * (lr_max - lr_min) * (1.0 + np.cos(np.pi * m / M)))


def amsgrad(theta, g, m1, m2, m2max, t, lr, beta1=BETA1, beta2=BETA2, eps=EPS):
    """One AMSGrad step (reading T3) at step number t >= 1.

    Returns (theta, m1, m2, m2max) after the step."""
    m1 = beta1 * m1 + (1.0 - beta1) * g
    m2 = beta2 * m2 + (1.0 - beta2) * g * g
    m2max = np.maximum(m2max, m2)
    step = lr / (1.0 - beta1 ** t)
    denom = np.sqrt(m2max / (1.0 - beta2 ** t)) + eps
    return theta - step * m1 / denom, m1, m2, m2max


# ---------------------------------------------------------------- sampler

def deviatoric_direction(beta):
    """Diagonal of the trace-free unit tensor N of Sec. 4.4: the spherical
    parameterisation (sin a cos b, sin a sin b, cos a) with the angle a in
    (0, pi) eliminated by the zero-trace condition
    sin a (cos b + sin b) + cos a = 0."""
    a = np.arctan2(1.0, -(np.cos(beta) + np.sin(beta)))
    return np.array([np.sin(a) * np.cos(beta), np.sin(a) * np.sin(beta), np.cos(a)])


def deviatoric_direction_closed_form(beta):
    """The closed form of the same diagonal printed in Sec. 4.4 (equal up to
    sign; undefined where cos beta + sin beta = 0)."""
    c, s = np.cos(beta), np.sin(beta)
    scale = 1.0 / np.sqrt((c * s + 1.0) / (2.0 * c * s + 1.0))
    return scale * np.array([-np.sqrt(2.0) * c / (2.0 * c + 2.0 * s),
                             -np.sqrt(2.0) * s / (2.0 * c + 2.0 * s),
                             1.0 / np.sqrt(2.0)])


def axis_angle_rotation(theta, psi, phi):
    """Matrix of x -> cos(theta) x + sin(theta) n x x + (1 - cos theta)(n . x) n
    with the axis n = (sin psi cos phi, sin psi sin phi, cos psi) (Sec. 4.4)."""
    n = np.array([np.sin(psi) * np.cos(phi), np.sin(psi) * np.sin(phi), np.cos(psi)])
    R = np.zeros((3, 3))
    for k in range(3):
        x = np.zeros(3)
        x[k] = 1.0
        R[:, k] = np.cos(theta) * x + np.sin(theta) * np.cross(n, x) \
            + (1.0 - np.cos(theta)) * np.dot(n, x) * n
    return R


def theta_from_unit(u):
    """theta in [0, pi] with theta - sin(theta) = pi u, by bisection (the left
    side increases monotonically on [0, pi])."""
    lo, hi = 0.0, np.pi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid - np.sin(mid) < np.pi * u:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def sample_parameters(u):
    """(a, e1, e2, e3, beta, theta, psi, phi) from a unit-cube point (reading T5)."""
    u = np.asarray(u, dtype=float)
    return (u[0], -3.0 + 6.0 * u[1], -3.0 + 6.0 * u[2], -3.0 + 6.0 * u[3],
            2.0 * np.pi * u[4], theta_from_unit(u[5]), np.pi * u[6], 2.0 * np.pi * u[7])


def sample_stiffness(u):
    """(C1, C2) of one unit-cube point (Sec. 4.4): C1 = 3 K1 P1 + 2 G1 P2 and
    C2 = 3 K2 P1 + 2 G2 (P2 - a N' (x) N') with N' = Q N Q^T."""
    a, e1, e2, e3, beta, theta, psi, phi = sample_parameters(u)
    K1, G1, K2, G2 = 1.0, 10.0 ** e1, 10.0 ** e2, 10.0 ** e3
    Q = axis_angle_rotation(theta, psi, phi)
    Nr = Q @ np.diag(deviatoric_direction(beta)) @ Q.T
    nv = sym_to_mandel(Nr)
    C1 = 3.0 * K1 * P1 + 2.0 * G1 * P2
    C2 = 3.0 * K2 * P1 + 2.0 * G2 * (P2 - a * np.outer(nv, nv))
    return C1, C2
