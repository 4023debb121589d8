"""Leaf laws: isotropic linear elastic fibre and J2 elasto-plastic matrix.

Matrix law (Sec. 4.1): small-strain J2 plasticity (von Mises yield
sqrt(3/2)|s| <= sigma_Y(p)) with exponential-linear isotropic hardening

    sigma_Y(p) = sigma0 + k_inf p + dsigma (1 - exp(-b p)),

integrated by implicit Euler (Sec. 3.2: the condensed energy of the implicit
Euler step gives the leaf stress).  The paper cites the classical radial
return (Simo-Hughes, Ch. 3) without printing it; this is that algorithm:
elastic trial state, consistency condition solved for the plastic multiplier
by a scalar Newton iteration, return along the trial deviator, and the
consistent (algorithmic) tangent.

Readings (not printed in the paper): p is the accumulated equivalent plastic
strain with dp = sqrt(2/3) |d eps_p|; the internal variables of one matrix
leaf are the traceless plastic strain (Mandel 6-vector) followed by p; a
trial state exactly on the yield surface (f = 0) counts as elastic; the
scalar Newton iteration starts at 0 and stops once the update is at most
1e-14 times q / (2G), the largest plastic multiplier the return admits (at
most max_iter iterations, 50 unless the caller caps it lower; a return that
has not met the test by then is reported as not converged).  A relative test on the iterate itself cannot be met
for small plastic increments: the consistency residual is a difference of
numbers of size q, so the update stalls at roundoff of q / (2G).

Complex-safe: every branch is decided on real parts, so complex-step
derivatives pass through.
"""
import numpy as np

from .mandel import DELTA6, P1, P2, bulk_shear

SQ23 = np.sqrt(2.0 / 3.0)
LOCAL_TOL = 1e-14
LOCAL_MAXIT = 50


class J2Material:
    def __init__(self, E, nu, sigma0, k_inf, dsigma, b):
        self.K, self.G = bulk_shear(E, nu)
        self.sigma0, self.k_inf, self.dsigma, self.b = sigma0, k_inf, dsigma, b

    def sigma_y(self, p):
        return self.sigma0 + self.k_inf * p + self.dsigma * (1.0 - np.exp(-self.b * p))

    def dsigma_y(self, p):
        return self.k_inf + self.dsigma * self.b * np.exp(-self.b * p)

    def elastic_stiffness(self):
        return 3.0 * self.K * P1 + 2.0 * self.G * P2


def j2_update(mat, eps, ep_n, p_n, max_iter=LOCAL_MAXIT):
    """One implicit Euler step of the J2 law at a single leaf.

    Returns dict(sigma[6], D[6,6], ep[6], p, plastic, margin, local_iters, ok),
    where margin = f / sigma_Y(p_n) is the relative trial yield value (its sign
    decides the branch) and ok is False when the scalar Newton iteration did
    not converge.
    """
    K, G = mat.K, mat.G
    e = eps - ep_n
    tr = e[0] + e[1] + e[2]
    s_tr = 2.0 * G * (e - tr / 3.0 * DELTA6)
    q = np.sqrt(s_tr @ s_tr)
    sy_n = mat.sigma_y(p_n)
    f = q - SQ23 * sy_n
    margin = np.real(f) / np.real(sy_n)
    if np.real(f) <= 0.0:
        sigma = K * tr * DELTA6 + s_tr
        D = 3.0 * K * P1 + 2.0 * G * P2
        return dict(sigma=sigma, D=D, ep=ep_n + 0.0 * e, p=p_n + 0.0 * q, plastic=False,
                    margin=margin, local_iters=0, ok=True)
    # Consistency condition g(x) = q - 2G x - sqrt(2/3) sigma_Y(p_n + sqrt(2/3) x) = 0
    x = 0.0 * q
    xtol = LOCAL_TOL * np.real(q) / (2.0 * G)
    ok = False
    it = 0
    for it in range(1, max_iter + 1):
        p = p_n + SQ23 * x
        g = q - 2.0 * G * x - SQ23 * mat.sigma_y(p)
        dg = -2.0 * G - (2.0 / 3.0) * mat.dsigma_y(p)
        dx = -g / dg
        x = x + dx
        if abs(np.real(dx)) <= xtol:
            ok = True
            break
    nhat = s_tr / q
    p = p_n + SQ23 * x
    theta = 1.0 - 2.0 * G * x / q
    theta_bar = 1.0 / (1.0 + mat.dsigma_y(p) / (3.0 * G)) - (1.0 - theta)
    sigma = K * tr * DELTA6 + theta * s_tr
    D = 3.0 * K * P1 + 2.0 * G * theta * P2 - 2.0 * G * theta_bar * np.outer(nhat, nhat)
    return dict(sigma=sigma, D=D, ep=ep_n + x * nhat, p=p, plastic=True, margin=margin,
                local_iters=it, ok=ok)


def elastic_update(C, eps):
    """Linear elastic leaf: sigma = C eps, tangent C."""
    return dict(sigma=C @ eps, D=C)
