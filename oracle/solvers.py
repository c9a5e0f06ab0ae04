"""Iterative solvers on a (local) operator W_L (test infrastructure only).

Objective (Section 2.3, eq. priorsys), taken literally - no 1/2 on the data term:

    min_{x in D}  ||h W_L x - h b||_2^2 + lambda * TV(x),   D = {x >= 0}.

h is the length unit of the data: the arrays W_L and b hold path lengths and line
integrals in pixels; with the image side as the unit of length (the default reading
of the solves, h = 1/N for an N x N grid) both carry the factor h.  h = 1 is the
pixel-unit problem.

Chambolle-Pock (the primal-dual method the paper cites among solvers for
eq. priorsys; Chambolle & Pock 2011, Algorithm 1 with theta = 1) on
K = [h W_L; grad], F(v, g) = ||v - h b||^2 + lambda sum_j ||g_j||_2, G = indicator(D):

    y  <- (y + sigma (h W_L xbar - h b)) / (1 + sigma/2)    prox of sigma F1*
    z  <- proj_{||z_j|| <= lambda}(z + sigma grad xbar)      prox of sigma F2*
    x+ <- max(0, x - tau (h W_L^T y - div z))                prox of tau G
    xbar <- x+ + theta (x+ - x);  x <- x+

Start x = xbar = 0, y = 0, z = 0 (the local iterations of the paper also start
from zero images).  Step sizes sigma = tau = 1/L (CP requires sigma tau ||K||^2 < 1)
with L^2 = 1.01 h^2 mu + 8, where mu = lambda_max(W_L^T W_L - Laplacian) comes from a
power iteration from the all-ones image: since mu >= ||W_L||^2 and ||grad||^2 <= 8
(each forward difference squared is at most twice the sum of its two squares), L^2
bounds ||K||^2 = ||h^2 W_L^T W_L - Laplacian|| from above.  In pixel units W_L^T W_L
dominates and the all-ones start finds mu quickly; the Laplacian's top eigenvector
(a checkerboard) is nearly orthogonal to that start, which is why its part is bounded
rather than iterated.

Nonnegative SIRT: eq. sirtit with the box projection of eq. sirtbox (l = 0,
r = +inf), alpha = 1/(N_theta N_d) as fixed in Section 3.1.
"""

import numpy as np

from .tv import grad, div, tv_iso, tv_aniso


def _apply_k(WL, shape, x):
    return WL @ x.ravel(), grad(x.reshape(shape))


def power_norm_sq(WL, shape, iters=100):
    """lambda_max(W_L^T W_L + grad^T grad) by power iteration from the all-ones image."""
    v = np.ones(shape)
    est = 0.0
    for _ in range(iters):
        w = (WL.T @ (WL @ v.ravel())).reshape(shape) - div(grad(v))
        est = float(np.linalg.norm(w) / np.linalg.norm(v))
        v = w / np.linalg.norm(w)
    return est


def cp_steps(WL, shape, iters=100, safety=1.01, h=1.0):
    """sigma = tau = 1 / L, L^2 = safety * h^2 * mu + 8 >= ||K||^2, K = [h W_L; grad]."""
    L2 = safety * h * h * power_norm_sq(WL, shape, iters) + 8.0
    s = 1.0 / np.sqrt(L2)
    return s, s


def cp_tv_nonneg(WL, b, shape, lam, sigma, tau, iters, theta=1.0, half=False, aniso=False,
                 nonneg=True, x0=None, callback=None, dual_callback=None, h=1.0):
    """K Chambolle-Pock iterations; returns the final primal iterate (rows, cols).

    h: length unit of the data (the objective's data term is ||h W_L x - h b||^2).
    half: data term 1/2 ||W_L x - b||^2 (prox of sigma F1* divides by 1 + sigma).
    aniso: anisotropic TV, whose dual prox clamps each component to [-lambda, lambda].
    callback(it, x) sees each new primal iterate; dual_callback(it, zt) sees the TV dual
    z + sigma grad xbar before its projection (so a caller can tell where it clips).
    """
    b = np.asarray(b, dtype=np.float64).ravel()
    x = np.zeros(shape) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    xbar = x.copy()
    y = np.zeros(WL.shape[0])
    z = np.zeros((2,) + tuple(shape))
    dual_scale = 1.0 + (sigma if half else sigma / 2.0)
    for it in range(iters):
        y = (y + sigma * h * (WL @ xbar.ravel() - b)) / dual_scale
        z = z + sigma * grad(xbar)
        if dual_callback is not None:
            dual_callback(it, z)
        if aniso:
            z = np.clip(z, -lam, lam)
        else:
            nrm = np.sqrt(z[0] ** 2 + z[1] ** 2)
            z = z / np.maximum(1.0, nrm / lam) if lam > 0 else np.zeros_like(z)
        xn = x - tau * (h * (WL.T @ y).reshape(shape) - div(z))
        if nonneg:
            xn = np.maximum(0.0, xn)
        xbar = xn + theta * (xn - x)
        x = xn
        if callback is not None:
            callback(it, x)
    return x


def cp_objective(WL, b, x, lam, half=False, aniso=False, h=1.0):
    r = h * (WL @ np.asarray(x).ravel() - np.asarray(b).ravel())
    data = float(r @ r) * (0.5 if half else 1.0)
    return data + lam * (tv_aniso(x) if aniso else tv_iso(x))


def sirt_nonneg(WL, b, shape, alpha, iters, lo=0.0, hi=np.inf, x0=None):
    """x <- clip(x + alpha W_L^T (b - W_L x), lo, hi), from x0 = 0."""
    b = np.asarray(b, dtype=np.float64).ravel()
    x = np.zeros(int(np.prod(shape))) if x0 is None else np.asarray(x0, np.float64).ravel().copy()
    for _ in range(iters):
        x = np.clip(x + alpha * (WL.T @ (b - WL @ x)), lo, hi)
    return x.reshape(shape)
