"""FGP total-variation denoiser and the paper's local FISTA-TV (TEST INFRASTRUCTURE ONLY).

Section 3.2 names FISTA with an FGP inner solver as an instance of the local method
for g(x) = ||grad x||_1 (Alg. 3, n_FGP FGP iterations per outer iteration).

FGP (Beck & Teboulle's fast gradient projection on the dual of the denoising problem)
solves   min_{l <= x <= r}  ||x - b||^2 + 2 gamma TV(x)
with the discrete gradient and divergence of oracle/tv.py.  In that notation the dual
variable p (one 2-vector per pixel, |p_j| <= 1) gives x = P_[l,r](b - gamma div p) and
its projected gradient step is p <- P_1(p - grad x / (8 gamma)); the dual iterates are
accelerated with the FISTA momentum t_{i+1} = (1 + sqrt(1 + 4 t_i^2)) / 2, from p = 0.

Local FISTA (Alg. 3) runs FISTA on eq. priorsys with g = TV, each gradient step being
one SIRT step S (step alpha = 1/(N_theta N_d)), written with the local operators:
    x_s   = FBP_L(p, u_k) = W_L^T C_{u_k} p                 (approximates S^k(0))
    q     = z_L - alpha W_L^T W_L z_L                         (A applied to the correction)
    x^k   = prox_{gamma TV}(x_s + q)   by n_FGP FGP iterations
    t^k   = (1 + sqrt(1 + 4 (t^{k-1})^2)) / 2
    z     = x^k + ((t^{k-1} - 1) / t^k) (x^k - x^{k-1})
    z_L   = z - x_s
from z_L = 0, x^0 = 0, t^0 = 1; returns x^n.  Readings: the printed recursion for t^k
lacks the square of the standard FISTA rule and the momentum line is garbled; both are
read as Beck & Teboulle's FISTA.  The SIRT step is a gradient step of step alpha/2 on
||W x - p||^2 (eq. priorsys has no 1/2), so the prox weight is gamma = alpha lambda / 2
(gamma = alpha lambda with the 1/2 data term).  Box constraints, when given, act in FGP.
"""

import numpy as np

from .geometry import roi_extend
from .projector import sparse_local
from .local import crop
from .tv import grad, div
from .filters import default_alpha, filter_apply


def _proj_unit(z, aniso):
    if aniso:
        return np.clip(z, -1.0, 1.0)
    nrm = np.sqrt(z[0] ** 2 + z[1] ** 2)
    return z / np.maximum(1.0, nrm)


def fgp(b, gamma, iters, lo=-np.inf, hi=np.inf, aniso=False):
    """FGP for min_{lo <= x <= hi} ||x - b||^2 + 2 gamma TV(x), `iters` dual steps from 0."""
    b = np.asarray(b, dtype=np.float64)
    if gamma <= 0:
        return np.clip(b, lo, hi)
    p = np.zeros((2,) + b.shape)
    r = p.copy()
    t = 1.0
    for _ in range(iters):
        x = np.clip(b - gamma * div(r), lo, hi)
        p_new = _proj_unit(r - grad(x) / (8.0 * gamma), aniso)
        t_new = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        r = p_new + ((t - 1.0) / t_new) * (p_new - p)
        p, t = p_new, t_new
    return np.clip(b - gamma * div(p), lo, hi)


def fgp_dual_gap(b, gamma, x, p, aniso=False):
    """Duality gap of the unconstrained denoising problem min 1/2||x - b||^2 + gamma TV(x)
    at primal x and dual w = -p:  P(x) - D(w) >= 0, with D(w) = 1/2||b||^2 - 1/2||b - gamma div p||^2."""
    g = grad(x)
    tv = np.sum(np.abs(g)) if aniso else np.sum(np.sqrt(g[0] ** 2 + g[1] ** 2))
    primal = 0.5 * np.sum((x - b) ** 2) + gamma * tv
    dual = 0.5 * np.sum(b ** 2) - 0.5 * np.sum((b - gamma * div(p)) ** 2)
    return primal - dual


def fgp_with_dual(b, gamma, iters, aniso=False):
    """FGP as above (no box), also returning the last dual iterate p."""
    b = np.asarray(b, dtype=np.float64)
    p = np.zeros((2,) + b.shape)
    r = p.copy()
    t = 1.0
    for _ in range(iters):
        x = b - gamma * div(r)
        p_new = _proj_unit(r - grad(x) / (8.0 * gamma), aniso)
        t_new = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        r = p_new + ((t - 1.0) / t_new) * (p_new - p)
        p, t = p_new, t_new
    return b - gamma * div(p), p


def prox_weight(geom, lam, alpha=None, half=False):
    alpha = default_alpha(geom) if alpha is None else alpha
    return alpha * lam if half else 0.5 * alpha * lam


def local_fista_tv(geom, sino, rect, margin, filters, lam, n_fgp, lo=-np.inf, hi=np.inf,
                   aniso=False, half=False, alpha=None, xs_iterates=None, full=False,
                   momentum=True):
    """Alg. 3 on the extended local part.  filters: U from sirt_filters (U[k-1] = u_k);
    xs_iterates (optional, [K, N, N]) replaces FBP_L(p, u_k) by those images."""
    gamma = prox_weight(geom, lam, alpha, half)
    return local_fista(geom, sino, rect, margin, filters,
                       lambda w: fgp(w, gamma, n_fgp, lo, hi, aniso), alpha, xs_iterates, full,
                       gamma, momentum)


def local_fista(geom, sino, rect, margin, filters, prox, alpha=None, xs_iterates=None,
                full=False, gamma=None, momentum=True):
    """Alg. 3 with any proximal step `prox` (image -> image) in place of FGP; without
    momentum (z = x^k) it is the ISTA form, eq. sirtista, of the same local method."""
    alpha = default_alpha(geom) if alpha is None else alpha
    ext = roi_extend(rect, margin, geom.n)
    r0, c0, rr, cc = ext
    WL = sparse_local(geom, ext)
    iters = len(filters) if xs_iterates is None else len(xs_iterates)
    sino = np.asarray(sino, dtype=np.float64)
    zl = np.zeros(rr * cc)
    x_prev = np.zeros(rr * cc)
    t = 1.0
    for k in range(iters):
        if xs_iterates is None:
            xs = WL.T @ filter_apply(geom, filters[k], sino).ravel()
        else:
            xs = np.asarray(xs_iterates[k])[r0:r0 + rr, c0:c0 + cc].ravel()
        q = zl - alpha * (WL.T @ (WL @ zl))
        x = np.asarray(prox((xs + q).reshape(rr, cc)), dtype=np.float64).ravel()
        t_new = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        z = x + ((t - 1.0) / t_new) * (x - x_prev) if momentum else x
        zl = z - xs
        x_prev, t = x, t_new
    x = x_prev.reshape(rr, cc)
    out = crop(x, ext, rect)
    if full:
        return dict(x=out, x_ext_full=x, ext=ext, WL=WL, gamma=gamma)
    return out
