"""Pins of the FGP denoiser and the local FISTA-TV oracle (Alg. 3).

  * FGP reaches the minimiser of the denoising problem: the duality gap between its
    primal and dual iterates (a certificate independent of the algorithm) falls to
    1e-9 of the objective, for isotropic and anisotropic TV;
  * with a large weight the minimiser is the constant mean(b) (closed form);
  * with the box [0, inf) FGP matches an independent ADMM minimiser of the
    nonnegative denoising problem;
  * Alg. 3 fed with the exact SIRT iterates on the whole grid is plain global FISTA
    (x = FGP(S(z)), z = x + beta (x - x_prev)), and on a local part it is FISTA on L
    whose exterior follows those iterates (b^k = p - W M_F x_s^{k-1}) -- the same
    bridge as for the box method, which checks the split z = x_s + z_L;
  * without TV the prox is the identity and Alg. 3 reduces to accelerated Alg. 2.
"""

import numpy as np
import pytest

from oracle import make_geometry, fp_ray, sparse_local, roi_extend
from oracle.local import exterior_subtract, crop
from oracle.tv import grad
from oracle.filters import default_alpha, sirt_filters, sirt_iterates, local_method_box
from oracle.fista import (fgp, fgp_with_dual, fgp_dual_gap, local_fista, local_fista_tv,
                          prox_weight)
from test_oracle_solvers import _admm_tv_nonneg


@pytest.mark.parametrize("aniso", [False, True])
@pytest.mark.parametrize("gamma", [0.05, 0.4])
def test_fgp_duality_gap_closes(aniso, gamma):
    rng = np.random.default_rng(11)
    b = rng.uniform(0.0, 1.0, (12, 9))
    b[3:8, 2:6] += 1.0
    x1, p1 = fgp_with_dual(b, gamma, 50, aniso)
    x2, p2 = fgp_with_dual(b, gamma, 10000, aniso)
    g1 = fgp_dual_gap(b, gamma, x1, p1, aniso)
    g2 = fgp_dual_gap(b, gamma, x2, p2, aniso)
    obj = 0.5 * np.sum(b ** 2)
    assert g1 >= -1e-12 and g2 >= -1e-12
    assert g2 <= 1e-9 * obj
    assert g2 < g1
    # fgp() returns the same primal iterate
    assert np.abs(fgp(b, gamma, 10000, aniso=aniso) - x2).max() <= 1e-14


def test_fgp_large_weight_gives_the_mean():
    rng = np.random.default_rng(12)
    b = rng.uniform(0.0, 1.0, (7, 8))
    x = fgp(b, 50.0, 20000)
    assert np.abs(x - b.mean()).max() <= 1e-7
    assert np.abs(grad(x)).max() <= 1e-7


def test_fgp_box_matches_admm():
    rng = np.random.default_rng(13)
    b = rng.normal(0.2, 0.5, (6, 7))
    gamma = 0.3
    x = fgp(b, gamma, 20000, 0.0, np.inf)
    # ||Ix - b||^2 + 2 gamma TV(x), x >= 0, by ADMM (W = I)
    ref = _admm_tv_nonneg(np.eye(b.size), b.ravel(), 6, 7, 2 * gamma, iters=20000)
    assert x.min() >= 0.0
    assert np.abs(x - ref).max() <= 1e-6


def test_fgp_zero_weight_is_the_box_projection():
    b = np.linspace(-1, 2, 20).reshape(4, 5)
    assert np.array_equal(fgp(b, 0.0, 10, 0.0, 1.0), np.clip(b, 0.0, 1.0))


def _phantom(n, seed):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2.0
    img = np.zeros((n, n))
    for _ in range(4):
        cx, cy = rng.uniform(-0.2, 0.2, 2) * n
        a, b = rng.uniform(0.08, 0.25, 2) * n
        img[((xx - cx) / a) ** 2 + ((yy - cy) / b) ** 2 < 1] = rng.uniform(0.3, 1.0)
    return img


@pytest.mark.parametrize("aniso,half", [(False, False), (True, True)])
def test_alg3_with_exact_sirt_on_the_whole_grid_is_global_fista(aniso, half):
    n = 16
    g = make_geometry(n, 12, 23)
    p = fp_ray(g, _phantom(n, 5))
    K, nf, lam = 6, 30, 40.0
    X = sirt_iterates(g, p, K)
    got = local_fista_tv(g, p, (0, 0, n, n), 0, None, lam, nf, aniso=aniso, half=half,
                         xs_iterates=X)
    W = sparse_local(g)
    alpha = default_alpha(g)
    gamma = prox_weight(g, lam, alpha, half)
    z = np.zeros(n * n)
    x_prev = np.zeros(n * n)
    t = 1.0
    for _ in range(K):
        s = z + alpha * (W.T @ (p.ravel() - W @ z))
        x = fgp(s.reshape(n, n), gamma, nf, aniso=aniso).ravel()
        t_new = (1 + np.sqrt(1 + 4 * t * t)) / 2
        z = x + ((t - 1) / t_new) * (x - x_prev)
        x_prev, t = x, t_new
    ref = x_prev.reshape(n, n)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert gamma == pytest.approx(alpha * lam * (1.0 if half else 0.5))


def test_alg3_with_exact_sirt_is_exterior_following_fista():
    n = 22
    g = make_geometry(n, 14, 31)
    p = fp_ray(g, _phantom(n, 6))
    rect, margin = (6, 5, 7, 8), 2
    K, nf, lam = 7, 25, 30.0
    X = sirt_iterates(g, p, K)
    got = local_fista_tv(g, p, rect, margin, None, lam, nf, lo=0.0, xs_iterates=X, full=True)
    ext = roi_extend(rect, margin, n)
    WL = sparse_local(g, ext)
    alpha = default_alpha(g)
    gamma = prox_weight(g, lam, alpha)
    shape = (ext[2], ext[3])
    z = np.zeros(ext[2] * ext[3])
    x_prev = z.copy()
    t = 1.0
    prev = np.zeros((n, n))
    for k in range(K):
        b = exterior_subtract(g, p, prev, ext).ravel()
        s = z + alpha * (WL.T @ (b - WL @ z))
        x = fgp(s.reshape(shape), gamma, nf, 0.0, np.inf).ravel()
        t_new = (1 + np.sqrt(1 + 4 * t * t)) / 2
        z = x + ((t - 1) / t_new) * (x - x_prev)
        x_prev, t = x, t_new
        prev = X[k]
    ref = x_prev.reshape(shape)
    assert np.abs(got["x_ext_full"] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(got["x"] - crop(ref, ext, rect)).max() <= 1e-12 * np.abs(ref).max()


def test_alg3_without_tv_is_accelerated_alg2():
    """lam = 0: the prox is the identity, so x^k = x_s + q and the momentum acts on the
    SIRT-type iteration; with one iteration it is exactly Alg. 2's first iterate."""
    n = 18
    g = make_geometry(n, 10, 27)
    p = fp_ray(g, _phantom(n, 7))
    U = sirt_filters(g, 4)
    rect, margin = (4, 4, 8, 9), 3
    a = local_fista_tv(g, p, rect, margin, U[:1], 0.0, 10)
    b = local_method_box(g, p, rect, margin, U[:1], -np.inf, np.inf)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    # more iterations: momentum makes it differ from Alg. 2 (t^1 = 1 gives no momentum
    # at k = 1, nonzero from k = 2 on)
    a4 = local_fista_tv(g, p, rect, margin, U, 0.0, 10)
    b4 = local_method_box(g, p, rect, margin, U, -np.inf, np.inf)
    assert np.abs(a4 - b4).max() > 1e-6 * np.abs(b4).max()


def test_outer_momentum_has_nesterov_asymptotics():
    """The outer momentum of Alg. 3, read off the method itself: with alpha = 0 and the
    identity as prox on one pixel, fed the SIRT iterates x_s^k = k, the output increments obey
    D_k = beta_{k-1} D_{k-1} + 1 (D_1 = 1), so beta_k = (D_{k+1} - 1) / D_k is visible in runs
    of K and K + 1 iterations.  Beck and Teboulle's rule gives t_k = (k + 1)/2 + O(log k), hence
    beta_1 = 0 and beta_k = 1 - 3/(k + 2) + O(log k / k^2), the momentum of Nesterov's method;
    a rule without the square tends to 1/2, a shifted index to 1 - 2/(k + 1)."""
    n = 4
    g = make_geometry(n, 3, 7)
    kmax = 121
    xs = [np.full((n, n), float(k + 1)) for k in range(kmax)]
    out = [0.0]
    for K in range(1, kmax + 1):
        x = local_fista(g, np.zeros((3, 7)), (1, 1, 1, 1), 0, None, lambda w: w, alpha=0.0,
                        xs_iterates=xs[:K])
        out.append(float(x[0, 0]))
    D = np.diff(out)   # D[k - 1] = D_k
    assert D[0] == pytest.approx(1.0) and D[1] == pytest.approx(1.0)   # beta_1 = 0
    beta = (D[1:] - 1.0) / D[:-1]                                       # beta[k - 1] = beta_k
    assert np.all(np.diff(beta) > 0) and beta[-1] < 1.0
    for k in (20, 60, 120):
        assert abs(beta[k - 1] - (1.0 - 3.0 / (k + 2))) < 2.0 * np.log(k) / k ** 2
