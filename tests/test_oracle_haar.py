"""Pins of the Haar l1 prior oracle.

  * the transform is orthonormal on any size (its explicit matrix satisfies B^T B = I)
    and the inverse undoes it;
  * on an 8 x 8 image with three levels, coefficients written out from the textbook Haar
    basis: the coarsest sum is sum(x)/8, a finest diagonal detail is
    (x00 - x01 - x10 + x11)/2, a coarsest horizontal detail is the difference of the
    left and right half sums over 8;
  * a constant image has no detail coefficients;
  * with L levels the transform of a region is the transform of its aligned 2^L tiles
    (the property the tiled GPU kernel uses), for ragged sizes too;
  * the prox is the minimiser of 1/2 ||x - w||^2 + gamma ||B x||_1 (no perturbation
    lowers the objective) and shrinks ||B x||_1;
  * the local FISTA with this prox, fed the exact SIRT iterates on the whole grid, is plain
    global FISTA with it.
"""

import numpy as np
import pytest

from oracle import make_geometry, fp_ray, sparse_local
from oracle.filters import default_alpha, sirt_iterates
from oracle.fista import prox_weight
from oracle.haar import haar_forward, haar_inverse, haar_prox, local_fista_haar


@pytest.mark.parametrize("shape,levels", [((8, 8), 3), ((5, 7), 2), ((13, 6), 4), ((1, 9), 3),
                                          ((16, 11), 5)])
def test_orthonormal_any_size(shape, levels):
    n = shape[0] * shape[1]
    B = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        B[:, j] = haar_forward(e.reshape(shape), levels).ravel()
    assert np.abs(B.T @ B - np.eye(n)).max() <= 1e-13
    x = np.random.default_rng(1).normal(size=shape)
    assert np.abs(haar_inverse(haar_forward(x, levels), levels) - x).max() <= 1e-13


def test_textbook_coefficients():
    x = np.random.default_rng(2).normal(size=(8, 8))
    c = haar_forward(x, 3)
    assert c[0, 0] == pytest.approx(x.sum() / 8, abs=1e-13)
    # finest level: block (0, 0), diagonal detail sits in the lower-right quadrant
    assert c[4, 4] == pytest.approx((x[0, 0] - x[0, 1] - x[1, 0] + x[1, 1]) / 2, abs=1e-13)
    # coarsest level: horizontal detail (difference along columns) of the whole image
    assert c[0, 1] == pytest.approx((x[:, :4].sum() - x[:, 4:].sum()) / 8, abs=1e-13)


def test_constant_image_has_no_details():
    c = haar_forward(np.full((12, 10), 0.7), 2)
    mask = np.zeros_like(c, dtype=bool)
    mask[:3, :3] = True               # the 12x10 -> 6x5 -> 3x3 block of sums
    assert np.abs(c[~mask]).max() <= 1e-13
    # each pairing multiplies a constant by sqrt 2; the third column of sums was unpaired
    # (odd width 5) at the second level
    assert np.abs(c[:3, :2] - 0.7 * 4).max() <= 1e-13
    assert np.abs(c[:3, 2] - 0.7 * 2 * np.sqrt(2)).max() <= 1e-13


@pytest.mark.parametrize("shape,levels", [((32, 48), 3), ((37, 29), 3), ((19, 40), 4)])
def test_tiles_are_independent(shape, levels):
    x = np.random.default_rng(3).normal(size=shape)
    T = 2 ** levels
    whole = haar_prox(x, 0.3, levels)
    tiled = np.empty_like(x)
    for r in range(0, shape[0], T):
        for c in range(0, shape[1], T):
            tiled[r:r + T, c:c + T] = haar_prox(x[r:r + T, c:c + T], 0.3, levels)
    assert np.abs(whole - tiled).max() <= 1e-13


def test_prox_minimises_its_objective():
    rng = np.random.default_rng(4)
    w = rng.normal(size=(9, 12))
    gamma, L = 0.4, 3
    f = lambda x: 0.5 * np.sum((x - w) ** 2) + gamma * np.abs(haar_forward(x, L)).sum()
    x = haar_prox(w, gamma, L)
    fx = f(x)
    for _ in range(200):
        assert fx <= f(x + 1e-3 * rng.normal(size=w.shape)) + 1e-12
    assert np.abs(haar_forward(x, L)).sum() < np.abs(haar_forward(w, L)).sum()


def test_local_fista_haar_bridge_to_global():
    n = 16
    g = make_geometry(n, 12, 23)
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2.0
    p = fp_ray(g, 1.0 * (xx ** 2 + yy ** 2 < 30))
    K, lam, L = 6, 300.0, 2
    X = sirt_iterates(g, p, K)
    got = local_fista_haar(g, p, (0, 0, n, n), 0, None, lam, L, xs_iterates=X)
    W = sparse_local(g)
    alpha = default_alpha(g)
    gamma = prox_weight(g, lam, alpha)
    z = np.zeros(n * n)
    x_prev = z.copy()
    t = 1.0
    for _ in range(K):
        s = z + alpha * (W.T @ (p.ravel() - W @ z))
        x = haar_prox(s.reshape(n, n), gamma, L).ravel()
        t_new = (1 + np.sqrt(1 + 4 * t * t)) / 2
        z = x + ((t - 1) / t_new) * (x - x_prev)
        x_prev, t = x, t_new
    assert np.abs(got - x_prev.reshape(n, n)).max() <= 1e-12 * np.abs(x_prev).max()


def test_ista_form_is_eq_sirtista_on_the_whole_grid():
    """Without momentum, with the exact SIRT iterates on the whole grid, the local method
    is eq. sirtista: x^{k+1} = B^-1 P(B S(x^k)) from x = 0."""
    n = 16
    g = make_geometry(n, 12, 23)
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2.0
    p = fp_ray(g, 1.0 * (xx ** 2 + yy ** 2 < 30))
    K, lam, L = 5, 300.0, 3
    X = sirt_iterates(g, p, K)
    got = local_fista_haar(g, p, (0, 0, n, n), 0, None, lam, L, xs_iterates=X, momentum=False)
    W = sparse_local(g)
    alpha = default_alpha(g)
    gamma = prox_weight(g, lam, alpha)
    x = np.zeros(n * n)
    for _ in range(K):
        s = x + alpha * (W.T @ (p.ravel() - W @ x))
        x = haar_inverse(np.sign(haar_forward(s.reshape(n, n), L)) *
                         np.maximum(np.abs(haar_forward(s.reshape(n, n), L)) - gamma, 0), L).ravel()
    assert np.abs(got - x.reshape(n, n)).max() <= 1e-12 * np.abs(x).max()
