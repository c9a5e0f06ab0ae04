"""Pins of the SIRT-filter oracle (Alg. 1, eq. sirtapp) and of the local method
(eq. localmethod, Alg. 2 with the box prior of eq. sirtbox).

  * Alg. 1 against the matrix-power definition u_k = alpha W sum_{j<k} A^j e with a
    brute-force dense W from the entry formula (eq. filtcalc, eq. sirtapp);
  * the detector convolution C_u against a plain double loop with the zero lag
    found by scanning the bins;
  * an exact identity at the impulse pixel: K SIRT iterations from zero give
    <u_K, p> there (A is symmetric), and FBP(p, u_K) gives sum_theta <u_K, p>_theta / m_theta
    (the pixel projects onto one bin centre per angle with weight 1/m_theta);
  * symmetry of the filters about the centre bin (the impulse sits on the grid
    centre, the projector is symmetric under a half turn);
  * Alg. 2 fed with the exact SIRT iterates equals projected SIRT on L whose
    exterior follows those iterates (b^k = p - W M_F x_s^{k-1}, eq. locouter) -- the
    bridge between the paper's method and exterior subtraction;
  * without a prior Alg. 2 returns FBP_L(p, u_K) (y stays zero);
  * the approximation itself: FBP(p, u_K) tracks K SIRT iterations.
"""

import numpy as np
import pytest

from oracle import make_geometry, fp_ray, bp_pixel, dense_matrix_hat, sparse_local, roi_extend
from oracle.local import exterior_subtract, crop
from oracle.filters import (default_alpha, impulse_pixel, filter_centres, sirt_filters,
                            filter_apply, fbp_filter, sirt_iterates, local_method_box)


def _phantom(n, seed=0):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2.0
    img = np.zeros((n, n))
    for _ in range(5):
        cx, cy = rng.uniform(-0.25, 0.25, 2) * n
        a, b = rng.uniform(0.05, 0.2, 2) * n
        img[((xx - cx) / a) ** 2 + ((yy - cy) / b) ** 2 < 1] = rng.uniform(0.2, 1.0)
    return img


def test_alg1_matches_matrix_powers():
    g = make_geometry(9, 6, 13)
    W = dense_matrix_hat(g)
    alpha = default_alpha(g)
    A = np.eye(W.shape[1]) - alpha * W.T @ W
    e = np.zeros(W.shape[1])
    r, c = impulse_pixel(g)
    e[r * g.n + c] = 1.0
    U = sirt_filters(g, 7)
    q = np.zeros_like(e)
    Ak = e.copy()
    for k in range(1, 8):
        q = q + Ak                     # q_k = sum_{j<k} A^j e
        Ak = A @ Ak
        u = alpha * (W @ q)
        assert np.abs(U[k - 1].ravel() - u).max() <= 1e-13 * np.abs(u).max()


@pytest.mark.parametrize("n,nd,off", [(9, 13, 0.0), (8, 10, 0.0), (7, 12, 0.3)])
def test_filter_apply_brute_force(n, nd, off):
    g = make_geometry(n, 5, nd, offset=off)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((5, nd))
    p = rng.standard_normal((5, nd))
    got = filter_apply(g, u, p)
    r, c = impulse_pixel(g)
    for k in range(5):
        t = (c - (n - 1) / 2.0) * g.cos[k] + (r - (n - 1) / 2.0) * g.sin[k]
        ctr = int(np.argmin(np.abs(g.s - t)))   # nearest bin centre (scan)
        assert ctr == filter_centres(g)[k]
        for i in range(nd):
            ref = 0.0
            for j in range(nd):
                lag = i - j + ctr
                if 0 <= lag < nd:
                    ref += u[k, lag] * p[k, j]
            assert abs(got[k, i] - ref) <= 1e-12 * (1 + abs(ref))


def test_impulse_pixel_identities():
    g = make_geometry(17, 12, 25)
    p = fp_ray(g, _phantom(17, 2))
    K = 9
    U = sirt_filters(g, K)
    X = sirt_iterates(g, p, K)
    r, c = impulse_pixel(g)
    assert np.all(filter_centres(g) == (g.n_det - 1) // 2)
    for k in (1, 4, K):
        sirt_c = float(np.sum(U[k - 1] * p))
        assert abs(X[k - 1][r, c] - sirt_c) <= 1e-12 * abs(sirt_c)
        fbp_c = float(np.sum(np.sum(U[k - 1] * p, axis=1) / g.m))
        got = fbp_filter(g, p, U[k - 1])[r, c]
        assert abs(got - fbp_c) <= 1e-12 * abs(fbp_c)


def test_filters_symmetric_about_centre():
    g = make_geometry(15, 8, 21)
    U = sirt_filters(g, 6)
    ctr = filter_centres(g)
    assert np.all(ctr == 10)
    for k in range(6):
        assert np.abs(U[k] - U[k][:, ::-1]).max() <= 1e-14 * np.abs(U[k]).max()
        assert U[k][:, ctr[0]].min() > 0


@pytest.mark.parametrize("lo,hi", [(0.0, np.inf), (0.1, 0.6)])
def test_alg2_with_exact_sirt_is_exterior_following_sirt(lo, hi):
    n = 24
    g = make_geometry(n, 16, 35)
    p = fp_ray(g, _phantom(n, 3))
    rect, margin = (7, 9, 6, 5), 2
    K = 8
    X = sirt_iterates(g, p, K)
    res = local_method_box(g, p, rect, margin, None, lo, hi, xs_iterates=X, full=True)
    # projected SIRT on L; at step k the exterior is that of x_s^{k-1} (x_s^0 = 0)
    ext = roi_extend(rect, margin, n)
    WL = sparse_local(g, ext)
    alpha = default_alpha(g)
    x = np.zeros(ext[2] * ext[3])
    prev = np.zeros((n, n))
    for k in range(K):
        b = exterior_subtract(g, p, prev, ext).ravel()
        x = np.clip(x + alpha * (WL.T @ (b - WL @ x)), lo, hi)
        prev = X[k]
    ref = x.reshape(ext[2], ext[3])
    assert np.abs(res["x_ext_full"] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(res["x"] - crop(ref, ext, rect)).max() <= 1e-12 * np.abs(ref).max()


def test_alg2_without_prior_is_local_fbp():
    n = 20
    g = make_geometry(n, 12, 29)
    p = fp_ray(g, _phantom(n, 4))
    rect, margin = (5, 6, 7, 6), 3
    U = sirt_filters(g, 5)
    x = local_method_box(g, p, rect, margin, U, -np.inf, np.inf)
    ext = roi_extend(rect, margin, n)
    xs = fbp_filter(g, p, U[-1], ext)
    assert np.abs(x - crop(xs, ext, rect)).max() <= 1e-12 * np.abs(xs).max()


def test_filtered_fbp_tracks_sirt():
    """Eq. sfbp: FBP(p, u_K) approximates K SIRT iterations.  With this projector the
    impulse's own column holds 1/m_theta on one bin per angle, so the filters carry
    about mean(1/m) = 1.12 times the mass of a typical pixel's response and the early
    iterates are over-scaled; the gap closes as K grows."""
    n = 33
    g = make_geometry(n, 32, 49)
    p = fp_ray(g, _phantom(n, 5))
    K = 60
    U = sirt_filters(g, K)
    X = sirt_iterates(g, p, K)
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2.0
    inner = xx ** 2 + yy ** 2 < (0.3 * n) ** 2
    errs = []
    for k in (5, 20, 60):
        f = fbp_filter(g, p, U[k - 1])
        errs.append(np.linalg.norm((f - X[k - 1])[inner]) / np.linalg.norm(X[k - 1][inner]))
    assert errs[0] < 0.16 and errs[2] < 0.08
    assert errs[2] < errs[0]
    # the one-pixel-shifted filter (a wrong zero lag) is far worse
    f = bp_pixel(g, np.roll(filter_apply(g, U[K - 1], p), 1, axis=1))
    bad = np.linalg.norm((f - X[K - 1])[inner]) / np.linalg.norm(X[K - 1][inner])
    assert bad > 2 * errs[2]
