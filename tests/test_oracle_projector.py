"""Pins for the oracle's projector (Section 2.1: W, W^T, W_L = W M_L, W = W_L + W_F)."""

import numpy as np
import pytest

import oracle
import synth


GEOMS = [(8, 4, 12), (8, 8, 13), (16, 8, 24), (16, 32, 25), (12, 7, 20)]


@pytest.mark.parametrize("n,na,nd", GEOMS)
def test_dense_brute_force_three_ways(n, na, nd):
    """Entry-by-entry loops, ray-driven impulse responses and the sparse pixel-driven
    matrix are the same W (angles 0, pi/4 and pi/2 occur for na = 4, 8, 32)."""
    g = oracle.make_geometry(n, na, nd)
    for rect in [(0, 0, n, n), (1, 2, n // 2, n // 2 + 1), (n - 3, 0, 3, n)]:
        Wh = oracle.dense_matrix_hat(g, rect)
        Wr = oracle.dense_matrix_ray(g, rect)
        Ws = oracle.sparse_local(g, rect).toarray()
        assert np.abs(Wh - Wr).max() < 1e-12
        assert np.abs(Wh - Ws).max() < 1e-12
        assert Wh.min() >= 0.0


def test_tie_at_45_degrees_is_row_stepping():
    g = oracle.make_geometry(16, 8, 24)
    k = 2   # theta = pi/4
    assert g.ystep[k] and np.isclose(g.m[k], np.sqrt(0.5))
    assert not g.ystep[6]   # 3pi/4 -> |sin| > |cos| in FP64


@pytest.mark.parametrize("n,na,nd", [(128, 32, 192), (1024, 128, 1536), (2048, 256, 3072),
                                     (4096, 512, 6144), (2048, 512, 3072)])
def test_adjoint_identity_ray_fp_vs_pixel_bp(n, na, nd):
    """<W_L x, y> = <x, W_L^T y> between the two independent codes, to 1e-12 relative,
    at every workload geometry, for ROIs in the interior and touching the edges."""
    g = oracle.make_geometry(n, na, nd)
    rng = np.random.default_rng(n + na)
    side = 12
    for rect in [(n // 2 - 5, n // 3, side, side + 3), (0, 0, side, side), (n - side, n - side - 1, side, side + 1)]:
        x = rng.random((rect[2], rect[3]))
        y = rng.random((na, nd))
        lhs = float(np.sum(oracle.fp_ray(g, x, rect) * y))
        rhs = float(np.sum(x * oracle.bp_pixel(g, y, rect)))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_constant_image_axis_angles_closed_form():
    """At theta = 0 and pi/2 the Joseph FP of a constant image is the number of
    rows the ray crosses: N for bins over the grid, N/2 for a ray on the outer
    half-pixel, 0 beyond."""
    n = 16
    ones = np.ones((n, n))
    g = oracle.make_geometry(n, 2, 24)   # bins aligned with pixel centres
    p = oracle.fp_ray(g, ones)
    exp = np.zeros(24)
    exp[4:20] = n
    assert np.allclose(p[0], exp, atol=1e-13) and np.allclose(p[1], exp, atol=1e-13)
    g = oracle.make_geometry(n, 2, 25)   # bins between pixel centres
    p = oracle.fp_ray(g, ones)
    exp = np.zeros(25)
    exp[5:20] = n
    exp[4] = exp[20] = n / 2
    assert np.allclose(p[0], exp, atol=1e-13) and np.allclose(p[1], exp, atol=1e-13)


def test_disc_chord_convergence():
    """Joseph FP of a finely sampled disc approaches the exact chord 2 sqrt(r^2 - s^2)
    as pixels shrink (disc radius fixed in physical units): the error falls at
    least by a factor 1.5 per halving of the pixel size."""
    errs = []
    for n in (32, 64, 128):
        r = 0.3 * n
        g = oracle.make_geometry(n, 16, int(1.5 * n))
        ell = synth.Ellipses(np.array([0.7]), np.array([-1.3]), np.array([r]), np.array([r]),
                             np.array([0.0]), np.array([1.0]))
        img = synth.raster(ell, n, supersample=8)
        exact = synth.analytic_sinogram(ell, 16, int(1.5 * n), subrays=1)
        p = oracle.fp_ray(g, img)
        errs.append(np.linalg.norm(p - exact) / np.linalg.norm(exact))
    assert errs[0] < 0.05
    assert errs[0] / errs[1] >= 1.5 and errs[1] / errs[2] >= 1.5, errs


def test_local_operator_is_masked_global():
    """W_L = W M_L (eq. 1): projecting a region equals projecting the full image
    with zeros outside; W = W_L + W_F (eq. locouter)."""
    g = oracle.make_geometry(24, 12, 36)
    rng = np.random.default_rng(1)
    x = rng.random((24, 24))
    rect = (5, 7, 9, 11)
    mask = np.zeros((24, 24), bool)
    mask[5:14, 7:18] = True
    pl = oracle.fp_ray(g, x[5:14, 7:18], rect)
    assert np.abs(pl - oracle.fp_ray(g, np.where(mask, x, 0.0))).max() < 1e-12
    pf = oracle.fp_ray(g, np.where(mask, 0.0, x))
    assert np.abs(pl + pf - oracle.fp_ray(g, x)).max() < 1e-12
    # W_L^T = M_L W^T
    y = rng.random((12, 36))
    assert np.abs(oracle.bp_pixel(g, y, rect) - oracle.bp_pixel(g, y)[5:14, 7:18]).max() < 1e-12


def test_band_is_nonzero_rows():
    g = oracle.make_geometry(40, 16, 60)
    rect = (3, 20, 10, 14)
    band = oracle.band_exact(g, rect)
    W = oracle.sparse_local(g, rect).tocoo()
    rows = np.unique(W.row)
    for k in range(16):
        rk = rows[(rows >= k * 60) & (rows < (k + 1) * 60)] - k * 60
        assert (band[k, 0], band[k, 1]) == (rk.min(), rk.max())
        assert len(rk) == rk.max() - rk.min() + 1   # contiguous
