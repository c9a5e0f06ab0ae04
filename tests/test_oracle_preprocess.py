"""Pins of the disc subtraction and the constant padding of truncated data (Section 3.3,
Section 4).

  * the disc value is the minimiser of the zero-frequency objective (checked against a
    numerical minimiser of that objective, not the closed form);
  * data that are exactly a multiple of the disc's projection give that multiple and a
    zero residual;
  * the disc image against a double loop of the definition, and its area against pi r^2;
  * the subtraction does what the paper uses it for: the filtered approximation of SIRT
    and the local method are closer to SIRT with it;
  * constant padding against a plain loop, identity without truncation, and on heavily
    truncated data (a third of the detector) the local reconstruction of the central part
    from padded data differs from the full-data one by a nearly constant offset, while
    zero-extended data leave the structured truncation error.
"""

import numpy as np
import pytest
import scipy.optimize as sopt

from oracle import make_geometry, fp_ray
from oracle.filters import sirt_filters, sirt_iterates, local_method_box, fbp_filter
from oracle.preprocess import disc_image, disc_value, disc_subtract, disc_add, pad_truncated


def _phantom(n):
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2.0
    return 0.6 * ((xx ** 2 + yy ** 2) < (0.45 * n) ** 2) + 0.4 * (((xx - 8) ** 2 + (yy + 5) ** 2) < 36)


def test_disc_value_minimises_the_zero_frequency_norm():
    g = make_geometry(33, 20, 49)
    rng = np.random.default_rng(4)
    p = fp_ray(g, _phantom(33)) + rng.normal(0, 0.1, (20, 49))
    D = fp_ray(g, disc_image(g))
    f = lambda c: float(np.sum(np.sum(p - c * D, axis=1) ** 2))
    c_num = sopt.minimize_scalar(f, bracket=(-10, 10), tol=1e-14).x
    c = disc_value(g, p)
    assert c == pytest.approx(c_num, rel=1e-7)
    assert f(c) <= f(c * (1 + 1e-4)) and f(c) <= f(c * (1 - 1e-4))


def test_multiple_of_the_disc():
    g = make_geometry(24, 16, 37)
    p = 0.37 * fp_ray(g, disc_image(g))
    q, c = disc_subtract(g, p)
    assert c == pytest.approx(0.37, rel=1e-13)
    assert np.abs(q).max() <= 1e-12


@pytest.mark.parametrize("n", [7, 8, 31])
def test_disc_image_definition(n):
    g = make_geometry(n, 4, 2 * n)
    d = disc_image(g)
    for r in range(n):
        for c in range(n):
            x, y = c - (n - 1) / 2.0, r - (n - 1) / 2.0
            assert d[r, c] == (1.0 if x * x + y * y <= n * n / 4.0 else 0.0)
    assert np.array_equal(d, d[::-1, ::-1]) and np.array_equal(d, d.T)
    if n == 31:
        assert abs(d.sum() - np.pi * n * n / 4) / (np.pi * n * n / 4) < 0.02


def test_disc_subtraction_improves_the_local_approximation():
    n, na, nd = 65, 48, 97
    g = make_geometry(n, na, nd)
    p = fp_ray(g, _phantom(n))
    q, c = disc_subtract(g, p)
    K = 40
    U = sirt_filters(g, K, workers=4)
    X = sirt_iterates(g, p, K, workers=4)
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2.0
    inner = xx ** 2 + yy ** 2 < (0.3 * n) ** 2
    for k in (4, 10):
        plain = fbp_filter(g, p, U[k - 1])
        with_disc = fbp_filter(g, q, U[k - 1]) + c * disc_image(g)
        e0 = np.linalg.norm((plain - X[k - 1])[inner]) / np.linalg.norm(X[k - 1][inner])
        e1 = np.linalg.norm((with_disc - X[k - 1])[inner]) / np.linalg.norm(X[k - 1][inner])
        assert e1 < 0.5 * e0
    rect, m = (20, 24, 20, 18), 5
    ref = X[-1][20:40, 24:42]
    a = local_method_box(g, p, rect, m, U, -np.inf, np.inf)
    b = disc_add(g, local_method_box(g, q, rect, m, U, -np.inf, np.inf), rect, c)
    assert np.linalg.norm(b - ref) < 0.7 * np.linalg.norm(a - ref)


def test_pad_truncated_definition():
    rng = np.random.default_rng(5)
    t = rng.normal(size=(3, 5))
    out = pad_truncated(t, 4, 12)
    for k in range(3):
        for i in range(12):
            j = min(max(i - 4, 0), 4)
            assert out[k, i] == t[k, j]
    assert np.array_equal(pad_truncated(t, 0, 5), t)


def test_padding_helps_truncated_local_reconstruction():
    n, na, nd = 65, 40, 97
    g = make_geometry(n, na, nd)
    p = fp_ray(g, _phantom(n))
    first, nb = 32, 33                      # the central 33 bins are measured
    trunc = p[:, first:first + nb]
    padded = pad_truncated(trunc, first, nd)
    zero = np.zeros_like(p)
    zero[:, first:first + nb] = trunc
    K = 30
    U = sirt_filters(g, K, workers=4)
    rect, m = (24, 24, 17, 17), 4           # inside the measured field of view
    full = local_method_box(g, p, rect, m, U, -np.inf, np.inf)
    a = local_method_box(g, padded, rect, m, U, -np.inf, np.inf)
    b = local_method_box(g, zero, rect, m, U, -np.inf, np.inf)
    # padding removes most of the structure of the truncation error (the cupping of
    # zero-extended data), leaving a nearly constant offset
    assert np.std(a - full) < 0.3 * np.std(b - full)
