"""Pins for the oracle's FBP (Section 2.2 eq. fbp) and TV operators (Section 2.3)."""

import numpy as np
import pytest

import oracle
import synth


def test_ramlak_frequency_response_is_ramp():
    """The DTFT of the Ram-Lak taps is the Fourier series of a triangle wave:
    sum_n h[n] e^{-i n w} = |w| / (2 pi) on [-pi, pi] (closed form), up to the
    truncation of the series at |n| < N_d (tail < 2 / (pi^2 N_d))."""
    nd = 1024
    n, h = oracle.ramlak_taps(nd)
    w = np.linspace(-np.pi, np.pi, 257)
    H = (h[None, :] * np.cos(np.outer(w, n))).sum(axis=1)
    assert np.abs(H - np.abs(w) / (2 * np.pi)).max() < 2.0 / (np.pi ** 2 * nd) + 1e-12
    assert abs(H[128]) < 1e-3   # zero DC response


def test_ramp_filter_linear_convolution_brute_force():
    g = oracle.make_geometry(8, 3, 9)
    rng = np.random.default_rng(2)
    p = rng.random((3, 9))
    q = oracle.ramp_filter(g, p, method="direct")
    ref = np.zeros_like(p)
    for k in range(3):
        for i in range(9):
            for j in range(9):
                d = i - j
                hv = 0.25 if d == 0 else (0.0 if d % 2 == 0 else -1.0 / (np.pi ** 2 * d * d))
                ref[k, i] += hv * p[k, j]
    assert np.abs(q - ref).max() < 1e-14
    g2 = oracle.make_geometry(600, 4, 700)
    p2 = rng.random((4, 700))
    assert np.abs(oracle.ramp_filter(g2, p2, "direct") - oracle.ramp_filter(g2, p2, "fft")).max() < 1e-12


@pytest.mark.parametrize("spacing", [1.0, 2.0])
def test_fbp_of_disc_recovers_value(spacing):
    """FBP of the exact sinogram of a uniform disc gives its value inside (interior mean
    within 2%) and ~0 outside; this fixes the pi/N_theta and spacing scale factors."""
    n, na = 128, 96
    nd = int(192 / spacing)
    g = oracle.make_geometry(n, na, nd, spacing=spacing)
    p = synth.disc_sinogram(40.0, 0.8, na, nd, spacing=spacing, subrays=4)
    x = oracle.fbp_ramlak(g, p)
    inner = x[64 - 20:64 + 20, 64 - 20:64 + 20].mean()
    assert abs(inner - 0.8) < 0.02 * 0.8
    assert abs(x[:12, :12].mean()) < 0.02
    assert np.abs(oracle.fbp_ramlak(g, np.zeros((na, nd)))).max() == 0.0


def test_fbp_linear():
    g = oracle.make_geometry(16, 8, 24)
    rng = np.random.default_rng(3)
    a, b = rng.random((8, 24)), rng.random((8, 24))
    lhs = oracle.fbp_ramlak(g, 2.0 * a - 3.0 * b)
    rhs = 2.0 * oracle.fbp_ramlak(g, a) - 3.0 * oracle.fbp_ramlak(g, b)
    assert np.abs(lhs - rhs).max() < 1e-12


def test_div_is_minus_grad_adjoint():
    rng = np.random.default_rng(4)
    for shape in [(1, 5), (5, 1), (7, 9), (16, 16)]:
        x = rng.standard_normal(shape)
        z = rng.standard_normal((2,) + shape)
        lhs = float(np.sum(oracle.grad(x) * z))
        rhs = -float(np.sum(x * oracle.div(z)))
        assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_tv_closed_forms():
    x = np.zeros((10, 12))
    x[:, 5:] = 2.0          # vertical edge of height 2 across 10 rows
    assert oracle.tv_iso(x) == pytest.approx(20.0)
    assert oracle.tv_aniso(x) == pytest.approx(20.0)
    r = np.add.outer(np.arange(6.0), np.arange(6.0))   # ramp x = r + c
    # forward differences 1 and 1 except the last row/column: iso = 25 sqrt(2) + 5 + 5
    assert oracle.tv_iso(r) == pytest.approx(25 * np.sqrt(2) + 10)
    assert oracle.tv_aniso(r) == pytest.approx(60.0)
