"""Filtered backprojection with the Ram-Lak filter (Section 2.2 eq. fbp; test infrastructure only).

FBP(p, h) = W^T C_h p, where C_h convolves every detector row (one angle)
with the 1D filter h.  The paper names the Ram-Lak filter and defers its
discretisation to Kak & Slaney; the oracle uses that book's spatial-domain
form for sampling interval tau = detector spacing:

    h[0] = 1/(4 tau^2),  h[n] = 0 for even n != 0,  h[n] = -1/(pi^2 n^2 tau^2) for odd n,

with filtered projection Q = tau * (h * p) as a *linear* (zero-padded, not
circular) convolution truncated to the N_d detector samples, and the
backprojection sum over angles weighted by pi / N_theta (angles uniform in
[0, pi)).  The Joseph weights of W^T sum, on average over a detector period,
to 1/tau per angle, so one more factor tau makes W^T an unbiased
backprojection: x_ext = (pi/N_theta) * tau * W^T Q, which for tau = 1 is
(pi/N_theta) W^T (h * p).
"""

import numpy as np


def ramlak_taps(n_det, spacing=1.0):
    """Offsets n = -(N_d-1)..N_d-1 and the Ram-Lak taps h[n]."""
    n = np.arange(-(n_det - 1), n_det)
    h = np.zeros(len(n))
    h[n == 0] = 1.0 / (4.0 * spacing * spacing)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (np.pi ** 2 * n[odd].astype(np.float64) ** 2 * spacing * spacing)
    return n, h


def ramp_filter(geom, sino, method="auto"):
    """Q[k, i] = spacing * sum_j h[i - j] p[k, j]  (linear convolution, N_d outputs)."""
    sino = np.asarray(sino, dtype=np.float64)
    nd = geom.n_det
    _, h = ramlak_taps(nd, geom.spacing)
    if method == "auto":
        method = "direct" if nd <= 512 else "fft"
    out = np.empty_like(sino)
    if method == "direct":
        for k in range(sino.shape[0]):
            out[k] = np.convolve(sino[k], h, mode="full")[nd - 1:2 * nd - 1]
    else:
        from scipy.signal import fftconvolve
        full = fftconvolve(sino, h[None, :], mode="full", axes=1)
        out[:] = full[:, nd - 1:2 * nd - 1]
    return out * geom.spacing


def fbp_ramlak(geom, sino, rect=None, workers=1):
    """x_ext = (pi / N_theta) * spacing * W^T Q on region rect (default: the whole grid)."""
    from .projector import bp_pixel
    q = ramp_filter(geom, sino)
    return (np.pi / geom.n_angles) * geom.spacing * bp_pixel(geom, q, rect, workers=workers)
