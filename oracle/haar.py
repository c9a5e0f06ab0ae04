"""Haar wavelet l1 prior and the local FISTA for it (TEST INFRASTRUCTURE ONLY).

Section 2.3 / Section 4: the penalty g(x) = ||B x||_1 with B a Haar wavelet decomposition,
minimised by ISTA (eq. sirtista: x <- B^-1 P(B S(x)), P soft thresholding) or, in the
experiments, FISTA.  B being orthonormal, the prox of gamma ||B x||_1 is exactly
B^T P_gamma(B w), so the local method (Alg. 3 with this prox in place of FGP) needs no
inner iteration.

Readings (the paper does not fix them): B is the separable 2D Haar transform with
`levels` levels on the extended local part (default 4); one level acts on the current
approximation block of h x w coefficients, first along rows then along columns, mapping
each pair (a, b) to ((a + b)/sqrt 2, (a - b)/sqrt 2) with the sums first and the
differences after them, and an unpaired last entry (odd length) passed on unchanged as
the last sum -- an orthonormal map for any size; the next level acts on the
ceil(h/2) x ceil(w/2) block of sums.  All coefficients, the coarsest sums included, enter
||B x||_1 (as written).  The threshold is gamma = alpha lambda / 2, the weight of the
SIRT step on eq. priorsys as for TV (eq. sirtista prints the threshold as lambda).
"""

import numpy as np

from .fista import local_fista, prox_weight

_S = 1.0 / np.sqrt(2.0)


def _fwd_1d(v):
    """One level along the last axis of v (..., n): [sums, (unpaired), differences]."""
    n = v.shape[-1]
    m = n // 2
    a = (v[..., 0:2 * m:2] + v[..., 1:2 * m:2]) * _S
    d = (v[..., 0:2 * m:2] - v[..., 1:2 * m:2]) * _S
    parts = [a] + ([v[..., n - 1:n]] if n % 2 else []) + [d]
    return np.concatenate(parts, axis=-1)


def _inv_1d(c):
    n = c.shape[-1]
    m = n // 2
    na = n - m                       # sums (and the unpaired entry)
    a, d = c[..., :m], c[..., na:]
    out = np.empty_like(c)
    out[..., 0:2 * m:2] = (a + d) * _S
    out[..., 1:2 * m:2] = (a - d) * _S
    if n % 2:
        out[..., n - 1] = c[..., m]
    return out


def haar_forward(x, levels):
    c = np.array(x, dtype=np.float64, copy=True)
    h, w = c.shape
    for _ in range(levels):
        if h < 1 or w < 1:
            break
        blk = c[:h, :w]
        blk = _fwd_1d(blk)                    # rows
        blk = _fwd_1d(blk.T).T                # columns
        c[:h, :w] = blk
        h, w = (h + 1) // 2, (w + 1) // 2
    return c


def haar_inverse(c, levels):
    x = np.array(c, dtype=np.float64, copy=True)
    h, w = x.shape
    sizes = []
    for _ in range(levels):
        sizes.append((h, w))
        h, w = (h + 1) // 2, (w + 1) // 2
    for h, w in reversed(sizes):
        blk = x[:h, :w]
        blk = _inv_1d(blk.T).T                # columns
        blk = _inv_1d(blk)                    # rows
        x[:h, :w] = blk
    return x


def soft(c, gamma):
    return np.sign(c) * np.maximum(np.abs(c) - gamma, 0.0)


def haar_prox(w, gamma, levels):
    """argmin_x 1/2 ||x - w||^2 + gamma ||B x||_1 = B^T soft(B w, gamma)."""
    return haar_inverse(soft(haar_forward(w, levels), gamma), levels)


def local_fista_haar(geom, sino, rect, margin, filters, lam, levels=4, half=False, alpha=None,
                     xs_iterates=None, full=False, momentum=True):
    """The local method (Alg. 3 form) with the Haar l1 prox; momentum=False gives the
    ISTA iteration of eq. sirtista."""
    gamma = prox_weight(geom, lam, alpha, half)
    return local_fista(geom, sino, rect, margin, filters,
                       lambda w: haar_prox(w, gamma, levels), alpha, xs_iterates, full, gamma,
                       momentum)
