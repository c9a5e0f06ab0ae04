"""Data preprocessing of the local method (TEST INFRASTRUCTURE ONLY).

Section 3.3 (implementation details): before a reconstruction with the local method the
projection of a disc centred on the rotation axis, of diameter N and constant value c, is
subtracted from the data, c chosen so that the zero-frequency components of all
projections have the least l2 norm afterwards; the disc is added back to the result.
Section 4 (truncated data): data cut off at the detector's edges are padded before the
filtered backprojection, and the local method uses the same padding.

Readings: the disc holds the pixels whose centres lie in the closed disc of radius N/2
about the grid centre, and "its forward projection" is W applied to that image (so that
adding c times the same pixels back undoes the subtraction exactly for a linear
reconstruction); the zero-frequency component of a projection is the sum of its bins, so
c = sum_k S_k T_k / sum_k T_k^2 with S_k, T_k the row sums of p and of W disc.
Constant padding extends each truncated row by its first and last measured values.
"""

import numpy as np

from .projector import fp_ray


def disc_image(geom):
    """1 on pixels whose centre is within N/2 of the grid centre, else 0."""
    n = geom.n
    x = geom.pixel_x(np.arange(n))
    return ((x[None, :] ** 2 + x[:, None] ** 2) <= (n / 2.0) ** 2).astype(np.float64)


def disc_value(geom, sino, disc_sino=None):
    """c minimising sum_k (sum_i (p - c D)[k, i])^2, D = W disc."""
    D = fp_ray(geom, disc_image(geom)) if disc_sino is None else disc_sino
    S = np.asarray(sino, dtype=np.float64).sum(axis=1)
    T = D.sum(axis=1)
    return float(np.dot(S, T) / np.dot(T, T))


def disc_subtract(geom, sino):
    """(p - c W disc, c)."""
    D = fp_ray(geom, disc_image(geom))
    c = disc_value(geom, sino, D)
    return np.asarray(sino, dtype=np.float64) - c * D, c


def disc_add(geom, img, rect, c):
    """img (the crop `rect` of the grid) plus c on the disc's pixels."""
    r0, c0, rr, cc = rect
    return np.asarray(img, dtype=np.float64) + c * disc_image(geom)[r0:r0 + rr, c0:c0 + cc]


def pad_truncated(trunc, first_bin, n_det):
    """Rows of a detector cut to bins [first_bin, first_bin + n_bins) extended to n_det
    bins with their edge values (constant padding)."""
    trunc = np.asarray(trunc, dtype=np.float64)
    nb = trunc.shape[1]
    idx = np.clip(np.arange(n_det) - first_bin, 0, nb - 1)
    return trunc[:, idx]
