"""Discrete gradient and divergence for total variation (Section 2.3; test infrastructure only).

The paper's TV penalty is g(x) = ||grad x||_1 with "a discrete gradient
operator" left unspecified.  The oracle uses forward differences with a zero
difference on the last row / column (Neumann boundary), restricted to the
local part, and the divergence div = -grad^T in the standard form of
Chambolle (2004):

    (grad x)_0[r, c] = x[r+1, c] - x[r, c]  (0 on the last row)
    (grad x)_1[r, c] = x[r, c+1] - x[r, c]  (0 on the last column)
    (div z)[r, c]    = d0 + d1 with
        d0 = z0[r, c] - z0[r-1, c] inside, z0[0, c] on the first row,
             -z0[rows-2, c] on the last row; d1 likewise along columns.

Isotropic TV sums the per-pixel Euclidean norm of the 2-vector; anisotropic
TV sums absolute values.
"""

import numpy as np


def grad(x):
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros((2,) + x.shape)
    g[0, :-1, :] = x[1:, :] - x[:-1, :]
    g[1, :, :-1] = x[:, 1:] - x[:, :-1]
    return g


def div(z):
    z = np.asarray(z, dtype=np.float64)
    rows, cols = z.shape[1:]
    d = np.zeros((rows, cols))
    z0, z1 = z[0], z[1]
    if rows > 1:
        d[0, :] += z0[0, :]
        d[1:-1, :] += z0[1:-1, :] - z0[:-2, :]
        d[-1, :] += -z0[-2, :]
    if cols > 1:
        d[:, 0] += z1[:, 0]
        d[:, 1:-1] += z1[:, 1:-1] - z1[:, :-2]
        d[:, -1] += -z1[:, -2]
    return d


def tv_iso(x):
    g = grad(x)
    return float(np.sum(np.sqrt(g[0] ** 2 + g[1] ** 2)))


def tv_aniso(x):
    g = grad(x)
    return float(np.sum(np.abs(g)))
