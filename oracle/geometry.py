"""Parallel-beam geometry (paper Section 2.1; test infrastructure only).

The paper fixes: 2D parallel beam with one rotation axis, N_d detectors,
N_theta angles, an N x N pixel grid, p with N_d N_theta entries, x with N^2
entries.  It leaves the coordinate conventions to the projector library, so
the oracle fixes them (the same conventions the `synth` generator states):

  pixel (r, c):  x = c - (N-1)/2,  y = r - (N-1)/2
  bin i:         s_i = (i - (N_d-1)/2) * spacing + offset
  angle k:       theta_k = k pi / N_theta unless given
  ray (k, i):    {x cos theta_k + y sin theta_k = s_i}

The Joseph projector steps along rows when |cos theta| >= |sin theta|
(evaluated in FP64 here; the tie at 45 degrees resolves by this comparison)
and along columns otherwise; m_k is the dominant |cos| or |sin|.
"""

from dataclasses import dataclass

import numpy as np


@dataclass
class Geometry:
    n: int
    n_angles: int
    n_det: int
    theta: np.ndarray
    cos: np.ndarray
    sin: np.ndarray
    spacing: float
    offset: float
    ystep: np.ndarray     # bool: step along rows (|cos| >= |sin|)
    m: np.ndarray         # |cos| if ystep else |sin|

    @property
    def s(self):
        return (np.arange(self.n_det) - (self.n_det - 1) / 2.0) * self.spacing + self.offset

    def pixel_x(self, cols):
        return np.asarray(cols, dtype=np.float64) - (self.n - 1) / 2.0

    def pixel_y(self, rows):
        return np.asarray(rows, dtype=np.float64) - (self.n - 1) / 2.0

    def bin_coord(self, t):
        """Real-valued bin index whose centre is at detector coordinate t."""
        return (np.asarray(t) - self.offset) / self.spacing + (self.n_det - 1) / 2.0


def make_geometry(n, n_angles, n_det, angles=None, spacing=1.0, offset=0.0):
    if n < 1 or n_angles < 1 or n_det < 1:
        raise ValueError("sizes must be positive")
    theta = (np.arange(n_angles, dtype=np.float64) * (np.pi / n_angles) if angles is None
             else np.asarray(angles, dtype=np.float64).copy())
    c, s = np.cos(theta), np.sin(theta)
    ystep = np.abs(c) >= np.abs(s)
    m = np.where(ystep, np.abs(c), np.abs(s))
    return Geometry(n, len(theta), n_det, theta, c, s, float(spacing), float(offset), ystep, m)


def roi_extend(rect, margin, n):
    """Extend a local part by `margin` pixels on each side and clip to the grid.

    Section 3.3: the local part is padded on each side and the result is
    cropped back afterwards, against edge artifacts of the prior.
    rect = (row0, col0, rows, cols), half-open on the global lattice.
    """
    r0, c0, rr, cc = rect
    a0, b0 = max(0, r0 - margin), max(0, c0 - margin)
    a1, b1 = min(n, r0 + rr + margin), min(n, c0 + cc + margin)
    return (a0, b0, a1 - a0, b1 - b0)


def band_exact(geom, rect):
    """Per angle, the inclusive range [lo, hi] of bins with a nonzero weight for
    some pixel of rect (brute force over all pixels); (0, -1) when empty.

    These are the nonzero rows of W_L (Section 2.1: many rows of W_L are zero).
    """
    r0, c0, rr, cc = rect
    xs = geom.pixel_x(np.arange(c0, c0 + cc))
    ys = geom.pixel_y(np.arange(r0, r0 + rr))
    out = np.zeros((geom.n_angles, 2), dtype=np.int64)
    s = geom.s
    for k in range(geom.n_angles):
        t = xs[None, :] * geom.cos[k] + ys[:, None] * geom.sin[k]
        tmin, tmax = t.min(), t.max()
        # candidate bins, then the exact strict test |s_i - t| < m for the nearest pixel
        lo = max(0, int(np.floor(geom.bin_coord(tmin - geom.m[k]))) - 1)
        hi = min(geom.n_det - 1, int(np.ceil(geom.bin_coord(tmax + geom.m[k]))) + 1)
        tv = np.sort(t.ravel())
        hit = []
        for i in range(lo, hi + 1):
            j = np.searchsorted(tv, s[i])
            d = min(abs(s[i] - tv[j]) if j < len(tv) else np.inf,
                    abs(s[i] - tv[j - 1]) if j > 0 else np.inf)
            if d < geom.m[k]:
                hit.append(i)
        out[k] = (hit[0], hit[-1]) if hit else (0, -1)
    return out
