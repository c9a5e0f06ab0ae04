"""SIRT-approximating FBP filters and the paper's local method (TEST INFRASTRUCTURE ONLY).

Section 3.1: K iterations of SIRT from zero are x_s^K = alpha sum_{k<K} A^k W^T p with
A = I - alpha W^T W (eq. sirtfull2).  Replacing sum_{k<K} A^k by a 2D convolution
whose kernel is its impulse response q_K (eq. filtcalc) makes them an FBP with the
angle-dependent filter u_K = alpha W q_K (eq. sirtapp, eq. sfbp); Alg. 1 computes
every u_k, k = 1..K, in one pass.  Evaluating that FBP on the local part only gives
the local SIRT approximation (eq. locsirtapp).

Section 3.2: the local method (eq. localmethod, Alg. 2) iterates a correction image
y on the local part L with the local operators only:
    x_s^k = FBP_L(p, u_k) = W_L^T C_{u_k} p
    y^k   = y^{k-1} - alpha W_L^T W_L y^{k-1} + d^k
    x^k   = x_s^k + y^k
where d^k carries the prior; for SIRT with box constraints [l, r] (eq. sirtbox)
d^k = P_[l,r](v) - v with v = x_s^k + y^{k-1} - alpha W_L^T W_L y^{k-1}, so
x^k = P_[l,r](v) and y^k = x^k - x_s^k.

Readings (the paper leaves them to its projector library):
  * the impulse of Alg. 1 is pixel (N // 2, N // 2), the grid centre for odd N;
  * C_u is a linear convolution along the detector, zero outside it, whose zero lag
    for angle k sits at the bin nearest the projection of that pixel's centre
    (exactly the central bin for odd N and odd N_d with no detector offset);
  * alpha = 1 / (N_theta N_d) as in Section 3.1.
"""

import numpy as np

from .geometry import roi_extend
from .projector import fp_ray, bp_pixel, sparse_local
from .local import crop


def default_alpha(geom):
    """alpha = (N_theta N_d)^-1 (Section 3.1)."""
    return 1.0 / (geom.n_angles * geom.n_det)


def impulse_pixel(geom):
    """(row, col) of the impulse image of Alg. 1."""
    return geom.n // 2, geom.n // 2


def filter_centres(geom):
    """Per angle, the bin index that is lag zero of the angle's filter."""
    r, c = impulse_pixel(geom)
    t = geom.pixel_x(c) * geom.cos + geom.pixel_y(r) * geom.sin
    return np.floor(geom.bin_coord(t) + 0.5).astype(np.int64)


def sirt_filters(geom, iters, alpha=None, workers=1):
    """Alg. 1, returning every filter: U[k - 1] = u_k for k = 1..iters, each [N_theta, N_d].

    q_0 = 0, c = e (impulse); for k = 1..K: q_k = q_{k-1} + c, c <- c - alpha W^T W c;
    u_k = alpha W q_k, accumulated as u_k = u_{k-1} + alpha W c_{k-1}.
    """
    alpha = default_alpha(geom) if alpha is None else alpha
    n = geom.n
    c = np.zeros((n, n))
    c[impulse_pixel(geom)] = 1.0
    u = np.zeros((geom.n_angles, geom.n_det))
    out = np.empty((iters, geom.n_angles, geom.n_det))
    for k in range(iters):
        t = fp_ray(geom, c)                      # W c_{k-1}
        u = u + alpha * t                        # u_k
        out[k] = u
        c = c - alpha * bp_pixel(geom, t, workers=workers)   # c_k
    return out


def filter_apply(geom, u, sino):
    """C_u p: row k of the sinogram convolved with row k of the filter, lag zero at
    filter_centres(geom)[k], linear (zero outside the detector), N_d outputs."""
    sino = np.asarray(sino, dtype=np.float64)
    ctr = filter_centres(geom)
    out = np.empty_like(sino)
    nd = geom.n_det
    for k in range(geom.n_angles):
        full = np.convolve(sino[k], u[k])        # full[m] = sum_j p[j] u[m - j]
        # out[i] = sum_j u[i - j + c] p[j] = full[i + c]; indices outside full are 0
        lo = ctr[k]
        idx = np.arange(nd) + lo
        ok = (idx >= 0) & (idx < full.size)
        row = np.zeros(nd)
        row[ok] = full[idx[ok]]
        out[k] = row
    return out


def fbp_filter(geom, sino, u, rect=None, workers=1):
    """FBP(p, u) = W^T C_u p (eq. sfbp); with rect, FBP_L evaluated on that region."""
    return bp_pixel(geom, filter_apply(geom, u, sino), rect, workers=workers)


def sirt_iterates(geom, sino, iters, alpha=None, workers=1):
    """Exact global SIRT from zero (eq. sirtit): returns x_s^1 .. x_s^K, [K, N, N]."""
    alpha = default_alpha(geom) if alpha is None else alpha
    n = geom.n
    x = np.zeros((n, n))
    out = np.empty((iters, n, n))
    sino = np.asarray(sino, dtype=np.float64)
    for k in range(iters):
        x = x + alpha * bp_pixel(geom, sino - fp_ray(geom, x), workers=workers)
        out[k] = x
    return out


def local_method_box(geom, sino, rect, margin, filters, lo=0.0, hi=np.inf, alpha=None,
                     xs_iterates=None, full=False):
    """Alg. 2 with the box prior of eq. sirtbox on the extended local part.

    filters: U from sirt_filters (U[k-1] = u_k); the iteration count is len(U).
    xs_iterates (optional, [K, N, N]): use these images for x_s^k instead of
    FBP_L(p, u_k) (the exact-SIRT form of the method).
    Returns the ROI crop, or with full=True a dict with the extended rect, the
    extended iterate and W_L.
    """
    alpha = default_alpha(geom) if alpha is None else alpha
    ext = roi_extend(rect, margin, geom.n)
    r0, c0, rr, cc = ext
    WL = sparse_local(geom, ext)
    iters = len(filters) if xs_iterates is None else len(xs_iterates)
    sino = np.asarray(sino, dtype=np.float64)
    y = np.zeros(rr * cc)
    x = y
    for k in range(iters):
        if xs_iterates is None:
            xs = WL.T @ filter_apply(geom, filters[k], sino).ravel()
        else:
            xs = np.asarray(xs_iterates[k])[r0:r0 + rr, c0:c0 + cc].ravel()
        v = xs + y - alpha * (WL.T @ (WL @ y))
        x = np.clip(v, lo, hi)
        y = x - xs
    x = x.reshape(rr, cc)
    out = crop(x, ext, rect)
    if full:
        return dict(x=out, x_ext_full=x, ext=ext, WL=WL)
    return out
