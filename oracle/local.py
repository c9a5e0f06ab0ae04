"""Local solve on an extended region after exterior subtraction (test infrastructure only).

Pieces and the passages they follow:
  * local part L = the requested ROI padded on each side and cropped back at the end
    (Section 3.3; the pad width is a parameter);
  * W = W_L + W_F (eq. locouter), hence the data the local part explains are
    b = p - W_F x_ext = p - W (M_F x_ext) for an estimate x_ext of the exterior;
  * the prior (TV, nonnegativity) acts only inside L and nothing outside L is
    updated (Section 3.2: prior only inside L; the effect on pixels outside L
    is ignored);
  * independent local parts are placed side by side without blending (Section 5.6).

The exterior estimate defaults to the Ram-Lak FBP of the whole sinogram.  The CP
solve's data term is measured with the image side as the unit of length (h = 1/N,
see solvers.py) unless h is given.
"""

import numpy as np

from .geometry import roi_extend
from .projector import fp_ray, sparse_local
from .fbp import fbp_ramlak
from .solvers import cp_steps, cp_tv_nonneg, sirt_nonneg


def exterior_subtract(geom, sino, x_ext, ext_rect, bins=None):
    """b = p - W (M_F x_ext): project the exterior (x_ext with L zeroed) and subtract.

    With bins (a boolean [N_theta, N_d] mask), only those rays are computed and
    b is zero elsewhere.
    """
    r0, c0, rr, cc = ext_rect
    xf = np.array(x_ext, dtype=np.float64, copy=True)
    xf[r0:r0 + rr, c0:c0 + cc] = 0.0
    fpf = fp_ray(geom, xf, None, bins)
    b = np.asarray(sino, dtype=np.float64) - fpf
    if bins is not None:
        b = np.where(bins, b, 0.0)
    return b


def crop(img, ext_rect, rect):
    """Crop the extended-region image back to the requested ROI."""
    dr, dc = rect[0] - ext_rect[0], rect[1] - ext_rect[1]
    return np.asarray(img)[dr:dr + rect[2], dc:dc + rect[3]]


def stitch(n, rects, crops, fill=0.0):
    """Place ROI crops into an n x n image side by side (no blending)."""
    out = np.full((n, n), fill, dtype=np.float64)
    for (r0, c0, rr, cc), x in zip(rects, crops):
        out[r0:r0 + rr, c0:c0 + cc] = x
    return out


def local_solve(geom, sino, rect, margin, method="cp", lam=0.0, iters=100, sigma=None,
                tau=None, x_ext=None, half=False, aniso=False, workers=1, full=False,
                dual_callback=None, h=None):
    """Reconstruct ROI rect: extend, subtract the exterior, iterate on L, crop.

    Returns the ROI crop (rows, cols), or with full=True a dict that also holds
    the extended rect, b, the step sizes, x_ext and the uncropped iterate.
    """
    ext = roi_extend(rect, margin, geom.n)
    if x_ext is None:
        x_ext = fbp_ramlak(geom, sino, workers=workers)
    WL = sparse_local(geom, ext)
    used = np.zeros(geom.n_angles * geom.n_det, dtype=bool)
    used[np.unique(WL.tocoo().row)] = True
    bins = used.reshape(geom.n_angles, geom.n_det)
    b = exterior_subtract(geom, sino, x_ext, ext, bins=bins)
    shape = (ext[2], ext[3])
    if h is None:
        h = 1.0 / geom.n
    if method == "cp":
        if sigma is None or tau is None:
            sigma, tau = cp_steps(WL, shape, h=h)
        x = cp_tv_nonneg(WL, b, shape, lam, sigma, tau, iters, half=half, aniso=aniso,
                         dual_callback=dual_callback, h=h)
    elif method == "sirt":
        alpha = 1.0 / (geom.n_angles * geom.n_det)
        x = sirt_nonneg(WL, b, shape, alpha, iters)
    else:
        raise ValueError(method)
    out = crop(x, ext, rect)
    if full:
        return dict(x=out, x_ext_full=x, ext=ext, b=b, sigma=sigma, tau=tau, x_ext=x_ext,
                    WL=WL, bins=bins, h=h)
    return out
