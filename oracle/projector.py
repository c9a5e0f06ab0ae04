"""Projection operators W, W^T and the local operators (Section 2.1; test infrastructure only).

The paper defines W as the N_d N_theta x N^2 matrix whose entry w_ij is the
contribution of pixel j to detector i, applied on the fly, and the local
operators W_L = W M_L, W_L^T = M_L W^T (eq. 1).  It does not fix the
discretisation (its experiments use a GPU toolbox).  The oracle uses
Joseph's method (linear interpolation between the two pixel centres the ray
passes between, on the row or column of the dominant direction, times the
path length per step 1/m):

    w[(k,i), (r,c)] = max(0, 1 - |s_i - t_rc| / m_k) / m_k,
    t_rc = x_c cos theta_k + y_r sin theta_k,  m_k = max(|cos|, |sin|).

The detector is sampled at bin centres (no bin-width integration) and pixels
outside the grid count as zero.

Two independent codes compute it:
  * fp_ray   - ray-driven: for every ray, step through the rows (or columns)
               and interpolate linearly between the two neighbouring pixels;
  * bp_pixel - pixel-driven: for every pixel and angle, evaluate the hat weight
               on the (at most two) bins it reaches and gather.
They share no helper, so the adjoint identity <W x, y> = <x, W^T y> between
them is a real check.  sparse_local builds W_L explicitly from the
pixel-driven weights (used by the iterative solvers: a sparse matrix-vector
product is a library primitive).
"""

import numpy as np
import scipy.sparse as sp

_TAPS = (-1, 0, 1, 2)   # bins around floor(u); covers every nonzero for spacing >= 1/2


def _full(geom):
    return (0, 0, geom.n, geom.n)


def hat_weight(geom, k, i, r, c):
    """Single entry w[(k,i),(r,c)] of W (global pixel indices)."""
    t = geom.pixel_x(c) * geom.cos[k] + geom.pixel_y(r) * geom.sin[k]
    s_i = (i - (geom.n_det - 1) / 2.0) * geom.spacing + geom.offset
    return max(0.0, 1.0 - abs(s_i - t) / geom.m[k]) / geom.m[k]


def fp_ray(geom, img, rect=None, bins=None, chunk=1024):
    """Ray-driven Joseph forward projection W_L x of a region image.

    img is the (rows, cols) image of region rect = (row0, col0, rows, cols);
    pixels outside the region are zero (this is W M_L).  bins, if given, is a
    boolean [N_theta, N_d] mask of the rays to compute (others are left 0).
    Returns the full sinogram [N_theta, N_d].
    """
    r0, c0, rr, cc = _full(geom) if rect is None else rect
    img = np.asarray(img, dtype=np.float64)
    assert img.shape == (rr, cc)
    out = np.zeros((geom.n_angles, geom.n_det))
    s_all = geom.s
    half = (geom.n - 1) / 2.0
    ys = geom.pixel_y(np.arange(r0, r0 + rr))      # row centres
    xs = geom.pixel_x(np.arange(c0, c0 + cc))      # column centres
    for k in range(geom.n_angles):
        idx = np.arange(geom.n_det) if bins is None else np.nonzero(bins[k])[0]
        ck, sk = geom.cos[k], geom.sin[k]
        for a in range(0, len(idx), chunk):
            ii = idx[a:a + chunk]
            s = s_all[ii][:, None]
            if geom.ystep[k]:
                # the ray crosses row y at x = (s - y sin)/cos; local column coordinate
                pos = (s - ys[None, :] * sk) / ck + half - c0
                lo = np.floor(pos).astype(np.int64)
                f = pos - lo
                acc = np.zeros(pos.shape)
                rows = np.broadcast_to(np.arange(rr)[None, :], pos.shape)
                for col, wgt in ((lo, 1.0 - f), (lo + 1, f)):
                    ok = (col >= 0) & (col < cc)
                    acc += np.where(ok, img[rows, np.clip(col, 0, cc - 1)] * wgt, 0.0)
            else:
                # the ray crosses column x at y = (s - x cos)/sin
                pos = (s - xs[None, :] * ck) / sk + half - r0
                lo = np.floor(pos).astype(np.int64)
                f = pos - lo
                acc = np.zeros(pos.shape)
                cols = np.broadcast_to(np.arange(cc)[None, :], pos.shape)
                for row, wgt in ((lo, 1.0 - f), (lo + 1, f)):
                    ok = (row >= 0) & (row < rr)
                    acc += np.where(ok, img[np.clip(row, 0, rr - 1), cols] * wgt, 0.0)
            out[k, ii] = acc.sum(axis=1) / geom.m[k]
    return out


def _bp_angles(geom, sino, rect, angles):
    r0, c0, rr, cc = rect
    xs = geom.pixel_x(np.arange(c0, c0 + cc))[None, :]
    ys = geom.pixel_y(np.arange(r0, r0 + rr))[:, None]
    out = np.zeros((rr, cc))
    for k in angles:
        t = xs * geom.cos[k] + ys * geom.sin[k]
        base = np.floor(geom.bin_coord(t)).astype(np.int64)
        for d in _TAPS:
            i = base + d
            ok = (i >= 0) & (i < geom.n_det)
            s_i = (i - (geom.n_det - 1) / 2.0) * geom.spacing + geom.offset
            w = np.maximum(0.0, 1.0 - np.abs(s_i - t) / geom.m[k]) / geom.m[k]
            out += np.where(ok, w * sino[k, np.clip(i, 0, geom.n_det - 1)], 0.0)
    return out


def _bp_worker(args):
    return _bp_angles(*args)


def bp_pixel(geom, sino, rect=None, workers=1):
    """Pixel-driven backprojection W_L^T y = M_L W^T y onto region rect.

    Returns the (rows, cols) region image.  workers > 1 splits the sum over
    angles across processes (the sum is the same up to FP64 rounding order).
    """
    assert geom.spacing >= 0.5, "tap set covers spacing >= 1/2"
    rect = _full(geom) if rect is None else rect
    sino = np.asarray(sino, dtype=np.float64)
    assert sino.shape == (geom.n_angles, geom.n_det)
    if workers <= 1:
        return _bp_angles(geom, sino, rect, range(geom.n_angles))
    import multiprocessing as mp
    parts = np.array_split(np.arange(geom.n_angles), workers)
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_bp_worker, [(geom, sino, rect, list(p)) for p in parts])
    return np.sum(res, axis=0)


def sparse_local(geom, rect=None):
    """W_L as a scipy CSR matrix [N_theta N_d, rows*cols] (pixel-driven weights).

    Column j is pixel (j // cols, j % cols) of the region; rows are k*N_d + i.
    """
    assert geom.spacing >= 0.5
    r0, c0, rr, cc = _full(geom) if rect is None else rect
    xs = geom.pixel_x(np.arange(c0, c0 + cc))[None, :]
    ys = geom.pixel_y(np.arange(r0, r0 + rr))[:, None]
    pix = np.arange(rr * cc, dtype=np.int64).reshape(rr, cc)
    R, C, V = [], [], []
    for k in range(geom.n_angles):
        t = xs * geom.cos[k] + ys * geom.sin[k]
        base = np.floor(geom.bin_coord(t)).astype(np.int64)
        for d in _TAPS:
            i = base + d
            s_i = (i - (geom.n_det - 1) / 2.0) * geom.spacing + geom.offset
            w = np.maximum(0.0, 1.0 - np.abs(s_i - t) / geom.m[k]) / geom.m[k]
            ok = (w > 0) & (i >= 0) & (i < geom.n_det)
            R.append((k * geom.n_det + i[ok]).astype(np.int64))
            C.append(pix[ok])
            V.append(w[ok])
    R, C, V = np.concatenate(R), np.concatenate(C), np.concatenate(V)
    return sp.csr_matrix((V, (R, C)), shape=(geom.n_angles * geom.n_det, rr * cc))


def dense_matrix_hat(geom, rect=None):
    """Brute-force dense W_L from the entry formula, with plain loops (tiny grids)."""
    r0, c0, rr, cc = _full(geom) if rect is None else rect
    W = np.zeros((geom.n_angles * geom.n_det, rr * cc))
    for k in range(geom.n_angles):
        for i in range(geom.n_det):
            for a in range(rr):
                for b in range(cc):
                    W[k * geom.n_det + i, a * cc + b] = hat_weight(geom, k, i, r0 + a, c0 + b)
    return W


def dense_matrix_ray(geom, rect=None):
    """Dense W_L whose columns are ray-driven projections of unit impulses."""
    r0, c0, rr, cc = _full(geom) if rect is None else rect
    W = np.zeros((geom.n_angles * geom.n_det, rr * cc))
    for j in range(rr * cc):
        e = np.zeros(rr * cc)
        e[j] = 1.0
        W[:, j] = fp_ray(geom, e.reshape(rr, cc), (r0, c0, rr, cc)).ravel()
    return W
