"""Random-ellipse phantoms and their exact line integrals.

The phantom is additive (as in the Shepp-Logan construction): every ellipse
adds its value to the pixels it covers, so the image is piecewise constant.
Sinograms are the exact line integrals of that continuous object, averaged
over sub-rays inside each detector bin; this mirrors the paper's practice of
simulating projections at a finer resolution and resampling (Section 4), and
keeps the data from being produced by the discrete projector under test.
"""

from dataclasses import dataclass

import numpy as np


def angles_uniform(n_angles):
    """theta_k = k*pi/N_theta, k = 0..N_theta-1 (uniform in [0, pi))."""
    return np.arange(n_angles, dtype=np.float64) * (np.pi / n_angles)


def bin_centres(n_det, spacing=1.0, offset=0.0):
    """Detector bin centres s_i = (i - (N_d-1)/2)*spacing + offset."""
    return (np.arange(n_det, dtype=np.float64) - (n_det - 1) / 2.0) * spacing + offset


@dataclass
class Ellipses:
    """Ellipse list: centre (cx, cy), semi-axes (a along phi, b across), value v."""
    cx: np.ndarray
    cy: np.ndarray
    a: np.ndarray
    b: np.ndarray
    phi: np.ndarray
    v: np.ndarray

    def __len__(self):
        return len(self.v)


def concat_ellipses(*parts):
    return Ellipses(*[np.concatenate([getattr(p, f) for p in parts])
                      for f in ("cx", "cy", "a", "b", "phi", "v")])


def _centres_in_disc(rng, radius):
    """One uniform point per entry of `radius` inside the disc of that radius."""
    cx = np.empty(len(radius))
    cy = np.empty(len(radius))
    for k, r in enumerate(radius):
        while True:
            x, y = rng.uniform(-r, r, 2)
            if x * x + y * y <= r * r:
                cx[k], cy[k] = x, y
                break
    return cx, cy


def random_ellipses(rng, n, count, axis_lo=None, axis_hi=None, vmin=0.0, vmax=1.0,
                    support=0.48):
    """`count` ellipses for an n x n grid.

    Semi-axes ~ U[n/32, n/4], orientation ~ U[0, pi), value ~ U[vmin, vmax];
    each ellipse lies inside the disc of radius support*n (centre drawn
    uniformly in the disc of radius support*n - max(a, b)), so the object is
    fully inside the reconstruction grid.
    """
    lo = n / 32.0 if axis_lo is None else axis_lo
    hi = n / 4.0 if axis_hi is None else axis_hi
    a = rng.uniform(lo, hi, count)
    b = rng.uniform(lo, hi, count)
    phi = rng.uniform(0.0, np.pi, count)
    v = rng.uniform(vmin, vmax, count)
    cx, cy = _centres_in_disc(rng, support * n - np.maximum(a, b))
    return Ellipses(cx, cy, a, b, phi, v)


def texture_ellipses(rng, n, count, std, axis_lo=1.0, axis_hi=3.0, support=0.46):
    """Fine additive texture: many small ellipses with values ~ N(0, std)."""
    a = rng.uniform(axis_lo, axis_hi, count)
    b = rng.uniform(axis_lo, axis_hi, count)
    phi = rng.uniform(0.0, np.pi, count)
    v = rng.normal(0.0, std, count)
    cx, cy = _centres_in_disc(rng, support * n - np.maximum(a, b))
    return Ellipses(cx, cy, a, b, phi, v)


def raster(ell, n, supersample=1):
    """Sample the additive ellipse phantom on an n x n grid (float64).

    With supersample = s > 1 each pixel is the mean of s x s point samples.
    """
    img = np.zeros((n, n), dtype=np.float64)
    s = int(supersample)
    offs = (np.arange(s) + 0.5) / s - 0.5
    half = (n - 1) / 2.0
    for k in range(len(ell)):
        cx, cy, a, b, phi, v = (ell.cx[k], ell.cy[k], ell.a[k], ell.b[k], ell.phi[k], ell.v[k])
        rad = max(a, b) + 1.0
        c0 = max(0, int(np.floor(cx - rad + half)))
        c1 = min(n, int(np.ceil(cx + rad + half)) + 1)
        r0 = max(0, int(np.floor(cy - rad + half)))
        r1 = min(n, int(np.ceil(cy + rad + half)) + 1)
        if c0 >= c1 or r0 >= r1:
            continue
        xs = np.arange(c0, c1) - half
        ys = np.arange(r0, r1) - half
        cphi, sphi = np.cos(phi), np.sin(phi)
        acc = np.zeros((r1 - r0, c1 - c0))
        for oy in offs:
            for ox in offs:
                dx = xs[None, :] + ox - cx
                dy = ys[:, None] + oy - cy
                u = dx * cphi + dy * sphi
                w = -dx * sphi + dy * cphi
                acc += ((u / a) ** 2 + (w / b) ** 2 <= 1.0)
        img[r0:r1, c0:c1] += v * acc / (s * s)
    return img


_CHUNK = 16   # ellipses per partial sum (fixed, so results do not depend on `workers`)


def _sino_chunk(args):
    ell, idx, th, n_det, spacing, offset, subrays = args
    n_angles = len(th)
    ct, st = np.cos(th), np.sin(th)
    q = (np.arange(subrays) + 0.5) / subrays - 0.5
    centre = (n_det - 1) / 2.0
    kk = np.arange(n_angles)
    cols, wts = [], []
    for e in idx:
        cx, cy, a, b, phi, v = (ell.cx[e], ell.cy[e], ell.a[e], ell.b[e], ell.phi[e], ell.v[e])
        proj = cx * ct + cy * st                      # centre's detector coordinate
        al = th - phi
        r2 = (a * np.cos(al)) ** 2 + (b * np.sin(al)) ** 2
        rmax = max(a, b)
        width = int(np.ceil(2 * rmax / spacing)) + 4
        i_start = np.floor((proj - rmax - offset) / spacing + centre).astype(np.int64) - 1
        ii = i_start[:, None] + np.arange(width)[None, :]          # [angles, width]
        s_bin = (ii - centre) * spacing + offset
        val = np.zeros(ii.shape)
        for qq in q:
            sp = s_bin + qq * spacing - proj[:, None]
            d = r2[:, None] - sp * sp
            val += np.where(d > 0, np.sqrt(np.maximum(d, 0.0)), 0.0)
        val *= (2.0 * a * b * v / subrays) / r2[:, None]
        ok = (ii >= 0) & (ii < n_det) & (val != 0)
        cols.append((kk[:, None] * n_det + ii)[ok])
        wts.append(val[ok])
    # one accumulation over the chunk: every bin appears at most once per ellipse and
    # bincount adds in input order, so each bin's sum runs over the ellipses in order.
    # Only the nonzero bins of the chunk's partial sum are returned (adding the zeros
    # would change nothing), which keeps the transfer from worker processes small.
    if not cols:
        return np.zeros(0, dtype=np.int64), np.zeros(0)
    part = np.bincount(np.concatenate(cols), weights=np.concatenate(wts),
                       minlength=n_angles * n_det)
    nz = np.flatnonzero(part)
    return nz, part[nz]


def analytic_sinogram(ell, n_angles, n_det, spacing=1.0, offset=0.0, subrays=4,
                      angles=None, workers=1):
    """Exact line integrals of the additive ellipse phantom, shape [N_theta, N_d].

    Each bin is the mean over `subrays` parallel rays at offsets
    ((q + 1/2)/subrays - 1/2) * spacing from the bin centre (for 4 sub-rays:
    +-1/8 and +-3/8 of a bin).  The line integral of an ellipse of value v
    along {x cos t + y sin t = s} is v * 2ab sqrt(r^2 - s'^2) / r^2 with
    s' = s - (cx cos t + cy sin t) and r^2 = a^2 cos^2(t-phi) + b^2 sin^2(t-phi).
    Ellipses are summed in fixed chunks, in order, whatever `workers` is.
    """
    th = angles_uniform(n_angles) if angles is None else np.asarray(angles, np.float64)
    chunks = [range(i, min(i + _CHUNK, len(ell))) for i in range(0, len(ell), _CHUNK)]
    jobs = [(ell, c, th, n_det, spacing, offset, subrays) for c in chunks]
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
            parts = pool.map(_sino_chunk, jobs)
    else:
        parts = [_sino_chunk(j) for j in jobs]
    flat = np.zeros(len(th) * n_det)
    for nz, val in parts:
        flat[nz] += val
    return flat.reshape(len(th), n_det)


def disc_sinogram(radius, value, n_angles, n_det, spacing=1.0, offset=0.0, cx=0.0, cy=0.0,
                  subrays=1):
    """Exact sinogram of a uniform disc: value * 2 sqrt(r^2 - s'^2)."""
    ell = Ellipses(np.array([cx]), np.array([cy]), np.array([radius]), np.array([radius]),
                   np.array([0.0]), np.array([value]))
    return analytic_sinogram(ell, n_angles, n_det, spacing, offset, subrays)


def add_gaussian_noise(rng, p, frac):
    """p + N(0, (frac * max p)^2), element-wise."""
    return p + rng.normal(0.0, frac * float(np.max(p)), p.shape)


def add_poisson_noise(rng, p, i0):
    """Photon-count noise: the largest count is I0 (Section 4).

    Counts c = I0 exp(-p / p_max); c' ~ Poisson(c);
    p' = -p_max ln(max(c', 1) / I0).  (The attenuation scale p_max and the
    clamp at one count are this generator's choices; the paper does not fix them.)
    """
    pmax = float(np.max(p))
    if pmax <= 0:
        return p.copy()
    counts = i0 * np.exp(-p / pmax)
    noisy = rng.poisson(counts).astype(np.float64)
    return -pmax * np.log(np.maximum(noisy, 1.0) / i0)
