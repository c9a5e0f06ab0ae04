"""The five synthetic workloads and their seeded inputs.

Every random draw comes from numpy.random.SeedSequence([1604, 2292, id]),
spawned into independent streams for the phantom, the noise, the ROI list and
the request arrivals, so that any process on any machine regenerates the same
arrays.  The workloads stand in for the paper's experiments (motor phantom,
1024 detectors, 512 angles, Poisson noise, 256^2 local parts, 128^2 tiles),
whose phantom and data are not available.
"""

import math

import numpy as np

from .phantom import (random_ellipses, texture_ellipses, concat_ellipses, raster,
                      analytic_sinogram, add_gaussian_noise, add_poisson_noise)

WORKLOADS = {
    # plain local method: one centred 32^2 ROI + 16 px margin, CP-TV 100 its
    "c1": dict(id=1, name="local-128-a32", n=128, n_ellipses=10, n_angles=32, n_det=192,
               noise=("gauss", 0.01), rois=[(48, 48, 32, 32)], margin=16, lam=0.05,
               iters=100),
    # single ROI solve: centred 128^2 ROI + 32 px margin on a 1024^2 grid, 300 its
    "c2": dict(id=2, name="roi128-n1024-a128", n=1024, n_ellipses=50, n_angles=128,
               n_det=1536, noise=("poisson", 1e4), rois=[(448, 448, 128, 128)], margin=32,
               lam=0.02, iters=300),
    # 64 uneven ROIs, sides in {32,64,128,256}, margin side/4, 200 its
    "c3": dict(id=3, name="batch64-n2048-a256", n=2048, n_ellipses=200, n_angles=256,
               n_det=3072, noise=("gauss", 0.02), n_rois=64, sides=(32, 64, 128, 256),
               margin_frac=0.25, lam=0.02, iters=200),
    # 16 x 16 tiles of 256^2 with a 32 px margin over 4096^2, 200 its
    "c4": dict(id=4, name="tiles256-n4096-a512", n=4096, n_ellipses=500, texture=0.01,
               n_texture=20000, n_angles=512, n_det=6144, noise=("poisson", 5e3), tile=256,
               margin=32, lam=0.01, iters=200),
    # serving: 64 resident 2048^2 slices, 512 x 3072 sinograms
    "c5": dict(id=5, name="serve-64x2048-a512", n=2048, n_slices=64, n_ellipses=30,
               n_angles=512, n_det=3072, noise=("poisson", 1e4), side=(32, 512),
               cp_frac=0.8, lam=0.02, iters=(100, 300)),
}


def workload(name):
    return dict(WORKLOADS[name])


def _streams(cfg_id):
    ss = np.random.SeedSequence([1604, 2292, cfg_id])
    return ss.spawn(4)   # phantom, noise, rois, arrivals


def _workers():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def make_inputs(name, subrays=4, with_image=True, slice_index=None, supersample=1,
                workers=None):
    """Phantom ellipses, ground-truth raster and noisy FP32-ready sinogram (float64).

    For the serving workload pass slice_index (0..63) to get one slice.  The
    result does not depend on `workers` (processes used for the line integrals).
    """
    workers = _workers() if workers is None else workers
    cfg = workload(name)
    ph_ss, no_ss, _, _ = _streams(cfg["id"])
    if slice_index is not None:
        ph_ss = ph_ss.spawn(cfg["n_slices"])[slice_index]
        no_ss = no_ss.spawn(cfg["n_slices"])[slice_index]
    rng = np.random.default_rng(ph_ss)
    n = cfg["n"]
    ell = random_ellipses(rng, n, cfg["n_ellipses"])
    if cfg.get("texture"):
        ell = concat_ellipses(ell, texture_ellipses(rng, n, cfg["n_texture"], cfg["texture"]))
    clean = analytic_sinogram(ell, cfg["n_angles"], cfg["n_det"], subrays=subrays,
                              workers=workers)
    nrng = np.random.default_rng(no_ss)
    kind, level = cfg["noise"]
    if kind == "gauss":
        sino = add_gaussian_noise(nrng, clean, level)
    else:
        sino = add_poisson_noise(nrng, clean, level)
    out = dict(cfg=cfg, ellipses=ell, sino_clean=clean, sino=sino)
    if with_image:
        out["image"] = raster(ell, n, supersample)
    return out


def _slice_job(args):
    name, k, subrays = args
    return make_inputs(name, subrays=subrays, with_image=False, slice_index=k, workers=1)["sino"]


def make_slices(name="c5", indices=None, subrays=4, workers=None):
    """Noisy sinograms of the serving workload's slices (float64 [N_theta, N_d] each),
    generated in parallel; identical to make_inputs(..., slice_index=k)["sino"]."""
    cfg = workload(name)
    indices = list(range(cfg["n_slices"])) if indices is None else list(indices)
    workers = _workers() if workers is None else workers
    jobs = [(name, k, subrays) for k in indices]
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
            return pool.map(_slice_job, jobs)
    return [_slice_job(j) for j in jobs]


def roi_list(name):
    """List of (row0, col0, rows, cols, margin) for the workload."""
    cfg = workload(name)
    n = cfg["n"]
    if "rois" in cfg:
        return [(r0, c0, rr, cc, cfg["margin"]) for (r0, c0, rr, cc) in cfg["rois"]]
    if name == "c3":
        _, _, roi_ss, _ = _streams(cfg["id"])
        rng = np.random.default_rng(roi_ss)
        out = []
        for _ in range(cfg["n_rois"]):
            side = int(rng.choice(cfg["sides"]))
            r0 = int(rng.integers(0, n - side + 1))
            c0 = int(rng.integers(0, n - side + 1))
            out.append((r0, c0, side, side, int(round(side * cfg["margin_frac"]))))
        return out
    if name == "c4":
        t = cfg["tile"]
        return [(i * t, j * t, t, t, cfg["margin"]) for i in range(n // t) for j in range(n // t)]
    raise KeyError(name)


def serving_requests(count, qps, name="c5", seed_offset=0):
    """Poisson-arrival request list for the serving workload.

    Each request: dict(t, slice, rect=(r0, c0, side, side), margin, method, lam, iters).
    Side ~ U{32..512}, random slice and centre (ROI inside the image),
    80% CP-TV (lambda 0.02), 20% nonnegative SIRT, iterations ~ U{100..300},
    margin ceil(side/4).
    """
    cfg = workload(name)
    _, _, _, arr_ss = _streams(cfg["id"])
    rng = np.random.default_rng(np.random.SeedSequence(arr_ss.entropy,
                                                       spawn_key=arr_ss.spawn_key + (seed_offset,)))
    n = cfg["n"]
    t = 0.0
    reqs = []
    for _ in range(count):
        t += rng.exponential(1.0 / qps) if qps > 0 else 0.0
        side = int(rng.integers(cfg["side"][0], cfg["side"][1] + 1))
        r0 = int(rng.integers(0, n - side + 1))
        c0 = int(rng.integers(0, n - side + 1))
        cp = bool(rng.random() < cfg["cp_frac"])
        reqs.append(dict(t=t, slice=int(rng.integers(0, cfg["n_slices"])),
                         rect=(r0, c0, side, side), margin=int(math.ceil(side / 4)),
                         method="cp" if cp else "sirt", lam=cfg["lam"] if cp else 0.0,
                         iters=int(rng.integers(cfg["iters"][0], cfg["iters"][1] + 1))))
    return reqs
