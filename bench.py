#!/usr/bin/env python3
"""Benchmark of the local-ROI hot path on one MI355X.

One step = one complete tiled reconstruction of a 4096^2 slice (512 angles, 6144
bins, Poisson noise I0 = 5e3): the Ram-Lak FBP exterior estimate of the whole
sinogram, the exterior residual, the band subtraction of 256 local parts (16 x 16
tiles of 256^2, each extended by a 32 px margin), 200 CP iterations of TV
(lambda = 0.01) + nonnegativity on all 256 parts together (one launch per operator
per iteration, captured in a hipGraph), and the crops stitched into the 4096^2 image
without blending.  The sinogram is resident in HBM before timing starts; the CP step
sizes are per-(geometry, shape) plans computed once by a power iteration and cached.
`value` = tile solves/s.

Secondary legs: the single 128^2 ROI of a 1024^2 slice solved one at a time (with a
quality comparison against the phantom and the global solve), 64 uneven ROIs of a
2048^2 slice batched (vs one at a time), the paper's own local method (Alg. 1, 2, 3)
on those ROIs, and serving of ROI requests over 64 resident 2048^2 slices.

Prints one JSON line.  --gpus N > 1 is refused: the benchmark runs on one GPU.
"""

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Roofline of the projectors.  Nothing here is a dense contraction, and a projector
# moves 0.03-0.2 B of compulsory HBM traffic per pixel-ray update, so the bound is the
# vector ALU: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.32e12 FP32 lane-instructions/s
# for one instruction per SIMD and cycle, and a minimal Joseph sample needs about 2.5 of
# them per update (coordinate step, floor, fraction, lerp and accumulate, shared by the
# two taps of an interpolation): 15.7e12 updates/s, the roof `frac` is taken against.
# gfx950 also pairs independent instructions of different classes from different waves
# (adds with anything, an FMA with a fraction or conversion), which doubles that issue
# rate to the 157.3 TFLOP/s of the published FP32 vector peak (78.6e12 lane-FMAs/s):
# `frac_paired_issue` is taken against that doubled roof, 31.5e12 updates/s.  The
# kernels here issue about 4.5 lane-instructions per update (the position is
# re-anchored, the band or image read is addressed, the weights are clamped); the share
# of the single-issue rate that corresponds to is reported as valu_frac_at_4_5.
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
OPS_PER_UPDATE = 2.5
PEAK_UPDATES = VALU_LANE_OPS / OPS_PER_UPDATE
KERNEL_OPS_PER_UPDATE = 4.5
HBM_PEAK_GBS = 8000.0


def alu_roofline(kernel, updates_per_launch, launch_us, traffic=None):
    """Roofline object of a projector kernel: algorithmic updates (the exact nonzero
    count of W_L over the launch's regions) per average launch duration."""
    rate = updates_per_launch / (launch_us * 1e-6)
    return {"bound": "alu", "kernel": kernel, "achieved": rate / 1e9,
            "peak": PEAK_UPDATES / 1e9, "unit": "Gupdate/s", "frac": rate / PEAK_UPDATES,
            "peak_paired_issue": 2 * PEAK_UPDATES / 1e9,
            "frac_paired_issue": rate / (2 * PEAK_UPDATES),
            "traffic": traffic, "avg_launch_us": launch_us,
            "updates_per_launch": updates_per_launch,
            "valu_frac_at_4_5": rate * KERNEL_OPS_PER_UPDATE / VALU_LANE_OPS}


def measured_peaks(torch, blocks=2048, iters=2048, reps=5):
    """What the chip sustains, measured beside the nominal figures: the rates at which
    it retires vector FP32 lane-instructions (the library's calibration kernels, blocks
    x 256 lanes each running iters x 128 independent-chain steps of one FMA, of an FMA
    and a fraction, or of one add, timed with events on their stream) and the HBM rate
    of a plain 1 GiB device-to-device copy (bytes read + written)."""
    from paper_1604_02292_amd import Context
    ctx = Context(0, workspace_bytes=1 << 20)
    try:
        out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        rates, ms = {}, {}
        for mode, name, per_step in ((0, "fma", 1), (1, "fma_fract", 2), (2, "add", 1)):
            ctx.tomo_valu_probe(blocks, iters, 0.999, 1e-3, out, mode=mode)   # warm-up
            ev0.record()
            for _ in range(reps):
                ctx.tomo_valu_probe(blocks, iters, 0.999, 1e-3, out, mode=mode)
            ev1.record()
            torch.cuda.synchronize()
            t = ev0.elapsed_time(ev1) * 1e-3 / reps
            rates[name] = blocks * 256 * iters * 128 * per_step / t
            ms[name] = 1e3 * t
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        ev0.record()
        for _ in range(reps):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        t_copy = ev0.elapsed_time(ev1) * 1e-3 / reps
        del src, dst
        rate = rates["fma"]
        return {"valu_lane_instr_per_s": rate, "valu_frac_of_nominal": rate / VALU_LANE_OPS,
                "updates_per_s_at_2_5": rate / OPS_PER_UPDATE,
                "valu_fma_fract_lane_instr_per_s": rates["fma_fract"],
                "valu_add_lane_instr_per_s": rates["add"],
                "valu_paired_frac_of_nominal": max(rates.values()) / (2 * VALU_LANE_OPS),
                "hbm_copy_gb_per_s": 2 * (1 << 30) / t_copy / 1e9,
                "hbm_copy_frac_of_nominal": 2 * (1 << 30) / t_copy / 1e9 / HBM_PEAK_GBS,
                "sample": f"{blocks} x 256 lanes x {iters * 128} steps of one FMA / an FMA and a "
                          f"fraction / one add, {reps} launches each ("
                          + ", ".join(f"{k} {v:.2f} ms" for k, v in ms.items())
                          + f"); 1 GiB copy x {reps}"}
    finally:
        ctx.close()


def total_nnz(ctx, g, exts, workers=16):
    """Exact nonzero count of W_L summed over the regions (host count, in threads: the
    library call releases the interpreter)."""
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        return int(sum(ex.map(lambda e: ctx.tomo_roi_nnz(g, e), exts)))


KERNEL_SOURCE = os.path.join(ROOT, "paper_1604_02292_amd", "csrc", "tomo_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def profiled_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summaries (FETCH_SIZE and WRITE_SIZE, each scaled by the
    reading of the same counter for a plain device copy of known size), or None
    when no summary matches the kernel source as it is now."""
    if not os.path.isdir(PROFILES):
        return None
    want = kernel_source_hash()
    for fn in sorted(os.listdir(PROFILES)):
        if not fn.endswith(".md"):
            continue
        with open(os.path.join(PROFILES, fn)) as f:
            for line in f:
                if not line.startswith("traffic-json: "):
                    continue
                rec = json.loads(line[len("traffic-json: "):])
                if (rec.get("workload") == workload and rec.get("kernel") == kernel and
                        rec.get("kernel_source_sha256") == want):
                    return rec["bytes_per_launch"]
    return None


def cpu_baseline(d, cfg, roi, margin):
    """The FP64 oracle on a bounded sample of the same workload: full FBP,
    exterior subtraction, step size and 10 of the 300 CP iterations; the full
    solve time is the sum with the iteration time scaled by 30."""
    import oracle
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    geo = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    sino = d["sino"].astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    xe = oracle.fbp_ramlak(geo, sino, workers=cores)
    t_fbp = time.perf_counter() - t0
    ext = oracle.roi_extend(roi, margin, cfg["n"])
    t0 = time.perf_counter()
    WL = oracle.sparse_local(geo, ext)
    used = np.zeros(geo.n_angles * geo.n_det, bool)
    used[np.unique(WL.tocoo().row)] = True
    b = oracle.exterior_subtract(geo, sino, xe, ext, bins=used.reshape(geo.n_angles, geo.n_det))
    t_ext = time.perf_counter() - t0
    shape = (ext[2], ext[3])
    t0 = time.perf_counter()
    h = 1.0 / cfg["n"]
    s, t = oracle.cp_steps(WL, shape, h=h)
    t_step = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.cp_tv_nonneg(WL, b, shape, cfg["lam"], s, t, 10, h=h)
    t_10 = time.perf_counter() - t0
    est = t_fbp + t_ext + t_step + t_10 * cfg["iters"] / 10.0
    log(f"cpu oracle: fbp {t_fbp:.2f}s ext {t_ext:.2f}s step {t_step:.2f}s 10 its {t_10:.2f}s "
        f"-> {est:.1f}s per solve")
    return {"value": 1.0 / est, "unit": "ROI solves/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 NumPy oracle: full Ram-Lak FBP (cores worker processes), exterior "
                      "subtraction, power-iteration step size and 10 of the 300 CP iterations "
                      "(single thread); the 300-iteration solve time is extrapolated "
                      f"(measured {t_fbp + t_ext + t_step + t_10:.1f}s)"}


def local_cpu_baseline(d, iters):
    """The FP64 oracle's Alg. 2 (oracle/filters.py, as it stands: every iteration
    convolves the whole sinogram with that iteration's filters and applies the sparse
    W_L) on a bounded sample of the 64-ROI batch: four iterations on one ROI of side 32
    and one of side 128 with filters of the workload's shape, the sparse W_L build timed
    apart; per-ROI cost a + b * area (b >= 0) fitted to the two and summed over the 64 ROIs
    times the iteration count.  The one-time filter recursion is not included."""
    import oracle
    import synth
    from oracle.filters import local_method_box
    cfg = d["cfg"]
    geo = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    sino = d["sino"].astype(np.float32).astype(np.float64)
    n_it = 4
    U = np.random.default_rng(0).normal(size=(n_it, cfg["n_angles"], cfg["n_det"])) * 1e-6
    rois = synth.roi_list("c3")
    pts = []
    for side in (32, 128):
        r0, c0, rr, cc, m = next(r for r in rois if r[2] == side)
        ext = oracle.roi_extend((r0, c0, rr, cc), m, cfg["n"])
        t0 = time.perf_counter()
        oracle.sparse_local(geo, ext)
        t_wl = time.perf_counter() - t0
        t0 = time.perf_counter()
        local_method_box(geo, sino, (r0, c0, rr, cc), m, U, 0.0, np.inf)
        t_2 = time.perf_counter() - t0
        pts.append((ext[2] * ext[3], t_wl, (t_2 - t_wl) / n_it))
    (a1, w1, i1), (a2, w2, i2) = pts
    def fit(v1, v2, area):   # nondecreasing in the area
        return v1 + max(v2 - v1, 0.0) * (area - a1) / (a2 - a1)
    total = 0.0
    for (r0, c0, rr, cc, m) in rois:
        e = oracle.roi_extend((r0, c0, rr, cc), m, cfg["n"])
        area = e[2] * e[3]
        total += max(fit(w1, w2, area), 0.0) + iters * max(fit(i1, i2, area), 0.0)
    log(f"cpu oracle (local method): iteration {i1:.2f}s (ext {a1} px) / {i2:.2f}s (ext {a2} px) "
        f"-> {total:.0f}s per batch")
    return {"value": len(rois) / total, "unit": "ROI solves/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 NumPy oracle Alg. 2 (whole-sinogram filter convolution and sparse "
                      "W_L products per iteration, single thread): 4 iterations on one 32^2 "
                      "and one 128^2 ROI plus their W_L builds, cost linear in the extended "
                      f"area fitted to those and summed over the 64 ROIs x {iters} iterations "
                      "(filter recursion excluded)"}


def _oracle_region_costs(geo, sino, ext, lam, h, n_it=3, n_ang_sample=32):
    """Single-thread FP64 oracle costs on one extended region: the sparse W_L build; the
    exterior subtraction over its band (from a zero exterior image: the same work) on
    n_ang_sample of the angles, scaled to all; and one power-iteration step, one CP-TV
    iteration and one SIRT iteration (each the mean of n_it)."""
    import oracle
    n, na = geo.n, geo.n_angles
    t0 = time.perf_counter()
    WL = oracle.sparse_local(geo, ext)
    t_wl = time.perf_counter() - t0
    used = np.zeros(na * geo.n_det, bool)
    used[np.unique(WL.tocoo().row)] = True
    used = used.reshape(na, geo.n_det)
    pick = np.arange(0, na, max(1, na // n_ang_sample))[:n_ang_sample]
    sample = np.zeros_like(used)
    sample[pick] = used[pick]
    t0 = time.perf_counter()
    oracle.exterior_subtract(geo, sino, np.zeros((n, n)), ext, bins=sample)
    t_ext = (time.perf_counter() - t0) * na / len(pick)
    shape = (ext[2], ext[3])
    t0 = time.perf_counter()
    oracle.power_norm_sq(WL, shape, n_it)
    t_pow = (time.perf_counter() - t0) / n_it
    bfull = np.zeros(na * geo.n_det)
    t0 = time.perf_counter()
    oracle.cp_tv_nonneg(WL, bfull, shape, lam, 0.35, 0.35, n_it, h=h)
    t_cp = (time.perf_counter() - t0) / n_it
    t0 = time.perf_counter()
    oracle.sirt_nonneg(WL, bfull, shape, 1e-6, n_it)
    t_sirt = (time.perf_counter() - t0) / n_it
    return {"area": ext[2] * ext[3], "side": max(ext[2], ext[3]), "wl": t_wl, "ext": t_ext,
            "power": t_pow, "cp": t_cp, "sirt": t_sirt}


def _fit(c1, c2):
    """Per-region oracle cost from two samples: W_L build, power, CP and SIRT steps linear
    in the extended area (their sparse products are), the exterior subtraction linear in
    the extended side (the band width); nondecreasing, never below the smaller sample."""
    def f(key, ext):
        x = "side" if key == "ext" else "area"
        v = ext[2] * ext[3] if x == "area" else max(ext[2], ext[3])
        x1, x2, v1, v2 = c1[x], c2[x], c1[key], c2[key]
        return max(v1, v1 + max(v2 - v1, 0.0) * (v - x1) / (x2 - x1))
    return f


def _oracle_fbp_cost(geo, sino, tile=256):
    """Single-thread oracle Ram-Lak FBP of the whole grid: the filter of the whole
    sinogram plus the backprojection of one tile x (n / tile)^2."""
    import oracle
    n = geo.n
    t0 = time.perf_counter()
    q = oracle.fbp.ramp_filter(geo, sino)
    t_ramp = time.perf_counter() - t0
    c = (n - tile) // 2
    t0 = time.perf_counter()
    oracle.bp_pixel(geo, q, (c, c, tile, tile), workers=1)
    return t_ramp + (time.perf_counter() - t0) * (n * n) / (tile * tile)


def batch_cpu_baseline(d):
    """The FP64 oracle, one thread, on a bounded sample of the 64-ROI batch: the FBP
    exterior (filter + one 256^2 tile of the backprojection), and for one ROI of side 32
    and one of side 128 the W_L build, exterior subtraction, and 3 power-iteration and 3
    CP steps; per-ROI costs fitted to those (linear in the extended area, the exterior
    subtraction in the side), summed over the 64 ROIs x 200 iterations plus 100 power
    steps per extended shape class."""
    import oracle
    import synth
    cfg = d["cfg"]
    n = cfg["n"]
    geo = oracle.make_geometry(n, cfg["n_angles"], cfg["n_det"])
    sino = d["sino"].astype(np.float32).astype(np.float64)
    rois = synth.roi_list("c3")
    t_meas = time.perf_counter()
    t_fbp = _oracle_fbp_cost(geo, sino)
    pts = []
    for side in (32, 128):
        r = next(q for q in rois if q[2] == side)
        pts.append(_oracle_region_costs(geo, sino, oracle.roi_extend(r[:4], r[4], n),
                                        cfg["lam"], 1.0 / n))
    f = _fit(*pts)
    total, shapes = t_fbp, set()
    for r in rois:
        e = oracle.roi_extend(r[:4], r[4], n)
        total += f("wl", e) + f("ext", e) + cfg["iters"] * f("cp", e)
        shapes.add((0, 0, min(n, (e[2] + 15) // 16 * 16), min(n, (e[3] + 15) // 16 * 16)))
    for e in shapes:
        total += 100 * f("power", e)
    t_meas = time.perf_counter() - t_meas
    log(f"cpu oracle (batch): {total:.0f}s per batch extrapolated (measured {t_meas:.1f}s)")
    return {"value": len(rois) / total, "unit": "ROI solves/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 NumPy oracle, single thread: Ram-Lak filter and one 256^2 tile of "
                      "the FBP backprojection (x 64 tiles); W_L build, exterior subtraction (32 "
                      "of 256 angles x 8), 3 power and 3 CP-TV steps on one side-32 and one "
                      "side-128 ROI; per-ROI costs linear in the extended area (the exterior "
                      "subtraction in the side), summed over the 64 ROIs x 200 "
                      f"iterations (extrapolation; measured {t_meas:.1f}s)"}


def serve_cpu_baseline(slices, reqs, cfg, n_ang_sample=16):
    """The FP64 oracle, one thread, on a bounded sample of the serving workload: per
    slice the FBP exterior and the residual over the whole detector (the residual on
    n_ang_sample of the 512 angles, x 512 / n_ang_sample); per request the W_L build,
    exterior subtraction and iterations (CP-TV or SIRT), with costs linear in the
    extended area (the exterior subtraction in the side) fitted to a side-32 and a
    side-128 request shape, plus 100 power steps per extended shape class; summed over
    the 64 slices and the request list."""
    import oracle
    n, na = cfg["n"], cfg["n_angles"]
    geo = oracle.make_geometry(n, na, cfg["n_det"])
    sino = slices[0].astype(np.float32).astype(np.float64)
    t_meas = time.perf_counter()
    t_fbp = _oracle_fbp_cost(geo, sino)
    pick = np.arange(0, na, na // n_ang_sample)[:n_ang_sample]
    bins = np.zeros((na, geo.n_det), bool)
    bins[pick] = True
    t0 = time.perf_counter()
    oracle.exterior_subtract(geo, sino, np.zeros((n, n)), (0, 0, 1, 1), bins=bins)
    t_resid = (time.perf_counter() - t0) * na / len(pick)
    pts = []
    for side in (32, 128):
        c = (n - side) // 2
        m = -(-side // 4)
        pts.append(_oracle_region_costs(geo, sino, oracle.roi_extend((c, c, side, side), m, n),
                                        0.02, 1.0 / n))
    f = _fit(*pts)
    total, shapes = len(slices) * (t_fbp + t_resid), set()
    for r in reqs:
        e = oracle.roi_extend(r["rect"], r["margin"], n)
        total += f("wl", e) + f("ext", e) + r["iters"] * f(r["method"], e)
        if r["method"] == "cp":
            shapes.add((0, 0, min(n, (e[2] + 15) // 16 * 16), min(n, (e[3] + 15) // 16 * 16)))
    for e in shapes:
        total += 100 * f("power", e)
    t_meas = time.perf_counter() - t_meas
    log(f"cpu oracle (serving): {total:.0f}s for {len(reqs)} requests extrapolated "
        f"(measured {t_meas:.1f}s)")
    return {"value": len(reqs) / total, "unit": "requests/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 NumPy oracle, single thread: per slice the Ram-Lak FBP (filter + "
                      "one 256^2 backprojection tile x 64) and the residual (16 of 512 angles "
                      "x 32); per request W_L build, exterior subtraction (32 of 512 angles x "
                      "16) and 3 steps of each solver on a side-32 and a side-128 request, "
                      "costs linear in the extended area (the exterior subtraction in the "
                      "side), summed over the 64 slices and the capacity run's "
                      f"requests (extrapolation; measured {t_meas:.1f}s)"}


def batched_leg(torch, d, reps=3, compare=True, iters=None, fixed_step=0.0, cpu=False):
    """64 uneven ROIs (sides 32..256, margin side/4) on a 2048^2 grid, 256 angles,
    3072 bins, 200 CP-TV iterations: one roi_solve_batch call vs the same ROIs
    solved one at a time, both from the same precomputed FBP exterior."""
    import synth
    from paper_1604_02292_amd import Context, make_params
    cfg = d["cfg"]
    ctx = Context(0, workspace_bytes=8 << 30)
    try:
        g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
        sino = torch.from_numpy(d["sino"].astype(np.float32)).cuda()
        xe = torch.empty((cfg["n"], cfg["n"]), dtype=torch.float32, device="cuda")
        ctx.tomo_fbp_ramlak(g, sino, xe)
        rois = synth.roi_list("c3")
        its = iters or cfg["iters"]
        params = [make_params(r[:4], r[4], "cp", cfg["lam"], its, fixed_step, fixed_step)
                  for r in rois]
        outs = [torch.empty((r[2], r[3]), dtype=torch.float32, device="cuda") for r in rois]
        log(f"batched: inputs ready, {len(rois)} ROIs, {its} iterations")
        nnz = total_nnz(ctx, g, [ctx.tomo_roi_ext(g, r[:4], r[4]) for r in rois])
        updates = 2 * its * nnz
        best, t_fp, t_bp = ctx.tomo_autotune(g, sino, params, outs, x_ext=xe)
        log(f"batched: autotune {best} (fp {1e3 * t_fp:.1f} us, bp {1e3 * t_bp:.1f} us per launch)")
        for _ in range(2):   # step sizes, then the graph capture
            ctx.roi_solve_batch(g, sino, params, outs, x_ext=xe)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.roi_solve_batch(g, sino, params, outs, x_ext=xe)
        torch.cuda.synchronize()
        t_batch = (time.perf_counter() - t0) / reps
        kern = {"launch": best, "fp_us": 1e3 * t_fp, "bp_us": 1e3 * t_bp,
                "fp_updates_per_s": nnz / (t_fp * 1e-3), "bp_updates_per_s": nnz / (t_bp * 1e-3)}
        # the batch's dominant iteration kernel against the ALU roof of the projectors
        dom_fp = t_fp >= t_bp
        fp_name = "fp_staged_kernel" if best.get("fp_rays_per_lane") == 4 else "fp_kernel"
        kname = fp_name if dom_fp else "bp_kernel"
        traffic = profiled_traffic("batch64-n2048-a256", kname)
        kern["roofline"] = alu_roofline(kname, nnz, 1e3 * (t_fp if dom_fp else t_bp), traffic)
        if traffic:
            kern["roofline"]["hbm_gb_per_s"] = traffic / ((t_fp if dom_fp else t_bp) * 1e-3) / 1e9
        if not compare:
            return {"roi_solves_per_s": len(rois) / t_batch, "ms_per_batch": 1e3 * t_batch,
                    "updates_per_s": updates / t_batch, **kern}
        one = [torch.empty_like(o) for o in outs]
        for p, o in zip(params, one):   # warm shapes
            ctx.roi_solve(g, sino, p, o, x_ext=xe)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p, o in zip(params, one):
            ctx.roi_solve(g, sino, p, o, x_ext=xe)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        diff = max(float((a - b).abs().max() / (b.abs().max() + 1e-30)) for a, b in zip(outs, one))
        log(f"batched: 64 ROIs {1e3 * t_batch:.1f} ms per batch; one at a time {1e3 * t_seq:.1f} ms; "
            f"{updates / t_batch / 1e9:.0f} Gupd/s")
        if cpu:
            kern["cpu_baseline"] = batch_cpu_baseline(d)
        return {"workload": "batch64-n2048-a256: 64 ROIs, sides {32,64,128,256}, margin side/4, "
                            "256 angles, 3072 bins, CP-TV 200 its",
                "roi_solves_per_s": len(rois) / t_batch, "ms_per_batch": 1e3 * t_batch,
                "one_at_a_time_roi_solves_per_s": len(rois) / t_seq,
                "speedup_vs_one_at_a_time": t_seq / t_batch,
                "updates_per_s": updates / t_batch,
                "max_rel_diff_batch_vs_single": diff, **kern}
    finally:
        ctx.close()


def local_leg(torch, d, reps=3, iters=None, compare=True, cpu=True):
    """The paper's own local method on the batch workload: SIRT-approximating filters
    (Alg. 1, once per geometry), the filtered data C_{u_k} p (once per sinogram), and
    Alg. 2 with a nonnegativity box for the 64 uneven ROIs in one roi_solve_local
    call; beside it the same ROIs by nonnegative SIRT after FBP exterior subtraction."""
    import synth
    from paper_1604_02292_amd import Context, make_params
    cfg = d["cfg"]
    ctx = Context(0, workspace_bytes=8 << 30)
    try:
        na, nd = cfg["n_angles"], cfg["n_det"]
        g = ctx.tomo_set_geometry(cfg["n"], na, nd)
        sino = torch.from_numpy(d["sino"].astype(np.float32)).cuda()
        its = iters or cfg["iters"]
        rois = synth.roi_list("c3")
        F = torch.empty((its, na, nd), dtype=torch.float32, device="cuda")
        D = torch.empty_like(F)
        ctx.tomo_sirt_filters(g, 2, F[:2])            # load the kernels
        ctx.tomo_sirt_filter_sino(g, F[:2], sino, D[:2])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.tomo_sirt_filters(g, its, F)
        torch.cuda.synchronize()
        t_filt = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.tomo_sirt_filter_sino(g, F, sino, D)
        torch.cuda.synchronize()
        t_conv = (time.perf_counter() - t0) / reps
        L = 1 << int(np.ceil(np.log2(2 * nd - 1)))
        # algorithmic traffic of the convolution: read the filters and the data
        # spectra once, write the filtered data
        conv_bytes = its * na * nd * 4 * 2 + na * L * 8 * 2 + na * nd * 4
        log(f"local: filters {its} x {na} x {nd} in {1e3 * t_filt:.1f} ms; filtered data "
            f"{1e3 * t_conv:.2f} ms ({conv_bytes / t_conv / 1e9:.0f} GB/s algorithmic)")
        params = [make_params(r[:4], r[4], "local", iters=its, box=(0.0, float("inf")))
                  for r in rois]
        outs = [torch.empty((r[2], r[3]), dtype=torch.float32, device="cuda") for r in rois]
        nnz = total_nnz(ctx, g, [ctx.tomo_roi_ext(g, r[:4], r[4]) for r in rois])
        for _ in range(2):   # the second call captures the iteration graph
            ctx.roi_solve_local(g, D, params, outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.roi_solve_local(g, D, params, outs)
        torch.cuda.synchronize()
        t_loc = (time.perf_counter() - t0) / reps
        ctx.tomo_kernel_timing(1)
        ctx.tomo_kernel_time(0, reset=True)
        ctx.roi_solve_local(g, D, params, outs)
        torch.cuda.synchronize()
        ctx.tomo_kernel_timing(0)
        n_fp, ms_fp = ctx.tomo_kernel_time(0)
        n_bp, ms_bp = ctx.tomo_kernel_time(1)
        fp_us, bp_us = 1e3 * ms_fp / max(1, n_fp), 1e3 * ms_bp / max(1, n_bp)
        log(f"local: 64 ROIs x {its} its {1e3 * t_loc:.1f} ms per batch; fp {fp_us:.1f} us, "
            f"two-channel bp {bp_us:.1f} us per launch")
        res = {"workload": "batch64-n2048-a256: 64 ROIs, sides {32,64,128,256}, margin side/4, "
                           f"256 angles, 3072 bins; Alg. 2 with box [0, inf), {its} its",
               "roi_solves_per_s": len(rois) / t_loc, "ms_per_batch": 1e3 * t_loc,
               "fp_us": fp_us, "bp_us": bp_us,
               "fp_updates_per_s": nnz / (fp_us * 1e-6), "bp_updates_per_s": nnz / (bp_us * 1e-6),
               "filters_ms": 1e3 * t_filt, "filtered_data_ms": 1e3 * t_conv,
               "filtered_data_gb_per_s": conv_bytes / t_conv / 1e9,
               "filtered_data_bytes": conv_bytes,
               # the iteration's dominant kernel against the ALU roof of the projectors
               # (both channels share one weight per update), and the filtered data
               # against HBM (algorithmic bytes: filters and data spectra read,
               # filtered data written)
               "roofline": alu_roofline("bp_kernel (two-channel)", nnz, bp_us,
                                        profiled_traffic("batch64-n2048-a256-alg2",
                                                         "bp_kernel (two-channel)")),
               "filtered_data_roofline": {"bound": "hbm", "kernel": "filter_conv_kernel",
                                          "achieved": conv_bytes / t_conv / 1e9,
                                          "peak": 8000.0, "unit": "GB/s",
                                          "frac": conv_bytes / t_conv / 8e12}}
        # local FISTA-TV (Alg. 3) on the same ROIs and filtered data: 100 FGP iterations
        # per outer iteration, TV prox weight gamma = alpha lambda / 2 = 0.02
        alpha = 1.0 / (na * nd)
        lam_f = 2 * 0.02 / alpha
        fparams = [make_params(r[:4], r[4], "fista", lam=lam_f, iters=its, inner_iters=100)
                   for r in rois]
        for _ in range(2):
            ctx.roi_solve_local(g, D, fparams, outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.roi_solve_local(g, D, fparams, outs)
        torch.cuda.synchronize()
        t_fista = (time.perf_counter() - t0) / reps
        ctx.tomo_kernel_timing(1)
        ctx.tomo_kernel_time(0, reset=True)
        ctx.roi_solve_local(g, D, fparams, outs)
        torch.cuda.synchronize()
        ctx.tomo_kernel_timing(0)
        n_g, ms_g = ctx.tomo_kernel_time(2)
        fgp_us = 1e3 * ms_g / max(1, n_g)
        log(f"local FISTA-TV: 64 ROIs x {its} its x 100 FGP {1e3 * t_fista:.1f} ms per batch; "
            f"FGP {fgp_us:.1f} us per outer iteration")
        res["fista_tv"] = {"roi_solves_per_s": len(rois) / t_fista, "ms_per_batch": 1e3 * t_fista,
                           "fgp_us_per_outer_iteration": fgp_us, "fgp_iterations": 100,
                           "gamma": 0.02, "lambda": lam_f}
        # the Haar l1 prior (4 levels, threshold gamma = 0.02) with the same local FISTA
        hparams = [make_params(r[:4], r[4], "haar", lam=lam_f, iters=its, inner_iters=4)
                   for r in rois]
        for _ in range(2):
            ctx.roi_solve_local(g, D, hparams, outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.roi_solve_local(g, D, hparams, outs)
        torch.cuda.synchronize()
        t_haar = (time.perf_counter() - t0) / reps
        ctx.tomo_kernel_timing(1)
        ctx.tomo_kernel_time(0, reset=True)
        ctx.roi_solve_local(g, D, hparams, outs)
        torch.cuda.synchronize()
        ctx.tomo_kernel_timing(0)
        n_h, ms_h = ctx.tomo_kernel_time(2)
        haar_us = 1e3 * ms_h / max(1, n_h)
        log(f"local FISTA-Haar: 64 ROIs x {its} its {1e3 * t_haar:.1f} ms per batch; "
            f"Haar prox {haar_us:.1f} us per outer iteration")
        res["fista_haar"] = {"roi_solves_per_s": len(rois) / t_haar, "ms_per_batch": 1e3 * t_haar,
                             "prox_us_per_outer_iteration": haar_us, "levels": 4,
                             "gamma": 0.02, "lambda": lam_f}
        # preprocessing of truncated data (once per sinogram): the central half of the
        # detector measured, constant padding, disc subtraction (Sections 3.3 and 4)
        first, nb = nd // 4, nd // 2
        trunc = sino[:, first:first + nb].contiguous()
        P = torch.empty_like(sino)
        val = torch.zeros(1, dtype=torch.float32, device="cuda")
        ctx.tomo_pad_truncated(g, trunc, first, P)
        ctx.tomo_disc_subtract(g, P, P, val)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.tomo_pad_truncated(g, trunc, first, P)
        torch.cuda.synchronize()
        t_pad = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.tomo_disc_subtract(g, P, P, val)
        torch.cuda.synchronize()
        t_disc = (time.perf_counter() - t0) / reps
        log(f"local: truncated-data preprocessing {na} x {nd}: padding {1e3 * t_pad:.3f} ms, "
            f"disc subtraction {1e3 * t_disc:.3f} ms (with the disc's full-grid projection)")
        res["preprocess"] = {"pad_ms": 1e3 * t_pad, "disc_subtract_ms": 1e3 * t_disc}
        if compare:
            xe = torch.empty((cfg["n"], cfg["n"]), dtype=torch.float32, device="cuda")
            ctx.tomo_fbp_ramlak(g, sino, xe)
            sp = [make_params(r[:4], r[4], "sirt", iters=its) for r in rois]
            so = [torch.empty_like(o) for o in outs]
            for _ in range(2):
                ctx.roi_solve_batch(g, sino, sp, so, x_ext=xe)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.roi_solve_batch(g, sino, sp, so, x_ext=xe)
            torch.cuda.synchronize()
            t_sirt = (time.perf_counter() - t0) / reps
            log(f"local: exterior-subtraction SIRT batch {1e3 * t_sirt:.1f} ms")
            res["exterior_sirt_ms_per_batch"] = 1e3 * t_sirt
        if cpu:
            res["cpu_baseline"] = local_cpu_baseline(d, its)
        return res
    finally:
        ctx.close()


def serving_leg(torch, slices, n_req=1000, n_warm=200, fractions=(0.25, 0.5, 0.75, 0.9),
                cpu=False, n_main=2000):
    """64 resident 2048^2 slices (512 angles x 3072 bins); requests with side
    U{32..512}, margin ceil(side/4), 80% CP-TV / 20% nonnegative SIRT, 100-300
    iterations.  Capacity = completion rate with all requests queued at once;
    latency = submit-to-done at Poisson arrivals of the given fractions of that
    rate (n_main requests at half of it, the point the line quotes, n_req at the
    others); plain = the first 200 of those requests solved one at a time with roi_solve; small
    budget = the capacity run again with a workspace that holds only a few
    slots next to two resident slices, so admission by HBM budget binds."""
    import synth
    from paper_1604_02292_amd import Context, make_params
    cfg = synth.workload("c5")

    def prm(r):
        return make_params(r["rect"], r["margin"], r["method"], r["lam"], r["iters"])

    def run(ctx, sids, reqs, open_loop, stages=None):
        outs = [torch.empty((r["rect"][2], r["rect"][3]), device="cuda") for r in reqs]
        lat, pend = [], {}
        i = 0
        t_start = time.perf_counter()
        while i < len(reqs) or pend:
            now = time.perf_counter() - t_start
            while i < len(reqs) and (not open_loop or reqs[i]["t"] <= now):
                t = ctx.roi_submit(sids[reqs[i]["slice"] % len(sids)], prm(reqs[i]), outs[i])
                pend[t] = i
                i += 1
                if i % 500 == 0:
                    log(f"serving: {i} of {len(reqs)} requests submitted")
            for t in list(pend):
                done, st = ctx.roi_poll_stages(t)
                if done:
                    lat.append(st["latency_ms"])
                    if stages is not None:
                        stages.append(st)
                    del pend[t]
            time.sleep(0.0002)
        return time.perf_counter() - t_start, lat, outs

    def pct(v, q):
        return float(np.percentile(v, q))

    sinos = [torch.from_numpy(s_.astype(np.float32)).cuda() for s_ in slices]
    ctx = Context(0, workspace_bytes=12 << 30)
    try:
        g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
        t0 = time.perf_counter()
        sids = [ctx.tomo_register_sinogram(g, s_) for s_ in sinos]
        t_reg = time.perf_counter() - t0
        run(ctx, sids, synth.serving_requests(n_warm, 1.0, seed_offset=1), False)
        reqs = synth.serving_requests(n_req, 1.0, seed_offset=2)
        t_cap, lat_cap, outs = run(ctx, sids, reqs, False)
        cap = n_req / t_cap
        sweep = []
        for k, fr in enumerate(fractions):
            n_fr = max(n_req, n_main) if fr == 0.5 else n_req
            reqs_open = synth.serving_requests(n_fr, fr * cap, seed_offset=3 + k)
            stages = []
            t_open, lat_open, _ = run(ctx, sids, reqs_open, True, stages)
            # where a request's time goes: queued (submit -> admitted), preparation
            # (admitted -> first iteration), iterations (-> done)
            split = {f"{key}_p50_ms": pct([q[key] for q in stages], 50)
                     for key in ("queued_ms", "prepare_ms", "run_ms")}
            split.update({f"{key}_p99_ms": pct([q[key] for q in stages], 99)
                          for key in ("queued_ms", "prepare_ms", "run_ms")})
            sweep.append({"fraction_of_capacity": fr, "offered_qps": fr * cap, "requests": n_fr,
                          "achieved_qps": n_fr / t_open, "p50_ms": pct(lat_open, 50),
                          "p99_ms": pct(lat_open, 99), "stages": split})
            log(f"serving: {fr:.2f} x capacity ({fr * cap:.1f} req/s): p50 {pct(lat_open, 50):.1f} "
                f"ms p99 {pct(lat_open, 99):.1f} ms")
        # plain one-at-a-time solves of the first n_plain capacity requests (same
        # exterior estimates)
        n_plain = min(len(reqs), 200)
        xes = {}
        for r in reqs[:n_plain]:
            if r["slice"] not in xes:
                xe = torch.empty((cfg["n"], cfg["n"]), device="cuda")
                ctx.tomo_fbp_ramlak(g, sinos[r["slice"]], xe)
                xes[r["slice"]] = xe
        torch.cuda.synchronize()
        plain_outs = [torch.empty_like(o) for o in outs[:n_plain]]
        t0 = time.perf_counter()
        for r, o in zip(reqs[:n_plain], plain_outs):
            ctx.roi_solve(g, sinos[r["slice"]], prm(r), o, x_ext=xes[r["slice"]])
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        diff = max(float((a - b).abs().max() / (b.abs().max() + 1e-30))
                   for a, b in zip(outs[:n_plain], plain_outs))
        del xes
    finally:
        ctx.close()
    # small HBM budget: two resident slices plus room for a few slots
    small = (2 * 60 << 20) + (96 << 20)
    ctx = Context(0, workspace_bytes=small)
    try:
        g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
        sids = [ctx.tomo_register_sinogram(g, s_) for s_ in sinos[:2]]
        reqs_small = synth.serving_requests(n_req // 2, 1.0, seed_offset=9)
        t_small, lat_small, _ = run(ctx, sids, reqs_small, False)
        peak = ctx.tomo_workspace_usage()
    finally:
        ctx.close()
    mid = next((p for p in sweep if p["fraction_of_capacity"] == 0.5), sweep[0])
    base = serve_cpu_baseline(slices, reqs, cfg) if cpu else None
    log(f"serving: register {t_reg:.2f}s; capacity {cap:.1f} req/s; plain {n_plain / t_plain:.1f} "
        f"req/s; {small >> 20} MiB budget: {len(reqs_small) / t_small:.1f} req/s")
    return {"workload": "serve-64x2048-a512: 64 resident slices, side U{32..512}, 80% CP-TV / "
                        "20% SIRT, 100-300 its",
            "capacity_solves_per_s": cap, "offered_qps": mid["offered_qps"],
            "p50_ms": mid["p50_ms"], "p99_ms": mid["p99_ms"], "latency_sweep": sweep,
            "saturated_p50_ms": pct(lat_cap, 50), "saturated_p99_ms": pct(lat_cap, 99),
            "one_at_a_time_solves_per_s": n_plain / t_plain, "one_at_a_time_requests": n_plain,
            "requests": n_req, "requests_at_half_capacity": mid["requests"],
            "warmup_requests": n_warm, "max_rel_diff_served_vs_plain": diff,
            "small_budget": {"workspace_mib": small >> 20, "resident_slices": 2,
                             "capacity_solves_per_s": len(reqs_small) / t_small,
                             "p50_ms": pct(lat_small, 50), "p99_ms": pct(lat_small, 99),
                             "workspace_usage": peak},
            **({"cpu_baseline": base} if base else {})}


def tiles_cpu_baseline(d, n_ang_sample=16, n_cp=3, n_pow=3):
    """The FP64 oracle, one thread, on a bounded sample of the tiled 4096^2 workload:
    the Ram-Lak filter of the whole sinogram; the pixel-driven backprojection of one
    256^2 tile of the grid (x 256 for the whole FBP); for one interior tile (extended
    320^2) the sparse W_L build, the exterior subtraction on n_ang_sample of the 512
    angles (x 512 / n_ang_sample), n_cp CP iterations (x 200 / n_cp) and n_pow
    power-iteration steps (x 100 / n_pow, once for each of the 4 extended shapes of the
    tiling).  The batch time is the sum with the tile costs times 256, a labelled
    extrapolation from the measured pieces."""
    import oracle
    import synth
    cfg = d["cfg"]
    n, na = cfg["n"], cfg["n_angles"]
    geo = oracle.make_geometry(n, na, cfg["n_det"])
    sino = d["sino"].astype(np.float32).astype(np.float64)
    rois = synth.roi_list("c4")
    tm = {}
    t0 = time.perf_counter()
    q = oracle.fbp.ramp_filter(geo, sino)
    tm["ramp_filter"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.bp_pixel(geo, q, (1920, 1920, 256, 256), workers=1)
    tm["bp_256"] = time.perf_counter() - t0
    r0, c0, rr, cc, m = rois[16 * 5 + 6]
    ext = oracle.roi_extend((r0, c0, rr, cc), m, n)
    t0 = time.perf_counter()
    WL = oracle.sparse_local(geo, ext)
    tm["wl_build"] = time.perf_counter() - t0
    used = np.zeros(na * geo.n_det, bool)
    used[np.unique(WL.tocoo().row)] = True
    used = used.reshape(na, geo.n_det)
    sample = np.zeros_like(used)
    pick = np.arange(0, na, na // n_ang_sample)[:n_ang_sample]
    sample[pick] = used[pick]
    xe = np.zeros((n, n))
    t0 = time.perf_counter()
    b = oracle.exterior_subtract(geo, sino, xe, ext, bins=sample)
    tm["exterior_sample"] = time.perf_counter() - t0
    shape, h = (ext[2], ext[3]), 1.0 / n
    t0 = time.perf_counter()
    oracle.power_norm_sq(WL, shape, n_pow)
    tm["power_sample"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.cp_tv_nonneg(WL, b, shape, cfg["lam"], 0.35, 0.35, n_cp, h=h)
    tm["cp_sample"] = time.perf_counter() - t0
    measured = sum(tm.values())
    t_fbp = tm["ramp_filter"] + tm["bp_256"] * (n * n) / (256 * 256)
    t_tile = (tm["wl_build"] + tm["exterior_sample"] * na / len(pick) +
              tm["cp_sample"] * cfg["iters"] / n_cp)
    t_power = 4 * tm["power_sample"] * 100 / n_pow
    t_batch = t_fbp + len(rois) * t_tile + t_power
    log(f"cpu oracle (tiles): {', '.join(f'{k} {v:.2f}s' for k, v in tm.items())} -> tile "
        f"{t_tile:.0f}s, batch {t_batch:.0f}s (one thread, extrapolated)")
    return {"value": len(rois) / t_batch, "unit": "tile solves/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 NumPy oracle on one thread: Ram-Lak filter of the whole sinogram, "
                      "backprojection of one 256^2 tile of the grid (x256 for the FBP), and for "
                      f"one interior tile the sparse W_L build, the exterior subtraction on "
                      f"{len(pick)} of {na} angles, {n_cp} CP iterations and {n_pow} power "
                      f"steps; measured {measured:.1f}s, extrapolated to the 256-tile batch "
                      f"({t_batch:.0f}s per batch, {t_tile:.0f}s per tile)",
            "pieces_s": tm, "tile_s": t_tile, "batch_s": t_batch}


def tiles_leg(torch, d, steps, warmup, quality=True):
    """Headline: the 4096^2 slice as 16 x 16 tiles of 256^2 + 32 px margin, 512 angles,
    6144 bins, 200 CP-TV iterations, stitched; each step one roi_solve_stitched call."""
    import synth
    from paper_1604_02292_amd import Context, make_params
    cfg = d["cfg"]
    n = cfg["n"]
    rois = synth.roi_list("c4")
    ctx = Context(0, workspace_bytes=16 << 30)
    try:
        g = ctx.tomo_set_geometry(n, cfg["n_angles"], cfg["n_det"])
        sino = torch.from_numpy(d["sino"].astype(np.float32)).cuda()
        params = [make_params(r[:4], r[4], "cp", cfg["lam"], cfg["iters"]) for r in rois]
        img = torch.zeros((n, n), dtype=torch.float32, device="cuda")
        t0 = time.perf_counter()
        nnz = total_nnz(ctx, g, [ctx.tomo_roi_ext(g, r[:4], r[4]) for r in rois])
        log(f"tiles: {len(rois)} tiles, nnz(W_L) summed {nnz} (counted in "
            f"{time.perf_counter() - t0:.1f}s)")
        launch = ctx.tomo_resolve_launch(g, params)
        for _ in range(max(2, warmup)):   # step sizes, then the graph capture
            ctx.roi_solve_stitched(g, sino, params, img)
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
            ctx.roi_solve_stitched(g, sino, params, img)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
        total = time.perf_counter() - t_start
        # kernel durations: the next solve first replays 50 back-to-back launches of each
        # iteration kernel on its own data between two HIP events on the solve's stream
        ctx.tomo_kernel_timing(2)
        ctx.tomo_kernel_time(0, reset=True)
        ctx.roi_solve_stitched(g, sino, params, img)
        torch.cuda.synchronize()
        ctx.tomo_kernel_timing(0)
        n_fp, ms_fp = ctx.tomo_kernel_time(0)
        n_bp, ms_bp = ctx.tomo_kernel_time(1)
        fp_us, bp_us = 1e3 * ms_fp / max(1, n_fp), 1e3 * ms_bp / max(1, n_bp)
        # the exterior estimate alone (Ram-Lak FBP of the whole sinogram)
        fbp = torch.empty((n, n), dtype=torch.float32, device="cuda")
        ctx.tomo_fbp_ramlak(g, sino, fbp)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(3):
            ctx.tomo_fbp_ramlak(g, sino, fbp)
        ev1.record()
        torch.cuda.synchronize()
        fbp_ms = ev0.elapsed_time(ev1) / 3
        dom_fp = fp_us >= bp_us
        fp_name = "fp_staged_kernel" if launch.get("fp_rays_per_lane") == 4 else "fp_kernel"
        kname = fp_name if dom_fp else "bp_kernel"
        traffic = profiled_traffic("tiles256-n4096-a512", kname)
        roof = alu_roofline(kname, nnz, fp_us if dom_fp else bp_us, traffic)
        if traffic:
            roof["hbm_gb_per_s"] = traffic / ((fp_us if dom_fp else bp_us) * 1e-6) / 1e9
        ms = 1e3 * total / steps
        log(f"tiles: {steps} steps {ms:.1f} ms/step ({len(rois) * steps / total:.1f} tile solves/s); "
            f"fp {fp_us:.1f} us, bp {bp_us:.1f} us per launch ({nnz / (fp_us * 1e-6) / 1e12:.2f} / "
            f"{nnz / (bp_us * 1e-6) / 1e12:.2f} T updates/s); FBP {fbp_ms:.2f} ms")
        res = {"value": len(rois) * steps / total, "ms_per_step": ms,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "launch": launch, "fp_us": fp_us, "bp_us": bp_us,
               "fp_updates_per_s": nnz / (fp_us * 1e-6), "bp_updates_per_s": nnz / (bp_us * 1e-6),
               "updates_per_s": 2 * cfg["iters"] * nnz / (total / steps), "fbp_ms": fbp_ms,
               "roofline": roof}
        if quality:
            # the global CP-TV solve of the whole slice (same lambda and iterations), the
            # FBP, and the stitched tiles, against each other and the phantom
            glob = torch.empty((n, n), dtype=torch.float32, device="cuda")
            gprm = make_params((0, 0, n, n), 0, "cp", cfg["lam"], cfg["iters"])
            ctx.roi_solve(g, sino, gprm, glob)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.roi_solve(g, sino, gprm, glob)
            torch.cuda.synchronize()
            t_glob = time.perf_counter() - t0
            fit = []
            for x in (img, glob):
                proj = torch.empty_like(sino)
                ctx.tomo_fp(g, (0, 0, n, n), x, proj)
                torch.cuda.synchronize()
                fit.append(float(torch.linalg.norm(proj - sino) / torch.linalg.norm(sino)))
            truth = d["image"]
            st, gl, fb = (t.double().cpu().numpy() for t in (img, glob, fbp))
            relq = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
            res["quality"] = {"stitched_vs_global_rel": relq(st, gl),
                              "stitched_vs_phantom_rel": relq(st, truth),
                              "global_vs_phantom_rel": relq(gl, truth),
                              "fbp_vs_phantom_rel": relq(fb, truth),
                              "data_residual_stitched": fit[0], "data_residual_global": fit[1],
                              "global_solve_ms": 1e3 * t_glob}
            log("tiles quality: " + ", ".join(f"{k} {v:.4g}" for k, v in res["quality"].items()))
        return res
    finally:
        ctx.close()


def single_roi_leg(torch, d, steps, warmup, autotune=False, quality=True, cpu=True):
    """One 128^2 ROI + 32 px margin of a 1024^2 slice (128 angles, 1536 bins), 300 CP-TV
    iterations, solved one at a time: FBP exterior, band subtraction, iterations, crop."""
    from paper_1604_02292_amd import Context, make_params
    cfg = d["cfg"]
    import synth
    r0, c0, rr, cc, margin = synth.roi_list("c2")[0]
    roi = (r0, c0, rr, cc)
    ctx = Context(0, workspace_bytes=8 << 30)
    try:
        g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
        prm = make_params(roi, margin, "cp", cfg["lam"], cfg["iters"])
        sino = torch.from_numpy(d["sino"].astype(np.float32)).cuda()
        out = torch.empty((rr, cc), dtype=torch.float32, device="cuda")
        ext = ctx.tomo_roi_ext(g, roi, margin)
        nnz = ctx.tomo_roi_nnz(g, ext)
        if autotune:
            best, t_fp, t_bp = ctx.tomo_autotune(g, sino, [prm], [torch.empty_like(out)])
            log(f"single ROI autotune: {best}")
        else:
            # the size heuristics' shapes (for this workload also the autotuner's), so that
            # a profiled run of this command runs the same kernels
            best = ctx.tomo_resolve_launch(g, [prm])
        for _ in range(max(2, warmup)):   # the second solve captures the iteration graph
            ctx.roi_solve(g, sino, prm, out)
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
            ctx.roi_solve(g, sino, prm, out)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
        total = time.perf_counter() - t_start
        ctx.tomo_kernel_timing(2)
        ctx.tomo_kernel_time(0, reset=True)
        for _ in range(3):
            ctx.roi_solve(g, sino, prm, out)
        torch.cuda.synchronize()
        ctx.tomo_kernel_timing(0)
        n_fp, ms_fp = ctx.tomo_kernel_time(0)
        n_bp, ms_bp = ctx.tomo_kernel_time(1)
        fp_us = 1e3 * ms_fp / max(1, n_fp)
        bp_us = 1e3 * ms_bp / max(1, n_bp)
        log(f"single ROI: {steps} steps {1e3 * total / steps:.3f} ms/step; fp {fp_us:.2f} us, "
            f"bp {bp_us:.2f} us per launch; nnz/launch {nnz}")
        dom_bp = ms_bp >= ms_fp
        kname = "bp_kernel" if dom_bp else "fp_kernel"
        res = {"workload": "single-roi-1024: 1024^2 grid, 128 angles, 1536 bins, 128^2 ROI + 32 px "
                           "margin, CP-TV lambda 0.02 + nonneg, 300 its, one ROI at a time",
               "roi_solves_per_s": steps / total, "ms_per_solve": 1e3 * total / steps,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "launch": best, "extended_roi": list(ext),
               "fp_updates_per_s": nnz / (fp_us * 1e-6), "bp_updates_per_s": nnz / (bp_us * 1e-6),
               "roofline": alu_roofline(kname, nnz, bp_us if dom_bp else fp_us,
                                        profiled_traffic("single-roi-1024", kname))}
        if quality:
            # the ROI of the global TV solve on the whole grid (same lambda and iterations),
            # the FBP and the paper's own local method (Alg. 1 filters, Alg. 2 with box
            # [0, inf), as many iterations), against the phantom inside the ROI
            n = cfg["n"]
            gout = torch.empty((n, n), dtype=torch.float32, device="cuda")
            gprm = make_params((0, 0, n, n), 0, "cp", cfg["lam"], cfg["iters"])
            ctx.roi_solve(g, sino, gprm, gout)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.roi_solve(g, sino, gprm, gout)
            torch.cuda.synchronize()
            t_glob = time.perf_counter() - t0
            fbp = torch.empty((n, n), dtype=torch.float32, device="cuda")
            ctx.tomo_fbp_ramlak(g, sino, fbp)
            its = cfg["iters"]
            F = torch.empty((its, cfg["n_angles"], cfg["n_det"]), dtype=torch.float32,
                            device="cuda")
            D = torch.empty_like(F)
            ctx.tomo_sirt_filters(g, its, F)
            ctx.tomo_sirt_filter_sino(g, F, sino, D)
            alg2 = torch.empty((rr, cc), dtype=torch.float32, device="cuda")
            ctx.roi_solve_local(g, D, [make_params(roi, margin, "local", iters=its,
                                                   box=(0.0, float("inf")))], [alg2])
            torch.cuda.synchronize()
            del F, D
            loc = out.double().cpu().numpy()
            glob = gout.double().cpu().numpy()[r0:r0 + rr, c0:c0 + cc]
            fbp_r = fbp.double().cpu().numpy()[r0:r0 + rr, c0:c0 + cc]
            truth = d["image"][r0:r0 + rr, c0:c0 + cc]
            alg2 = alg2.double().cpu().numpy()
            relq = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
            res["quality"] = {"local_vs_global_rel": relq(loc, glob),
                              "fbp_vs_global_rel": relq(fbp_r, glob),
                              "local_vs_phantom_rel": relq(loc, truth),
                              "global_vs_phantom_rel": relq(glob, truth),
                              "fbp_vs_phantom_rel": relq(fbp_r, truth),
                              "alg2_vs_phantom_rel": relq(alg2, truth),
                              "global_solve_ms": 1e3 * t_glob}
            log("single ROI quality: " + ", ".join(f"{k} {v:.4g}" for k, v in res["quality"].items()))
    finally:
        ctx.close()
    if cpu:
        res["cpu_baseline"] = cpu_baseline(d, cfg, roi, margin)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-single", action="store_true")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--skip-local", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests per serving load point (at least 2000 at half of capacity)")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the untimed quality comparisons (global solves, FBP, Alg. 2 "
                         "against the phantom)")
    ap.add_argument("--only", choices=["tiles", "single", "batch", "serve", "local", "peaks"],
                    default=None,
                    help="run only one leg (for profiling) and print its JSON")
    ap.add_argument("--iters", type=int, default=None,
                    help="override the iteration count of the batch and local legs (profiling)")
    ap.add_argument("--fixed-step", type=float, default=0.0,
                    help="explicit CP step for the batch leg, skipping the power iteration")
    ap.add_argument("--gen-workers", type=int, default=0,
                    help="processes for input generation (0 = one per core, at most 16)")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the launch shapes of the single-ROI leg before timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy 5 times (the "
                         "reference kernel for scaling HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        # two plain copies of 256 MiB each: the runtime's blit copy and an
        # elementwise kernel (y = 1 * x), 3 times each
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "ROI solves are independent and would be sharded across GPUs without "
              "per-iteration communication, but no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    if args.only == "peaks":
        import torch
        print(json.dumps(measured_peaks(torch)), flush=True)
        return
    import synth
    gw = args.gen_workers or None
    want = (lambda leg: args.only == leg) if args.only else (lambda leg: True)
    quality = not args.no_quality
    # all inputs are generated before the GPU is initialised (the generator forks)
    t0 = time.perf_counter()
    d4 = synth.make_inputs("c4", with_image=quality and args.only is None,
                           workers=gw) if want("tiles") else None
    d2 = (synth.make_inputs("c2", with_image=quality, workers=1)
          if want("single") and not args.skip_single else None)
    d3 = (synth.make_inputs("c3", with_image=False, workers=gw)
          if (want("batch") and not args.skip_batch) or (want("local") and not args.skip_local)
          else None)
    slices = (synth.make_slices("c5", workers=gw)
              if want("serve") and not args.skip_serve else None)
    log(f"inputs generated ({time.perf_counter() - t0:.1f}s)")
    import torch

    if args.only == "batch":
        print(json.dumps(batched_leg(torch, d3, reps=args.steps, compare=False, iters=args.iters,
                                     fixed_step=args.fixed_step)), flush=True)
        return
    if args.only == "serve":
        print(json.dumps(serving_leg(torch, slices, args.serve_requests, args.serve_warmup)),
              flush=True)
        return
    if args.only == "local":
        print(json.dumps(local_leg(torch, d3, reps=args.steps, iters=args.iters, compare=False,
                                   cpu=False)), flush=True)
        return
    if args.only == "single":
        print(json.dumps(single_roi_leg(torch, d2, args.steps, args.warmup, args.autotune,
                                        quality=False, cpu=False)), flush=True)
        return

    t = tiles_leg(torch, d4, args.steps, args.warmup, quality=quality and args.only is None)
    cfg4 = d4["cfg"]
    res = {
        "metric": "tile solves/s (4096^2 slice as 256 local parts, 200 CP-TV iterations each, "
                  "FBP exterior, stitched)",
        "value": t.pop("value"), "unit": "tile solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded random-ellipse phantom + texture, exact line integrals, "
                "Poisson noise)",
        "config": {"workload": "tiles256-n4096-a512: 4096^2 grid, 512 angles, 6144 bins, "
                               "16 x 16 tiles of 256^2 + 32 px margin, CP-TV lambda "
                               f"{cfg4['lam']} + nonneg, {cfg4['iters']} its, stitched",
                   "tiles": 256, "launch": t.pop("launch")},
        "p50_ms": t.pop("p50_ms"), "p99_ms": t.pop("p99_ms"),
        "roofline": t.pop("roofline"),
    }
    res.update(t)
    try:
        peaks = measured_peaks(torch)
        res["measured_peaks"] = peaks
        res["roofline"]["frac_of_measured_alu"] = (res["roofline"]["achieved"] * 1e9 /
                                                   peaks["updates_per_s_at_2_5"])
    except Exception as e:   # the headline line must still print
        res["measured_peaks"] = {"error": repr(e)}
    if args.only == "tiles":
        print(json.dumps(res), flush=True)
        return
    if not args.skip_single:
        try:
            res["single_roi"] = single_roi_leg(torch, d2, max(5, args.steps), args.warmup,
                                               args.autotune, quality=quality,
                                               cpu=not args.no_cpu_baseline)
        except Exception as e:   # the headline line must still print
            res["single_roi"] = {"error": repr(e)}
    if not args.skip_batch:
        try:
            res["batched"] = batched_leg(torch, d3, cpu=not args.no_cpu_baseline)
        except Exception as e:
            res["batched"] = {"error": repr(e)}
    if not args.skip_local:
        try:
            res["local_method"] = local_leg(torch, d3, cpu=not args.no_cpu_baseline)
        except Exception as e:
            res["local_method"] = {"error": repr(e)}
    if not args.skip_serve:
        try:
            res["serving"] = serving_leg(torch, slices, args.serve_requests, args.serve_warmup,
                                         cpu=not args.no_cpu_baseline)
        except Exception as e:
            res["serving"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = tiles_cpu_baseline(d4)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
