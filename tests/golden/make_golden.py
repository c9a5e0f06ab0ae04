"""Write expected values for the full-size parity tests.

Every stored value is computed by the FP64 oracle (`oracle/`) from the seeded
generator (`synth/`); nothing here touches the HIP library.

    python tests/golden/make_golden.py [c2] [c3] [c4] [c5] [c3local]
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

WORKERS = min(8, os.cpu_count() or 1)


def golden_workload(name, roi_indices=None, lam_scale=1.0, iters=None):
    t0 = time.time()
    d = synth.make_inputs(name, with_image=False)
    cfg = d["cfg"]
    g = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    xe = oracle.fbp_ramlak(g, d["sino"], workers=WORKERS)
    rois = synth.roi_list(name)
    if roi_indices is None:
        roi_indices = list(range(len(rois)))
    out = {}
    for i in roi_indices:
        r0, c0, rr, cc, m = rois[i]
        res = oracle.local_solve(g, d["sino"], (r0, c0, rr, cc), m, lam=cfg["lam"] * lam_scale,
                                 iters=iters or cfg["iters"], x_ext=xe, full=True)
        out[f"x_{i}"] = res["x"].astype(np.float32)
        out[f"sigma_{i}"] = np.float64(res["sigma"])
        out[f"rect_{i}"] = np.array([r0, c0, rr, cc, m])
        print(f"{name} roi {i} ext {res['ext']} sigma {res['sigma']:.6g} "
              f"({time.time() - t0:.1f}s)", flush=True)
    out["x_ext_samples"] = xe[:: max(1, cfg["n"] // 64), :: max(1, cfg["n"] // 64)].astype(np.float32)
    np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), **out)


def c5_sample(n=8, cp_count=6, max_side=256, n_slices=4):
    """Requests of the serving workload's capacity stream for the served-parity test: the
    first ones in stream order that fill two per side class ([32, 64), [64, 128),
    [128, 192), [192, max_side]) with cp_count CP-TV and n - cp_count SIRT requests, on at
    most n_slices slices (each slice costs the oracle one FBP)."""
    reqs = synth.serving_requests(4000, 1.0, seed_offset=2)
    edges = [32, 64, 128, 192, max_side + 1]
    need = {c: n // 4 for c in range(4)}
    cp_left, sirt_left = cp_count, n - cp_count
    slices, pick = [], []
    for i, r in enumerate(reqs):
        side = r["rect"][2]
        if side > max_side:
            continue
        c = next(k for k in range(4) if edges[k] <= side < edges[k + 1])
        if need[c] == 0:
            continue
        if r["method"] == "cp" and cp_left == 0 or r["method"] == "sirt" and sirt_left == 0:
            continue
        if r["slice"] not in slices and len(slices) == n_slices:
            continue
        if r["slice"] not in slices:
            slices.append(r["slice"])
        need[c] -= 1
        if r["method"] == "cp":
            cp_left -= 1
        else:
            sirt_left -= 1
        pick.append(i)
        if len(pick) == n:
            break
    return reqs, pick


def golden_serving():
    t0 = time.time()
    cfg = synth.workload("c5")
    g = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    reqs, pick = c5_sample()
    slices = sorted({reqs[i]["slice"] for i in pick})
    sinos = dict(zip(slices, synth.make_slices("c5", indices=slices)))
    xes = {k: oracle.fbp_ramlak(g, v.astype(np.float32).astype(np.float64), workers=WORKERS)
           for k, v in sinos.items()}
    print(f"c5 slices {slices}: FBPs ({time.time() - t0:.1f}s)", flush=True)
    out = {"pick": np.array(pick)}
    for i in pick:
        r = reqs[i]
        p = sinos[r["slice"]].astype(np.float32).astype(np.float64)
        res = oracle.local_solve(g, p, r["rect"], r["margin"], method=r["method"], lam=r["lam"],
                                 iters=r["iters"], x_ext=xes[r["slice"]], full=True)
        out[f"x_{i}"] = res["x"].astype(np.float32)
        out[f"sigma_{i}"] = np.float64(res["sigma"] if r["method"] == "cp" else 0.0)
        out[f"req_{i}"] = np.array([r["slice"], *r["rect"], r["margin"], r["iters"],
                                    1 if r["method"] == "cp" else 0])
        print(f"c5 request {i} slice {r['slice']} rect {r['rect']} {r['method']} "
              f"{r['iters']} its ({time.time() - t0:.1f}s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "c5_oracle.npz"), **out)


LOCAL_K = 20
LOCAL_ROIS = (1, 0)     # batch ROIs of side 64 and 128


def golden_local_depth():
    """The paper's local methods at full batch size after LOCAL_K iterations on two sampled
    ROIs: the oracle's Alg. 1 filters u_1..u_K of the 2048^2 geometry, then Alg. 2 with the
    box [0, inf), local FISTA-TV (100 FGP steps, prox weight 0.02) and local FISTA with the
    4-level Haar prior (threshold 0.02) on each ROI."""
    from oracle.filters import sirt_filters, local_method_box
    from oracle.fista import local_fista_tv
    from oracle.haar import local_fista_haar
    t0 = time.time()
    d = synth.make_inputs("c3", with_image=False)
    cfg = d["cfg"]
    na, nd = cfg["n_angles"], cfg["n_det"]
    g = oracle.make_geometry(cfg["n"], na, nd)
    p = d["sino"].astype(np.float32).astype(np.float64)
    U = sirt_filters(g, LOCAL_K, workers=WORKERS)
    print(f"c3local: {LOCAL_K} filters ({time.time() - t0:.1f}s)", flush=True)
    lam = 2 * 0.02 * na * nd
    rois = synth.roi_list("c3")
    out = {"rois": np.array(LOCAL_ROIS), "iters": np.int64(LOCAL_K)}
    for i in LOCAL_ROIS:
        r0, c0, rr, cc, m = rois[i]
        rect = (r0, c0, rr, cc)
        out[f"alg2_{i}"] = local_method_box(g, p, rect, m, U, 0.0, np.inf).astype(np.float32)
        out[f"fista_{i}"] = local_fista_tv(g, p, rect, m, U, lam, 100).astype(np.float32)
        out[f"haar_{i}"] = local_fista_haar(g, p, rect, m, U, lam, 4).astype(np.float32)
        out[f"rect_{i}"] = np.array([r0, c0, rr, cc, m])
        print(f"c3local roi {i} {rois[i]} ({time.time() - t0:.1f}s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "c3_local_oracle.npz"), **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2"]
    if "c2" in which:
        golden_workload("c2")
    if "c3" in which:
        rois = synth.roi_list("c3")
        # two ROIs per side class
        pick = []
        for side in (32, 64, 128, 256):
            pick += [i for i, r in enumerate(rois) if r[2] == side][:2]
        golden_workload("c3", pick)
    if "c4" in which:
        # corner, edge and two interior tiles of the 16 x 16 grid
        golden_workload("c4", [0, 7, 16 * 5 + 6, 16 * 10 + 9])
    if "c5" in which:
        golden_serving()
    if "c3local" in which:
        golden_local_depth()
