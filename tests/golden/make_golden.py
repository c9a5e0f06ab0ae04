"""Write expected values for the full-size parity tests.

Every stored value is computed by the FP64 oracle (`oracle/`) from the seeded
generator (`synth/`); nothing here touches the HIP library.

    python tests/golden/make_golden.py [c2] [c3] [c4]
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
