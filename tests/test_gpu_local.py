"""GPU parity of the paper's own local method against the FP64 oracle
(oracle/filters.py): the SIRT-approximating filters (Alg. 1), the filtered data
C_{u_k} p (detector convolutions by FFT), and Alg. 2 with the box prior, each
through the C ABI.  Also the general box of the SIRT solve and the error paths.

Bars: the filters and the reconstructions are iterated FP32 results (1e-4 and the
1e-3 reconstruction bar); one convolution call is held to 1e-5 per plane.
"""

import os
import subprocess
import sys

import numpy as np
import pytest

import synth
import oracle
from oracle.filters import sirt_filters, filter_apply, local_method_box
from oracle.fista import local_fista_tv
from oracle.haar import local_fista_haar

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def ctx():
    from paper_1604_02292_amd import Context
    c = Context(0, workspace_bytes=4 << 30)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c1():
    return synth.make_inputs("c1", with_image=False)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("n,na,nd,K", [(128, 32, 192, 40), (65, 24, 97, 25), (40, 9, 61, 3)])
def test_sirt_filters_match_oracle(ctx, n, na, nd, K):
    print(f"[filters] n={n} na={na} nd={nd} K={K}", flush=True)
    geo = oracle.make_geometry(n, na, nd)
    U = sirt_filters(geo, K, workers=4)
    g = ctx.tomo_set_geometry(n, na, nd)
    F = torch.empty((K, na, nd), dtype=torch.float32, device="cuda")
    ctx.tomo_sirt_filters(g, K, F)
    torch.cuda.synchronize()
    got = F.double().cpu().numpy()
    errs = [rel(got[k], U[k]) for k in range(K)]
    print(f"    max plane rel {max(errs):.2e} (first {errs[0]:.2e}, last {errs[-1]:.2e})")
    assert max(errs) <= 1e-4


@pytest.mark.parametrize("n,na,nd,count,offset", [
    # L >= 512: radix-16 stages plus one radix-2 / 4 / 8 stage (none when log2 L is a
    # multiple of 4); below, radix-4 stages plus one radix-2 stage
    (128, 32, 192, 7, 0.0),      # L = 512 (radix 2 + 16 + 16), odd filter count
    (64, 5, 300, 3, 0.0),        # L = 1024 (radix 4 + 16 + 16)
    (64, 5, 700, 3, 25.0),       # L = 2048 (radix 8 + 16 + 16), detector offset
    (64, 4, 1536, 2, 0.0),       # L = 4096 (radix 16 x 3)
    (40, 4, 1100, 1, 900.0),     # L = 4096, impulse projects off the detector
    (65, 24, 97, 4, 0.0),        # L = 256
    (65, 24, 97, 3, 60.0),       # impulse projects off the detector: lag beyond the rows
    (64, 6, 3072, 2, 0.0),       # L = 8192
    (96, 3, 6144, 3, 0.0),       # L = 16384
    (8, 5, 1, 1, 0.0),           # one bin: L = 4
])
def test_filter_sino_matches_oracle(ctx, n, na, nd, count, offset):
    print(f"[filter_sino] n={n} na={na} nd={nd} count={count} offset={offset}", flush=True)
    geo = oracle.make_geometry(n, na, nd, offset=offset)
    rng = np.random.default_rng(7)
    u = rng.standard_normal((count, na, nd)) * np.exp(-np.abs(np.arange(nd) - nd / 2) / 20.0)
    p = rng.uniform(0.0, 5.0, (na, nd))
    g = ctx.tomo_set_geometry(n, na, nd, det_offset=offset)
    out = torch.empty((count, na, nd), dtype=torch.float32, device="cuda")
    u32 = u.astype(np.float32).astype(np.float64)
    p32 = p.astype(np.float32).astype(np.float64)
    ctx.tomo_sirt_filter_sino(g, _gpu(u32), _gpu(p32), out)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    for k in range(count):
        ref = filter_apply(geo, u32[k], p32)
        e = rel(got[k], ref)
        print(f"    plane {k} rel {e:.2e}")
        assert e <= 1e-5


ROIS_C1 = [  # (r0, c0, rows, cols, margin, iters, box)
    (48, 48, 32, 32, 16, 50, (0.0, float("inf"))),
    (0, 90, 20, 38, 8, 37, (0.1, 0.8)),       # at the grid edge (extension clipped)
    (70, 5, 9, 1, 4, 50, (-float("inf"), float("inf"))),   # one column, no prior
    (100, 100, 28, 3, 0, 12, (0.0, 0.5)),
]


def _local_oracle(geo, p, rois, U):
    out = []
    for (r0, c0, rr, cc, m, it, box) in rois:
        out.append(local_method_box(geo, p, (r0, c0, rr, cc), m, U[:it], box[0], box[1]))
    return out


def _local_gpu(ctx, cfg, p32, rois, K):
    from paper_1604_02292_amd import make_params
    g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    F = torch.empty((K, cfg["n_angles"], cfg["n_det"]), dtype=torch.float32, device="cuda")
    ctx.tomo_sirt_filters(g, K, F)
    D = torch.empty_like(F)
    ctx.tomo_sirt_filter_sino(g, F, _gpu(p32), D)
    params, outs = [], []
    for (r0, c0, rr, cc, m, it, box) in rois:
        params.append(make_params((r0, c0, rr, cc), m, "local", iters=it, box=box))
        outs.append(torch.empty((rr, cc), dtype=torch.float32, device="cuda"))
    ctx.roi_solve_local(g, D, params, outs)
    torch.cuda.synchronize()
    return [o.double().cpu().numpy() for o in outs], g, D


def test_local_method_matches_oracle(ctx, c1):
    cfg = c1["cfg"]
    p32 = c1["sino"].astype(np.float32).astype(np.float64)
    geo = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    K = max(r[5] for r in ROIS_C1)
    U = sirt_filters(geo, K, workers=4)
    ref = _local_oracle(geo, p32, ROIS_C1, U)
    print("[local] batch of", len(ROIS_C1), "ROIs", flush=True)
    got, _, _ = _local_gpu(ctx, cfg, p32, ROIS_C1, K)
    for roi, a, b in zip(ROIS_C1, got, ref):
        e = rel(a, b) if np.linalg.norm(b) > 0 else float(np.abs(a).max())
        print(f"    roi {roi[:4]} iters {roi[5]} box {roi[6]} rel {e:.2e}")
        assert e <= 1e-3
        lo, hi = np.float32(roi[6][0]), np.float32(roi[6][1])   # the bounds as the GPU holds them
        assert a.min() >= lo and a.max() <= hi
    # one ROI alone gives the same result as inside the batch (same launch shape)
    from paper_1604_02292_amd import make_params
    print("[local] single-ROI call", flush=True)
    got1, _, _ = _local_gpu(ctx, cfg, p32, ROIS_C1[:1], K)
    assert rel(got1[0], ref[0]) <= 1e-3


# groups = 8 has no two-channel kernel of its own: its tiles are those of 4 groups, which
# the two-channel band then uses
@pytest.mark.parametrize("variant,groups,ppt", [(1, 1, 1), (1, 2, 1), (1, 4, 1), (1, 8, 1),
                                                (1, 1, 2), (1, 2, 2), (1, 4, 2), (1, 8, 2),
                                                (2, 1, 1), (2, 1, 2)])
def test_local_method_every_backprojector_shape(ctx, c1, variant, groups, ppt):
    cfg = c1["cfg"]
    p32 = c1["sino"].astype(np.float32).astype(np.float64)
    geo = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    rois = ROIS_C1[:2]
    K = 50
    U = sirt_filters(geo, K, workers=4)
    ref = _local_oracle(geo, p32, rois, U)
    print(f"[local shape] variant={variant} groups={groups} ppt={ppt}", flush=True)
    ctx.tomo_set_launch(bp_variant=variant, bp_groups=groups, bp_pixels_per_thread=ppt)
    try:
        got, _, _ = _local_gpu(ctx, cfg, p32, rois, K)
    finally:
        ctx.tomo_set_launch()
    for a, b in zip(got, ref):
        assert rel(a, b) <= 1e-3


# (r0, c0, rows, cols, margin, iters, lam, n_fgp, box, flags); flags 1 = 1/2 data term,
# 2 = anisotropic TV.  Extended parts of 1x1 to 2x2 FGP tiles; FGP counts that end
# inside a launch (9, 20), on a launch boundary (16) and the default (0 = 100).
FISTA_C1 = [
    (48, 48, 32, 32, 16, 30, 500.0, 0, None, 0),
    (0, 90, 20, 38, 8, 25, 2000.0, 20, (0.0, 1.0), 2),
    (70, 5, 9, 1, 4, 30, 300.0, 16, None, 0),
    (100, 100, 28, 3, 6, 12, 100.0, 9, (0.0, float("inf")), 1),
]


@pytest.mark.parametrize("variant", [1, 2])
def test_local_fista_tv_matches_oracle(ctx, c1, variant):
    from paper_1604_02292_amd import make_params
    cfg = c1["cfg"]
    p32 = c1["sino"].astype(np.float32).astype(np.float64)
    geo = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    K = max(r[5] for r in FISTA_C1)
    U = sirt_filters(geo, K, workers=4)
    ref = []
    for (r0, c0, rr, cc, m, it, lam, nf, box, fl) in FISTA_C1:
        lo, hi = box if box else (-np.inf, np.inf)
        ref.append(local_fista_tv(geo, p32, (r0, c0, rr, cc), m, U[:it], lam, nf or 100, lo, hi,
                                  aniso=bool(fl & 2), half=bool(fl & 1)))
    # one local-SIRT request in the same batch
    sirt_roi = ROIS_C1[0][:5] + (20,) + ROIS_C1[0][6:]
    ref_sirt = _local_oracle(geo, p32, [sirt_roi], U)[0]
    g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    F = torch.empty((K, cfg["n_angles"], cfg["n_det"]), dtype=torch.float32, device="cuda")
    ctx.tomo_sirt_filters(g, K, F)
    D = torch.empty_like(F)
    ctx.tomo_sirt_filter_sino(g, F, _gpu(p32), D)
    params, outs = [], []
    for (r0, c0, rr, cc, m, it, lam, nf, box, fl) in FISTA_C1:
        params.append(make_params((r0, c0, rr, cc), m, "fista", lam=lam, iters=it, flags=fl,
                                  box=box, inner_iters=nf))
        outs.append(torch.empty((rr, cc), dtype=torch.float32, device="cuda"))
    r0, c0, rr, cc, m, it, box = sirt_roi
    params.append(make_params((r0, c0, rr, cc), m, "local", iters=it, box=box))
    outs.append(torch.empty((rr, cc), dtype=torch.float32, device="cuda"))
    print(f"[fista] batch of {len(params)} requests, backprojector variant {variant}", flush=True)
    ctx.tomo_set_launch(bp_variant=variant)
    try:
        ctx.roi_solve_local(g, D, params, outs)
        torch.cuda.synchronize()
    finally:
        ctx.tomo_set_launch()
    for roi, o, b in zip(FISTA_C1 + [None], outs, ref + [ref_sirt]):
        a = o.double().cpu().numpy()
        assert np.linalg.norm(b) > 0
        e = rel(a, b)
        print(f"    {roi if roi else 'local sirt'} rel {e:.2e}", flush=True)
        assert e <= 1e-3
    # the TV prior acts: the first request differs from unregularised Alg. 2
    plain = _local_oracle(geo, p32, [(48, 48, 32, 32, 16, 30, (-np.inf, np.inf))], U)[0]
    assert rel(ref[0], plain) > 1e-2


# (r0, c0, rows, cols, margin, iters, lam, levels, flags): extended parts of one full
# 64^2 tile (6 levels), ragged 36 x 54, 17 x 9 and 40 x 15 parts, the default level
# count (0 = 4); regions inside the object, where the thresholds leave a nonzero result
HAAR_C1 = [
    (48, 48, 32, 32, 16, 30, 300.0, 6, 0),
    (40, 70, 20, 38, 8, 25, 150.0, 3, 1),
    (70, 45, 9, 1, 4, 30, 60.0, 0, 0),
    (60, 60, 28, 3, 6, 12, 100.0, 1, 0),
]


def test_local_fista_haar_matches_oracle(ctx, c1):
    from paper_1604_02292_amd import make_params
    cfg = c1["cfg"]
    p32 = c1["sino"].astype(np.float32).astype(np.float64)
    geo = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    K = max(r[5] for r in HAAR_C1)
    U = sirt_filters(geo, K, workers=4)
    ref = [local_fista_haar(geo, p32, (r0, c0, rr, cc), m, U[:it], lam, lv or 4, half=bool(fl & 1))
           for (r0, c0, rr, cc, m, it, lam, lv, fl) in HAAR_C1]
    # a TV request in the same batch
    tv = FISTA_C1[0]
    ref_tv = local_fista_tv(geo, p32, tv[:4], tv[4], U[:tv[5]], tv[6], 100)
    g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    F = torch.empty((K, cfg["n_angles"], cfg["n_det"]), dtype=torch.float32, device="cuda")
    ctx.tomo_sirt_filters(g, K, F)
    D = torch.empty_like(F)
    ctx.tomo_sirt_filter_sino(g, F, _gpu(p32), D)
    params, outs = [], []
    for (r0, c0, rr, cc, m, it, lam, lv, fl) in HAAR_C1:
        params.append(make_params((r0, c0, rr, cc), m, "haar", lam=lam, iters=it, flags=fl,
                                  inner_iters=lv))
        outs.append(torch.empty((rr, cc), dtype=torch.float32, device="cuda"))
    params.append(make_params(tv[:4], tv[4], "fista", lam=tv[6], iters=tv[5]))
    outs.append(torch.empty((tv[2], tv[3]), dtype=torch.float32, device="cuda"))
    print(f"[haar] batch of {len(params)} requests", flush=True)
    ctx.roi_solve_local(g, D, params, outs)
    torch.cuda.synchronize()
    for roi, o, b in zip(HAAR_C1 + [None], outs, ref + [ref_tv]):
        a = o.double().cpu().numpy()
        assert np.linalg.norm(b) > 0
        e = rel(a, b)
        print(f"    {roi if roi else 'fista-tv'} rel {e:.2e}", flush=True)
        assert e <= 1e-3
    # the threshold acts: the first request differs from unregularised Alg. 2
    plain = _local_oracle(geo, p32, [(48, 48, 32, 32, 16, 30, (-np.inf, np.inf))], U)[0]
    assert rel(ref[0], plain) > 1e-2


def test_local_ista_form_matches_oracle(ctx, c1):
    """ROI_FLAG_NO_MOMENTUM: the ISTA form (eq. sirtista) of both l1 priors."""
    from paper_1604_02292_amd import make_params
    cfg = c1["cfg"]
    p32 = c1["sino"].astype(np.float32).astype(np.float64)
    geo = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    K = 20
    U = sirt_filters(geo, K, workers=4)
    rect, m = (48, 48, 32, 32), 16
    ref_h = local_fista_haar(geo, p32, rect, m, U, 300.0, 3, momentum=False)
    ref_t = local_fista_tv(geo, p32, rect, m, U, 500.0, 40, momentum=False)
    g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    F = torch.empty((K, cfg["n_angles"], cfg["n_det"]), dtype=torch.float32, device="cuda")
    ctx.tomo_sirt_filters(g, K, F)
    D = torch.empty_like(F)
    ctx.tomo_sirt_filter_sino(g, F, _gpu(p32), D)
    outs = [torch.empty((32, 32), dtype=torch.float32, device="cuda") for _ in range(2)]
    ctx.roi_solve_local(g, D, [make_params(rect, m, "haar", lam=300.0, iters=K, inner_iters=3,
                                           flags=8),
                               make_params(rect, m, "fista", lam=500.0, iters=K, inner_iters=40,
                                           flags=8)], outs)
    torch.cuda.synchronize()
    for o, b, name in zip(outs, (ref_h, ref_t), ("ista-haar", "ista-tv")):
        e = rel(o.double().cpu().numpy(), b)
        print(f"[{name}] rel {e:.2e}", flush=True)
        assert e <= 1e-3
    # the flag changes the result (momentum acts from the second iteration on)
    assert rel(local_fista_haar(geo, p32, rect, m, U, 300.0, 3), ref_h) > 1e-3


def test_local_haar_errors(ctx):
    from paper_1604_02292_amd import make_params, TomoError
    g = ctx.tomo_set_geometry(64, 8, 96)
    D = torch.zeros((5, 8, 96), dtype=torch.float32, device="cuda")
    out = torch.empty((8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(TomoError, match="EINVAL"):   # too many levels
        ctx.roi_solve_local(g, D, [make_params((0, 0, 8, 8), 2, "haar", iters=5, inner_iters=7)],
                            [out])
    with pytest.raises(TomoError, match="EINVAL"):   # no box with the Haar prior
        ctx.roi_solve_local(g, D, [make_params((0, 0, 8, 8), 2, "haar", iters=5,
                                               box=(0.0, 1.0))], [out])
    with pytest.raises(TomoError, match="EINVAL"):   # no momentum to drop in Alg. 2
        ctx.roi_solve_local(g, D, [make_params((0, 0, 8, 8), 2, "local", iters=5, flags=8)],
                            [out])


def test_local_fista_timing_kind(ctx, c1):
    from paper_1604_02292_amd import make_params
    cfg = c1["cfg"]
    p32 = c1["sino"].astype(np.float32)
    g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    K = 5
    F = torch.empty((K, cfg["n_angles"], cfg["n_det"]), dtype=torch.float32, device="cuda")
    ctx.tomo_sirt_filters(g, K, F)
    D = torch.empty_like(F)
    ctx.tomo_sirt_filter_sino(g, F, _gpu(p32), D)
    out = torch.empty((32, 32), dtype=torch.float32, device="cuda")
    ctx.tomo_kernel_timing(1)
    ctx.tomo_kernel_time(0, reset=True)
    ctx.roi_solve_local(g, D, [make_params((48, 48, 32, 32), 16, "fista", lam=500.0, iters=K)],
                        [out])
    torch.cuda.synchronize()
    ctx.tomo_kernel_timing(0)
    assert ctx.tomo_kernel_time(0)[0] == K
    assert ctx.tomo_kernel_time(1)[0] == K
    n, ms = ctx.tomo_kernel_time(2)
    assert n == K and ms > 0


def test_box_sirt_matches_oracle(ctx, c1):
    from paper_1604_02292_amd import make_params
    cfg = c1["cfg"]
    p32 = c1["sino"].astype(np.float32)
    geo = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    r0, c0, rr, cc, m = synth.roi_list("c1")[0]
    iters, lo, hi = 60, 0.05, 0.6
    res = oracle.local_solve(geo, p32.astype(np.float64), (r0, c0, rr, cc), m, method="sirt",
                             iters=1, full=True)
    ext = res["ext"]
    x = oracle.sirt_nonneg(res["WL"], res["b"].ravel(), (ext[2], ext[3]),
                           1.0 / (cfg["n_angles"] * cfg["n_det"]), iters, lo, hi)
    ref = oracle.crop(np.asarray(x).reshape(ext[2], ext[3]), ext, (r0, c0, rr, cc))
    g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    out = torch.empty((rr, cc), dtype=torch.float32, device="cuda")
    print("[box sirt]", flush=True)
    ctx.roi_solve(g, _gpu(p32), make_params((r0, c0, rr, cc), m, "sirt", iters=iters,
                                            box=(lo, hi)), out)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    e = rel(got, ref)
    print(f"    rel {e:.2e}")
    assert e <= 1e-3
    assert got.min() >= np.float32(lo) and got.max() <= np.float32(hi)


def test_local_method_errors(ctx):
    from paper_1604_02292_amd import make_params, TomoError
    g = ctx.tomo_set_geometry(64, 8, 96)
    D = torch.zeros((5, 8, 96), dtype=torch.float32, device="cuda")
    out = torch.empty((8, 8), dtype=torch.float32, device="cuda")
    sino = torch.zeros((8, 96), dtype=torch.float32, device="cuda")
    with pytest.raises(TomoError, match="EINVAL"):   # wrong method
        ctx.roi_solve_local(g, D, [make_params((0, 0, 8, 8), 2, "sirt", iters=5)], [out])
    with pytest.raises(TomoError, match="EINVAL"):   # more iterations than planes
        ctx.roi_solve_local(g, D, [make_params((0, 0, 8, 8), 2, "local", iters=6)], [out])
    with pytest.raises(TomoError, match="EINVAL"):   # box with lo > hi
        ctx.roi_solve_local(g, D, [make_params((0, 0, 8, 8), 2, "local", iters=5,
                                               box=(1.0, 0.0))], [out])
    with pytest.raises(TomoError, match="EINVAL"):   # the local method through roi_solve
        ctx.roi_solve(g, sino, make_params((0, 0, 8, 8), 2, "local", iters=5), out)
    with pytest.raises(TomoError, match="EINVAL"):   # box for CP
        ctx.roi_solve(g, sino, make_params((0, 0, 8, 8), 2, "cp", iters=5, box=(0, 1)), out)
    with pytest.raises(TomoError, match="EINVAL"):
        ctx.tomo_sirt_filters(g, 0, torch.empty((0, 8, 96), device="cuda"))
    gbig = ctx.tomo_set_geometry(16, 2, 8193)
    with pytest.raises(TomoError, match="EINVAL"):
        ctx.tomo_sirt_filter_sino(gbig, torch.zeros((1, 2, 8193), device="cuda"),
                                  torch.zeros((2, 8193), device="cuda"),
                                  torch.zeros((1, 2, 8193), device="cuda"))


def _sino_in_subprocess(name, tmpdir):
    path = os.path.join(str(tmpdir), f"{name}_sino.npy")
    code = ("import sys, numpy; sys.path.insert(0, %r); import synth; "
            "numpy.save(%r, synth.make_inputs(%r, with_image=False)['sino'])"
            % (os.path.dirname(HERE), path, name))
    subprocess.run([sys.executable, "-c", code], check=True, timeout=600)
    return np.load(path)


@pytest.mark.parametrize("name,sampled", [("c3", (0, 17, 40, 63)), ("c4", (0, 7, 86, 169))])
def test_local_methods_full_size_first_iterate(ctx, tmp_path_factory, name, sampled):
    """The batched workloads at full size in the launch shape of the benchmark (64 uneven
    ROIs on 2048^2, 256 angles, 3072 bins; 256 tiles on 4096^2, 512 angles, 6144 bins, the
    16384-point FFT), one iteration of each local method: with u_1 = alpha W e and
    d_1 = C_{u_1} p, x^1 = P(W_L^T d_1) (Alg. 2, a box that clips part of the values),
    FGP(W_L^T d_1) (Alg. 3, TV) and
    B^T soft(B W_L^T d_1) (Haar).  The oracle computes u_1 from the impulse's own column
    of W and each method's first iterate on the sampled ROIs; the depth of the filter
    recursion and of the iterations is covered at the smaller sizes."""
    from paper_1604_02292_amd import make_params
    from oracle.fista import fgp, prox_weight
    from oracle.haar import haar_prox
    cfg = synth.workload(name)
    n, na, nd = cfg["n"], cfg["n_angles"], cfg["n_det"]
    print(f"[local {name}] generating inputs", flush=True)
    p32 = _sino_in_subprocess(name, tmp_path_factory.mktemp(name + "l")).astype(np.float32)
    geo = oracle.make_geometry(n, na, nd)
    ci = n // 2
    u1 = (1.0 / (na * nd)) * oracle.fp_ray(geo, np.ones((1, 1)), (ci, ci, 1, 1))
    g = ctx.tomo_set_geometry(n, na, nd)
    F = torch.empty((1, na, nd), dtype=torch.float32, device="cuda")
    ctx.tomo_sirt_filters(g, 1, F)
    torch.cuda.synchronize()
    e = rel(F[0].double().cpu().numpy(), u1)
    print(f"    u_1 rel {e:.2e}", flush=True)
    assert e <= 1e-5
    D = torch.empty_like(F)
    ctx.tomo_sirt_filter_sino(g, _gpu(u1[None]), torch.from_numpy(p32).cuda(), D)
    torch.cuda.synchronize()
    d1 = filter_apply(geo, u1.astype(np.float32).astype(np.float64), p32.astype(np.float64))
    e = rel(D[0].double().cpu().numpy(), d1)
    print(f"    C_u1 p rel {e:.2e}", flush=True)
    assert e <= 1e-5
    del F, D
    rois = synth.roi_list(name)
    d1g = _gpu(d1[None])
    lam = 2 * 0.02 * na * nd          # prox weight gamma = alpha lam / 2 = 0.02
    gamma = prox_weight(geo, lam)
    xs_of = {}
    for i in sampled:
        r0, c0, rr, cc, m = rois[i]
        ext = oracle.roi_extend((r0, c0, rr, cc), m, n)
        xs_of[i] = (ext, oracle.bp_pixel(geo, d1, ext))
    # an upper bound that clips about half of the first sampled ROI's first iterate
    top = float(np.median(xs_of[sampled[0]][1]))
    for method in ("local", "fista", "haar"):
        params, outs = [], []
        for (r0, c0, rr, cc, m) in rois:
            if method == "local":
                params.append(make_params((r0, c0, rr, cc), m, "local", iters=1, box=(0.0, top)))
            else:
                params.append(make_params((r0, c0, rr, cc), m, method, lam=lam, iters=1,
                                          inner_iters=100 if method == "fista" else 4))
            outs.append(torch.empty((rr, cc), dtype=torch.float32, device="cuda"))
        ctx.roi_solve_local(g, d1g, params, outs)
        torch.cuda.synchronize()
        for i in sampled:
            r0, c0, rr, cc, m = rois[i]
            ext, xs = xs_of[i]
            if method == "local":
                ref_ext, bar = np.clip(xs, 0.0, np.float32(top)), 1e-5
            elif method == "fista":
                ref_ext, bar = fgp(xs, gamma, 100), 1e-4
            else:
                ref_ext, bar = haar_prox(xs, gamma, 4), 1e-5
            ref = oracle.crop(ref_ext, ext, (r0, c0, rr, cc))
            e = rel(outs[i].double().cpu().numpy(), ref)
            print(f"    {method} roi {i} {rois[i]} rel {e:.2e}", flush=True)
            assert e <= bar
        del outs


def test_local_methods_full_size_depth(ctx, tmp_path_factory):
    """The batched workload at full size (64 uneven ROIs on 2048^2, 256 angles, 3072 bins)
    in the benchmark's launch shape (all 64 ROIs in one call), 20 iterations of Alg. 2
    (box [0, inf)), local FISTA-TV (100 FGP steps, prox weight 0.02) and FISTA with the
    4-level Haar prior, each from the library's own Alg. 1 filters and filtered data, on
    two sampled ROIs (sides 64 and 128) against the oracle's results with its own filters
    (tests/golden/make_golden.py c3local) at the 1e-3 reconstruction bar."""
    from paper_1604_02292_amd import make_params
    path = os.path.join(HERE, "golden", "c3_local_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("no stored oracle result for the local methods at full size")
    gold = np.load(path)
    K = int(gold["iters"])
    cfg = synth.workload("c3")
    n, na, nd = cfg["n"], cfg["n_angles"], cfg["n_det"]
    print(f"[local depth] generating inputs", flush=True)
    p32 = _sino_in_subprocess("c3", tmp_path_factory.mktemp("c3d")).astype(np.float32)
    g = ctx.tomo_set_geometry(n, na, nd)
    F = torch.empty((K, na, nd), dtype=torch.float32, device="cuda")
    ctx.tomo_sirt_filters(g, K, F)
    D = torch.empty_like(F)
    ctx.tomo_sirt_filter_sino(g, F, torch.from_numpy(p32).cuda(), D)
    del F
    rois = synth.roi_list("c3")
    lam = 2 * 0.02 * na * nd          # prox weight gamma = alpha lam / 2 = 0.02
    for method, key in (("local", "alg2"), ("fista", "fista"), ("haar", "haar")):
        params, outs = [], []
        for (r0, c0, rr, cc, m) in rois:
            if method == "local":
                params.append(make_params((r0, c0, rr, cc), m, "local", iters=K,
                                          box=(0.0, float("inf"))))
            else:
                params.append(make_params((r0, c0, rr, cc), m, method, lam=lam, iters=K,
                                          inner_iters=100 if method == "fista" else 4))
            outs.append(torch.empty((rr, cc), dtype=torch.float32, device="cuda"))
        ctx.roi_solve_local(g, D, params, outs)
        torch.cuda.synchronize()
        for i in (int(v) for v in gold["rois"]):
            assert tuple(gold[f"rect_{i}"]) == tuple(rois[i])
            e = rel(outs[i].double().cpu().numpy(), gold[f"{key}_{i}"])
            print(f"    {method} roi {i} {rois[i]} {K} its: rel {e:.2e}", flush=True)
            assert e <= 1e-3
        del outs
