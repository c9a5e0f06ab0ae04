"""Host-side checks of the C ABI: the library loads, exports every call of
include/tomo.h, and its planning logic (bands, extended rects, validation)
agrees with the oracle.  No GPU is touched (host-only context, device = -1)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1604_02292_amd import _lib
from paper_1604_02292_amd.tomo import Context, TomoError

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "tomo.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:tomo|roi)_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_call():
    lib = _lib.load()
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, n


def test_host_context_rejects_gpu_calls():
    ctx = Context(device=-1)
    g = ctx.tomo_set_geometry(64, 8, 96)
    lib = ctx.lib
    st = lib.tomo_fp(ctx.h, g, _lib.tomo_rect(0, 0, 4, 4), None, None, 0, None)
    assert st == _lib.TOMO_ESTATE
    st = lib.tomo_synchronize(ctx.h)
    assert st == _lib.TOMO_ESTATE


@pytest.mark.parametrize("n,na,nd", [(128, 32, 192), (1024, 128, 1536), (2048, 256, 3072),
                                     (4096, 512, 6144)])
def test_band_covers_exact_nonzero_rows(n, na, nd):
    """Every nonzero row of W_L (the oracle's brute-force band) lies inside the
    library's band, which is at most 2 bins wider on each side."""
    ctx = Context(device=-1)
    g = ctx.tomo_set_geometry(n, na, nd)
    geo = oracle.make_geometry(n, na, nd)
    rng = np.random.default_rng(n)
    rects = [(0, 0, 9, 13), (n - 7, n - 11, 7, 11),
             (int(rng.integers(0, n - 20)), int(rng.integers(0, n - 20)), 20, 17)]
    for rect in rects:
        i0, w = ctx.tomo_roi_band(g, rect)
        exact = oracle.band_exact(geo, rect)
        for k in range(na):
            lo, hi = exact[k]
            assert i0[k] <= lo and hi <= i0[k] + w[k] - 1
            assert lo - i0[k] <= 3 and (i0[k] + w[k] - 1) - hi <= 3


def test_roi_ext_matches_oracle():
    ctx = Context(device=-1)
    g = ctx.tomo_set_geometry(128, 4, 192)
    for roi, m in [((48, 48, 32, 32), 16), ((0, 100, 32, 28), 16), ((0, 0, 128, 128), 16),
                   ((120, 3, 8, 8), 0)]:
        assert ctx.tomo_roi_ext(g, roi, m) == oracle.roi_extend(roi, m, 128)


def test_argument_validation():
    ctx = Context(device=-1)
    with pytest.raises(TomoError) as e:
        ctx.tomo_set_geometry(0, 8, 8)
    assert e.value.status == _lib.TOMO_EINVAL
    with pytest.raises(TomoError) as e:
        ctx.tomo_set_geometry(64, 8, 96, det_spacing=0.5)
    assert e.value.status == _lib.TOMO_EINVAL
    g = ctx.tomo_set_geometry(64, 8, 96)
    for bad in [(0, 0, 0, 4), (-1, 0, 4, 4), (60, 60, 8, 8)]:
        with pytest.raises(TomoError) as e:
            ctx.tomo_roi_band(g, bad)
        assert e.value.status == _lib.TOMO_EINVAL
    with pytest.raises(TomoError) as e:
        ctx.tomo_roi_ext(g, (0, 0, 4, 4), -1)
    assert e.value.status == _lib.TOMO_EINVAL
    lib = ctx.lib
    i0 = (C.c_int32 * 8)()
    w = (C.c_int32 * 8)()
    assert lib.tomo_roi_band(ctx.h, 7, _lib.tomo_rect(0, 0, 4, 4), i0, w) == _lib.TOMO_ENOENT
    assert lib.tomo_create(-2, None, 0, C.byref(C.c_void_p())) == _lib.TOMO_EINVAL
    assert b"unknown geometry" in lib.tomo_last_error(ctx.h)


@pytest.mark.parametrize("n,na,nd,rect", [(128, 32, 192, (32, 32, 64, 64)),
                                          (64, 45, 90, (0, 10, 20, 33)),
                                          (1024, 128, 1536, (416, 416, 40, 48))])
def test_nnz_count_matches_oracle(n, na, nd, rect):
    """The library's algorithmic update count is the nonzero count of the oracle's W_L."""
    ctx = Context(device=-1)
    g = ctx.tomo_set_geometry(n, na, nd)
    WL = oracle.sparse_local(oracle.make_geometry(n, na, nd), rect)
    assert ctx.tomo_roi_nnz(g, rect) == WL.nnz


def test_launch_shapes_by_problem_size():
    """The size heuristics: a single small region (the 1024^2 workload's 192^2 extended ROI,
    128 angles: 35 k rays, 37 k pixels) gets the most waves per ray and per pixel (8
    forward-projector segments, 8 backprojector angle groups, direct band reads); the
    256 tiles of 4096^2 (extended parts up to 320^2) and the 64-ROI batch on 2048^2
    (extended parts up to 384^2, staged 24 lines at a time) get the LDS-staged forward
    projector (rays per lane 4), a region wider than 16-line stages hold two rays per lane,
    also when the staged projector is forced; all get the LDS-staged backprojector with two
    pixels per thread.  Forced knobs are validated and kept."""
    import synth
    from paper_1604_02292_amd.tomo import make_params
    ctx = Context(device=-1)
    g = ctx.tomo_set_geometry(1024, 128, 1536)
    small = ctx.tomo_resolve_launch(g, [make_params((448, 448, 128, 128), 32, "cp", 0.02, 300)])
    assert (small["fp_segments"], small["fp_rays_per_lane"]) == (8, 1)
    assert (small["bp_variant"], small["bp_groups"], small["bp_pixels_per_thread"]) == (1, 8, 1)
    g3 = ctx.tomo_set_geometry(2048, 256, 3072)
    batch = [make_params(r[:4], r[4], "cp", 0.02, 200) for r in synth.roi_list("c3")]
    big = ctx.tomo_resolve_launch(g3, batch)
    assert (big["fp_segments"], big["fp_rays_per_lane"]) == (1, 4)
    assert (big["bp_variant"], big["bp_groups"], big["bp_pixels_per_thread"]) == (2, 1, 2)
    g4 = ctx.tomo_set_geometry(4096, 512, 6144)
    tiles = [make_params(r[:4], r[4], "cp", 0.01, 200) for r in synth.roi_list("c4")]
    t4 = ctx.tomo_resolve_launch(g4, tiles)
    assert (t4["fp_segments"], t4["fp_rays_per_lane"]) == (1, 4)
    assert (t4["bp_variant"], t4["bp_groups"], t4["bp_pixels_per_thread"]) == (2, 1, 2)
    # many jobs: the forward projector's items round-robin over the XCDs, the
    # backprojector's (equal tiles) in contiguous eighths
    assert (t4["fp_xcd_order"], t4["bp_xcd_order"]) == (2, 1)
    assert (big["fp_xcd_order"], big["bp_xcd_order"]) == (2, 1)
    wide = batch + [make_params((500, 500, 800, 800), 64, "cp", 0.02, 200)]   # 928^2
    assert ctx.tomo_resolve_launch(g3, wide)["fp_rays_per_lane"] == 2
    ctx.tomo_set_launch(fp_rays_per_lane=4)
    assert ctx.tomo_resolve_launch(g3, wide)["fp_rays_per_lane"] == 2
    assert ctx.tomo_resolve_launch(g3, batch)["fp_rays_per_lane"] == 4
    ctx.tomo_set_launch(fp_rays_per_lane=2)
    assert ctx.tomo_resolve_launch(g4, tiles)["fp_rays_per_lane"] == 2
    ctx.tomo_set_launch()
    ctx.tomo_set_launch(fp_segments=4, bp_groups=2)
    forced = ctx.tomo_resolve_launch(g, [make_params((448, 448, 128, 128), 32, "cp", 0.02, 300)])
    assert (forced["fp_segments"], forced["bp_groups"]) == (4, 2)
    for bad in [dict(fp_segments=3), dict(fp_segments=16), dict(bp_groups=16),
                dict(bp_pixels_per_thread=3), dict(bp_variant=5), dict(fp_rays_per_lane=3)]:
        with pytest.raises(TomoError) as e:
            ctx.tomo_set_launch(**bad)
        assert e.value.status == _lib.TOMO_EINVAL
    assert ctx.tomo_get_launch()["fp_segments"] == 4   # a rejected call changes nothing
    ctx.tomo_set_launch()
