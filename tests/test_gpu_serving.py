"""Serving: resident sinograms, roi_submit / roi_poll with continuous batching.

Each request's result must be the same alone and in a mix (bit-identical:
a slot's arithmetic never depends on the other slots), agree with roi_solve
on the same request (up to FP32 rounding of the exterior data), and match the
FP64 oracle at the 1e-3 reconstruction bar.
"""

import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def wait_all(ctx, tickets, timeout=120.0):
    lat = {}
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            done, ms = ctx.roi_poll(t)
            if done:
                lat[t] = ms
                pending.discard(t)
        if time.time() - t0 > timeout:
            raise AssertionError(f"{len(pending)} requests not done after {timeout}s")
        time.sleep(0.0005)
    return lat


@pytest.fixture(scope="module")
def served():
    from paper_1604_02292_amd import Context
    ctx = Context(0, workspace_bytes=2 << 30)
    d = synth.make_inputs("c1")
    cfg = d["cfg"]
    g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    p32 = d["sino"].astype(np.float32)
    sino = dev(p32)
    sid = ctx.tomo_register_sinogram(g, sino)
    yield ctx, g, sid, sino, p32, cfg
    ctx.tomo_synchronize()
    ctx.tomo_unregister_sinogram(sid)
    ctx.close()


REQS = [((48, 48, 32, 32), 16, "cp", 0.05, 100), ((0, 0, 24, 40), 6, "sirt", 0.0, 60),
        ((90, 10, 30, 30), 8, "cp", 5.0, 77), ((60, 100, 16, 20), 4, "cp", 0.05, 33),
        ((5, 90, 40, 36), 10, "sirt", 0.0, 120), ((64, 64, 64, 64), 16, "cp", 0.05, 51)]


def test_alone_equals_mix_and_matches_roi_solve(served):
    from paper_1604_02292_amd import make_params
    ctx, g, sid, sino, p32, cfg = served
    params = [make_params(r, m, meth, lam, it) for r, m, meth, lam, it in REQS]
    alone = []
    for p in params:
        o = torch.empty((p.roi.rows, p.roi.cols), device="cuda")
        wait_all(ctx, [ctx.roi_submit(sid, p, o)])
        alone.append(o.clone())
    outs = [torch.empty((p.roi.rows, p.roi.cols), device="cuda") for p in params]
    tickets = [ctx.roi_submit(sid, p, o) for p, o in zip(params, outs)]
    lat = wait_all(ctx, tickets)
    assert all(v is not None and v > 0 for v in lat.values())
    torch.cuda.synchronize()
    for a, b in zip(alone, outs):
        assert torch.equal(a, b)
    # permuted submission order
    perm = [5, 2, 0, 4, 1, 3]
    outs2 = [None] * len(params)
    tickets = []
    for i in perm:
        outs2[i] = torch.empty((params[i].roi.rows, params[i].roi.cols), device="cuda")
        tickets.append(ctx.roi_submit(sid, params[i], outs2[i]))
    wait_all(ctx, tickets)
    torch.cuda.synchronize()
    for a, b in zip(alone, outs2):
        assert torch.equal(a, b)
    # same requests through roi_solve (FBP exterior recomputed there).  The serving loop
    # picks its launch shapes for the batch it runs and roi_solve for the single request
    # (e.g. 4 or 8 forward-projector segments per ray): different FP32 summation orders,
    # which 30-120 iterations amplify to ~1e-5 relative; each path is held to the oracle
    # at 1e-3 elsewhere
    for p, a in zip(params, alone):
        o = torch.empty((p.roi.rows, p.roi.cols), device="cuda")
        ctx.roi_solve(g, sino, p, o)
        torch.cuda.synchronize()
        assert rel(o.double().cpu().numpy(), a.double().cpu().numpy()) <= 1e-4


def test_uneven_slots_alone_equal_mix():
    """Slots of very different sizes (an 800^2 region beside 96^2 and 280 x 230 ones,
    CP and SIRT) share ticks; every result is bit-identical alone and in the mix."""
    from paper_1604_02292_amd import Context, make_params
    ctx = Context(0, workspace_bytes=4 << 30)
    try:
        g = ctx.tomo_set_geometry(1024, 128, 1536)
        rng = np.random.default_rng(1604)
        sino = dev(10.0 * rng.random((128, 1536)))
        sid = ctx.tomo_register_sinogram(g, sino)
        reqs = [make_params((100, 100, 800, 800), 0, "cp", 0.05, 12),
                make_params((40, 900, 64, 64), 16, "cp", 0.05, 20),
                make_params((700, 20, 200, 150), 40, "sirt", 0.0, 16)]
        print("[serving] wide + narrow slots", flush=True)
        alone = []
        for p in reqs:
            o = torch.empty((p.roi.rows, p.roi.cols), device="cuda")
            wait_all(ctx, [ctx.roi_submit(sid, p, o)])
            alone.append(o.clone())
        outs = [torch.empty((p.roi.rows, p.roi.cols), device="cuda") for p in reqs]
        wait_all(ctx, [ctx.roi_submit(sid, p, o) for p, o in zip(reqs, outs)])
        torch.cuda.synchronize()
        for a, b in zip(alone, outs):
            assert bool(torch.isfinite(a).all())
            assert torch.equal(a, b)
        ctx.tomo_synchronize()
        ctx.tomo_unregister_sinogram(sid)
    finally:
        ctx.close()


def test_request_timeline(served):
    """roi_poll_stages on the GPU path: every finished request reports its queueing,
    preparation and iteration times, which add up to its latency; a request that waited
    behind a full slot set shows it as queueing time."""
    from paper_1604_02292_amd import make_params
    ctx, g, sid, sino, p32, cfg = served
    ctx.tomo_serving_config(max_slots=2)
    try:
        params = [make_params(r, m, meth, lam, it) for r, m, meth, lam, it in REQS]
        outs = [torch.empty((p.roi.rows, p.roi.cols), device="cuda") for p in params]
        tickets = [ctx.roi_submit(sid, p, o) for p, o in zip(params, outs)]
        got, t0 = {}, time.time()
        while len(got) < len(tickets) and time.time() - t0 < 120:
            for t in tickets:
                if t not in got:
                    done, st = ctx.roi_poll_stages(t)
                    if done:
                        got[t] = st
            time.sleep(0.0005)
        assert len(got) == len(tickets)
        for t in tickets:
            st = got[t]
            assert min(st.values()) >= 0.0 and st["run_ms"] > 0.0
            assert abs(st["queued_ms"] + st["prepare_ms"] + st["run_ms"] - st["latency_ms"]) < 1.0
        # two slots: the last request waited for earlier ones to retire
        assert got[tickets[-1]]["queued_ms"] > 0.5 * min(got[t]["run_ms"] for t in tickets[:2])
    finally:
        ctx.tomo_serving_config(max_slots=32)


def test_served_matches_oracle(served):
    from paper_1604_02292_amd import make_params
    ctx, g, sid, sino, p32, cfg = served
    geo = oracle.make_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    for (roi, m, meth, lam, it) in [REQS[0], REQS[1], REQS[2]]:
        ref = oracle.local_solve(geo, p32.astype(np.float64), roi, m, method=meth, lam=lam,
                                 iters=it, full=True)
        s = ref["sigma"] if meth == "cp" else 0.0
        p = make_params(roi, m, meth, lam, it, s, s)
        o = torch.empty((roi[2], roi[3]), device="cuda")
        wait_all(ctx, [ctx.roi_submit(sid, p, o)])
        e = rel(o.double().cpu().numpy(), ref["x"])
        print(f"[serve] {roi} {meth} rel {e:.2e}", flush=True)
        assert e <= 1e-3


def test_admission_errors(served):
    from paper_1604_02292_amd import Context, TomoError, make_params, _lib
    ctx, g, sid, sino, p32, cfg = served
    # unknown sinogram / ticket
    p = make_params((0, 0, 8, 8), 2, "cp", 0.05, 10)
    o = torch.empty((8, 8), device="cuda")
    with pytest.raises(TomoError) as e:
        ctx.roi_submit(999, p, o)
    assert e.value.status == _lib.TOMO_ENOENT
    with pytest.raises(TomoError) as e:
        ctx.roi_poll(123456789)
    assert e.value.status == _lib.TOMO_ENOENT
    # a sinogram with a NaN or an infinity is refused and nothing stays registered
    for bad in (float("nan"), float("inf")):
        ctx.tomo_synchronize()
        used0, _ = ctx.tomo_workspace_usage()
        poisoned = sino.clone()
        poisoned[3, 17] = bad
        with pytest.raises(TomoError) as e:
            ctx.tomo_register_sinogram(g, poisoned)
        assert e.value.status == _lib.TOMO_EINVAL
        ctx.tomo_synchronize()
        assert ctx.tomo_workspace_usage()[0] == used0
    # invalid request
    o16 = torch.empty((16, 16), device="cuda")
    with pytest.raises(TomoError) as e:
        ctx.roi_submit(sid, make_params((120, 120, 16, 16), 2, "cp", 0.05, 10), o16)
    assert e.value.status == _lib.TOMO_EINVAL
    # busy: unregister while requests are queued
    outs = [torch.empty((32, 32), device="cuda") for _ in range(16)]
    tickets = [ctx.roi_submit(sid, make_params((40, 40, 32, 32), 16, "cp", 0.05, 200), q)
               for q in outs]
    with pytest.raises(TomoError) as e:
        ctx.tomo_unregister_sinogram(sid)
    assert e.value.status == _lib.TOMO_EBUSY
    wait_all(ctx, tickets)
    # a request larger than the whole workspace is refused at submission
    small = Context(0, workspace_bytes=24 << 20)
    try:
        g2 = small.tomo_set_geometry(1024, 128, 1536)
        s2 = torch.zeros((128, 1536), device="cuda")
        sid2 = small.tomo_register_sinogram(g2, s2)
        big = torch.empty((1024, 1024), device="cuda")
        with pytest.raises(TomoError) as e:
            small.roi_submit(sid2, make_params((0, 0, 1024, 1024), 0, "cp", 0.02, 5), big)
        assert e.value.status == _lib.TOMO_ENOMEM
        small.tomo_unregister_sinogram(sid2)
    finally:
        small.close()


def test_small_budget_admission(served):
    """With a workspace that holds the resident sinogram and only about one
    slot (state plus its step-size power iteration), requests of shapes whose
    step size is not cached yet are admitted one or two at a time and all
    complete with the same results as roi_solve."""
    from paper_1604_02292_amd import Context, make_params
    ctx, g, sid, sino, p32, cfg = served
    small = Context(0, workspace_bytes=1 << 20)
    try:
        g2 = small.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
        sid2 = small.tomo_register_sinogram(g2, sino)
        rects = [(40 + k, 36 + 2 * k, 24 + 3 * k, 20 + 5 * k) for k in range(6)]
        params = [make_params(r, 8 + k, "cp", cfg["lam"], 40) for k, r in enumerate(rects)]
        outs = [torch.empty((r[2], r[3]), device="cuda") for r in rects]
        tickets = [small.roi_submit(sid2, p, o) for p, o in zip(params, outs)]
        wait_all(small, tickets)
        used, peak = small.tomo_workspace_usage()
        assert peak <= 1 << 20
        torch.cuda.synchronize()
        for p, o in zip(params, outs):
            ref = torch.empty_like(o)
            ctx.roi_solve(g, sino, p, ref)
            torch.cuda.synchronize()
            assert rel(o.double().cpu().numpy(), ref.double().cpu().numpy()) <= 1e-5
        small.tomo_unregister_sinogram(sid2)
    finally:
        small.close()


def _slices_in_subprocess(indices, tmpdir):
    """The serving workload's slices, generated in a fresh process (the generator forks
    worker processes, which must not inherit this process's GPU state)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = os.path.join(str(tmpdir), "c5_slices.npy")
    code = ("import sys, numpy; sys.path.insert(0, %r); import synth; "
            "numpy.save(%r, numpy.stack(synth.make_slices('c5', indices=%r)))"
            % (root, path, list(indices)))
    subprocess.run([sys.executable, "-c", code], check=True, timeout=600)
    return dict(zip(indices, np.load(path)))


def test_full_size_served_requests_match_oracle(tmp_path_factory):
    """The serving workload at full size (2048^2 slices, 512 angles x 3072 bins): eight
    sampled requests of its request stream (sides 41-200, 6 CP-TV and 2 SIRT, 161-292
    iterations, on 4 resident slices), submitted interleaved with 24 other requests of the
    same stream on the same slices, each against the stored FP64 oracle result at the 1e-3
    reconstruction bar (tests/golden/make_golden.py c5; the oracle's FBP exterior, the
    library's own resident FBP and residual on the GPU)."""
    import os
    from paper_1604_02292_amd import Context, make_params
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("no stored oracle result for the serving workload")
    gold = np.load(path)
    pick = [int(i) for i in gold["pick"]]
    cfg = synth.workload("c5")
    reqs = synth.serving_requests(4000, 1.0, seed_offset=2)
    slices = sorted({reqs[i]["slice"] for i in pick})
    others = [i for i in range(len(reqs)) if reqs[i]["slice"] in slices and i not in pick][:24]
    print(f"[serve c5] slices {slices}: generating", flush=True)
    data = _slices_in_subprocess(slices, tmp_path_factory.mktemp("c5"))
    ctx = Context(0, workspace_bytes=4 << 30)
    try:
        g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
        sinos = {k: dev(v) for k, v in data.items()}
        sids = {k: ctx.tomo_register_sinogram(g, s) for k, s in sinos.items()}
        order = sorted(pick + others)   # stream order: sampled requests among the others
        outs, tickets = {}, []
        for i in order:
            r = reqs[i]
            s = float(gold[f"sigma_{i}"]) if i in pick and r["method"] == "cp" else 0.0
            p = make_params(r["rect"], r["margin"], r["method"], r["lam"], r["iters"], s, s)
            outs[i] = torch.empty((r["rect"][2], r["rect"][3]), device="cuda")
            tickets.append(ctx.roi_submit(sids[r["slice"]], p, outs[i]))
        wait_all(ctx, tickets, timeout=300.0)
        torch.cuda.synchronize()
        for i in pick:
            r = reqs[i]
            assert tuple(gold[f"req_{i}"][1:5]) == tuple(r["rect"])
            e = rel(outs[i].double().cpu().numpy(), gold[f"x_{i}"])
            print(f"    request {i} slice {r['slice']} {r['rect']} {r['method']} "
                  f"{r['iters']} its: rel {e:.2e}", flush=True)
            assert e <= 1e-3
        for i in others:
            assert torch.isfinite(outs[i]).all()
        ctx.tomo_synchronize()
        for sid in sids.values():
            ctx.tomo_unregister_sinogram(sid)
    finally:
        ctx.close()
