"""The serving scheduler on the host, without a GPU: a host-only context with the test
executor (tomo_serving_fake) runs the real admission, continuous batching, workspace
budget accounting, ticket lifecycle and retirement code, while a tick launches nothing
and a retired request's output holds the number of iterations its slot ran."""

import ctypes
import time

import numpy as np
import pytest
import torch

from paper_1604_02292_amd import Context, TomoError, make_params
from paper_1604_02292_amd._lib import (TOMO_EAGAIN, TOMO_EBUSY, TOMO_EHIP, TOMO_EINVAL,
                                      TOMO_ENOENT, TOMO_ENOMEM, TOMO_ESTATE)

N, NA, ND = 128, 32, 192


def fake_ctx(budget=256 << 20, tick_us=0, n=N, na=NA, nd=ND):
    ctx = Context(device=-1)
    ctx.tomo_serving_fake(budget, tick_us)
    g = ctx.tomo_set_geometry(n, na, nd)
    return ctx, g


def sino_of(na=NA, nd=ND):
    return torch.zeros((na, nd), dtype=torch.float32)


def req(side=32, iters=8, r0=40, c0=40, margin=8):
    return make_params((r0, c0, side, side), margin, "cp", 0.05, iters)


def wait(ctx, tickets, timeout=30.0):
    res, pending, t0 = {}, list(tickets), time.time()
    while pending:
        for t in list(pending):
            done, st = ctx.roi_poll_stages(t)
            if done:
                res[t] = st
                pending.remove(t)
        if pending and time.time() - t0 > timeout:
            raise TimeoutError(f"{len(pending)} requests pending after {timeout} s")
        time.sleep(0.001)
    return res


def usage(ctx):
    return ctx.tomo_workspace_usage()


def prime(ctx, sid):
    """Occupy the stalled scheduler with a one-iteration request, so that requests
    submitted next all wait in the queue and meet the admission rules together."""
    out = torch.zeros((8, 8))
    t = ctx.roi_submit(sid, req(8, 1, 0, 0, 0), out)
    time.sleep(0.05)
    return t, out


def test_each_request_runs_exactly_its_iterations():
    ctx, g = fake_ctx()
    try:
        ctx.tomo_serving_config(max_slots=5, iters_per_tick=4)
        sid = ctx.tomo_register_sinogram(g, sino_of())
        rng = np.random.default_rng(7)
        outs, tickets = [], []
        for k in range(40):
            side = int(rng.integers(8, 64))
            it = int(rng.integers(1, 41))
            out = torch.full((side, side), -1.0)
            p = req(side, it, int(rng.integers(0, N - side)), int(rng.integers(0, N - side)))
            tickets.append(ctx.roi_submit(sid, p, out))
            outs.append((out, it))
        wait(ctx, tickets)
        for out, it in outs:
            assert torch.all(out == float(it)), (it, out.unique())
        ctx.tomo_synchronize()   # idle: only the registration is held
        assert usage(ctx)[0] == usage_after_register(ctx, g)
    finally:
        ctx.close()


def usage_after_register(ctx, g):
    """Bytes a fresh context holds with one registered sinogram of geometry g."""
    c2, g2 = fake_ctx(n=ctx.geoms[g][0], na=ctx.geoms[g][1], nd=ctx.geoms[g][2])
    try:
        c2.tomo_register_sinogram(g2, sino_of(*c2.geoms[g2][1:]))
        return usage(c2)[0]
    finally:
        c2.close()


def test_slot_limit_and_fifo_admission():
    ctx, g = fake_ctx(tick_us=-1)   # stalled: the first admitted slots wait
    try:
        ctx.tomo_serving_config(max_slots=3, iters_per_tick=4)
        sid = ctx.tomo_register_sinogram(g, sino_of())
        p_t, p_out = prime(ctx, sid)
        outs = [torch.zeros((16, 16)) for _ in range(7)]
        tickets = [ctx.roi_submit(sid, req(16, 8), o) for o in outs]
        time.sleep(0.3)
        for t in tickets:
            assert ctx.roi_poll_stages(t) == (False, None)
        ctx.tomo_serving_fake(0, 5000)   # release: 5 ms per iteration, 40 ms per request
        st = wait(ctx, [p_t] + tickets)
        queued = [st[t]["queued_ms"] for t in tickets]
        # three at a time in submission order (first in, first admitted), each wave
        # when the previous one retired
        waves = [queued[0:3], queued[3:6], queued[6:]]
        for w in waves:
            assert max(w) - min(w) < 15.0, queued
        assert min(waves[1]) > max(waves[0]) + 30.0, queued
        assert min(waves[2]) > max(waves[1]) + 30.0, queued
        for t in tickets:
            s = st[t]
            assert min(s.values()) >= 0.0
            assert abs(s["queued_ms"] + s["prepare_ms"] + s["run_ms"] - s["latency_ms"]) < 1.0
        assert all(torch.all(o == 8.0) for o in outs)
    finally:
        ctx.close()


def test_admission_respects_the_workspace_budget():
    # measure what one admitted slot holds, then give room for two and a half
    ctx, g = fake_ctx(tick_us=-1)
    try:
        sid = ctx.tomo_register_sinogram(g, sino_of())
        base = usage(ctx)[0]
        out = torch.zeros((96, 96))   # alive until the ticket is done
        t = ctx.roi_submit(sid, req(96, 4, 10, 10), out)
        time.sleep(0.2)
        one = usage(ctx)[0] - base
        assert one > 0
        ctx.tomo_serving_fake(0, 0)
        wait(ctx, [t])
    finally:
        ctx.close()
    budget = max(base + int(2.5 * one) + (1 << 16), 1 << 20)
    ctx, g = fake_ctx(budget=budget, tick_us=-1)
    try:
        ctx.tomo_serving_config(max_slots=8)
        sid = ctx.tomo_register_sinogram(g, sino_of())
        p_t, p_out = prime(ctx, sid)
        outs = [torch.zeros((96, 96)) for _ in range(6)]
        tickets = [ctx.roi_submit(sid, req(96, 4, 10, 10), o) for o in outs]
        time.sleep(0.3)
        assert usage(ctx)[0] <= budget
        ctx.tomo_serving_fake(0, 5000)
        st = wait(ctx, [p_t] + tickets)
        queued = [st[t]["queued_ms"] for t in tickets]
        # two at a time (the budget, not the slot limit of 8, holds the rest back)
        for w in (queued[0:2], queued[2:4], queued[4:6]):
            assert max(w) - min(w) < 10.0, queued
        assert min(queued[2:4]) > max(queued[0:2]) + 15.0, queued
        assert min(queued[4:6]) > max(queued[2:4]) + 15.0, queued
        assert usage(ctx)[1] <= budget   # the peak never passed the budget
        assert all(torch.all(o == 4.0) for o in outs)
    finally:
        ctx.close()


def test_queue_full_is_eagain():
    ctx, g = fake_ctx(tick_us=-1)
    try:
        ctx.tomo_serving_config(max_slots=1)
        sid = ctx.tomo_register_sinogram(g, sino_of())
        out = torch.zeros((8, 8))
        p = req(8, 1)
        tickets = []
        with pytest.raises(TomoError) as e:
            for _ in range(9000):
                tickets.append(ctx.roi_submit(sid, p, out))
        assert e.value.status == TOMO_EAGAIN
        assert len(tickets) in (8192, 8193)   # the queue, plus the one admitted slot
        ctx.tomo_serving_fake(0, 0)
        wait(ctx, tickets, timeout=120.0)
        assert torch.all(out == 1.0)
    finally:
        ctx.close()


def test_requests_that_cannot_fit():
    ctx, g = fake_ctx(budget=16 << 20, n=1024, na=128, nd=1536)
    try:
        # registration larger than the budget
        g2 = ctx.tomo_set_geometry(2048, 256, 3072)
        with pytest.raises(TomoError) as e:
            ctx.tomo_register_sinogram(g2, sino_of(256, 3072))
        assert e.value.status == TOMO_ENOMEM
        used0 = usage(ctx)[0]
        sid = ctx.tomo_register_sinogram(g, sino_of(128, 1536))
        assert usage(ctx)[0] > used0
        # larger than the whole workspace: refused at submission
        with pytest.raises(TomoError) as e:
            ctx.roi_submit(sid, make_params((0, 0, 1024, 1024), 0, "cp", 0.02, 10),
                           torch.zeros((1024, 1024)))
        assert e.value.status == TOMO_ENOMEM
        # fits the workspace but never next to the resident sinogram: fails when admitted
        side = 400
        big = torch.zeros((side, side))
        t = ctx.roi_submit(sid, make_params((100, 100, side, side), 32, "cp", 0.02, 10), big)
        with pytest.raises(TomoError) as e:
            wait(ctx, [t])
        assert e.value.status == TOMO_EHIP and "does not fit" in str(e.value)
        # a small request still runs afterwards
        out = torch.zeros((32, 32))
        wait(ctx, [ctx.roi_submit(sid, make_params((10, 10, 32, 32), 8, "cp", 0.02, 6), out)])
        assert torch.all(out == 6.0)
    finally:
        ctx.close()


def test_ticket_lifecycle_and_registration_rules():
    ctx, g = fake_ctx(tick_us=-1)
    try:
        with pytest.raises(TomoError) as e:
            ctx.roi_poll_stages(12345)
        assert e.value.status == TOMO_ENOENT
        bad = sino_of()
        bad[3, 5] = float("nan")
        used0 = usage(ctx)[0]
        with pytest.raises(TomoError) as e:
            ctx.tomo_register_sinogram(g, bad)
        assert e.value.status == TOMO_EINVAL and "NaN" in str(e.value)
        assert usage(ctx)[0] == used0
        sid = ctx.tomo_register_sinogram(g, sino_of())
        out = torch.zeros((16, 16))
        t = ctx.roi_submit(sid, req(16, 4), out)
        with pytest.raises(TomoError) as e:
            ctx.tomo_unregister_sinogram(sid)   # a live request holds it
        assert e.value.status == TOMO_EBUSY
        with pytest.raises(TomoError) as e:
            ctx.roi_submit(sid + 1, req(16, 4), out)
        assert e.value.status == TOMO_ENOENT
        with pytest.raises(TomoError) as e:
            ctx.roi_submit(sid, make_params((120, 120, 16, 16), 4, "cp", 0.05, 4), out)
        assert e.value.status == TOMO_EINVAL   # outside the grid
        ctx.tomo_serving_fake(0, 0)
        wait(ctx, [t])
        with pytest.raises(TomoError) as e:
            ctx.roi_poll_stages(t)   # reported once, then forgotten
        assert e.value.status == TOMO_ENOENT
        ctx.tomo_synchronize()
        ctx.tomo_unregister_sinogram(sid)
        with pytest.raises(TomoError) as e:
            ctx.tomo_unregister_sinogram(sid)
        assert e.value.status == TOMO_ENOENT
        assert usage(ctx)[0] == used0
        with pytest.raises(TomoError) as e:
            ctx.tomo_serving_fake(64 << 20, 0)   # set up once only
        assert e.value.status == TOMO_ESTATE
    finally:
        ctx.close()


def test_executor_setup_rules():
    ctx = Context(device=-1)
    try:
        with pytest.raises(TomoError) as e:
            ctx.tomo_serving_fake(0, 0)
        assert e.value.status == TOMO_ESTATE
        with pytest.raises(TomoError) as e:
            ctx.tomo_serving_fake(1000, 0)
        assert e.value.status == TOMO_EINVAL
        g = ctx.tomo_set_geometry(N, NA, ND)
        with pytest.raises(ValueError):   # the binding wants GPU memory here
            ctx.tomo_register_sinogram(g, sino_of())
        sino = sino_of()
        sid = ctypes.c_int32()
        st = ctx.lib.tomo_register_sinogram(ctx.h, g, ctypes.c_void_p(sino.data_ptr()),
                                            ctypes.byref(sid))
        assert st == TOMO_ESTATE   # a host-only context without the executor
    finally:
        ctx.close()


def test_stalled_executor_times_out_then_drains():
    ctx, g = fake_ctx(tick_us=-1)
    try:
        sid = ctx.tomo_register_sinogram(g, sino_of())
        outs = [torch.zeros((16, 16)) for _ in range(4)]
        tickets = [ctx.roi_submit(sid, req(16, 12), o) for o in outs]
        with pytest.raises(TimeoutError):
            wait(ctx, tickets, timeout=0.3)
        ctx.tomo_serving_fake(0, 2000)   # 2 ms per iteration from now on
        st = wait(ctx, tickets)
        for t in tickets:
            assert st[t]["run_ms"] >= 12 * 2.0 * 0.9
        assert all(torch.all(o == 12.0) for o in outs)
    finally:
        ctx.close()


def test_destroy_ends_a_stall():
    ctx, g = fake_ctx(tick_us=-1)
    sid = ctx.tomo_register_sinogram(g, sino_of())
    outs = [torch.zeros((16, 16)) for _ in range(40)]
    for o in outs:
        ctx.roi_submit(sid, req(16, 100), o)
    t0 = time.time()
    ctx.close()
    assert time.time() - t0 < 10.0
