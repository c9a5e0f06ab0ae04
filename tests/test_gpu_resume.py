"""Pause and resume: a CP-TV or SIRT solve run as K1 iterations, then K2 more from the
saved iteration state (roi_solve_resume), gives the bits of one solve of K1 + K2
iterations, and the state after K1 gives the bits of a K1-iteration solve's crop."""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.fixture(scope="module")
def setup():
    from paper_1604_02292_amd import Context
    ctx = Context(0, workspace_bytes=1 << 30)
    d = synth.make_inputs("c1", with_image=False)
    cfg = d["cfg"]
    g = ctx.tomo_set_geometry(cfg["n"], cfg["n_angles"], cfg["n_det"])
    yield ctx, g, dev(d["sino"])
    ctx.close()


@pytest.mark.parametrize("method,lam,rect,splits", [
    ("cp", 0.05, (48, 48, 32, 32), (37, 63)),
    ("cp", 0.05, (0, 70, 40, 58), (50, 1, 49)),
    ("cp", 5.0, (20, 30, 24, 40), (10, 10, 10, 10)),
    ("sirt", 0.0, (48, 48, 32, 32), (33, 67)),
])
def test_pieces_equal_one_solve(setup, method, lam, rect, splits):
    from paper_1604_02292_amd import make_params
    ctx, g, sino = setup
    K = sum(splits)
    whole = torch.empty((rect[2], rect[3]), device="cuda")
    ctx.roi_solve(g, sino, make_params(rect, 16, method, lam, K), whole)
    first = torch.empty_like(whole)
    ctx.roi_solve(g, sino, make_params(rect, 16, method, lam, splits[0]), first)
    nbytes = ctx.roi_state_bytes(g, make_params(rect, 16, method, lam, K))
    state = torch.full((nbytes // 4,), float("nan"), device="cuda")   # ignored at done = 0
    out = torch.empty_like(whole)
    done = 0
    for k, it in enumerate(splits):
        ctx.roi_solve_resume(g, sino, make_params(rect, 16, method, lam, it), done, state, out)
        done += it
        if k == 0:
            torch.cuda.synchronize()
            assert torch.equal(out, first)
    torch.cuda.synchronize()
    print(f"    {method} {rect} {splits}: max |diff| "
          f"{(out - whole).abs().max().item():.3g}", flush=True)
    assert torch.isfinite(out).all()
    assert torch.equal(out, whole)


def test_state_size_and_arguments(setup):
    from paper_1604_02292_amd import TomoError, make_params
    ctx, g, sino = setup
    p = make_params((48, 48, 32, 32), 16, "cp", 0.05, 10)
    nbytes = ctx.roi_state_bytes(g, p)
    # x, two xbar buffers, xbar^T, two TV duals (2 planes), the band dual
    assert nbytes >= 4 * (64 * 64 * 7 + 32 * 64)
    with pytest.raises(TomoError):
        ctx.roi_state_bytes(g, make_params((48, 48, 32, 32), 16, "local", 0.0, 10))
    state = torch.zeros((nbytes // 4,), device="cuda")
    out = torch.empty((32, 32), device="cuda")
    with pytest.raises(TomoError):
        ctx.roi_solve_resume(g, sino, p, -1, state, out)
