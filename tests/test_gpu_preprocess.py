"""GPU parity of the local method's preprocessing against the FP64 oracle
(oracle/preprocess.py): disc subtraction and its undo (Section 3.3), constant padding of
truncated data (Section 4), and the whole truncated-data pipeline of the paper's
experiment (pad, subtract the disc, filter, Alg. 3, add the disc back)."""

import numpy as np
import pytest

import synth
import oracle
from oracle.filters import sirt_filters
from oracle.fista import local_fista_tv
from oracle.preprocess import disc_subtract, disc_add, pad_truncated

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.fixture(scope="module")
def ctx():
    from paper_1604_02292_amd import Context
    c = Context(0, workspace_bytes=2 << 30)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c1():
    return synth.make_inputs("c1", with_image=False)


@pytest.mark.parametrize("n,na,nd,inplace", [(128, 32, 192, False), (65, 24, 97, True),
                                             (64, 7, 200, False)])
def test_disc_subtract_matches_oracle(ctx, n, na, nd, inplace):
    print(f"[disc] n={n} na={na} nd={nd} inplace={inplace}", flush=True)
    geo = oracle.make_geometry(n, na, nd)
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2.0
    img = 0.7 * (xx ** 2 + yy ** 2 < (0.4 * n) ** 2) + 0.3 * ((xx - 3) ** 2 + yy ** 2 < 16)
    p32 = oracle.fp_ray(geo, img).astype(np.float32).astype(np.float64)
    ref, c_ref = disc_subtract(geo, p32)
    g = ctx.tomo_set_geometry(n, na, nd)
    sino = _gpu(p32)
    out = sino if inplace else torch.empty_like(sino)
    val = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.tomo_disc_subtract(g, sino, out, val)
    torch.cuda.synchronize()
    c = float(val.item())
    print(f"    c {c:.8f} (oracle {c_ref:.8f}); data rel {rel(out.cpu().numpy(), ref):.2e}")
    assert abs(c - c_ref) <= 1e-6 * abs(c_ref)
    # the residual is a small difference of large terms: compare it against the data's scale
    assert np.linalg.norm(out.double().cpu().numpy() - ref) <= 1e-6 * np.linalg.norm(p32)
    # undo on a region at the grid's corner and one across the centre
    for rect in [(0, 0, 9, 13), (n // 2 - 5, n // 2 - 7, 11, 15)]:
        r0, c0, rr, cc = rect
        base = np.random.default_rng(1).normal(size=(rr, cc)).astype(np.float32)
        x = _gpu(base)
        ctx.tomo_disc_add(g, rect, val, x)
        torch.cuda.synchronize()
        want = disc_add(geo, base.astype(np.float64), rect, c)
        assert np.abs(x.double().cpu().numpy() - want).max() <= 1e-6 * (1 + abs(c))


def test_pad_truncated_is_exact(ctx):
    g = ctx.tomo_set_geometry(64, 5, 101)
    rng = np.random.default_rng(2)
    for first, nb in [(40, 21), (0, 101), (0, 1), (100, 1), (3, 60)]:
        t = rng.normal(size=(5, nb)).astype(np.float32)
        out = torch.empty((5, 101), dtype=torch.float32, device="cuda")
        ctx.tomo_pad_truncated(g, _gpu(t), first, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), pad_truncated(t, first, 101).astype(np.float32))


def test_preprocess_errors(ctx):
    from paper_1604_02292_amd import TomoError
    g = ctx.tomo_set_geometry(64, 5, 101)
    out = torch.empty((5, 101), dtype=torch.float32, device="cuda")
    with pytest.raises(TomoError, match="EINVAL"):
        ctx.tomo_pad_truncated(g, torch.zeros((5, 30), device="cuda"), 80, out)
    with pytest.raises(TomoError, match="EINVAL"):
        ctx.tomo_disc_add(g, (60, 0, 8, 8), torch.zeros(1, device="cuda"),
                          torch.zeros((8, 8), device="cuda"))


def test_truncated_data_pipeline_matches_oracle(ctx, c1):
    """The paper's truncated-data experiment at the small size: the central half of the
    detector measured, padded, disc subtracted, filtered, local FISTA-TV on the central
    part, disc added back."""
    from paper_1604_02292_amd import make_params
    cfg = c1["cfg"]
    n, na, nd = cfg["n"], cfg["n_angles"], cfg["n_det"]
    first, nb = 48, 96
    trunc = c1["sino"][:, first:first + nb].astype(np.float32)
    geo = oracle.make_geometry(n, na, nd)
    K, lam, nf = 25, 400.0, 40
    rect, m = (40, 40, 48, 48), 8
    padded = pad_truncated(trunc, first, nd)
    q, c = disc_subtract(geo, padded)
    U = sirt_filters(geo, K, workers=4)
    ref = disc_add(geo, local_fista_tv(geo, q, rect, m, U, lam, nf, 0.0, np.inf), rect, c)
    g = ctx.tomo_set_geometry(n, na, nd)
    P = torch.empty((na, nd), dtype=torch.float32, device="cuda")
    ctx.tomo_pad_truncated(g, _gpu(trunc), first, P)
    val = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.tomo_disc_subtract(g, P, P, val)
    F = torch.empty((K, na, nd), dtype=torch.float32, device="cuda")
    ctx.tomo_sirt_filters(g, K, F)
    D = torch.empty_like(F)
    ctx.tomo_sirt_filter_sino(g, F, P, D)
    out = torch.empty((rect[2], rect[3]), dtype=torch.float32, device="cuda")
    ctx.roi_solve_local(g, D, [make_params(rect, m, "fista", lam=lam, iters=K, inner_iters=nf,
                                           box=(0.0, float("inf")))], [out])
    ctx.tomo_disc_add(g, rect, val, out)
    torch.cuda.synchronize()
    e = rel(out.cpu().numpy(), ref)
    print(f"[truncated pipeline] c {val.item():.6f} (oracle {c:.6f}) rel {e:.2e}", flush=True)
    assert e <= 1e-3
