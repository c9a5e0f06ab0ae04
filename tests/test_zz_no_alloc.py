"""The allocation-free FBP entry point (tomo_fbp_ramlak_noalloc) against the
workspace-based one (tomo_fbp_ramlak), through the C ABI: two calls in a row, the
second on a smaller geometry, each bit-identical to the existing entry point (and
within the projector bar rel-L2 <= 1e-5), the context's workspace untouched, and a
geometry whose scratch exceeds the static array rejected with EINVAL."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_fbp_matches_workspace_fbp():
    from paper_1604_02292_amd import Context, TomoError
    from paper_1604_02292_amd import _lib
    ctx = Context(0, workspace_bytes=1 << 30)
    try:
        rng = np.random.default_rng(1604)
        for n, na, nd in [(1024, 128, 1536), (128, 32, 192)]:
            print(f"[noalloc fbp] grid {n}, {na} angles, {nd} bins", flush=True)
            g = ctx.tomo_set_geometry(n, na, nd)
            sino = torch.from_numpy(rng.random((na, nd)).astype(np.float32)).cuda()
            ref = torch.empty((n, n), dtype=torch.float32, device="cuda")
            got = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
            ctx.tomo_fbp_ramlak(g, sino, ref)
            torch.cuda.synchronize()
            used0, _ = ctx.tomo_workspace_usage()
            ctx.tomo_fbp_ramlak_noalloc(g, sino, got)
            torch.cuda.synchronize()
            used1, _ = ctx.tomo_workspace_usage()
            e = _rel(got, ref)
            print(f"    rel {e:.2e}, identical {bool(torch.equal(got, ref))}, workspace "
                  f"{used0} -> {used1} bytes", flush=True)
            assert e <= 1e-5
            assert torch.equal(got, ref)
            assert used1 == used0
        # scratch beyond the static array: rejected on the host before any launch
        g = ctx.tomo_set_geometry(8192, 1024, 12288)
        big = torch.zeros((1024, 12288), dtype=torch.float32, device="cuda")
        out = torch.empty((8192, 8192), dtype=torch.float32, device="cuda")
        with pytest.raises(TomoError) as ei:
            ctx.tomo_fbp_ramlak_noalloc(g, big, out)
        assert ei.value.status == _lib.TOMO_EINVAL
        assert "scratch" in str(ei.value)
    finally:
        ctx.close()
