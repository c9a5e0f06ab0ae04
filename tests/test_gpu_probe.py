"""The ALU-roof calibration kernels (tomo_valu_probe) compute what they claim: every
lane's eight chains of v <- v a + b (mode 0), v <- fract(v a + b) (mode 1; the values
stay in [0, 1), so the fraction keeps them) and v <- v + b (mode 2), summed, against
the same recurrences in FP64 on the host (the only difference is FP32 rounding, far
below the bar), and their arguments are checked."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_valu_probe_computes_its_chains(mode):
    from paper_1604_02292_amd import Context, TomoError
    ctx = Context(0, workspace_bytes=1 << 20)
    try:
        blocks, iters, a, b = 3, 5, 0.999, 1e-3
        print(f"[valu probe] mode {mode}, {blocks} blocks, {iters} x 128 steps per lane", flush=True)
        out = torch.full((blocks * 256,), float("nan"), dtype=torch.float32, device="cuda")
        ctx.tomo_valu_probe(blocks, iters, a, b, out, mode=mode)
        torch.cuda.synchronize()
        af, bf = float(np.float32(a)), float(np.float32(b))
        lane = np.arange(256, dtype=np.float64)
        v = np.stack([np.float32(1e-3) * (lane + i).astype(np.float32) for i in range(8)])
        v = v.astype(np.float64)
        for _ in range(iters * 16):
            v = v + bf if mode == 2 else v * af + bf
        ref = np.tile(v.sum(axis=0), blocks)
        got = out.double().cpu().numpy()
        err = float(np.max(np.abs(got - ref) / np.abs(ref)))
        print(f"    max rel error {err:.2e}", flush=True)
        assert err <= 1e-5
        with pytest.raises(TomoError):
            ctx.tomo_valu_probe(0, iters, a, b, torch.empty(0, device="cuda"), mode=mode)
        with pytest.raises(TomoError):
            ctx.tomo_valu_probe(blocks, iters, a, b, out, mode=3)
    finally:
        ctx.close()
