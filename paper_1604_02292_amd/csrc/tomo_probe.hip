// Calibration of the projectors' ALU roof.  Not a step of the reconstruction: kernels
// whose lanes issue nothing but one or two classes of FP32 vector instructions, so
// that the rates at which the chip retires them can be measured on the same build and
// clock as the projectors, beside the nominal figures derived from the unit counts
// (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz per issue slot).
#include "tomo_runtime.h"

namespace tomo {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 8;    // independent dependency chains per lane
constexpr int kProbeUnroll = 16;   // steps per chain per loop trip

// Each lane runs iters x kProbeUnroll steps on each of eight independent chains
// (enough to cover the latency at one wave per SIMD), then stores the chains' sum so
// that none of the work is dead.  A step is, by MODE:
//   0  one FMA, v = v a + b                       (one class, a scalar operand)
//   1  an FMA then a fraction, v = fract(v a + b) (two classes the chip can pair)
//   2  one add, v = v + b                         (one class, a scalar operand: adds
//                                                  with vector operands only pair)
template <int MODE>
__global__ __launch_bounds__(kProbeThreads) void valu_probe_kernel(float* __restrict__ out,
                                                                   int iters, float a, float b) {
    float v[kProbeChains];
#pragma unroll
    for (int i = 0; i < kProbeChains; ++i) v[i] = (float)(threadIdx.x + i) * 1.0e-3f;
    for (int k = 0; k < iters; ++k) {
#pragma unroll
        for (int r = 0; r < kProbeUnroll; ++r)
#pragma unroll
            for (int i = 0; i < kProbeChains; ++i) {
                if constexpr (MODE == 0) v[i] = fmaf(v[i], a, b);
                if constexpr (MODE == 1) v[i] = __builtin_amdgcn_fractf(fmaf(v[i], a, b));
                if constexpr (MODE == 2) v[i] = v[i] + b;
            }
    }
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] =
        ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
}

}  // namespace
}  // namespace tomo

using namespace tomo;

extern "C" tomo_status tomo_valu_probe(tomo_ctx* ctx, int32_t blocks, int32_t iters, int32_t mode,
                                       float a, float b, float* out, void* hip_stream) {
    tomo_status st = need_gpu(ctx);
    if (st != TOMO_OK) return st;
    if (!out) return fail(ctx, TOMO_EINVAL, "null pointer");
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
        return fail(ctx, TOMO_EINVAL, "blocks and iters must lie in [1, 2^20]");
    const hipStream_t s = (hipStream_t)hip_stream;
    switch (mode) {
        case 0:
            hipLaunchKernelGGL(valu_probe_kernel<0>, dim3(blocks), dim3(kProbeThreads), 0, s, out,
                               iters, a, b);
            break;
        case 1:
            hipLaunchKernelGGL(valu_probe_kernel<1>, dim3(blocks), dim3(kProbeThreads), 0, s, out,
                               iters, a, b);
            break;
        case 2:
            hipLaunchKernelGGL(valu_probe_kernel<2>, dim3(blocks), dim3(kProbeThreads), 0, s, out,
                               iters, a, b);
            break;
        default:
            return fail(ctx, TOMO_EINVAL, "mode must be 0 (FMA), 1 (FMA + fraction) or 2 (add)");
    }
    TOMO_HIP(ctx, hipGetLastError());
    return TOMO_OK;
}
