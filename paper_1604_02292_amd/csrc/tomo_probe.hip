// Calibration of the projectors' ALU roof.  Not a step of the reconstruction: one
// kernel whose lanes issue nothing but FP32 fused multiply-adds, so that the rate
// at which the chip retires vector FP32 lane-instructions can be measured on the
// same build and clock as the projectors, beside the nominal figure derived from
// the unit counts (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz).
#include "tomo_runtime.h"

namespace tomo {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 8;    // independent dependency chains per lane
constexpr int kProbeUnroll = 16;   // FMAs per chain per loop trip

// Each lane runs iters x kProbeUnroll x kProbeChains FMAs v = v a + b over eight
// independent chains (enough to cover the FMA latency at one wave per SIMD), then
// stores the chains' sum so that none of the work is dead.
__global__ __launch_bounds__(kProbeThreads) void valu_probe_kernel(float* __restrict__ out,
                                                                   int iters, float a, float b) {
    float v[kProbeChains];
#pragma unroll
    for (int i = 0; i < kProbeChains; ++i) v[i] = (float)(threadIdx.x + i) * 1.0e-3f;
    for (int k = 0; k < iters; ++k) {
#pragma unroll
        for (int r = 0; r < kProbeUnroll; ++r)
#pragma unroll
            for (int i = 0; i < kProbeChains; ++i) v[i] = fmaf(v[i], a, b);
    }
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] =
        ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
}

}  // namespace
}  // namespace tomo

using namespace tomo;

extern "C" tomo_status tomo_valu_probe(tomo_ctx* ctx, int32_t blocks, int32_t iters, float a,
                                       float b, float* out, void* hip_stream) {
    tomo_status st = need_gpu(ctx);
    if (st != TOMO_OK) return st;
    if (!out) return fail(ctx, TOMO_EINVAL, "null pointer");
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
        return fail(ctx, TOMO_EINVAL, "blocks and iters must lie in [1, 2^20]");
    hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0,
                       (hipStream_t)hip_stream, out, iters, a, b);
    TOMO_HIP(ctx, hipGetLastError());
    return TOMO_OK;
}
