// HIP kernels for gfx950 (MI355X): Joseph forward projection, matched
// backprojection with the fused TV / prox epilogues of the Chambolle-Pock and
// SIRT iterations, the Ram-Lak filter and small helpers.
//
// Operators (paper Section 2.1): W with entries
//   w[(k,i),(r,c)] = max(0, 1 - |s_i - t_rc| / m_k) / m_k,  t_rc = x_c cos + y_r sin,
// applied on the fly; local operators W_L = W M_L, W_L^T = M_L W^T.
// Everything here is FP32 arithmetic except the ray / pixel positions, which
// are anchored in FP64: a 4096-pixel grid needs more than FP32's 24 bits to
// place a ray to 1e-5 of a pixel.
//
// Nothing here is a dense contraction, so there is no MFMA: the projectors are
// gathers bound by the vector ALU and the load path, the epilogues by HBM.

#include <algorithm>
#include <type_traits>

#include "tomo_internal.h"

namespace tomo {

namespace {

// Logical work item for hardware block b.  The grid is a multiple of 8 and
// consecutive blocks are dealt round-robin to the 8 XCDs.  With `contiguous`
// set, XCD x gets the x-th eighth of the item list, so the items of one ROI
// (adjacent in the list) share that XCD's L2; otherwise item b runs on XCD
// b mod 8, which balances the XCDs for any mix of item costs.
__device__ __forceinline__ int xcd_remap(int b, int G, int contiguous) {
    return contiguous ? (b & 7) * (G >> 3) + (b >> 3) : b;
}

// Smallest s with s * s > v (compile time).
constexpr int isqrt_above(int v) {
    int s = 0;
    while (s * s <= v) ++s;
    return s;
}

// Neumaier's compensated sum: s + c carries s + t with the rounding error of
// the FP32 addition kept in c (Neumaier 1974, improved Kahan-Babuska sum).
__device__ __forceinline__ void comp_add(float& s, float& c, float t) {
    const float u = s + t;
    c += (fabsf(s) >= fabsf(t)) ? ((s - u) + t) : ((t - u) + s);
    s = u;
}

__device__ __forceinline__ int uniform_int(int v) {
    return __builtin_amdgcn_readfirstlane(v);
}

// Address-space views: tables and job descriptors are read through the
// constant space (scalar loads into SGPRs), images and bands through the
// global space (global_load with a scalar base), not through flat pointers.
#if defined(__HIP_DEVICE_COMPILE__)
#define CONST_AS __attribute__((address_space(4)))
#define GLOBAL_AS __attribute__((address_space(1)))
#define LDS_AS __attribute__((address_space(3)))
#else   // the host pass only needs the declarations
#define CONST_AS
#define GLOBAL_AS
#define LDS_AS
#endif
typedef const GLOBAL_AS float gcfloat;

template <typename T>
__device__ __forceinline__ const CONST_AS T* cview(const T* p) {
    return (const CONST_AS T*)(p);
}
__device__ __forceinline__ gcfloat* gview(const float* p) { return (gcfloat*)(p); }

// Raw buffer loads: a scalar resource for the whole array, a 32-bit per-lane
// byte offset and a scalar byte offset for the row.  Word 3 is the raw
// 32-bit-data format of gfx9-family buffer resources.
typedef float v2f __attribute__((ext_vector_type(2)));

// A tile's per-angle anchor in LDS: FP32 fraction (+ shift PSH) and the
// integer part I as the byte offset 4 (I - PSH).
struct Anchor {
    float f;
    int i4;
};
// A staged band window in LDS: the anchor fraction (+ shift) and the LDS byte
// address that band coordinate (integer part of the anchor - shift) maps to.
struct WinMeta {
    float f;
    unsigned base;
};
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float* p, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}
#if defined(__HIP_DEVICE_COMPILE__)   // distinct from const float* only in the device pass
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(gcfloat* p, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}
#endif
__device__ __forceinline__ v2f load2(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}
typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4f load4(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
}

// Epilogue operands of ray j (band position) of angle k: the values the forward
// projector's mode combines with the ray sum (0 for rays off the band or detector).
__device__ __forceinline__ void fp_operands(const CONST_AS Job* J, const AngFP& A, int k, int j,
                                            int step, float& pre0, float& pre1) {
    const int gi = A.i0 + j;
    if (j >= A.w || gi < 0 || gi >= J->n_det) return;
    const size_t bidx = (size_t)k * J->bpitch + 1 + j;
    const size_t gidx = (size_t)k * J->n_det + gi;
    switch (J->fp_mode) {
        case FP_ACCUM: pre0 = J->gout[gidx]; break;
        case FP_BAND_FROM_GLOBAL:
        case FP_RESID:
        case FP_FILTER: pre0 = J->gbase[gidx]; break;
        case FP_LOCAL:
            pre0 = J->gbase[(size_t)(step + J->dk0) * (size_t)J->gstride + gidx];
            break;
        case FP_BAND_ADD: pre0 = J->y[bidx]; break;
        case FP_CP_DUAL: pre0 = J->y[bidx]; pre1 = J->b[bidx]; break;
        case FP_SIRT: pre1 = J->b[bidx]; break;
        default: break;
    }
}

// The forward projector's fused epilogue for ray j of angle k with ray sum acc.
__device__ __forceinline__ void fp_store(const CONST_AS Job* J, const AngFP& A, int k, int j,
                                         float acc, float pre0, float pre1) {
    float* y = J->y;
    float* gout = J->gout;
    const int gi = A.i0 + j;
    const bool ondet = (gi >= 0) && (gi < J->n_det);
    const size_t bidx = (size_t)k * J->bpitch + 1 + j;
    const size_t gidx = (size_t)k * J->n_det + gi;
    const float fpv = acc * A.inv_m;
    const int mode = J->fp_mode;
    switch (mode) {
        case FP_STORE:
            if (ondet) gout[gidx] = fpv;
            break;
        case FP_ACCUM:
            if (ondet) gout[gidx] = pre0 + fpv;
            break;
        case FP_BAND_FROM_GLOBAL:
            y[bidx] = ondet ? pre0 + J->scale * fpv : 0.f;
            break;
        case FP_BAND_ADD:
            y[bidx] = ondet ? pre0 + J->scale * fpv : 0.f;
            break;
        case FP_CP_DUAL:
            // prox of sigma F1*, F1(v) = ||v - h b||^2 (or 1/2 ||v - h b||^2) on the rows
            // h W_L of K, kept as B * h y: h y <- (h y + sigma h^2 (W_L xbar - b)) / (1 + sigma/2)
            y[bidx] = ondet ? (pre0 + (J->sigma_y * A.bscale) * (fpv - pre1)) * J->dual_div : 0.f;
            break;
        case FP_SIRT:
            y[bidx] = ondet ? (J->alpha * A.bscale) * (pre1 - fpv) : 0.f;
            break;
        case FP_BAND_STORE:
            y[bidx] = ondet ? A.bscale * fpv : 0.f;
            break;
        case FP_RESID:
            if (ondet) gout[gidx] = pre0 + J->scale * fpv;
            break;
        case FP_FILTER:
            // one step of the filter recursion: the band carries -alpha W c for
            // the update of c, the filter accumulates alpha W c
            y[bidx] = ondet ? -(J->alpha * A.bscale) * fpv : 0.f;
            if (ondet) gout[gidx] = pre0 + J->alpha * fpv;
            break;
        case FP_LOCAL: {
            // two-channel band: (d - alpha W_L v, d), d the filtered data
            const float d = ondet ? pre0 : 0.f;
            const v2f o = ondet ? v2f{A.bscale * (d - J->alpha * fpv), A.bscale * d}
                                : v2f{0.f, 0.f};
            *(v2f*)(y + 2 * bidx) = o;
        } break;
        default:
            break;
    }
}

// ---------------------------------------------------------------------------
// Forward projection.  One block = one angle of one job and 64 * max(4, SEG) / SEG
// rays (4 waves, or SEG waves when SEG > 4); each ray is split into SEG consecutive
// segments of outer lines (rows, or columns for |sin| > |cos|) handled by different
// waves and summed in a fixed order.  A wave's 64 lanes are 64 adjacent rays, so at every outer line they
// read nearly contiguous pixels of one image row (the transposed copy of the
// image serves the column-stepping angles, keeping those reads contiguous).
// ---------------------------------------------------------------------------
template <int SEG>
constexpr int fp_threads() { return SEG > 4 ? 64 * SEG : 256; }

template <int SEG, int RP>
__global__ __launch_bounds__(fp_threads<SEG>()) void fp_kernel(const Job* __restrict__ jobs,
                                                 const Item* __restrict__ items, int n_items,
                                                 int step, int contiguous) {
    constexpr int NT = fp_threads<SEG>(), SUBS = NT / 64 / SEG;
    __shared__ float red[SEG > 1 ? RP * NT : 1];
    const int bid = xcd_remap(blockIdx.x, gridDim.x, contiguous);
    if (bid >= n_items) return;
    const Item it = cview(items)[bid];
    const CONST_AS Job* J = cview(jobs) + it.job;
    const int k = it.a;
    const AngFP A = *cview((const AngFP*)it.tab);
    const int lane = threadIdx.x & 63;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int seg = wave % SEG;
    const int sub = wave / SEG;
    const int jfirst = (it.b * SUBS + sub) * 64 * RP;   // a wave: 64 RP adjacent rays
    const int j0 = jfirst + RP * lane;                  // this lane: rays j0 .. j0 + RP - 1
    const int rpar = (step + J->parity0) & 1;
    gcfloat* img = gview(A.tr ? J->xt : J->xb[rpar]);
    const int pitch = A.tr ? J->tp : J->xp;
    const int n_outer = A.tr ? J->nc : J->nr;
    const int n_inner = A.tr ? J->nr : J->nc;

    // Epilogue operands are independent of the ray sums: fetch them first so
    // their memory latency overlaps the loop.
    float pre0[RP], pre1[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
        pre0[r] = pre1[r] = 0.f;
        if (seg == 0) fp_operands(J, A, k, j0 + r, step, pre0[r], pre1[r]);
    }

    float acc[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) acc[r] = 0.f;
    if (jfirst < A.w) {
        const int jlast = min(jfirst + 64 * RP - 1, A.w - 1);
        // Outer lines where some ray of this wave lies strictly inside the image
        // columns' interpolation range (kLpad - 1, n_inner + kLpad) of storage
        // coordinates; outside it every weight is 0.
        const double pa = A.a0 + (double)jfirst * A.aj;
        const double pb = A.a0 + (double)jlast * A.aj;
        const double lo_in = (double)(kLpad - 1), hi_in = (double)(n_inner + kLpad);
        int o_lo = 0, o_hi = 0;
        if (A.step == 0.0) {
            const bool any = (fmax(pa, pb) > lo_in) && (fmin(pa, pb) < hi_in);
            o_hi = any ? n_outer : 0;
        } else {
            const double inv = 1.0 / A.step;
            const double t1 = (lo_in - pa) * inv, t2 = (hi_in - pa) * inv;
            const double t3 = (lo_in - pb) * inv, t4 = (hi_in - pb) * inv;
            double lo = fmin(fmin(t1, t2), fmin(t3, t4));
            double hi = fmax(fmax(t1, t2), fmax(t3, t4));
            lo = fmin(fmax(lo, -2.0), (double)n_outer + 2.0);
            hi = fmin(fmax(hi, -2.0), (double)n_outer + 2.0);
            o_lo = max(0, (int)floor(lo) - 1);
            o_hi = min(n_outer, (int)ceil(hi) + 2);
        }
        o_lo = uniform_int(o_lo);
        o_hi = uniform_int(o_hi);
        const int len = max(0, o_hi - o_lo);
        const int s0 = o_lo + (len * seg) / SEG;
        const int s1 = o_lo + (len * (seg + 1)) / SEG;
        const float stepf = (float)A.step;
        const unsigned rowb = (unsigned)pitch * 4u;
        // Each outer line is read through its own buffer resource whose range is
        // that line: a read past its end returns 0 per element from the hardware
        // range check, and the line holds kLpad zeros before its first pixel
        // (so no read starts before it), so no position clamp is needed.
        // 32 outer lines per FP64 anchor: pos = I + loc with loc within 64 +- 34,
        // so the FP32 part carries a few 1e-6 of a pixel at any grid size; the
        // +64 shift makes truncation a floor and fract the interpolation weight.
        if constexpr (RP == 1) {
            const double pj = A.a0 + (double)j0 * A.aj;
            for (int oc = s0; oc < s1; oc += 32) {
                const double p0 = fma((double)oc, A.step, pj);
                const double fl0 = fmin(fmax(floor(p0), -1.0e6), 1.0e6);
                const float base64 = (float)(p0 - fl0) + 64.f;
                unsigned ib4 = (unsigned)((int)fl0 - 64) * 4u;
                asm("" : "+v"(ib4));   // keeps (index << 2) + ib4 a single shift-add
                const int cnt = min(32, s1 - oc);
                gcfloat* line = img + (size_t)oc * pitch;
                // two-level sum: the chunk's terms first, then the chunk into the ray
                // (long rays of a large grid keep a few ulp of the full sum)
                float cs = 0.f;
                int q = 0;
                if (cnt == 32) {
                    // a full chunk: all 32 paired loads issue before the first is used
                    float f[32];
                    v2f v[32];
#pragma unroll
                    for (int u = 0; u < 32; ++u) {
                        const float loc = fmaf((float)u, stepf, base64);
                        f[u] = __builtin_amdgcn_fractf(loc);
                        const unsigned off = ((unsigned)loc << 2) + ib4;
                        v[u] = load2(make_rsrc(line + (size_t)u * pitch, rowb), off, 0);
                    }
#pragma unroll
                    for (int u = 0; u < 32; ++u) cs += fmaf(f[u], v[u].y - v[u].x, v[u].x);
                    q = 32;
                }
                for (; q + 8 <= cnt; q += 8) {
                    const float b8 = fmaf((float)q, stepf, base64);
                    float f[8];
                    v2f v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float loc = fmaf((float)u, stepf, b8);
                        f[u] = __builtin_amdgcn_fractf(loc);
                        const unsigned off = ((unsigned)loc << 2) + ib4;
                        v[u] = load2(make_rsrc(line + (size_t)(q + u) * pitch, rowb), off, 0);
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) cs += fmaf(f[u], v[u].y - v[u].x, v[u].x);
                }
                for (; q < cnt; ++q) {
                    const float loc = fmaf((float)q, stepf, base64);
                    const float f = __builtin_amdgcn_fractf(loc);
                    const unsigned off = ((unsigned)loc << 2) + ib4;
                    const v2f v = load2(make_rsrc(line + (size_t)q * pitch, rowb), off, 0);
                    cs += fmaf(f, v.y - v.x, v.x);
                }
                acc[0] += cs;
            }
        } else if (fabs(A.aj) >= 2.0) {
            // detector spacing of sqrt 2 pixels or more: the two rays are too far
            // apart for one 4-pixel read, so each reads its own pairs
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const double pj = A.a0 + (double)(j0 + r) * A.aj;
                for (int oc = s0; oc < s1; oc += 32) {
                    const double p0 = fma((double)oc, A.step, pj);
                    const double fl0 = fmin(fmax(floor(p0), -1.0e6), 1.0e6);
                    const float base64 = (float)(p0 - fl0) + 64.f;
                    const unsigned ib4 = (unsigned)((int)fl0 - 64) * 4u;
                    const int cnt = min(32, s1 - oc);
                    gcfloat* line = img + (size_t)oc * pitch;
                    float cs = 0.f;
                    for (int q = 0; q < cnt; ++q) {
                        const float loc = fmaf((float)q, stepf, base64);
                        const float f = __builtin_amdgcn_fractf(loc);
                        const unsigned off = ((unsigned)loc << 2) + ib4;
                        const v2f v = load2(make_rsrc(line + (size_t)q * pitch, rowb), off, 0);
                        cs += fmaf(f, v.y - v.x, v.x);
                    }
                    acc[r] += cs;
                }
            }
        } else {
            // Two adjacent rays per lane from one 4-pixel read: at every line the
            // lower-positioned ray sits at loc (pixels i, i+1 of the read) and the
            // other at loc + |aj|, 1 <= |aj| < 2 bins apart, i.e. at t = f + |aj| - 1
            // in [0, 2) from pixel i+1: the piecewise-linear interpolation
            // v1 + clamp(t)(v2 - v1) + clamp(t - 1)(v3 - v2) over the same read.
            const int lo_r = A.aj < 0.0 ? 1 : 0;      // which of the two is lower
            const double pj = A.a0 + (double)(j0 + lo_r) * A.aj;
            const float c1 = (float)(fabs(A.aj) - 1.0);
            const float c2 = (float)(fabs(A.aj) - 2.0);
            float cl = 0.f, ch = 0.f;
            for (int oc = s0; oc < s1; oc += 32) {
                const double p0 = fma((double)oc, A.step, pj);
                const double fl0 = fmin(fmax(floor(p0), -1.0e6), 1.0e6);
                const float base64 = (float)(p0 - fl0) + 64.f;
                unsigned ib4 = (unsigned)((int)fl0 - 64) * 4u;
                asm("" : "+v"(ib4));
                const int cnt = min(32, s1 - oc);
                gcfloat* line = img + (size_t)oc * pitch;
                float sl = 0.f, sh = 0.f;
                int q = 0;
                auto term = [&](float f, v4f v) {
                    sl += fmaf(f, v.y - v.x, v.x);
                    const float w1 = __builtin_amdgcn_fmed3f(f + c1, 0.f, 1.f);
                    const float w2 = __builtin_amdgcn_fmed3f(f + c2, 0.f, 1.f);
                    sh += v.y;
                    sh = fmaf(w1, v.z - v.y, sh);
                    sh = fmaf(w2, v.w - v.z, sh);
                };
                if (cnt == 32) {
                    float f[32];
                    v4f v[32];
#pragma unroll
                    for (int u = 0; u < 32; ++u) {
                        const float loc = fmaf((float)u, stepf, base64);
                        f[u] = __builtin_amdgcn_fractf(loc);
                        const unsigned off = ((unsigned)loc << 2) + ib4;
                        v[u] = load4(make_rsrc(line + (size_t)u * pitch, rowb), off, 0);
                    }
#pragma unroll
                    for (int u = 0; u < 32; ++u) term(f[u], v[u]);
                    q = 32;
                }
                for (; q + 8 <= cnt; q += 8) {
                    const float b8 = fmaf((float)q, stepf, base64);
                    float f[8];
                    v4f v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float loc = fmaf((float)u, stepf, b8);
                        f[u] = __builtin_amdgcn_fractf(loc);
                        const unsigned off = ((unsigned)loc << 2) + ib4;
                        v[u] = load4(make_rsrc(line + (size_t)(q + u) * pitch, rowb), off, 0);
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) term(f[u], v[u]);
                }
                for (; q < cnt; ++q) {
                    const float loc = fmaf((float)q, stepf, base64);
                    const unsigned off = ((unsigned)loc << 2) + ib4;
                    term(__builtin_amdgcn_fractf(loc),
                         load4(make_rsrc(line + (size_t)q * pitch, rowb), off, 0));
                }
                cl += sl;
                ch += sh;
            }
            acc[lo_r] = cl;
            acc[1 - lo_r] = ch;
        }
    }
    if (SEG > 1) {
#pragma unroll
        for (int r = 0; r < RP; ++r) red[r * NT + threadIdx.x] = acc[r];
        __syncthreads();
        if (seg != 0) return;
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            acc[r] = 0.f;
#pragma unroll
            for (int q = 0; q < SEG; ++q) acc[r] += red[r * NT + (sub * SEG + q) * 64 + lane];
        }
    }

#pragma unroll
    for (int r = 0; r < RP; ++r) {
        if (j0 + r >= A.w) break;
        fp_store(J, A, k, j0 + r, acc[r], pre0[r], pre1[r]);
    }
}

// ---------------------------------------------------------------------------
// Forward projection, LDS-staged (the throughput shape for batches).  One block =
// a group of angles of one job that step along the same image lines (rows, or
// columns through the transposed copy) and all rays of their bands.  The block
// copies L whole padded lines of the region at a time into LDS with
// coalesced reads - each pixel is read once per group instead of once per ray that
// crosses it - stored column-major with an odd stride, so that a ray's two taps are
// one ds_read2 and adjacent rays fall on distinct banks.  The (angle, ray) pairs of
// the group are dealt to the threads in rounds, the angles of one ray adjacent, and
// every pair takes its interpolation steps from LDS.  A wave skips a stage when none
// of its rays meets the image inside the staged lines; zero columns on both sides of
// the staged lines give the exact zeros that the direct kernel's range-checked reads
// give, so no tap index is clamped.  Ray sums run in the same two levels as
// fp_kernel: per chunk of staged lines, then into the ray.
// ---------------------------------------------------------------------------
// Six waves per SIMD (three eight-wave blocks per CU, which the LDS stages allow):
// gfx950 pairs independent VALU instructions of different waves (an FMA with a
// fraction or conversion, adds with anything), and this kernel's mix needs that many
// waves to keep both issue slots busy.
template <int L>
__global__ __launch_bounds__(kFpsThreads, 6) void fp_staged_kernel(const Job* __restrict__ jobs,
                                                                const Item* __restrict__ items,
                                                                int n_items, int step,
                                                                int contiguous) {
    // [ZP + pitch + ZP][STR]: the staged lines, column-major, with
    // zero columns on both sides
    extern __shared__ float fps_lds[];
    constexpr int NT = kFpsThreads, STR = L + 1, ZP = L + 2;
    static_assert(L <= 32, "a stage's rays must stay inside the zero columns");
    static_assert(L % 8 == 0, "a full stage runs in chunks of eight lines");
    const int bid = xcd_remap(blockIdx.x, gridDim.x, contiguous);
    if (bid >= n_items) return;
    const Item it = cview(items)[bid];
    const CONST_AS Job* J = cview(jobs) + it.job;
    const int k0 = it.a, W = it.b, nang = it.pad;   // angles k0 .. k0 + nang - 1, W pair slots each
    if (W <= 0 || nang <= 0) return;
    const AngFP* tabs = (const AngFP*)it.tab;
    const int t = threadIdx.x, lane = t & 63;
    const int tr = cview(tabs)[0].tr;
    const int rpar = (step + J->parity0) & 1;
    gcfloat* img = gview(tr ? J->xt : J->xb[rpar]);
    const int pitch = tr ? J->tp : J->xp;
    const int n_outer = tr ? J->nc : J->nr;
    const int n_inner = tr ? J->nr : J->nc;
    const int npairs = nang * W;
    const int rounds = (npairs + NT - 1) / NT;
    if (rounds > kFpsMaxRounds) return;   // the host never builds such a group
    LDS_AS float* S = (LDS_AS float*)fps_lds + ZP * STR;   // column 0 of the line
    const unsigned s_base = (unsigned)(size_t)S;
    // pair p = ray j * nang + angle a: a wave holds the same few rays of every angle of
    // the group, whose line ranges nearly coincide (adjacent rays of one angle enter and
    // leave the region over a slanted front, which would idle lanes of a wave), and whose
    // taps fall on few adjacent columns (distinct banks, or the same address)
    const float rcp_n = 1.0f / (float)nang;
    const unsigned rowb = (unsigned)pitch * 4u;
    const __amdgpu_buffer_rsrc_t img_rs = make_rsrc(img, (size_t)n_outer * rowb);

    // Lines on which some ray of the group lies strictly inside the interpolation
    // range (kLpad - 1, n_inner + kLpad) of storage coordinates: lane a of every wave
    // takes angle a (rays 0 and w - 1 bound its range), then a wave-wide min / max.
    const double lo_in = (double)(kLpad - 1), hi_in = (double)(n_inner + kLpad);
    int o_lo = n_outer, o_hi = 0;
    for (int a0 = 0; a0 < nang; a0 += 64) {
        const int a = a0 + lane;
        int lo_a = n_outer, hi_a = 0;
        if (a < nang) {
            const AngFP A = tabs[a];
            if (A.w > 0) {
                const double pa = A.a0, pb = A.a0 + (double)(A.w - 1) * A.aj;
                if (A.step == 0.0) {
                    if ((fmax(pa, pb) > lo_in) && (fmin(pa, pb) < hi_in)) {
                        lo_a = 0;
                        hi_a = n_outer;
                    }
                } else {
                    const double inv = 1.0 / A.step;
                    const double t1 = (lo_in - pa) * inv, t2 = (hi_in - pa) * inv;
                    const double t3 = (lo_in - pb) * inv, t4 = (hi_in - pb) * inv;
                    double lo = fmin(fmin(t1, t2), fmin(t3, t4));
                    double hi = fmax(fmax(t1, t2), fmax(t3, t4));
                    lo = fmin(fmax(lo, -2.0), (double)n_outer + 2.0);
                    hi = fmin(fmax(hi, -2.0), (double)n_outer + 2.0);
                    lo_a = max(0, (int)floor(lo) - 1);
                    hi_a = min(n_outer, (int)ceil(hi) + 2);
                    if (hi_a <= lo_a) {
                        lo_a = n_outer;
                        hi_a = 0;
                    }
                }
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            lo_a = min(lo_a, __shfl_xor(lo_a, d));
            hi_a = max(hi_a, __shfl_xor(hi_a, d));
        }
        o_lo = min(o_lo, lo_a);
        o_hi = max(o_hi, hi_a);
    }
    o_lo = uniform_int(o_lo);
    o_hi = uniform_int(o_hi);
    // The zero columns: a ray that meets the image inside a stage stays within L - 1
    // line steps (|step| <= 1) of it, so its taps fall in [2 - L, pitch + L] and need no
    // clamp (the first four and last two entries of a padded line are zeros too).
    for (int e = t; e < ZP * STR; e += NT) {
        S[-ZP * STR + e] = 0.f;
        S[pitch * STR + e] = 0.f;
    }
    // Per round: this thread's pair (angle a, ray j), its ray's storage coordinate at
    // line o_lo and step per line (FP64), kept in registers across the stages.
    double pb[kFpsMaxRounds], ps[kFpsMaxRounds];
    float acc[kFpsMaxRounds];
    bool val[kFpsMaxRounds];
#pragma unroll
    for (int r = 0; r < kFpsMaxRounds; ++r) {
        acc[r] = 0.f;
        pb[r] = 0.0;
        ps[r] = 0.0;
        val[r] = false;
        if (r < rounds) {
            const int p = r * NT + t;
            const int j = (int)(((float)p + 0.5f) * rcp_n);   // exact: p < 2^12, nang <= 64
            const int a = p - j * nang;
            const AngFP A = tabs[a];
            val[r] = (p < npairs) && (j < A.w);
            pb[r] = fma((double)o_lo, A.step, fma((double)j, A.aj, A.a0));
            ps[r] = A.step;
        }
    }

    for (int oc = o_lo; oc < o_hi; oc += L) {
        const int cnt = min(L, o_hi - oc);
        __syncthreads();   // the previous stage's readers are done
        // (lines past the region's last read 0 from the buffer's range check; lines
        // past the stage's count are staged but never read)
        for (int i = t; i < pitch; i += NT) {
            float v[L];
#pragma unroll
            for (int u = 0; u < L; ++u)
                v[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                     img_rs, (unsigned)i * 4u,
                                                     (unsigned)(oc + u) * rowb, 0));
#pragma unroll
            for (int u = 0; u < L; ++u) S[i * STR + u] = v[u];
        }
        __syncthreads();
        const double doc = (double)(oc - o_lo);
#pragma unroll
        for (int r = 0; r < kFpsMaxRounds; ++r) {
            if (r >= rounds) break;
            // storage coordinate of the ray at line oc, and at the stage's last line
            double p0 = fma(doc, ps[r], pb[r]);
            double dp = ps[r];
            const double p1 = fma((double)(cnt - 1), dp, p0);
            const double pmin = fmin(p0, p1), pmax = fmax(p0, p1);
            const bool touches = val[r] && (pmax > lo_in - 1.0) && (pmin < hi_in + 1.0);
            if (__ballot(touches) == 0) continue;   // only exact zeros on these lines
            if (!touches) {   // reads of the leading zeros, discarded or adding 0
                p0 = 2.0;
                dp = 0.0;
            }
            const double fl0 = floor(p0);
            const float base64 = (float)(p0 - fl0) + 64.f;
            const float stepf = (float)dp;
            const int ib = (int)fl0 - 64;
            // loc = base64 + u step lies in [65 - L, 63 + L) (|step| <= 1, u < L <= 32):
            // positive, so the truncation below is a floor
            const unsigned lb = (unsigned)(ib * STR) * 4u + s_base;
            // four partial sums (independent add chains), combined in a fixed order
            float c4[4] = {0.f, 0.f, 0.f, 0.f};
            if (cnt == L) {
                // line u of the tap's column sits u floats further: an immediate offset
                // of the ds_read2 (u, u + STR dwords).  Eight lines' operands at a time
                // keep the registers few enough for several waves per SIMD (the summation
                // order is the same as for the whole stage at once).
#pragma unroll
                for (int u0 = 0; u0 < L; u0 += 8) {
                    float f[8], v0[8], v1[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int u = u0 + e;
                        const float loc = fmaf((float)u, stepf, base64);
                        f[e] = __builtin_amdgcn_fractf(loc);
                        const LDS_AS float* col = (const LDS_AS float*)(size_t)(
                            __umul24((unsigned)loc, STR * 4u) + lb);
                        v0[e] = col[u];
                        v1[e] = col[u + STR];
                    }
#pragma unroll
                    for (int e = 0; e < 8; ++e) c4[e & 3] += fmaf(f[e], v1[e] - v0[e], v0[e]);
                }
            } else {
                // the stage's last lines: four at a time into the four sums, the rest
                // into the first
                auto tap = [&](int u) {
                    const float loc = fmaf((float)u, stepf, base64);
                    const float f = __builtin_amdgcn_fractf(loc);
                    const LDS_AS float* col = (const LDS_AS float*)(size_t)(
                        __umul24((unsigned)loc, STR * 4u) + lb + 4u * (unsigned)u);
                    return fmaf(f, col[STR] - col[0], col[0]);
                };
                int u = 0;
                for (; u + 4 <= cnt; u += 4) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) c4[q] += tap(u + q);
                }
                for (; u < cnt; ++u) c4[0] += tap(u);
            }
            acc[r] += (c4[0] + c4[1]) + (c4[2] + c4[3]);
        }
    }
    // fused epilogue of every valid pair
#pragma unroll
    for (int r = 0; r < kFpsMaxRounds; ++r) {
        if (r >= rounds) break;
        const int p = r * NT + t;
        if (!val[r]) continue;
        const int j = (int)(((float)p + 0.5f) * rcp_n);
        const int a = p - j * nang;
        const AngFP A = tabs[a];
        float pre0 = 0.f, pre1 = 0.f;
        fp_operands(J, A, k0 + a, j, step, pre0, pre1);
        fp_store(J, A, k0 + a, j, acc[r], pre0, pre1);
    }
}

// ---------------------------------------------------------------------------
// Backprojection (pixel-driven gather: no atomics, bit-reproducible).  One
// block = one tile of 256/AG threads of one job (64 when AG = 8: 8-wave
// blocks), each thread owning PPT vertically adjacent pixels; each pixel's
// angles are split into AG contiguous groups summed in a fixed order.  For the CP mode the block first computes
// the TV dual update on its tile plus a one-pixel top/left halo (from the
// previous xbar and z, which are double-buffered so neighbouring tiles never
// see half-updated values), takes its divergence, then applies the primal
// prox and the extrapolation to its own pixels.
// ---------------------------------------------------------------------------
template <int AG>
constexpr int bp_threads() { return AG > 4 ? 64 * AG : 256; }

template <int AG, int PPT, bool STAGED, bool COMP, bool TWO>
__global__ __launch_bounds__(bp_threads<AG>(), STAGED ? (TWO ? 6 : 8) : 1) void bp_kernel(const Job* __restrict__ jobs,
                                                 const Item* __restrict__ items, int n_items,
                                                 int step, int contiguous) {
    constexpr int NT = bp_threads<AG>();     // 4 waves, or one wave per group beyond 4
    constexpr int P = NT / AG;               // threads per angle group (a multiple of 64)
    constexpr int TW = (AG >= 4) ? 8 : 16;
    constexpr int TH = (P / TW) * PPT;       // pixel rows of the tile
    __shared__ float xs[TH + 2][TW + 2];
    __shared__ float zs0[TH + 1][TW + 1];
    __shared__ float zs1[TH + 1][TW + 1];
    __shared__ float red[PPT][AG > 1 ? NT : 1];   // group partial sums (and the power sums)
    __shared__ float red2[PPT][(AG > 1 && TWO) ? NT : 1];   // second channel's partial sums
    static_assert(!TWO || !COMP, "two-channel bands are not compensated");
    constexpr int CH = TWO ? 2 : 1;   // floats per band entry
    // Per-angle anchors of the tile, ANC per pass (AG groups x PA angles).
    constexpr int ANC = STAGED ? 256 : 512, PA = ANC / AG;   // (sized for LDS occupancy)
    // Staged band windows: WS entries per angle starting SHIFT below the
    // anchor; a pixel's offset from the anchor is at most
    // sqrt((TW/2)^2 + (TH/2)^2) <= 18 bins, so its pair lies inside the window.
    // In FP32 the anchor fraction carries the smaller shift PSH (> that offset),
    // which keeps the coordinate positive and its rounding error small.
    constexpr int SHIFT = 32, WS = 64;
    constexpr int PSH = isqrt_above((TW / 2) * (TW / 2) + (TH / 2) * (TH / 2)) + 1;
    static_assert(PSH <= SHIFT, "pixel offsets exceed the window");
    // per stage: angles per group, windows, windows per wave.  16 windows of 64 entries
    // keep the single-channel block at 18 KB of LDS and, with the launch bounded to
    // eight waves per SIMD, 62 VGPRs: eight blocks per CU, which pays for the extra
    // stage barriers (32 windows per stage allowed six).  The two-channel block (27 KB)
    // is bounded to six waves, the most its LDS allows.
    constexpr int KA = 16 / AG, NW = AG * KA, WPW = NW / 4;
    static_assert(TW * TW + TH * TH <= 36 * 36, "tile too large for the band window");
    __shared__ Anchor anc[ANC];
    // [guard][buffer 0: NW windows][buffer 1][guard]: stray lanes of ragged tiles
    // stay inside the guards
    __shared__ float win[STAGED ? (2 * NW + 2) * WS * CH : 1];
    __shared__ WinMeta wmeta[2][STAGED ? NW : 1];

    const int bid = xcd_remap(blockIdx.x, gridDim.x, contiguous);
    if (bid >= n_items) return;
    const Item it = cview(items)[bid];
    const CONST_AS Job* J = cview(jobs) + it.job;
    const int R0 = it.a * TH, C0 = it.b * TW;
    const int t = threadIdx.x;
    const int g = uniform_int(t / P);      // P is a multiple of 64: one group per wave
    const int p = t % P;
    const int tr = (p / TW) * PPT, tc = p % TW;   // first own pixel in the tile
    const int c = C0 + tc;
    const int nr = J->nr, nc = J->nc;
    const int mode = J->bp_mode;
    const int rpar = (step + J->parity0) & 1, wpar = rpar ^ 1;
    const bool tv = (mode == BP_CP) || (mode == BP_POWER);
    bool inside[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) inside[q] = (R0 + tr + q < nr) && (c < nc);

    // Tile anchors (FP64): the padded band coordinate of the tile's reference
    // point (C0 + TW/2, R0 + TH/2) for each angle, split into an integer part kept
    // and a fraction + PSH in FP32.  A pixel's coordinate is
    // the anchor plus its offset inside the tile, |offset| <= max(TW, TH)/2 * sqrt 2
    // < PSH, so the FP32 value stays positive (truncation = floor) and small.
    const int na = J->n_angles;
    const CONST_AS AngBP* tab = cview((const AngBP*)it.tab);
    const int npass = ((na + AG - 1) / AG + PA - 1) / PA;
    auto fill_anchors = [&](int pass) {
        for (int e = t; e < ANC; e += NT) {
            const int gg = e / PA;
            const int kk = (na * gg) / AG + pass * PA + e % PA;
            if (kk < (na * (gg + 1)) / AG) {
                const double T = fma((double)C0 + 0.5 * TW, tab[kk].cud,
                                     fma((double)R0 + 0.5 * TH, tab[kk].sud, tab[kk].u0));
                const double fl = fmin(fmax(floor(T), -1.0e6), 1.0e6);
                anc[e].f = (float)(T - fl) + (float)PSH;
                anc[e].i4 = ((int)fl - PSH) * 4;
            }
        }
    };
    fill_anchors(0);

    // Every load that does not depend on another one is issued here, before the
    // first barrier: the primal values of the own pixels, the xbar tile with its
    // halo, and the old TV dual of the tile plus top/left halo.
    float xo[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        xo[q] = 0.f;
        if (inside[q] && (mode == BP_CP || mode == BP_SIRT || mode == BP_ACCUM))
            xo[q] = J->x[(size_t)(R0 + tr + q) * J->ldx + c];
        if (inside[q] && (mode == BP_LOCAL || mode == BP_FISTA))   // correction v (padded)
            xo[q] = J->xb[rpar][(size_t)(R0 + tr + q) * J->xp + c + kLpad];
    }
    constexpr int NZ = ((TH + 1) * (TW + 1) + NT - 1) / NT;
    float zq0[NZ], zq1[NZ];
    float divv[PPT], zn0[PPT], zn1[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) divv[q] = zn0[q] = zn1[q] = 0.f;
    if (tv) {
        gcfloat* xb = gview(J->xb[rpar]);
        const int xp = J->xp;
        const size_t plane = (size_t)nr * nc;
        gcfloat* zo = gview(J->z[rpar]);
#pragma unroll
        for (int u = 0; u < NZ; ++u) {
            const int q = t + NT * u;
            const int lr = q / (TW + 1), lc = q % (TW + 1);
            const int rr = R0 - 1 + lr, cc = C0 - 1 + lc;
            zq0[u] = 0.f;
            zq1[u] = 0.f;
            if (mode == BP_CP && q < (TH + 1) * (TW + 1) && rr >= 0 && rr < nr && cc >= 0 &&
                cc < nc) {
                const size_t zi = (size_t)rr * nc + cc;
                zq0[u] = zo[zi];
                zq1[u] = zo[plane + zi];
            }
        }
        for (int q = t; q < (TH + 2) * (TW + 2); q += NT) {
            const int lr = q / (TW + 2), lc = q % (TW + 2);
            const int rr = R0 - 1 + lr, cc = C0 - 1 + lc;
            float v = 0.f;
            if (rr >= 0 && rr < nr && cc >= -1 && cc <= nc) v = xb[(size_t)rr * xp + cc + kLpad];
            xs[lr][lc] = v;
        }
        __syncthreads();
        const float lam = J->lam, sigma = J->sigma;
        const int aniso = J->flags & JF_ANISO;
#pragma unroll
        for (int u = 0; u < NZ; ++u) {
            const int q = t + NT * u;
            if (q >= (TH + 1) * (TW + 1)) break;
            const int lr = q / (TW + 1), lc = q % (TW + 1);
            const int rr = R0 - 1 + lr, cc = C0 - 1 + lc;
            float q0 = 0.f, q1 = 0.f;
            if (rr >= 0 && rr < nr && cc >= 0 && cc < nc) {
                const float xc = xs[lr][lc];
                // forward differences, zero on the last row / column (Neumann)
                const float g0 = (rr < nr - 1) ? xs[lr + 1][lc] - xc : 0.f;
                const float g1 = (cc < nc - 1) ? xs[lr][lc + 1] - xc : 0.f;
                if (mode == BP_POWER) {
                    q0 = g0;
                    q1 = g1;
                } else {
                    q0 = zq0[u] + sigma * g0;
                    q1 = zq1[u] + sigma * g1;
                    if (aniso) {
                        q0 = fminf(fmaxf(q0, -lam), lam);
                        q1 = fminf(fmaxf(q1, -lam), lam);
                    } else if (lam > 0.f) {
                        // projection of each pixel's 2-vector onto the lambda-ball
                        const float sc = fmaxf(1.f, sqrtf(q0 * q0 + q1 * q1) / lam);
                        q0 = q0 / sc;
                        q1 = q1 / sc;
                    } else {
                        q0 = 0.f;
                        q1 = 0.f;
                    }
                }
            }
            zs0[lr][lc] = q0;
            zs1[lr][lc] = q1;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            if (!inside[q]) continue;
            const int lr = tr + q + 1, lc = tc + 1;
            zn0[q] = zs0[lr][lc];
            zn1[q] = zs1[lr][lc];
            // div = -grad^T (z is 0 outside the region and on its last row/column)
            divv[q] = (zn0[q] - zs0[lr - 1][lc]) + (zn1[q] - zs1[lr][lc - 1]);
        }
    }

    if (!tv) __syncthreads();   // anchors of the first pass

    float acc[PPT], cacc[PPT], acc2[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) acc[q] = cacc[q] = acc2[q] = 0.f;
    // one pixel-angle term w0 y0 + w1 y1; COMP keeps the sum compensated (the
    // filtered-backprojection sums cancel to values far below their terms)
    auto accum = [&](int q, float w0, float y0, float w1, float y1) {
        if constexpr (COMP) {
            comp_add(acc[q], cacc[q], fmaf(w0, y0, w1 * y1));
        } else {
            acc[q] = fmaf(w0, y0, acc[q]);
            acc[q] = fmaf(w1, y1, acc[q]);
        }
    };
    const int kg0 = (na * g) / AG, kg1 = (na * (g + 1)) / AG;   // this group's angles
    const float dcf = (float)(tc - TW / 2), drf = (float)(tr - TH / 2);
    if constexpr (!STAGED) {
    // ---- backprojection, direct: every pixel reads its band pair from global
    // memory (fewest dependent steps: the latency-bound shape) ----
    const int bpitch = J->bpitch;
    const unsigned rowb = (unsigned)bpitch * 4u;
    gcfloat* yband = gview(J->y);
    for (int pass = 0; pass < npass; ++pass) {
        if (pass > 0) {
            __syncthreads();
            fill_anchors(pass);
            __syncthreads();
        }
        const int ka = kg0 + pass * PA, kb = min(kg1, ka + PA);
        const Anchor* an = anc + g * PA - ka;
        if (!inside[0]) continue;
        if constexpr (TWO) {
            // (g, d) pairs: one 16-byte read gives both channels of both taps
            const unsigned rowb2 = 2u * rowb;
            constexpr int UA = 8 / PPT;
            int k = ka;
            for (; k + UA <= kb; k += UA) {
                float f[UA][PPT];
                v4f yv[UA][PPT];
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const Anchor A = an[k + u];
                    const __amdgpu_buffer_rsrc_t rs =
                        make_rsrc(yband + (size_t)(k + u) * 2 * bpitch, rowb2);
                    float loc = fmaf(dcf, tab[k + u].cu, fmaf(drf, tab[k + u].su, A.f));
#pragma unroll
                    for (int q = 0; q < PPT; ++q) {
                        if (q) loc += tab[k + u].su;
                        f[u][q] = __builtin_amdgcn_fractf(loc);
                        yv[u][q] = load4(rs, ((unsigned)loc << 3) + 2u * (unsigned)A.i4, 0);
                    }
                }
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const float r = tab[k + u].r, rm1 = tab[k + u].rm1;
#pragma unroll
                    for (int q = 0; q < PPT; ++q) {
                        const float w0 = __builtin_amdgcn_fmed3f(r - f[u][q], 0.f, 1.f);
                        const float w1 = __builtin_amdgcn_fmed3f(f[u][q] + rm1, 0.f, 1.f);
                        acc[q] = fmaf(w0, yv[u][q].x, acc[q]);
                        acc[q] = fmaf(w1, yv[u][q].z, acc[q]);
                        acc2[q] = fmaf(w0, yv[u][q].y, acc2[q]);
                        acc2[q] = fmaf(w1, yv[u][q].w, acc2[q]);
                    }
                }
            }
            for (; k < kb; ++k) {
                const Anchor A = an[k];
                const __amdgpu_buffer_rsrc_t rs = make_rsrc(yband + (size_t)k * 2 * bpitch, rowb2);
                const float r = tab[k].r, rm1 = tab[k].rm1;
                float loc = fmaf(dcf, tab[k].cu, fmaf(drf, tab[k].su, A.f));
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    if (q) loc += tab[k].su;
                    const float f = __builtin_amdgcn_fractf(loc);
                    const v4f yv = load4(rs, ((unsigned)loc << 3) + 2u * (unsigned)A.i4, 0);
                    const float w0 = __builtin_amdgcn_fmed3f(r - f, 0.f, 1.f);
                    const float w1 = __builtin_amdgcn_fmed3f(f + rm1, 0.f, 1.f);
                    acc[q] = fmaf(w0, yv.x, acc[q]);
                    acc[q] = fmaf(w1, yv.z, acc[q]);
                    acc2[q] = fmaf(w0, yv.y, acc2[q]);
                    acc2[q] = fmaf(w1, yv.w, acc2[q]);
                }
            }
            continue;
        }
        // Each band row is read through its own buffer resource whose range is
        // that row, so a stray coordinate reads 0 instead of a neighbouring row.
        constexpr int UA = 16 / PPT;   // angles per step: 16 paired band loads in flight
        int k = ka;
        for (; k + UA <= kb; k += UA) {
            float f[UA][PPT];
            v2f yv[UA][PPT];
#pragma unroll
            for (int u = 0; u < UA; ++u) {
                const Anchor A = an[k + u];
                const __amdgpu_buffer_rsrc_t rs = make_rsrc(yband + (size_t)(k + u) * bpitch, rowb);
                float loc = fmaf(dcf, tab[k + u].cu, fmaf(drf, tab[k + u].su, A.f));
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    if (q) loc += tab[k + u].su;
                    f[u][q] = __builtin_amdgcn_fractf(loc);
                    yv[u][q] = load2(rs, ((unsigned)loc << 2) + (unsigned)A.i4, 0);
                }
            }
#pragma unroll
            for (int u = 0; u < UA; ++u) {
                const float r = tab[k + u].r, rm1 = tab[k + u].rm1;
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    // clamp to [0, 1] == max(0, .) here: r <= 1 and f >= 0
                    const float w0 = __builtin_amdgcn_fmed3f(r - f[u][q], 0.f, 1.f);
                    const float w1 = __builtin_amdgcn_fmed3f(f[u][q] + rm1, 0.f, 1.f);
                    accum(q, w0, yv[u][q].x, w1, yv[u][q].y);
                }
            }
        }
        for (; k < kb; ++k) {
            const Anchor A = an[k];
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(yband + (size_t)k * bpitch, rowb);
            const float r = tab[k].r, rm1 = tab[k].rm1;
            float loc = fmaf(dcf, tab[k].cu, fmaf(drf, tab[k].su, A.f));
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                if (q) loc += tab[k].su;
                const float f = __builtin_amdgcn_fractf(loc);
                const v2f yv = load2(rs, ((unsigned)loc << 2) + (unsigned)A.i4, 0);
                const float w0 = __builtin_amdgcn_fmed3f(r - f, 0.f, 1.f);
                const float w1 = __builtin_amdgcn_fmed3f(f + rm1, 0.f, 1.f);
                accum(q, w0, yv.x, w1, yv.y);
            }
        }
    }
    } else {
    // ---- backprojection, staged: band windows in LDS, KA angles per group per
    // stage, double-buffered; each window is one coalesced 64-entry row read,
    // and every pixel-angle reads its pair from LDS (the throughput shape) ----
    const int wv = uniform_int(t >> 6), lane = t & 63;
    const int bpitch = J->bpitch;
    const int wsmax = bpitch - WS;           // bpitch >= WS by construction
    const unsigned rowb = (unsigned)bpitch * 4u * CH;
    gcfloat* yband = gview(J->y);
    const __amdgpu_buffer_rsrc_t rs_band =
        make_rsrc(yband, (size_t)na * bpitch * CH * sizeof(float));
    LDS_AS float* const wl = (LDS_AS float*)win + WS * CH;
    const unsigned wl_bytes = (unsigned)(size_t)wl;
    for (int pass = 0; pass < npass; ++pass) {
        if (pass > 0) {
            __syncthreads();
            fill_anchors(pass);
            __syncthreads();
        }
        // angles of group gg in this pass: [lo(gg), hi(gg)); stage s covers
        // lo + s KA .. lo + s KA + KA - 1
        const int span = min(PA, (na + AG - 1) / AG - pass * PA);   // upper bound over groups
        const int nst = (max(span, 0) + KA - 1) / KA;
        // Window w of stage st holds angle slot w % KA of group w / KA.  Only the
        // staged values stay live across a stage; the rest is recomputed at
        // store time from the anchors (read together, before any is used).
        auto win_kk = [&](int st, int w, bool* ok) {
            const int gg = w / KA, j = w % KA;
            const int lo = (na * gg) / AG + pass * PA;
            const int hi = min((na * (gg + 1)) / AG, lo + PA);
            *ok = lo + st * KA + j < hi;
            return lo + st * KA + j;
        };
        auto win_anchors = [&](int st, Anchor* A) {
#pragma unroll
            for (int i = 0; i < WPW; ++i) {
                const int w = wv * WPW + i;
                A[i] = anc[min((w / KA) * PA + st * KA + w % KA, ANC - 1)];
            }
        };
        float sv[WPW];
        v2f sv2[TWO ? WPW : 1];
        auto stage_load = [&](int st) {
            Anchor A[WPW];
            win_anchors(st, A);
#pragma unroll
            for (int i = 0; i < WPW; ++i) {
                bool ok;
                const int kk = win_kk(st, wv * WPW + i, &ok);
                if constexpr (TWO) sv2[i] = v2f{0.f, 0.f};
                else sv[i] = 0.f;
                if (ok) {   // the window lies inside its band row: ws in [0, bpitch - WS]
                    const int ws = min(max((uniform_int(A[i].i4) >> 2) + PSH - SHIFT, 0), wsmax);
                    const unsigned soff = (unsigned)kk * rowb + (unsigned)ws * 4u * CH;
                    if constexpr (TWO)
                        sv2[i] = load2(rs_band, (unsigned)lane * 8u, soff);
                    else
                        sv[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                             rs_band, (unsigned)lane * 4u, soff, 0));
                }
            }
        };
        auto stage_store = [&](int st, int buf) {
            Anchor A[WPW];
            win_anchors(st, A);
#pragma unroll
            for (int i = 0; i < WPW; ++i) {
                const int w = wv * WPW + i;
                bool ok;
                (void)win_kk(st, w, &ok);
                if (!ok) continue;
                const int I = (uniform_int(A[i].i4) >> 2) + PSH;
                const int ws = min(max(I - SHIFT, 0), wsmax);
                const int slot = (buf * NW + w) * WS;
                if constexpr (TWO) ((LDS_AS v2f*)wl)[slot + lane] = sv2[i];
                else wl[slot + lane] = sv[i];
                if (lane == 0) {
                    wmeta[buf][w].f = A[i].f;
                    wmeta[buf][w].base = wl_bytes + (unsigned)(slot + I - PSH - ws) * 4u * CH;
                }
            }
        };
        if (nst > 0) {
            stage_load(0);
            stage_store(0, 0);
        }
        __syncthreads();
        for (int st = 0; st < nst; ++st) {
            const int buf = st & 1;
            if (st + 1 < nst) stage_load(st + 1);   // in flight while this stage computes
            const int kfirst = kg0 + pass * PA + st * KA;
            const int nj = max(0, min(KA, min(kg1, kg0 + pass * PA + PA) - kfirst));
            if (inside[0]) {
                const WinMeta* wm = wmeta[buf] + g * KA;
                constexpr int UA = 8 / PPT;   // LDS latency is short: 8 pair reads in flight
                // the band pair of a pixel-angle: (y0, y1), or (g0, d0, g1, d1) for two channels
                using Pair = typename std::conditional<TWO, v4f, v2f>::type;
                auto fetch = [&](float loc, unsigned base) -> Pair {
                    if constexpr (TWO) {
                        const LDS_AS v2f* pp =
                            (const LDS_AS v2f*)(size_t)(((unsigned)loc << 3) + base);
                        const v2f e0 = pp[0], e1 = pp[1];
                        return v4f{e0.x, e0.y, e1.x, e1.y};
                    } else {
                        const LDS_AS float* pp =
                            (const LDS_AS float*)(size_t)(((unsigned)loc << 2) + base);
                        return v2f{pp[0], pp[1]};
                    }
                };
                auto apply = [&](int q, float w0, float w1, const Pair& v) {
                    if constexpr (TWO) {
                        acc[q] = fmaf(w0, v.x, acc[q]);
                        acc[q] = fmaf(w1, v.z, acc[q]);
                        acc2[q] = fmaf(w0, v.y, acc2[q]);
                        acc2[q] = fmaf(w1, v.w, acc2[q]);
                    } else {
                        accum(q, w0, v.x, w1, v.y);
                    }
                };
                int j = 0;
                for (; j + UA <= nj; j += UA) {
                    float f[UA][PPT];
                    Pair yv[UA][PPT];
#pragma unroll
                    for (int u = 0; u < UA; ++u) {
                        const WinMeta M = wm[j + u];
                        const AngBP a = tab[kfirst + j + u];
                        float loc = fmaf(dcf, a.cu, fmaf(drf, a.su, M.f));
#pragma unroll
                        for (int q = 0; q < PPT; ++q) {
                            if (q) loc += a.su;
                            f[u][q] = __builtin_amdgcn_fractf(loc);
                            yv[u][q] = fetch(loc, M.base);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < UA; ++u) {
                        const float r = tab[kfirst + j + u].r, rm1 = tab[kfirst + j + u].rm1;
#pragma unroll
                        for (int q = 0; q < PPT; ++q) {
                            // clamp to [0, 1] == max(0, .) here: r <= 1 and f >= 0
                            const float w0 = __builtin_amdgcn_fmed3f(r - f[u][q], 0.f, 1.f);
                            const float w1 = __builtin_amdgcn_fmed3f(f[u][q] + rm1, 0.f, 1.f);
                            apply(q, w0, w1, yv[u][q]);
                        }
                    }
                }
                for (; j < nj; ++j) {
                    const WinMeta M = wm[j];
                    const AngBP a = tab[kfirst + j];
                    float loc = fmaf(dcf, a.cu, fmaf(drf, a.su, M.f));
#pragma unroll
                    for (int q = 0; q < PPT; ++q) {
                        if (q) loc += a.su;
                        const float f = __builtin_amdgcn_fractf(loc);
                        const Pair v = fetch(loc, M.base);
                        const float w0 = __builtin_amdgcn_fmed3f(a.r - f, 0.f, 1.f);
                        const float w1 = __builtin_amdgcn_fmed3f(f + a.rm1, 0.f, 1.f);
                        apply(q, w0, w1, v);
                    }
                }
            }
            if (st + 1 < nst) stage_store(st + 1, (st + 1) & 1);
            __syncthreads();
        }
    }
    }
    if constexpr (COMP) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) acc[q] += cacc[q];
    }
    if (AG > 1) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            red[q][t] = acc[q];
            if constexpr (TWO) red2[q][t] = acc2[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            acc[q] = 0.f;
            acc2[q] = 0.f;
            if (g == 0) {
#pragma unroll
                for (int h = 0; h < AG; ++h) {
                    acc[q] += red[q][h * P + p];
                    if constexpr (TWO) acc2[q] += red2[q][h * P + p];
                }
            }
        }
    }

    float sq = 0.f;
    if (g == 0) {
        float* x = J->x;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            if (!inside[q]) continue;
            const int r = R0 + tr + q;
            const size_t xi = (size_t)r * J->ldx + c;
            switch (mode) {
                case BP_STORE: {
                    const float v = J->scale * acc[q];
                    x[xi] = v;
                    float* xb0 = J->xb[0];
                    float* xt = J->xt;
                    if (xb0) xb0[(size_t)r * J->xp + c + kLpad] = v;
                    if (xt) xt[(size_t)c * J->tp + r + kLpad] = v;
                } break;
                case BP_ACCUM:
                    x[xi] = xo[q] + J->scale * acc[q];
                    break;
                case BP_CP: {
                    const float xn = fmaxf(0.f, xo[q] - J->tau * (acc[q] - divv[q]));
                    x[xi] = xn;
                    const float xbn = 2.f * xn - xo[q];   // theta = 1
                    float* xbw = J->xb[wpar];
                    float* xt = J->xt;
                    float* zw = J->z[wpar];
                    xbw[(size_t)r * J->xp + c + kLpad] = xbn;
                    xt[(size_t)c * J->tp + r + kLpad] = xbn;
                    const size_t zi = (size_t)r * nc + c;
                    zw[zi] = zn0[q];
                    zw[(size_t)nr * nc + zi] = zn1[q];
                } break;
                case BP_SIRT: {
                    const float xn = fminf(fmaxf(xo[q] + acc[q], J->lo), J->hi);
                    x[xi] = xn;
                    float* xbw = J->xb[wpar];
                    float* xt = J->xt;
                    xbw[(size_t)r * J->xp + c + kLpad] = xn;
                    xt[(size_t)c * J->tp + r + kLpad] = xn;
                } break;
                case BP_LOCAL: {
                    // x = P_[lo,hi](v + W_L^T g); the new correction v = x - W_L^T d
                    const float xn = fminf(fmaxf(xo[q] + acc[q], J->lo), J->hi);
                    x[xi] = xn;
                    const float vn = xn - acc2[q];
                    J->xb[wpar][(size_t)r * J->xp + c + kLpad] = vn;
                    J->xt[(size_t)c * J->tp + r + kLpad] = vn;
                } break;
                case BP_FISTA: {
                    // FGP input x_s + q = v + W_L^T (d - alpha W_L v), and x_s = W_L^T d
                    const size_t pi = (size_t)r * nc + c;
                    J->w[pi] = xo[q] + acc[q];
                    J->xs[pi] = acc2[q];
                } break;
                case BP_POWER: {
                    const float w = acc[q] - divv[q];
                    x[xi] = w;
                    sq += w * w;
                } break;
                default:
                    break;
            }
        }
    }
    if (mode == BP_POWER) {
        // block sum of the squares, in the anchor table's LDS (no longer needed)
        static_assert(sizeof(anc) >= NT * sizeof(float), "anchor table too small to reuse");
        float* psum = (float*)anc;
        __syncthreads();
        psum[t] = sq;
        __syncthreads();
        for (int h = NT / 2; h > 0; h >>= 1) {
            if (t < h) psum[t] += psum[t + h];
            __syncthreads();
        }
        if (t == 0) {
            float* part = J->part;
            part[it.a * J->ntc + it.b] = psum[0];
        }
    }
}

__global__ void fill_kernel(float* __restrict__ p, size_t n, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Interior of the padded buffers set to v, padding to 0.
__global__ void fill_padded_kernel(float* __restrict__ xb, float* __restrict__ xt, int nr, int nc,
                                   int xp, int tp, float v) {
    const size_t nb = (size_t)nr * xp, nt = xt ? (size_t)nc * tp : 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb + nt;
         i += (size_t)gridDim.x * blockDim.x) {
        if (i < nb) {
            const int cc = (int)(i % xp);
            xb[i] = (cc >= kLpad && cc < nc + kLpad) ? v : 0.f;
        } else {
            const size_t q = i - nb;
            const int rr = (int)(q % tp);
            xt[q] = (rr >= kLpad && rr < nr + kLpad) ? v : 0.f;
        }
    }
}

// Region [r0, r0+nr) x [c0, c0+nc) of src -> padded xbar (+ transposed, + plain).
__global__ void pad_copy_kernel(const float* __restrict__ src, int lds, int r0, int c0, int nr,
                                int nc, float* __restrict__ xb, int xp, float* __restrict__ xt,
                                int tp, float* __restrict__ dst, int ldd) {
    __shared__ float tile[32][33];
    const int bc = blockIdx.x * 32, br = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int q = ty; q < 32; q += 8) {
        const int rr = br + q, cc = bc + tx;
        float v = 0.f;
        if (rr < nr && cc < nc) {
            v = src[(size_t)(r0 + rr) * lds + c0 + cc];
            if (xb) xb[(size_t)rr * xp + cc + kLpad] = v;
            if (dst) dst[(size_t)rr * ldd + cc] = v;
        }
        tile[q][tx] = v;
    }
    if (!xt) return;
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int cc = bc + q, rr = br + tx;
        if (rr < nr && cc < nc) xt[(size_t)cc * tp + rr + kLpad] = tile[tx][q];
    }
}

// *flag = 1 when any of the n values is NaN or infinite (a plain store from every
// lane that finds one: all write the same value).
__global__ void check_finite_kernel(const float* __restrict__ p, size_t n,
                                    unsigned* __restrict__ flag) {
    bool bad = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(p[i]);
    if (bad) *flag = 1u;
}

__global__ void crop_kernel(const float* __restrict__ x, int ldx, int dr, int dc, int rows,
                            int cols, float* __restrict__ out, int ldo) {
    const size_t n = (size_t)rows * cols;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int rr = (int)(i / cols), cc = (int)(i % cols);
        out[(size_t)rr * ldo + cc] = x[(size_t)(rr + dr) * ldx + cc + dc];
    }
}

// Full-detector sinogram rows -> band layout for the backprojector (band
// position j at j + 1, scaled by the angle's B; zeros off the detector and in
// the padding).
__global__ void band_gather_kernel(const float* __restrict__ sino, int n_det,
                                   const AngFP* __restrict__ afp, float* __restrict__ band,
                                   int bpitch) {
    const int k = blockIdx.x;
    const int i0 = afp[k].i0, w = afp[k].w;
    const float bs = afp[k].bscale;
    for (int q = threadIdx.x; q < bpitch; q += blockDim.x) {
        const int j = q - 1, gi = i0 + j;
        float v = 0.f;
        if (j >= 0 && j < w && gi >= 0 && gi < n_det) v = bs * sino[(size_t)k * n_det + gi];
        band[(size_t)k * bpitch + q] = v;
    }
}

__global__ void band_scatter_kernel(const float* __restrict__ band, int bpitch,
                                    const AngFP* __restrict__ afp, float* __restrict__ sino,
                                    int n_det, int accumulate) {
    const int k = blockIdx.x;
    const int i0 = afp[k].i0, w = afp[k].w;
    for (int j = threadIdx.x; j < w; j += blockDim.x) {
        const int gi = i0 + j;
        if (gi < 0 || gi >= n_det) continue;
        const float v = band[(size_t)k * bpitch + 1 + j];
        if (accumulate)
            sino[(size_t)k * n_det + gi] += v;
        else
            sino[(size_t)k * n_det + gi] = v;
    }
}

// Ram-Lak filtering: block (chunk, angle) produces 256 consecutive outputs of
// one detector row as a linear (zero-padded) convolution along the detector,
// q[i] = taps[0] p[i] + sum_{odd d} taps[d] (p[i-d] + p[i+d]), written (times
// the angle's B) into the band layout of the receiving backprojection.
// Ram-Lak filter of one sinogram row, linear (zero outside the detector).  The
// centre tap and the negative odd taps cancel to a small filtered value, so
// the sum over the near taps (offset below kRampNear) is compensated and those
// taps are FP32 pairs hi + lo: the FP32 result then agrees with an exact
// convolution of the FP32 data to a few ulp.  The far taps are below
// 2 / (pi^2 kRampNear^2) ~ 5e-5 of the centre's scale each and sum to under
// 2e-3 of it in magnitude, so a plain FP32 sum of them adds no more than
// 1e-9 of the data's scale in error.  Every lane runs the same offsets
// 1, 3, .., n_det - 1 (uniform tap loads); a neighbour off the detector reads
// one of the two zeros around the row.
constexpr int kRampNear = 64;
__global__ __launch_bounds__(256) void ramp_kernel(const float* __restrict__ sino, int n_det,
                                                   const float* __restrict__ taps,
                                                   const AngFP* __restrict__ afp,
                                                   float* __restrict__ band, int bpitch) {
    extern __shared__ float prow[];   // n_det + 2: a zero, the row, a zero
    const int k = blockIdx.y;
    for (int i = threadIdx.x; i < n_det + 2; i += blockDim.x)
        prow[i] = (i >= 1 && i <= n_det) ? sino[(size_t)k * n_det + i - 1] : 0.f;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_det) return;
    const float* row = prow + 1;      // row[-1] = row[n_det] = 0
    const CONST_AS float* h = cview(taps);   // tap index is uniform: scalar loads
    const int i0 = afp[k].i0, w = afp[k].w;
    const float p0 = row[i];
    float s = h[0] * p0, c = fmaf(h[1], p0, fmaf(h[0], p0, -s));
    float lo = 0.f, far = 0.f;
    const int dmax = n_det - 1, dnear = min(dmax, kRampNear - 1);
    int d = 1;
    for (; d <= dnear; d += 2) {
        const float P = row[max(i - d, -1)] + row[min(i + d, n_det)];
        const float t = h[2 * d] * P;
        comp_add(s, c, t);
        c += fmaf(h[2 * d], P, -t);        // rounding of the product
        lo = fmaf(h[2 * d + 1], P, lo);    // the taps' low parts
    }
#pragma unroll 8
    for (; d <= dmax; d += 2)
        far = fmaf(h[2 * d], row[max(i - d, -1)] + row[min(i + d, n_det)], far);
    comp_add(s, c, far);
    const float q = s + (c + lo);
    const int j = i - i0;
    if (j >= 0 && j < w) band[(size_t)k * bpitch + 1 + j] = afp[k].bscale * q;
}

// Power iteration: v = w / ||w||, ||w|| from the per-tile partial sums (summed
// in the same fixed order by every block), written into the padded buffers.
// ---------------------------------------------------------------------------
// Preprocessing of the local method (Section 3.3 disc subtraction; Section 4
// constant padding of truncated data).  A pixel belongs to the disc of
// diameter n about the grid centre when (2c - n + 1)^2 + (2r - n + 1)^2 <= n^2,
// decided exactly in integers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool in_disc(int n, int r, int c) {
    const long long dx = 2LL * c - (n - 1), dy = 2LL * r - (n - 1);
    return dx * dx + dy * dy <= (long long)n * n;
}

// img[r][c] (region (r0, c0) of the grid, pitch ld): add = 0 writes the disc
// indicator; add = 1 adds *value on the disc's pixels.
__global__ void disc_kernel(float* __restrict__ img, int ld, int n, int r0, int c0, int rows,
                            int cols, const float* __restrict__ value, int add) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= cols || r >= rows) return;
    const bool in = in_disc(n, r0 + r, c0 + c);
    float* q = img + (size_t)r * ld + c;
    if (add) {
        if (in) *q += *value;
    } else {
        *q = in ? 1.f : 0.f;
    }
}

// Row sums of the data and of the disc's projection, in FP64: st[2a] = sum_i p[a][i],
// st[2a + 1] = sum_i D[a][i].  One block per angle.
__global__ __launch_bounds__(256) void disc_sums_kernel(const float* __restrict__ p,
                                                        const float* __restrict__ D, int nd,
                                                        double* __restrict__ st) {
    __shared__ double s0[256], s1[256];
    const int a = blockIdx.x, t = threadIdx.x;
    double u = 0.0, v = 0.0;
    for (int i = t; i < nd; i += 256) {
        u += (double)p[(size_t)a * nd + i];
        v += (double)D[(size_t)a * nd + i];
    }
    s0[t] = u;
    s1[t] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            s0[t] += s0[t + h];
            s1[t] += s1[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        st[2 * a] = s0[0];
        st[2 * a + 1] = s1[0];
    }
}

// value = sum_a S_a T_a / sum_a T_a^2 (one block).
__global__ __launch_bounds__(256) void disc_value_kernel(const double* __restrict__ st, int na,
                                                         float* __restrict__ value) {
    __shared__ double s0[256], s1[256];
    const int t = threadIdx.x;
    double u = 0.0, v = 0.0;
    for (int a = t; a < na; a += 256) {
        u += st[2 * a] * st[2 * a + 1];
        v += st[2 * a + 1] * st[2 * a + 1];
    }
    s0[t] = u;
    s1[t] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            s0[t] += s0[t + h];
            s1[t] += s1[t + h];
        }
        __syncthreads();
    }
    if (t == 0) *value = s1[0] > 0.0 ? (float)(s0[0] / s1[0]) : 0.f;
}

__global__ void disc_apply_kernel(const float* __restrict__ p, const float* __restrict__ D,
                                  size_t n, const float* __restrict__ value, float* out) {
    const float v = *value;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = fmaf(-v, D[i], p[i]);
}

// out[a][i] = trunc[a][clamp(i - first, 0, nb - 1)]
__global__ void pad_truncated_kernel(const float* __restrict__ trunc, int nb, int first, int nd,
                                     float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, a = blockIdx.y;
    if (i >= nd) return;
    const int j = min(max(i - first, 0), nb - 1);
    out[(size_t)a * nd + i] = trunc[(size_t)a * nb + j];
}

// ---------------------------------------------------------------------------
// FGP (fast gradient projection on the dual of TV denoising, the inner solver of
// the paper's local FISTA-TV, Alg. 3): min_{lo <= x <= hi} ||x - b||^2 + 2 gamma TV(x),
//   x = P(b - gamma div r),  p' = P_1(r - grad x / (8 gamma)),  r = p' + beta_i (p' - p).
// Temporal blocking: a block loads its 32 x 32 tile with a halo of kFgpSteps + 1
// pixels into LDS and runs kFgpSteps dual iterations there (each iteration's valid
// area shrinks by one pixel per side), then writes p and r of its tile; no
// neighbour exchange is needed within a launch.  Outside the region p = r = b = 0;
// the gradient is zero on the region's last row / column (Neumann), so the duals
// stay zero there, as in the CP kernel's TV.
// ---------------------------------------------------------------------------
constexpr int kFgpThreads = 1024;   // 16 waves; two blocks per CU: eight waves per SIMD

__global__ __launch_bounds__(kFgpThreads) void fgp_kernel(const Job* __restrict__ jobs,
                                                  const Item* __restrict__ items, int n_items,
                                                  int step, int i0) {
    constexpr int H = kFgpSteps + 1, RW = kFgpTile + 2 * H, RN = RW * RW;
    constexpr int NQ = (RN + kFgpThreads - 1) / kFgpThreads;   // region pixels per thread
    // Each thread keeps its own pixels' b, p and r in registers; only x and r,
    // which neighbours read, go through LDS.  The arrays are padded so that every
    // neighbour read stays in bounds without a test: r0 of pixel q sits at
    // sr0[RW + q] (the up neighbour of the first row reads the zero row in front),
    // r1 at sr1[1 + q], and x has a zero row behind the window.  A neighbour read
    // that crosses the window's edge returns another finite pixel's value instead of
    // zero; it only feeds pixels on the window's rim, which are outside the exact
    // area from the first step on.
    __shared__ float sx[RN + RW], sr0[RW + RN], sr1[1 + RN];
    const int bid = blockIdx.x;
    if (bid >= n_items) return;
    const Item it = cview(items)[bid];
    const CONST_AS Job* J = cview(jobs) + it.job;
    const int nf = J->n_fgp;
    // this launch's iterations of the job; the launch covering the last one finishes
    if (!(i0 < nf || (nf == 0 && i0 == 0))) return;
    const int i1 = min(nf, i0 + kFgpSteps);
    const bool last = i1 >= nf;
    const int nr = J->nr, nc = J->nc;
    const int R0 = it.a * kFgpTile - H, C0 = it.b * kFgpTile - H;
    const size_t plane = (size_t)nr * nc;
    const float gamma = J->gamma;
    const int t = threadIdx.x;
    if (t < RW) {
        sr0[t] = 0.f;
        sx[RN + t] = 0.f;
    }
    if (t == 0) sr1[0] = 0.f;
    // per own pixel: its window row (bits 0-7; RW past the last pixel) and whether the
    // gradient row / column is taken (bits 8, 9: inside the region and not on its last
    // row / column), b, p and r
    static_assert(RW < 256, "window row must fit in 8 bits");
    int meta[NQ];
    float b[NQ], p0[NQ], p1[NQ], r0[NQ], r1[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = t + kFgpThreads * u;
        const int lr = q / RW, lc = q % RW;
        const int rr = R0 + lr, cc = C0 + lc;
        meta[u] = q < RN ? lr : RW;   // past the last row: outside every window
        b[u] = p0[u] = p1[u] = r0[u] = r1[u] = 0.f;
        if (q < RN) {
            if (rr >= 0 && rr < nr && cc >= 0 && cc < nc) {
                meta[u] |= (rr < nr - 1 && lr + 1 < RW ? 256 : 0) |
                           (cc < nc - 1 && lc + 1 < RW ? 512 : 0);
                const size_t pi = (size_t)rr * nc + cc;
                b[u] = J->w[pi];
                if (i0 > 0 && gamma > 0.f) {
                    p0[u] = J->fp[pi];
                    p1[u] = J->fp[plane + pi];
                    r0[u] = J->fr[pi];
                    r1[u] = J->fr[plane + pi];
                }
            }
            sr0[RW + q] = r0[u];
            sr1[1 + q] = r1[u];
        }
    }
    __syncthreads();
    const float lo = J->lo, hi = J->hi;
    if (gamma > 0.f && i1 > i0) {
        const float inv8g = 1.f / (8.f * gamma);
        const bool aniso = (J->flags & JF_ANISO) != 0;
#pragma unroll 1
        for (int i = i0; i < i1; ++i) {
            // Values stay exact on rows / columns [s, RW - 1 - s] after the s-th step of
            // this launch; rows outside [s - 1, RW - s] are not needed by any later step.
            const int s = i - i0 + 1, wlo = s - 1, whi = RW - s;
            // x = P(b - gamma div r); div r = r0 - r0(up) + r1 - r1(left), zero outside
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int q = t + kFgpThreads * u;
                const int lr = meta[u] & 255;
                if (lr >= wlo && lr <= whi) {
                    const float up = sr0[q], left = sr1[q];
                    const float d = (r0[u] - up) + (r1[u] - left);
                    sx[q] = fminf(fmaxf(b[u] - gamma * d, lo), hi);
                }
            }
            __syncthreads();
            const float beta = J->beta_in[i];
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int q = t + kFgpThreads * u;
                const int lr = meta[u] & 255;
                if (lr < wlo || lr > whi) continue;
                const float xq = sx[q];
                const float dn = sx[q + RW] - xq, rt = sx[q + 1] - xq;
                const float g0 = (meta[u] & 256) ? dn : 0.f;
                const float g1 = (meta[u] & 512) ? rt : 0.f;
                // outside the region r stays zero: no gradient is taken there
                float n0 = r0[u] - g0 * inv8g;
                float n1 = r1[u] - g1 * inv8g;
                if (aniso) {
                    n0 = fminf(fmaxf(n0, -1.f), 1.f);
                    n1 = fminf(fmaxf(n1, -1.f), 1.f);
                } else {
                    // onto the unit ball: scale by 1/|n| only where |n| > 1
                    const float q2 = fmaf(n0, n0, n1 * n1);
                    const float sc = q2 > 1.f ? __builtin_amdgcn_rsqf(q2) : 1.f;
                    n0 *= sc;
                    n1 *= sc;
                }
                r0[u] = n0 + beta * (n0 - p0[u]);
                r1[u] = n1 + beta * (n1 - p1[u]);
                p0[u] = n0;
                p1[u] = n1;
                sr0[RW + q] = r0[u];
                sr1[1 + q] = r1[u];
            }
            __syncthreads();
        }
    }
    if (last) {   // p (not r) forms the result: share it through the r arrays
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int q = t + kFgpThreads * u;
            if (q < RN) {
                sr0[RW + q] = p0[u];
                sr1[1 + q] = p1[u];
            }
        }
        __syncthreads();
    }
    // the tile's own pixels
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = t + kFgpThreads * u;
        if (q >= RN) continue;
        const int lr = q / RW, lc = q % RW;
        if (lr < H || lr >= H + kFgpTile || lc < H || lc >= H + kFgpTile) continue;
        const int rr = R0 + lr, cc = C0 + lc;
        if (rr >= nr || cc >= nc) continue;
        const size_t pi = (size_t)rr * nc + cc;
        if (!last) {
            J->fp[pi] = p0[u];
            J->fp[plane + pi] = p1[u];
            J->fr[pi] = r0[u];
            J->fr[plane + pi] = r1[u];
            continue;
        }
        // x = P(b - gamma div p), then the FISTA momentum point z and v = z - x_s
        const float d = (p0[u] - sr0[q]) + (p1[u] - sr1[q]);
        const float x = fminf(fmaxf(b[u] - gamma * d, lo), hi);
        const size_t xi = (size_t)rr * J->ldx + cc;
        const float xo = J->x[xi];
        const float beta = (J->flags & JF_NO_MOMENTUM) ? 0.f : J->beta_out[step];
        const float z = x + beta * (x - xo);
        const float v = z - J->xs[pi];
        J->x[xi] = x;
        const int wpar = ((step + J->parity0) & 1) ^ 1;
        J->xb[wpar][(size_t)rr * J->xp + cc + kLpad] = v;
        J->xt[(size_t)cc * J->tp + rr + kLpad] = v;
    }
}

// ---------------------------------------------------------------------------
// Haar l1 prior (eq. sirtista with FISTA): the prox of gamma ||B x||_1 is
// B^T soft(B w, gamma) for the orthonormal Haar transform B.  With L levels, B acts
// independently on the region's aligned 2^L x 2^L tiles (a level-j pair always lies in
// one aligned 2^j block), so one block transforms one tile in LDS: per level, rows
// then columns of the current block of sums, (a, b) -> ((a + b)/sqrt 2, (a - b)/sqrt 2)
// with the sums first, an unpaired last entry passed on as the last sum; threshold;
// inverse; then the FISTA momentum point and the new correction v.
// ---------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(256) void haar_kernel(const Job* __restrict__ jobs,
                                                   const Item* __restrict__ items, int n_items,
                                                   int step) {
    constexpr int T = 1 << L, P = T + 1;
    __shared__ float A[T * P], Bf[T * P];
    const int bid = blockIdx.x;
    if (bid >= n_items) return;
    const Item it = cview(items)[bid];
    const CONST_AS Job* J = cview(jobs) + it.job;
    const int nr = J->nr, nc = J->nc;
    const int R0 = it.a * T, C0 = it.b * T;
    const int th = min(T, nr - R0), tw = min(T, nc - C0);
    const int t = threadIdx.x;
    const float s2 = 0.70710678118654752f;
    for (int q = t; q < T * T; q += 256) {
        const int lr = q / T, lc = q % T;
        A[lr * P + lc] = (lr < th && lc < tw) ? J->w[(size_t)(R0 + lr) * nc + C0 + lc] : 0.f;
    }
    __syncthreads();
    int hs[L], ws[L];
    {
        int h = th, w = tw;
        for (int l = 0; l < L; ++l) {
            hs[l] = h;
            ws[l] = w;
            h = (h + 1) / 2;
            w = (w + 1) / 2;
        }
    }
    // forward
    for (int l = 0; l < L; ++l) {
        const int h = hs[l], w = ws[l];
        const int mw = w / 2, aw = w - mw, mh = h / 2, ah = h - mh;
        for (int q = t; q < h * w; q += 256) {   // rows: A -> Bf
            const int r = q / w, j = q % w;
            float v;
            if (j < mw) v = (A[r * P + 2 * j] + A[r * P + 2 * j + 1]) * s2;
            else if (j < aw) v = A[r * P + w - 1];
            else v = (A[r * P + 2 * (j - aw)] - A[r * P + 2 * (j - aw) + 1]) * s2;
            Bf[r * P + j] = v;
        }
        __syncthreads();
        for (int q = t; q < h * w; q += 256) {   // columns: Bf -> A
            const int i = q / w, c = q % w;
            float v;
            if (i < mh) v = (Bf[2 * i * P + c] + Bf[(2 * i + 1) * P + c]) * s2;
            else if (i < ah) v = Bf[(h - 1) * P + c];
            else v = (Bf[2 * (i - ah) * P + c] - Bf[(2 * (i - ah) + 1) * P + c]) * s2;
            A[i * P + c] = v;
        }
        __syncthreads();
    }
    const float gam = J->gamma;
    for (int q = t; q < th * tw; q += 256) {
        const int r = q / tw, c = q % tw;
        const float v = A[r * P + c];
        A[r * P + c] = copysignf(fmaxf(fabsf(v) - gam, 0.f), v);
    }
    __syncthreads();
    // inverse
    for (int l = L - 1; l >= 0; --l) {
        const int h = hs[l], w = ws[l];
        const int mw = w / 2, aw = w - mw, mh = h / 2, ah = h - mh;
        for (int q = t; q < h * w; q += 256) {   // columns: A -> Bf
            const int r = q / w, c = q % w;
            float v;
            if (r < 2 * mh) {
                const float a = A[(r >> 1) * P + c], d = A[(ah + (r >> 1)) * P + c];
                v = (r & 1) ? (a - d) * s2 : (a + d) * s2;
            } else {
                v = A[mh * P + c];
            }
            Bf[r * P + c] = v;
        }
        __syncthreads();
        for (int q = t; q < h * w; q += 256) {   // rows: Bf -> A
            const int r = q / w, c = q % w;
            float v;
            if (c < 2 * mw) {
                const float a = Bf[r * P + (c >> 1)], d = Bf[r * P + aw + (c >> 1)];
                v = (c & 1) ? (a - d) * s2 : (a + d) * s2;
            } else {
                v = Bf[r * P + mw];
            }
            A[r * P + c] = v;
        }
        __syncthreads();
    }
    const int wpar = ((step + J->parity0) & 1) ^ 1;
    for (int q = t; q < th * tw; q += 256) {
        const int lr = q / tw, lc = q % tw;
        const int rr = R0 + lr, cc = C0 + lc;
        const float x = A[lr * P + lc];
        const size_t pi = (size_t)rr * nc + cc;
        const size_t xi = (size_t)rr * J->ldx + cc;
        const float xo = J->x[xi];
        const float beta = (J->flags & JF_NO_MOMENTUM) ? 0.f : J->beta_out[step];
        const float z = x + beta * (x - xo);
        const float v = z - J->xs[pi];
        J->x[xi] = x;
        J->xb[wpar][(size_t)rr * J->xp + cc + kLpad] = v;
        J->xt[(size_t)cc * J->tp + rr + kLpad] = v;
    }
}

// ---------------------------------------------------------------------------
// Detector convolutions by FFT: C_u p for a whole bank of angle-dependent
// filters u_k (Section 3.1, eq. sirtapp; Section 3.3: the convolved data are
// computed once and shared by every local part).  A linear convolution of two
// n_det-long rows equals the circular one of length L >= 2 n_det - 1, so one
// complex transform of length L = 2^LOG per filter PAIR does two rows at once:
// the pair is packed as u_{2h} + i u_{2h+1}, multiplied by the spectrum of the
// real data row, and transformed back; the real and imaginary parts are the
// two convolutions.  The transform lives in LDS: each radix-4 (one radix-2
// when LOG is odd) self-sorting Stockham stage reads all its butterfly inputs
// into registers, synchronises, and writes the outputs back in place.
// ---------------------------------------------------------------------------
constexpr int kFftThreads = 512;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// Twiddles from two small LDS tables: exp(-2 pi i m / L) = t1[m / kTw2] t2[m % kTw2]
// (kTw2 = min(64, L) entries of fine angles, L / kTw2 of coarse ones), loaded from the
// full FP32 table tw[m] = exp(-2 pi i m / L) at the block's start.
template <int LOG>
struct FftTw {
    static constexpr int L = 1 << LOG;
    static constexpr int N2 = L < 64 ? L : 64, N1 = L / N2;
    float2 t1[N1], t2[N2];
    __device__ void load(const float2* __restrict__ tw) {
        for (int i = threadIdx.x; i < N1; i += blockDim.x) t1[i] = tw[i * N2];
        for (int i = threadIdx.x; i < N2; i += blockDim.x) t2[i] = tw[i];
    }
    __device__ float2 operator()(int m) const;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b);

template <int LOG>
__device__ float2 FftTw<LOG>::operator()(int m) const {
    return cmul(t1[m / N2], t2[m % N2]);
}

// LDS index of transform entry i: one padding entry per 32 breaks the bank
// conflicts of the strided writes of the first stages.
__device__ __forceinline__ int fpad(int i) { return i + (i >> 5); }
template <int L>
struct FftLds {
    static constexpr int N = L + L / 32;
};

// Forward DFT (exp(-2 pi i f n / L)) of z[0..L) in place (stored at fpad(i)), twiddles
// from `tw`.
template <int LOG>
__device__ void fft_lds(float2* z, const FftTw<LOG>& tw) {
    constexpr int L = 1 << LOG, T = kFftThreads;
    const int t = threadIdx.x;
    int ns = 1;   // length of the sub-transforms already done
    if constexpr (LOG & 1) {
        constexpr int NB = (L / 2 + T - 1) / T;
        float2 a[NB], b[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * T;
            if (j < L / 2) {
                a[i] = z[fpad(j)];
                b[i] = z[fpad(j + L / 2)];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * T;
            if (j < L / 2) {
                z[fpad(2 * j)] = make_float2(a[i].x + b[i].x, a[i].y + b[i].y);
                z[fpad(2 * j + 1)] = make_float2(a[i].x - b[i].x, a[i].y - b[i].y);
            }
        }
        __syncthreads();
        ns = 2;
    }
    constexpr int NB = (L / 4 + T - 1) / T;
#pragma unroll 1
    for (; ns < L; ns <<= 2) {
        float2 v[NB][4];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * T;
            if (j < L / 4) {
                const int k = j & (ns - 1);
                const int m = (L / (4 * ns)) * k;   // twiddle of input r: r m < L
                v[i][0] = z[fpad(j)];
                v[i][1] = cmul(z[fpad(j + L / 4)], tw(m));
                v[i][2] = cmul(z[fpad(j + L / 2)], tw(2 * m));
                v[i][3] = cmul(z[fpad(j + 3 * (L / 4))], tw(3 * m));
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * T;
            if (j < L / 4) {
                const int k = j & (ns - 1);
                const float2 a0 = make_float2(v[i][0].x + v[i][2].x, v[i][0].y + v[i][2].y);
                const float2 a1 = make_float2(v[i][0].x - v[i][2].x, v[i][0].y - v[i][2].y);
                const float2 a2 = make_float2(v[i][1].x + v[i][3].x, v[i][1].y + v[i][3].y);
                // -i (v1 - v3)
                const float2 a3 = make_float2(v[i][1].y - v[i][3].y, v[i][3].x - v[i][1].x);
                const int base = ((j - k) << 2) + k;
                z[fpad(base)] = make_float2(a0.x + a2.x, a0.y + a2.y);
                z[fpad(base + ns)] = make_float2(a1.x + a3.x, a1.y + a3.y);
                z[fpad(base + 2 * ns)] = make_float2(a0.x - a2.x, a0.y - a2.y);
                z[fpad(base + 3 * ns)] = make_float2(a1.x - a3.x, a1.y - a3.y);
            }
        }
        __syncthreads();
    }
}

// spec[a][0..L) = FFT of sinogram row a, zero-padded to L.
template <int LOG>
__global__ __launch_bounds__(kFftThreads, 4) void spectra_kernel(const float* __restrict__ sino,
                                                              int n_det,
                                                              const float2* __restrict__ tw,
                                                              float2* __restrict__ spec) {
    constexpr int L = 1 << LOG;
    __shared__ float2 z[FftLds<L>::N];
    __shared__ FftTw<LOG> twl;
    twl.load(tw);
    const int a = blockIdx.x;
    const float* row = sino + (size_t)a * n_det;
    for (int i = threadIdx.x; i < L; i += kFftThreads)
        z[fpad(i)] = make_float2(i < n_det ? row[i] : 0.f, 0.f);
    __syncthreads();
    fft_lds<LOG>(z, twl);
    float2* o = spec + (size_t)a * L;
    for (int i = threadIdx.x; i < L; i += kFftThreads) o[i] = z[fpad(i)];
}

// Block (a, h): rows a of filters 2h and 2h + 1 convolved with data row a.
// out[k][a][i] = sum_j filt[k][a][i - j + ctr[a]] p[a][j] = (u * p)[i + ctr[a]],
// zero where i + ctr[a] falls outside the 2 n_det - 1 samples of the linear
// convolution.
template <int LOG>
__global__ __launch_bounds__(kFftThreads, 4) void filter_conv_kernel(
    const float* __restrict__ filt, int n_filt, int n_angles, int n_det,
    const int* __restrict__ ctr, const float2* __restrict__ tw, const float2* __restrict__ spec,
    float* __restrict__ out) {
    constexpr int L = 1 << LOG;
    __shared__ float2 z[FftLds<L>::N];
    __shared__ FftTw<LOG> twl;
    twl.load(tw);
    const int npairs = (n_filt + 1) / 2;
    const int a = blockIdx.x / npairs, h = blockIdx.x % npairs;
    const int k0 = 2 * h;
    const bool second = k0 + 1 < n_filt;
    const size_t plane = (size_t)n_angles * n_det;
    const float* f0 = filt + (size_t)k0 * plane + (size_t)a * n_det;
    for (int i = threadIdx.x; i < L; i += kFftThreads) {
        float2 v = make_float2(0.f, 0.f);
        if (i < n_det) v = make_float2(f0[i], second ? f0[plane + i] : 0.f);
        z[fpad(i)] = v;
    }
    __syncthreads();
    fft_lds<LOG>(z, twl);
    // times the data spectrum; the inverse transform is conj(FFT(conj(.))) / L
    const float2* sp = spec + (size_t)a * L;
    for (int i = threadIdx.x; i < L; i += kFftThreads) {
        const float2 w = cmul(z[fpad(i)], sp[i]);
        z[fpad(i)] = make_float2(w.x, -w.y);
    }
    __syncthreads();
    fft_lds<LOG>(z, twl);
    const float inv = 1.f / (float)L;
    const int c = ctr[a];
    float* o0 = out + (size_t)k0 * plane + (size_t)a * n_det;
    for (int i = threadIdx.x; i < n_det; i += kFftThreads) {
        const int m = i + c;
        const bool ok = m >= 0 && m <= 2 * n_det - 2;
        const float2 v = ok ? z[fpad(m)] : make_float2(0.f, 0.f);
        o0[i] = v.x * inv;
        if (second) o0[plane + i] = -v.y * inv;
    }
}

// The same convolution for L >= 512 with radix-16 stages (one radix-2, 4 or 8 stage
// covers the remaining bits): at L = 8192 four passes per transform instead of seven.  The
// forward transform's first stage reads the filter rows straight from global memory;
// its last stage, the product with the data spectrum and the inverse transform's first
// stage run on the same registers (the last stage of a self-sorting transform leaves
// entry j + r L/16 with the thread that the next transform's first stage gives it);
// the inverse's last stage writes the outputs straight to global memory.
__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
    return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
    return make_float2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ float2 cmi(float2 a) { return make_float2(a.y, -a.x); }   // -i a
__device__ __forceinline__ float2 cmulc(float2 a, float wr, float wi) {
    return make_float2(fmaf(a.x, wr, -a.y * wi), fmaf(a.x, wi, a.y * wr));
}
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
    const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = cmi(csub(x1, x3));
    x0 = cadd(a0, a2);
    x1 = cadd(a1, a3);
    x2 = csub(a0, a2);
    x3 = csub(a1, a3);
}
// Forward DFT of v[0..R) in registers (exp(-2 pi i n k / R)), natural order.
template <int R>
__device__ __forceinline__ void dft_reg(float2* v);
template <>
__device__ __forceinline__ void dft_reg<2>(float2* v) {
    const float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}
template <>
__device__ __forceinline__ void dft_reg<4>(float2* v) {
    dft4(v[0], v[1], v[2], v[3]);
}
template <>
__device__ __forceinline__ void dft_reg<8>(float2* v) {
    // n = 2 n1 + n2, k = k1 + 4 k2: 4-point DFTs over n1, twiddles W8^(n2 k1), pairs
    constexpr float H = 0.70710678118654752f;
    dft4(v[0], v[2], v[4], v[6]);
    dft4(v[1], v[3], v[5], v[7]);
    v[3] = cmulc(v[3], H, -H);
    v[5] = cmi(v[5]);
    v[7] = cmulc(v[7], -H, -H);
    float2 o[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        o[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
        o[k1 + 4] = csub(v[2 * k1], v[2 * k1 + 1]);
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = o[r];
}
template <>
__device__ __forceinline__ void dft_reg<16>(float2* v) {
    // n = 4 n1 + n2, k = k1 + 4 k2: 4-point DFTs over n1, twiddles W16^(n2 k1), 4-point
    // DFTs over n2
    constexpr float C = 0.92387953251128676f, S = 0.38268343236508977f,
                    H = 0.70710678118654752f;
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
    // Y[n2][k1] sits at v[n2 + 4 k1]
    v[5] = cmulc(v[5], C, -S);      // W^1
    v[9] = cmulc(v[9], H, -H);      // W^2
    v[13] = cmulc(v[13], S, -C);    // W^3
    v[6] = cmulc(v[6], H, -H);      // W^2
    v[10] = cmi(v[10]);             // W^4
    v[14] = cmulc(v[14], -H, -H);   // W^6
    v[7] = cmulc(v[7], S, -C);      // W^3
    v[11] = cmulc(v[11], -H, -H);   // W^6
    v[15] = cmulc(v[15], -C, S);    // W^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
        dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // X[k1 + 4 k2] sits at v[4 k1 + k2]
    float2 o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = o[r];
}
// v[r] *= exp(-2 pi i r m / L) for r = 1 .. R-1 (r m < L): four table twiddles at most,
// the others as products of two of them.
template <int LOG, int R>
__device__ __forceinline__ void twiddle_reg(float2* v, int m, const FftTw<LOG>& tw) {
    float2 w[R];
    w[1] = tw(m);
    if constexpr (R >= 4) {
        w[2] = tw(2 * m);
        w[3] = cmul(w[1], w[2]);
    }
    if constexpr (R >= 8) {
        w[4] = tw(4 * m);
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
    }
    if constexpr (R >= 16) {
        w[8] = tw(8 * m);
#pragma unroll
        for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
    }
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
}
// One self-sorting radix-R stage through LDS: R sub-transforms of length ns become one
// of length R ns.
template <int LOG, int R>
__device__ void fft_stage_lds(float2* z, int ns, const FftTw<LOG>& tw) {
    constexpr int L = 1 << LOG, NBF = L / R, NB = (NBF + kFftThreads - 1) / kFftThreads;
    const int t = threadIdx.x;
    float2 v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * kFftThreads;
        if (j < NBF) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = z[fpad(j + r * NBF)];
            twiddle_reg<LOG, R>(v[i], (L / (R * ns)) * (j & (ns - 1)), tw);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * kFftThreads;
        if (j < NBF) {
            const int k = j & (ns - 1);
            dft_reg<R>(v[i]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) z[fpad(base + r * ns)] = v[i][r];
        }
    }
    __syncthreads();
}

template <int LOG>
__global__ __launch_bounds__(kFftThreads, 4) void filter_conv16_kernel(
    const float* __restrict__ filt, int n_filt, int n_angles, int n_det,
    const int* __restrict__ ctr, const float2* __restrict__ tw, const float2* __restrict__ spec,
    float* __restrict__ out) {
    static_assert(LOG >= 9, "the radix-16 path takes L >= 512");
    constexpr int L = 1 << LOG, Q = LOG / 4, RB = LOG % 4;
    constexpr int RE = RB ? (1 << RB) : 16;   // radix of the first forward / last inverse stage
    constexpr int NMID = RB ? Q - 1 : Q - 2;   // radix-16 stages through LDS per transform
    __shared__ float2 z[FftLds<L>::N];
    __shared__ FftTw<LOG> twl;
    twl.load(tw);
    const int npairs = (n_filt + 1) / 2;
    const int a = blockIdx.x / npairs, h = blockIdx.x % npairs;
    const int k0 = 2 * h;
    const bool second = k0 + 1 < n_filt;
    const size_t plane = (size_t)n_angles * n_det;
    const float* f0 = filt + (size_t)k0 * plane + (size_t)a * n_det;
    const int t = threadIdx.x;
    // forward, first stage (ns = 1, no twiddles) from the filter pair u_{2h} + i u_{2h+1}
    {
        constexpr int NBF = L / RE, NB = (NBF + kFftThreads - 1) / kFftThreads;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * kFftThreads;
            if (j < NBF) {
                float2 v[RE];
#pragma unroll
                for (int r = 0; r < RE; ++r) {
                    const int e = j + r * NBF;
                    v[r] = e < n_det ? make_float2(f0[e], second ? f0[plane + e] : 0.f)
                                     : make_float2(0.f, 0.f);
                }
                dft_reg<RE>(v);
#pragma unroll
                for (int r = 0; r < RE; ++r) z[fpad(j * RE + r)] = v[r];
            }
        }
        __syncthreads();
    }
    int ns = RE;
#pragma unroll 1
    for (int q = 0; q < NMID; ++q, ns *= 16) fft_stage_lds<LOG, 16>(z, ns, twl);
    // forward last stage (ns = L / 16: twiddle index j, outputs at j + r L / 16), times
    // the data spectrum, conjugated (the inverse is conj(FFT(conj(.))) / L), and the
    // inverse's first stage (ns = 1, inputs at j + r L / 16)
    {
        constexpr int NBF = L / 16, NB = (NBF + kFftThreads - 1) / kFftThreads;
        float2 v[NB][16];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * kFftThreads;
            if (j < NBF) {
#pragma unroll
                for (int r = 0; r < 16; ++r) v[i][r] = z[fpad(j + r * NBF)];
                twiddle_reg<LOG, 16>(v[i], j, twl);
            }
        }
        __syncthreads();
        const float2* sp = spec + (size_t)a * L;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * kFftThreads;
            if (j < NBF) {
                dft_reg<16>(v[i]);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float2 w = cmul(v[i][r], sp[j + r * NBF]);
                    v[i][r] = make_float2(w.x, -w.y);
                }
                dft_reg<16>(v[i]);
#pragma unroll
                for (int r = 0; r < 16; ++r) z[fpad(j * 16 + r)] = v[i][r];
            }
        }
        __syncthreads();
    }
    ns = 16;
#pragma unroll 1
    for (int q = 0; q < NMID; ++q, ns *= 16) fft_stage_lds<LOG, 16>(z, ns, twl);
    // inverse last stage (ns = L / RE: twiddle index j, outputs at j + r L / RE) straight
    // to the filtered data: out[k][a][i] = full[i + ctr[a]], zero off the 2 n_det - 1
    // samples of the linear convolution
    const float inv = 1.f / (float)L;
    const int c = ctr[a];
    float* o0 = out + (size_t)k0 * plane + (size_t)a * n_det;
    {
        constexpr int NBF = L / RE, NB = (NBF + kFftThreads - 1) / kFftThreads;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * kFftThreads;
            if (j < NBF) {
                float2 v[RE];
#pragma unroll
                for (int r = 0; r < RE; ++r) v[r] = z[fpad(j + r * NBF)];
                twiddle_reg<LOG, RE>(v, j, twl);
                dft_reg<RE>(v);
#pragma unroll
                for (int r = 0; r < RE; ++r) {
                    const int m = j + r * NBF, o = m - c;
                    if (m <= 2 * n_det - 2 && o >= 0 && o < n_det) {
                        o0[o] = v[r].x * inv;
                        if (second) o0[plane + o] = -v[r].y * inv;
                    }
                }
            }
        }
    }
    for (int i = t; i < n_det; i += kFftThreads) {
        const int m = i + c;
        if (m < 0 || m > 2 * n_det - 2) {
            o0[i] = 0.f;
            if (second) o0[plane + i] = 0.f;
        }
    }
}

__global__ __launch_bounds__(256) void power_normalize_kernel(
    const float* __restrict__ w, int ldx, int nr, int nc, const float* __restrict__ part,
    int n_part, float* __restrict__ xb, int xp, float* __restrict__ xt, int tp,
    float* __restrict__ est) {
    __shared__ double red[256];
    double s = 0.0;
    for (int q = threadIdx.x; q < n_part; q += 256) s += (double)part[q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double nrm = sqrt(red[0]);
    const float inv = nrm > 0.0 ? (float)(1.0 / nrm) : 0.f;
    if (blockIdx.x == 0 && threadIdx.x == 0) *est = (float)nrm;
    const size_t n = (size_t)nr * nc;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int rr = (int)(i / nc), cc = (int)(i % nc);
        const float v = w[(size_t)rr * ldx + cc] * inv;
        xb[(size_t)rr * xp + cc + kLpad] = v;
        xt[(size_t)cc * tp + rr + kLpad] = v;
    }
}

inline unsigned grid_for(size_t n, unsigned block, unsigned cap = 8192) {
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

inline unsigned pad8(int n) { return (unsigned)((n + 7) & ~7); }

}  // namespace

hipError_t launch_fp(const Job* jobs, const Item* items, int n_items, int step, int segments,
                     hipStream_t s, int contiguous, int rays_per_lane, int stage_pitch) {
    if (n_items <= 0) return hipSuccess;
    const dim3 grid(pad8(n_items));
    if (rays_per_lane == kFpStaged) {
        if (stage_pitch < 1 || stage_pitch > kFpsMaxPitch16) return hipErrorInvalidValue;
        const size_t lds = fps_lds_bytes(stage_pitch);
        const int L = fps_lines(stage_pitch);
        if (L == 32)
            hipLaunchKernelGGL(fp_staged_kernel<32>, grid, dim3(kFpsThreads), lds, s, jobs,
                               items, n_items, step, contiguous);
        else if (L == 24)
            hipLaunchKernelGGL(fp_staged_kernel<24>, grid, dim3(kFpsThreads), lds, s, jobs,
                               items, n_items, step, contiguous);
        else
            hipLaunchKernelGGL(fp_staged_kernel<16>, grid, dim3(kFpsThreads), lds, s, jobs,
                               items, n_items, step, contiguous);
        return hipGetLastError();
    }
#define TOMO_FP(SG, R)                                                                 \
    hipLaunchKernelGGL((fp_kernel<SG, R>), grid, dim3(fp_threads<SG>()), 0, s, jobs, items, \
                       n_items, step, contiguous)
    if (rays_per_lane == 2) {   // one segment per ray
        TOMO_FP(1, 2);
    } else {
        switch (segments) {
            case 1: TOMO_FP(1, 1); break;
            case 2: TOMO_FP(2, 1); break;
            case 8: TOMO_FP(8, 1); break;
            default: TOMO_FP(4, 1); break;
        }
    }
#undef TOMO_FP
    return hipGetLastError();
}

hipError_t launch_bp(const Job* jobs, const Item* items, int n_items, int step, int groups,
                     int ppt, hipStream_t s, int contiguous, int staged, int compensated,
                     int two_channel) {
    if (n_items <= 0) return hipSuccess;
    const dim3 grid(pad8(n_items));
#define TOMO_BP_T(AGV, PPTV, ST, CO, TW)                                                   \
    hipLaunchKernelGGL((bp_kernel<AGV, PPTV, ST, CO, TW>), grid, dim3(bp_threads<AGV>()), 0, \
                       s, jobs, items, n_items, step, contiguous)
#define TOMO_BP(AGV, PPTV, ST, CO) TOMO_BP_T(AGV, PPTV, ST, CO, false)
    if (two_channel && staged) {   // (g, d) pairs staged in LDS
        if (ppt == 2) TOMO_BP_T(1, 2, true, false, true);
        else TOMO_BP_T(1, 1, true, false, true);
    } else if (two_channel) {   // direct reads of (g, d) pairs
        if (ppt == 2) {
            switch (groups) {
                case 1: TOMO_BP_T(1, 2, false, false, true); break;
                case 2: TOMO_BP_T(2, 2, false, false, true); break;
                default: TOMO_BP_T(4, 2, false, false, true); break;
            }
        } else {
            switch (groups) {
                case 1: TOMO_BP_T(1, 1, false, false, true); break;
                case 2: TOMO_BP_T(2, 1, false, false, true); break;
                default: TOMO_BP_T(4, 1, false, false, true); break;
            }
        }
    } else if (compensated) {   // one shape only: staged, one group, two pixels per thread
        TOMO_BP(1, 2, true, true);
    } else if (staged) {   // one angle group: a stage's windows serve the whole tile
        if (ppt == 2) TOMO_BP(1, 2, true, false);
        else TOMO_BP(1, 1, true, false);
    } else if (ppt == 2) {
        switch (groups) {
            case 1: TOMO_BP(1, 2, false, false); break;
            case 2: TOMO_BP(2, 2, false, false); break;
            case 8: TOMO_BP(8, 2, false, false); break;
            default: TOMO_BP(4, 2, false, false); break;
        }
    } else {
        switch (groups) {
            case 1: TOMO_BP(1, 1, false, false); break;
            case 2: TOMO_BP(2, 1, false, false); break;
            case 8: TOMO_BP(8, 1, false, false); break;
            default: TOMO_BP(4, 1, false, false); break;
        }
    }
#undef TOMO_BP
#undef TOMO_BP_T
    return hipGetLastError();
}

hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_padded(float* xb, float* xt, int nr, int nc, int xp, int tp, float v,
                              hipStream_t s) {
    const size_t n = (size_t)nr * xp + (xt ? (size_t)nc * tp : 0);
    hipLaunchKernelGGL(fill_padded_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, xb, xt, nr,
                       nc, xp, tp, v);
    return hipGetLastError();
}

hipError_t launch_pad_copy(const float* src, int lds, int r0, int c0, int nr, int nc, float* xb,
                           int xp, float* xt, int tp, float* dst, int ldd, hipStream_t s) {
    const dim3 grid((nc + 31) / 32, (nr + 31) / 32);
    hipLaunchKernelGGL(pad_copy_kernel, grid, dim3(256), 0, s, src, lds, r0, c0, nr, nc, xb, xp,
                       xt, tp, dst, ldd);
    return hipGetLastError();
}

hipError_t launch_crop(const float* x, int ldx, int dr, int dc, int rows, int cols, float* out,
                       int ldo, hipStream_t s) {
    hipLaunchKernelGGL(crop_kernel, dim3(grid_for((size_t)rows * cols, 256)), dim3(256), 0, s, x,
                       ldx, dr, dc, rows, cols, out, ldo);
    return hipGetLastError();
}

hipError_t launch_check_finite(const float* p, size_t n, unsigned* flag, hipStream_t s) {
    hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, flag);
    return hipGetLastError();
}

hipError_t launch_band_gather(const float* sino, int n_det, const AngFP* afp, int n_angles,
                              float* band, int bpitch, hipStream_t s) {
    hipLaunchKernelGGL(band_gather_kernel, dim3(n_angles), dim3(256), 0, s, sino, n_det, afp,
                       band, bpitch);
    return hipGetLastError();
}

hipError_t launch_band_scatter(const float* band, int bpitch, const AngFP* afp, int n_angles,
                               float* sino, int n_det, int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(band_scatter_kernel, dim3(n_angles), dim3(256), 0, s, band, bpitch, afp,
                       sino, n_det, accumulate);
    return hipGetLastError();
}

hipError_t launch_ramp(const float* sino, int n_angles, int n_det, const float* taps,
                       const AngFP* afp, float* band, int bpitch, hipStream_t s) {
    const size_t lds = (size_t)(n_det + 2) * sizeof(float);
    hipLaunchKernelGGL(ramp_kernel, dim3((n_det + 255) / 256, n_angles), dim3(256), lds, s, sino,
                       n_det, taps, afp, band, bpitch);
    return hipGetLastError();
}

hipError_t launch_power_normalize(const float* w, int ldx, int nr, int nc, const float* part,
                                  int n_part, float* xb, int xp, float* xt, int tp, float* est,
                                  hipStream_t s) {
    hipLaunchKernelGGL(power_normalize_kernel, dim3(grid_for((size_t)nr * nc, 256, 256)),
                       dim3(256), 0, s, w, ldx, nr, nc, part, n_part, xb, xp, xt, tp, est);
    return hipGetLastError();
}

hipError_t launch_fgp(const Job* jobs, const Item* items, int n_items, int step, int i0,
                      hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(fgp_kernel, dim3(n_items), dim3(kFgpThreads), 0, s, jobs, items, n_items,
                       step, i0);
    return hipGetLastError();
}

hipError_t launch_disc(float* img, int ld, int n, int r0, int c0, int rows, int cols,
                       const float* value, int add, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(disc_kernel, dim3((cols + 255) / 256, rows), dim3(256), 0, s, img, ld, n,
                       r0, c0, rows, cols, value, add);
    return hipGetLastError();
}

hipError_t launch_disc_value(const float* p, const float* D, int na, int nd, double* st,
                             float* value, hipStream_t s) {
    if (na <= 0) return hipSuccess;
    hipLaunchKernelGGL(disc_sums_kernel, dim3(na), dim3(256), 0, s, p, D, nd, st);
    hipLaunchKernelGGL(disc_value_kernel, dim3(1), dim3(256), 0, s, st, na, value);
    return hipGetLastError();
}

hipError_t launch_disc_apply(const float* p, const float* D, size_t n, const float* value,
                             float* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(disc_apply_kernel, dim3(blocks), dim3(256), 0, s, p, D, n, value, out);
    return hipGetLastError();
}

hipError_t launch_pad_truncated(const float* trunc, int na, int nb, int first, int nd,
                                float* out, hipStream_t s) {
    if (na <= 0 || nd <= 0) return hipSuccess;
    hipLaunchKernelGGL(pad_truncated_kernel, dim3((nd + 255) / 256, na), dim3(256), 0, s, trunc,
                       nb, first, nd, out);
    return hipGetLastError();
}

hipError_t launch_haar(const Job* jobs, const Item* items, int n_items, int step, int levels,
                       hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    switch (levels) {
#define X(LV)                                                                                  \
    case LV:                                                                                   \
        hipLaunchKernelGGL(haar_kernel<LV>, dim3(n_items), dim3(256), 0, s, jobs, items,       \
                           n_items, step);                                                     \
        break;
        X(1) X(2) X(3) X(4) X(5) X(6)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define TOMO_FFT_CASES(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#define TOMO_FFT_SMALL(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#define TOMO_FFT_LARGE(X) X(9) X(10) X(11) X(12) X(13) X(14)

hipError_t launch_spectra(const float* sino, int n_angles, int n_det, int log2_len,
                          const float2* tw, float2* spec, hipStream_t s) {
    if (n_angles <= 0) return hipSuccess;
    switch (log2_len) {
#define X(LG)                                                                                  \
    case LG:                                                                                   \
        hipLaunchKernelGGL(spectra_kernel<LG>, dim3(n_angles), dim3(kFftThreads), 0, s, sino,  \
                           n_det, tw, spec);                                                   \
        break;
        TOMO_FFT_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_filter_conv(const float* filters, int n_filt, int n_angles, int n_det,
                              const int* ctr, int log2_len, const float2* tw, const float2* spec,
                              float* out, hipStream_t s) {
    if (n_filt <= 0 || n_angles <= 0) return hipSuccess;
    const dim3 grid((unsigned)(n_angles * ((n_filt + 1) / 2)));
    switch (log2_len) {
#define X(LG)                                                                                  \
    case LG:                                                                                   \
        hipLaunchKernelGGL(filter_conv_kernel<LG>, grid, dim3(kFftThreads), 0, s, filters,     \
                           n_filt, n_angles, n_det, ctr, tw, spec, out);                       \
        break;
        TOMO_FFT_SMALL(X)
#undef X
#define X(LG)                                                                                  \
    case LG:                                                                                   \
        hipLaunchKernelGGL(filter_conv16_kernel<LG>, grid, dim3(kFftThreads), 0, s, filters,   \
                           n_filt, n_angles, n_det, ctr, tw, spec, out);                       \
        break;
        TOMO_FFT_LARGE(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef TOMO_FFT_CASES
#undef TOMO_FFT_SMALL
#undef TOMO_FFT_LARGE

}  // namespace tomo
