// Internal types shared by the HIP kernels and the host runtime.
//
// A "job" is one image region with its detector band: the extended local part
// of one ROI solve, or the whole grid (FBP, exterior projection).  The two
// batched kernels take an array of jobs and a flat list of work items, so one
// launch serves any number of ROIs of any size (Section 5.6: independent local
// parts reconstructed in parallel).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tomo {

// Padded image layout (xbar [n_r][xp], xbar^T [n_c][tp]): column c of a row is
// stored at c + kLpad, with zeros before it and at least two zeros after the
// last column, so an interpolation read that starts up to 3 entries left of
// the first column stays inside the row.
constexpr int kLpad = 4;

// Per (job, angle) table of the ray-driven forward projector (Joseph, Section 2.1).
// Ray j of the band crosses outer line o (a row, or a column when tr = 1) at the
// storage coordinate  pos = a0 + j * aj + o * step  (inner index + kLpad).
struct AngFP {
    double a0;
    double aj;
    double step;
    float inv_m;      // 1 / max(|cos|, |sin|): path length per outer step
    int32_t w;        // band width (rays)
    int32_t i0;       // global bin of band position 0 (may lie off the detector)
    int32_t tr;       // 1: step along columns, read the transposed image
    float bscale;     // B = spacing / m^2: band arrays read by the backprojector hold B * y
    int32_t pad1;
};
static_assert(sizeof(AngFP) == 48, "AngFP layout");

// Per (job, angle) table of the pixel-driven backprojector.  Pixel (r, c) of the
// region lands at padded band coordinate u = c * cu + r * su + u0 and touches band
// entries floor(u) and floor(u) + 1.  With f = u - floor(u), A = 1/m and
// B = spacing / m^2, the hat max(0, 1 - |s_i - t| / m) / m gives the weights
//   max(0, A - f B) = B max(0, r - f)   and   max(0, (A - B) + f B) = B max(0, f + r - 1),
// r = A / B = m / spacing.  Band arrays read by the backprojector store B * y, so
// the kernel only evaluates max(0, r - f) and max(0, f + rm1), rm1 = r - 1.
// The FP64 terms place a tile's reference point; the FP32 copies of cu and su
// carry the small offsets of the tile's pixels from it.
struct AngBP {
    float cu, su, r, rm1;     // FP32: read as one 16-byte scalar load per angle
    double cud, sud, u0;      // FP64: per-tile anchors
    double pad;
};
static_assert(sizeof(AngBP) == 48, "AngBP layout");

enum FpMode : int32_t {
    FP_STORE = 0,            // gout[k][i] = fp (on-detector bins of the band)
    FP_ACCUM = 1,            // gout[k][i] += fp
    FP_BAND_FROM_GLOBAL = 2, // y[k][j] = gbase[k][i] + scale * fp
    FP_BAND_ADD = 3,         // y[k][j] += scale * fp
    FP_CP_DUAL = 4,          // y <- (y + sigma (fp - b)) * dual_div
    FP_SIRT = 5,             // y <- alpha (b - fp)
    FP_BAND_STORE = 6,       // y = fp
    FP_RESID = 7,            // gout[k][i] = gbase[k][i] + scale * fp
    FP_FILTER = 8,           // y = -alpha fp;  gout[k][i] = gbase[k][i] + alpha fp
    FP_LOCAL = 9             // y = (d - alpha fp, d), d = plane (step + dk0) of gbase
};

enum BpMode : int32_t {
    BP_STORE = 0,   // x = scale * bp   (optional padded copies)
    BP_ACCUM = 1,   // x += scale * bp
    BP_CP = 2,      // TV dual + primal prox + extrapolation
    BP_SIRT = 3,    // x = clamp(x + bp, lo, hi)
    BP_POWER = 4,   // x = bp - div grad v, per-tile sums of x^2
    BP_LOCAL = 5,   // two-channel band (g, d): x = clamp(v + bp_g, lo, hi), v <- x - bp_d
    BP_FISTA = 6    // two-channel band (g, d): w = v + bp_g, xs = bp_d (FGP input and x_s)
};

enum JobFlags : int32_t { JF_HALF = 1, JF_ANISO = 2, JF_NO_MOMENTUM = 8, JF_PIXEL_UNITS = 16 };

struct Job {
    int32_t nr, nc;          // region rows, cols
    int32_t xp, tp;          // pitch of padded xbar [nr][xp] (col c at c + kLpad) and of xbarT [nc][tp]
    int32_t n_angles;        // band rows
    int32_t bpitch;          // band pitch (band position j stored at j + 1)
    int32_t n_det;           // detector bins (off-detector band entries are kept at 0)
    int32_t fp_mode, bp_mode;
    int32_t flags;
    int32_t parity0;         // xbar/z buffer read at launch step s: (s + parity0) & 1
    int32_t ldx;             // pitch of x
    int32_t ntc;             // tiles per row of the BP work decomposition
    int32_t dk0;             // FP_LOCAL: plane of gbase read at launch step s is s + dk0
    float sigma, tau, lam, dual_div, alpha, scale;
    float sigma_y;           // CP data-dual step: sigma h^2 (the dual is stored as h y)
    float lo, hi;            // box of the SIRT-type updates
    int64_t gstride;         // FP_LOCAL: floats between planes of gbase
    const AngFP* afp;
    const AngBP* abp;
    float* x;                // primal / output image [nr][ldx]
    float* xb[2];            // padded xbar, ping-pong
    float* xt;               // padded transposed xbar
    float* z[2];             // TV dual [2][nr][nc], ping-pong
    float* y;                // band array [n_angles][bpitch] (dual / FP output / BP input);
                             // two-channel modes: [n_angles][bpitch][2]
    const float* b;          // band data [n_angles][bpitch]
    float* gout;             // full-detector sinogram output [n_angles][n_det]
    const float* gbase;      // full-detector sinogram base
    float* part;             // per-tile partial sums (BP_POWER)
    // local FISTA-TV (BP_FISTA + fgp_kernel)
    float* w;                // FGP input x_s + q [nr][nc]
    float* xs;               // x_s = W_L^T d [nr][nc]
    float* fp;               // FGP dual p [2][nr][nc]
    float* fr;               // FGP dual momentum point r [2][nr][nc]
    const float* beta_in;    // FGP momentum per inner iteration
    const float* beta_out;   // FISTA momentum per outer iteration
    float gamma;             // prox weight of TV / threshold of the Haar coefficients
    int32_t n_fgp;           // FGP iterations per outer iteration
    int32_t levels;          // Haar levels (local FISTA with the Haar l1 prior)
};

// One block's work.  `tab` points at the block's table (FP: the AngFP entry of
// its angle; BP: the job's AngBP array) so the kernel can fetch the job
// descriptor and the table at the same time.
struct Item {
    int32_t job, a, b, pad;  // FP: angle, ray chunk; BP: tile row, tile col
    const void* tab;
    int64_t pad2;
};
static_assert(sizeof(Item) == 32, "Item layout");

// LDS-staged forward projector: L image lines per stage (stride L + 1, L + 2 zero
// columns on each side), kFpsThreads threads, at most kFpsMaxPairs (angle, ray) pairs per
// block.  32 lines per stage for line pitches up to kFpsMaxPitch, 24 up to
// kFpsMaxPitch24, 16 up to kFpsMaxPitch16: each keeps the LDS of a block under a third
// of the CU's 160 KB (beyond 752 entries, 16-line stages fit two blocks per CU).
constexpr int kFpStaged = 4;   // the rays_per_lane value that selects it
constexpr int kFpsThreads = 512;   // eight waves: three blocks per CU give six waves per SIMD
constexpr int kFpsMaxRounds = 8, kFpsMaxPairs = kFpsMaxRounds * kFpsThreads;
constexpr int kFpsMaxPitch = 336;     // (336 + 68) x 33 x 4 B = 53.3 KB
constexpr int kFpsMaxPitch24 = 480;   // (480 + 52) x 25 x 4 B = 53.2 KB
constexpr int kFpsMaxPitch16 = 784;   // (784 + 36) x 17 x 4 B = 55.8 KB
inline int fps_lines(int pitch) {
    return pitch <= kFpsMaxPitch ? 32 : pitch <= kFpsMaxPitch24 ? 24 : 16;
}
inline size_t fps_lds_bytes(int pitch) {
    const int L = fps_lines(pitch);
    return (size_t)(pitch + 2 * (L + 2)) * (L + 1) * sizeof(float);
}

// Launchers (tomo_kernels.hip).
// contiguous = 1: each XCD runs one contiguous eighth of the items (L2
// locality for many small jobs); 0: item b runs on XCD b mod 8 (balanced).
// rays_per_lane = 2: each lane projects two adjacent rays from 4-pixel reads
// (segments must be 1; the items must be built for 512 rays per block).
// rays_per_lane = kFpStaged: the LDS-staged forward projector (items from fps_items;
// stage_pitch = the largest line pitch, xp or tp, of the launch's jobs, at most
// kFpsMaxPitch16; a larger value than the jobs need only selects shorter stages).
hipError_t launch_fp(const Job* jobs, const Item* items, int n_items, int step, int segments,
                     hipStream_t s, int contiguous = 1, int rays_per_lane = 1,
                     int stage_pitch = 0);
// staged = 1: band windows staged in LDS (one angle group; throughput shape),
// 0: direct band reads (any group count; latency shape).  Same results.
// compensated = 1: compensated sums over angles, staged, groups 1, ppt 2 only
// (the items must be built for that tiling).
// two_channel = 1: the band holds (g, d) pairs (BP_LOCAL / BP_FISTA jobs only); staged
// or direct reads.
hipError_t launch_bp(const Job* jobs, const Item* items, int n_items, int step, int groups,
                     int ppt, hipStream_t s, int contiguous = 1, int staged = 0,
                     int compensated = 0, int two_channel = 0);
// FGP iterations [i0, i0 + kFgpSteps) of every FISTA job, on tiles of
// kFgpTile x kFgpTile pixels (items: job, tile row, tile column); the launch that
// reaches a job's last inner iteration also forms x, the FISTA momentum point and
// the new correction v (written to the padded copies read at step + 1).  48-pixel tiles
// recompute a smaller share of halo pixels than 32-pixel ones (66^2 windows against 50^2)
// and, with 1024-thread blocks, keep five pixels per thread in registers.
constexpr int kFgpTile = 48, kFgpSteps = 8;
hipError_t launch_fgp(const Job* jobs, const Item* items, int n_items, int step, int i0,
                      hipStream_t s);
// Haar l1 prox of local FISTA: per aligned 2^levels tile of the job (items: job, tile
// row, tile column), forward transform, soft threshold gamma, inverse, then the FISTA
// momentum point and the new correction v (as the last FGP launch).  levels 1..6.
constexpr int kHaarMaxLevels = 6;
hipError_t launch_haar(const Job* jobs, const Item* items, int n_items, int step, int levels,
                       hipStream_t s);
// Disc of diameter n about the grid centre (exact integer test): add = 0 writes its
// indicator into the region (r0, c0, rows, cols) of img (pitch ld); add = 1 adds *value
// on its pixels.
hipError_t launch_disc(float* img, int ld, int n, int r0, int c0, int rows, int cols,
                       const float* value, int add, hipStream_t s);
// *value = sum_a S_a T_a / sum_a T_a^2 with S, T the FP64 row sums of p and D (st: 2 na doubles).
hipError_t launch_disc_value(const float* p, const float* D, int na, int nd, double* st,
                             float* value, hipStream_t s);
// out = p - *value * D (out may be p).
hipError_t launch_disc_apply(const float* p, const float* D, size_t n, const float* value,
                             float* out, hipStream_t s);
// Rows of nb measured bins starting at detector bin `first`, extended to nd bins with
// their edge values.
hipError_t launch_pad_truncated(const float* trunc, int na, int nb, int first, int nd,
                                float* out, hipStream_t s);
hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s);
hipError_t launch_fill_padded(float* xb, float* xt, int nr, int nc, int xp, int tp, float v,
                              hipStream_t s);
hipError_t launch_pad_copy(const float* src, int lds, int r0, int c0, int nr, int nc,
                           float* xb, int xp, float* xt, int tp, float* dst, int ldd,
                           hipStream_t s);
// out[r][c] (row pitch ldo) = x[r + dr][c + dc] (row pitch ldx), r < rows, c < cols.
hipError_t launch_crop(const float* x, int ldx, int dr, int dc, int rows, int cols, float* out,
                       int ldo, hipStream_t s);
// *flag = 1 when any of p[0 .. n) is NaN or infinite (flag left as it is otherwise).
hipError_t launch_check_finite(const float* p, size_t n, unsigned* flag, hipStream_t s);
hipError_t launch_band_gather(const float* sino, int n_det, const AngFP* afp, int n_angles,
                              float* band, int bpitch, hipStream_t s);
hipError_t launch_band_scatter(const float* band, int bpitch, const AngFP* afp, int n_angles,
                               float* sino, int n_det, int accumulate, hipStream_t s);
hipError_t launch_ramp(const float* sino, int n_angles, int n_det, const float* taps,
                       const AngFP* afp, float* band, int bpitch, hipStream_t s);
// Detector convolutions by FFT (length L = 2^log2_len >= 2 n_det - 1, twiddles
// tw[m] = exp(-2 pi i m / L) in FP32).  spectra: spec[a][L] = FFT of sino row a
// (zero-padded).  filter_conv: for each angle a and filter pair (2h, 2h + 1) of
// `filters` [n_filt][n_angles][n_det], out[k][a][i] = sum_j filt[k][a][i - j + ctr[a]] sino[a][j].
hipError_t launch_spectra(const float* sino, int n_angles, int n_det, int log2_len,
                          const float2* tw, float2* spec, hipStream_t s);
hipError_t launch_filter_conv(const float* filters, int n_filt, int n_angles, int n_det,
                              const int* ctr, int log2_len, const float2* tw, const float2* spec,
                              float* out, hipStream_t s);
hipError_t launch_power_normalize(const float* w, int ldx, int nr, int nc, const float* part,
                                  int n_part, float* xb, int xp, float* xt, int tp, float* est,
                                  hipStream_t s);

}  // namespace tomo
