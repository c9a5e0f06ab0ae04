// Allocation-free Ram-Lak FBP, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// tomo_fbp_ramlak keeps its scratch (the work list, the job descriptor, the
// per-angle tables and the filtered band) in blocks of the context's workspace.
// The variant here keeps the same scratch in one static device array per GPU,
// fills it with kernels and copies from host tables that live as long as the
// geometry, and then runs the same three kernels (fill, Ram-Lak filter,
// compensated staged backprojection), so its result has the same bits.
#include <cinttypes>
#include <cmath>

#include "tomo_runtime.h"

namespace tomo {

constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

// Every GPU the library runs on holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in, never the device memory: the
// device address comes from hipGetSymbolAddress (scratch_ptr below).
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

char* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

// Work items of the backprojector over the whole grid, in the order bp_items
// lists them: tile row a, tile column b, item a * ntc + b.
__global__ void fbp_items_kernel(Item* items, int n_items, int ntc, const AngBP* tab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    Item it;
    it.job = 0;
    it.a = i / ntc;
    it.b = i % ntc;
    it.pad = 0;
    it.tab = tab;
    it.pad2 = 0;
    items[i] = it;
}

// The job descriptor arrives as a kernel argument; one lane per 32-bit word stores it.
constexpr int kJobWords = (int)(sizeof(Job) / 4);
static_assert(sizeof(Job) % 4 == 0, "Job is a whole number of words");
struct JobWords {
    uint32_t w[kJobWords];
};

__global__ void store_job_kernel(uint32_t* dst, JobWords j) {
    const int i = threadIdx.x;
    if (i < kJobWords) dst[i] = j.w[i];
}

}  // namespace

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return hipSuccess;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = (char*)p;
    return hipSuccess;
}

}  // namespace tomo

using namespace tomo;

extern "C" tomo_status tomo_fbp_ramlak_noalloc(tomo_ctx* ctx, int32_t geom, const float* sino,
                                               float* img, void* hip_stream) {
    tomo_status st = need_gpu(ctx);
    if (st != TOMO_OK) return st;
    if (!img || !sino) return fail(ctx, TOMO_EINVAL, "null pointer");
    GUARD_BEGIN
    const Geom* gp;
    if ((st = get_geom(ctx, geom, &gp)) != TOMO_OK) return st;
    const Geom& g = *gp;
    if (g.nd > 16384) return fail(ctx, TOMO_EINVAL, "FBP supports at most 16384 detector bins");
    char* base = scratch_ptr(ctx->device);
    if (!base) return fail(ctx, TOMO_EHIP, "no scratch address for device %d", ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const Plan& P = g.full;
    // the shape of tomo_fbp_ramlak: staged band windows, one angle group, two pixels
    // per thread, compensated angle sums; the XCD order as the size heuristic picks it
    LaunchCfg L = choose_launch(ctx, 0, (long long)g.n * g.n);
    L.staged = 1;
    L.ag = 1;
    L.ppt = 2;
    int th, tw;
    bp_tile(L.ag, L.ppt, &th, &tw);
    const int ntr = (g.n + th - 1) / th, ntc = (g.n + tw - 1) / tw;
    const size_t n_items = (size_t)ntr * ntc;
    const size_t o_job = 0;
    const size_t o_afp = align_up(sizeof(Job), 256);
    const size_t o_abp = o_afp + align_up((size_t)g.na * sizeof(AngFP), 256);
    const size_t o_it = o_abp + align_up((size_t)g.na * sizeof(AngBP), 256);
    const size_t o_band = o_it + align_up(n_items * sizeof(Item), 256);
    const size_t n_band = (size_t)g.na * P.bpitch;
    const size_t need = o_band + n_band * sizeof(float);
    if (need > kScratchBytes || n_items > (size_t)INT32_MAX)
        return fail(ctx, TOMO_EINVAL,
                    "the allocation-free FBP needs %zu bytes of scratch for a %dx%d grid with %d "
                    "angles and %d bins; its limit is %zu bytes",
                    need, g.n, g.n, g.na, g.nd, kScratchBytes);
    AngFP* d_afp = (AngFP*)(base + o_afp);
    AngBP* d_abp = (AngBP*)(base + o_abp);
    Item* d_items = (Item*)(base + o_it);
    float* band = (float*)(base + o_band);
    Job J;
    std::memset(&J, 0, sizeof J);
    J.nr = g.n;
    J.nc = g.n;
    J.xp = P.xp;
    J.tp = P.tp;
    J.n_angles = g.na;
    J.bpitch = P.bpitch;
    J.n_det = g.nd;
    J.bp_mode = BP_STORE;
    J.ldx = g.n;
    J.scale = (float)(M_PI / g.na * g.spacing);
    J.afp = d_afp;
    J.abp = d_abp;
    J.x = img;
    J.y = band;
    JobWords jw;
    std::memcpy(jw.w, &J, sizeof J);
    // the host tables belong to the geometry, which lives as long as the context
    TOMO_HIP(ctx, hipMemcpyAsync(d_afp, P.afp.data(), (size_t)g.na * sizeof(AngFP),
                                 hipMemcpyHostToDevice, s));
    TOMO_HIP(ctx, hipMemcpyAsync(d_abp, P.abp.data(), (size_t)g.na * sizeof(AngBP),
                                 hipMemcpyHostToDevice, s));
    fbp_items_kernel<<<(unsigned)((n_items + 255) / 256), 256, 0, s>>>(d_items, (int)n_items, ntc,
                                                                       d_abp);
    TOMO_HIP(ctx, hipGetLastError());
    store_job_kernel<<<1, ((kJobWords + 63) / 64) * 64, 0, s>>>((uint32_t*)(base + o_job), jw);
    TOMO_HIP(ctx, hipGetLastError());
    TOMO_HIP(ctx, launch_fill(band, n_band, 0.f, s));
    TOMO_HIP(ctx, launch_ramp(sino, g.na, g.nd, g.d_taps, d_afp, band, P.bpitch, s));
    TOMO_HIP(ctx, launch_bp((const Job*)(base + o_job), d_items, (int)n_items, 0, L.ag, L.ppt, s,
                            L.cbp, 1, 1));
    return TOMO_OK;
    GUARD_END(ctx)
}
