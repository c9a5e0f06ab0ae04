// Host runtime internals: geometry, planning tables, the workspace arena and
// the context.  Shared by the C ABI (tomo_capi.cpp) and the serving scheduler
// (tomo_serve.cpp).
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/tomo.h"
#include "tomo_internal.h"

namespace tomo {

struct Rect {
    int r0, c0, rows, cols;
};

// Host tables of one job: an image region and the detector band of a (possibly
// different) band source region.
struct Plan {
    Rect reg{};
    std::vector<AngFP> afp;
    std::vector<AngBP> abp;
    int wmax = 0;
    int bpitch = 0;
    int xp = 0, tp = 0;
};

// Parallel-beam geometry (Section 2.1); the row/column-stepping branch of
// Joseph's method is decided here, once, in FP64.
struct Geom {
    int n = 0, na = 0, nd = 0;
    double spacing = 1.0, offset = 0.0;
    std::vector<double> th, c, s, m;
    std::vector<int> ystep;
    float* d_taps = nullptr;   // Ram-Lak taps h[d] / spacing as FP32 pairs (hi, lo), d < nd
                               // (device, GPU contexts)
    size_t taps_off = 0;
    Plan full;                 // tables of the whole grid (FBP), made once with the geometry
};

void band_of(const Geom& g, const Rect& b, int k, int* i0, int* w);
Plan make_plan(const Geom& g, const Rect& reg, const Rect& band_src);
Rect extend_rect(const Rect& roi, int margin, int n);

// First-fit allocator over the caller's workspace.  Frees are deferred until
// an event recorded on the stream that last used the memory has completed, so
// memory is only reused in stream order.
class Arena {
public:
    void init(char* base, size_t bytes);
    // Returns nullptr when the request does not fit even after reclaiming all
    // completed deferred frees (waiting for them when `wait` is true).
    char* alloc(size_t bytes, bool wait = true);
    void free_now(char* p);
    void free_after(std::vector<char*> ps, hipStream_t s);
    void reclaim(bool wait);
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t capacity() const { return size_; }
    size_t largest_free() const;

private:
    char* base_ = nullptr;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> live_;   // offset -> length
    std::deque<std::pair<hipEvent_t, std::vector<char*>>> pending_;
    std::recursive_mutex mu_;
    void release_locked(size_t off);
};

// Pinned host staging for small uploads (tables, job descriptors, work lists).
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool ev_live = false;
    hipError_t upload(void* dev, const void* src, size_t bytes, hipStream_t s);
    void destroy();
};

struct SinoState;
struct ServeState;

// A captured hipGraph of a whole iteration loop (all FP / BP launches of a
// solve), replayed for later solves with the same work-list layout.  Its job
// and item arrays live in `dbuf` (owned by the entry); each solve uploads its
// own descriptors there before replaying.
struct GraphEntry {
    char* dbuf = nullptr;
    size_t bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t last = nullptr;
    long long stamp = 0;
};

}  // namespace tomo

struct tomo_ctx {
    tomo_ctx();
    ~tomo_ctx();   // defined where the serving state is a complete type
    int device = -1;
    bool host_only = true;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    tomo::Arena arena;
    tomo::Staging staging;
    std::string err;
    std::recursive_mutex mu;   // geometry list, caches, registrations
    std::deque<tomo::Geom> geoms;   // deque: references stay valid while serving reads them
    // lambda_max(W_L^T W_L - Laplacian) by (geometry, rounded rows, rounded cols)
    std::map<std::tuple<int, int, int>, float> step_cache;
    tomo_launch knobs{};   // launch shape forced by the user; 0 fields = automatic
    std::map<std::tuple<int, int, int>, tomo_launch> tuned;   // autotuner results by class
    std::map<int, std::unique_ptr<tomo::SinoState>> sinos;
    int next_sino = 1;
    std::unique_ptr<tomo::ServeState> serve;
    // cached iteration graphs, keyed by the work-list layout
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    std::map<std::vector<long long>, tomo::GraphEntry> graphs;
    std::map<std::vector<long long>, int> graph_seen;
    long long graph_clock = 0;
    // kernel timing (measurement hook)
    int timing_mode = 0;   // 0 off, 1 events around every launch, 2 graph-bracketed pass
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::tuple<hipEvent_t, hipEvent_t, int>> ev_pending;
    long long t_launches[3] = {0, 0, 0};   // fp, bp, fgp
    double t_ms[3] = {0.0, 0.0, 0.0};
};

namespace tomo {

tomo_status fail(tomo_ctx* ctx, tomo_status st, const char* fmt, ...);

// A named host range for profilers that record ROCTx markers (rocprofv3
// --marker-trace): pushed on construction, popped on destruction.
class TraceRange {
public:
    TraceRange(const char* fmt, ...) {
        char buf[160];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        roctxRangePushA(buf);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

#define TOMO_HIP(ctx, expr)                                                                 \
    do {                                                                                     \
        hipError_t e__ = (expr);                                                             \
        if (e__ != hipSuccess)                                                               \
            return ::tomo::fail((ctx), TOMO_EHIP, "%s failed: %s", #expr, hipGetErrorString(e__)); \
    } while (0)

// Host exceptions never cross the C ABI.
#define GUARD_BEGIN try {
#define GUARD_END(ctx)                                                                  \
    }                                                                                   \
    catch (const std::bad_alloc&) {                                                     \
        return fail((ctx), TOMO_ENOMEM, "host allocation failed");                      \
    }                                                                                   \
    catch (...) {                                                                       \
        return fail((ctx), TOMO_EINVAL, "unexpected host exception");                   \
    }

tomo_status need_gpu(tomo_ctx* ctx);   // GPU context with its device made current

// Looks up, once per device (the device current), the address of the static scratch array
// of the allocation-free entry point (tomo_noalloc.hip).
hipError_t noalloc_setup(int device);

// Returns the listed workspace blocks to the arena after the work already queued
// on `s` when the scope ends (also on an early error return).
struct ArenaRelease {
    tomo_ctx* ctx;
    hipStream_t s;
    std::vector<char*> ptrs;
    ~ArenaRelease();
};
tomo_status get_geom(tomo_ctx* ctx, int32_t gid, const Geom** g);

// ---- solve pipeline shared by roi_solve, roi_solve_batch and serving ----

struct RoiState {
    roi_params prm{};
    Rect roi{}, ext{};
    Plan plan;            // ext region, ext band
    Plan plan_full;       // full grid, ext band (exterior projection)
    // device
    char* block = nullptr;   // contiguous zero-initialised state
    size_t state_floats = 0;   // x .. y (re-zeroed before iterating)
    size_t total_floats = 0;   // x .. part
    float *x = nullptr, *xb0 = nullptr, *xb1 = nullptr, *xt = nullptr, *z0 = nullptr,
          *z1 = nullptr, *y = nullptr, *b = nullptr, *part = nullptr;
    AngFP* d_afp = nullptr;
    AngBP* d_abp = nullptr;
    AngFP* d_afp_full = nullptr;
    float sigma = 0.f, tau = 0.f;
    int ntr = 0, ntc = 0;
};

struct LaunchCfg {
    int seg = 4, ag = 4, ppt = 1;
    int rp = 1;             // forward projector rays per lane (2 only with seg 1)
    int cfp = 1, cbp = 1;   // XCD order of FP / BP items: 1 contiguous, 0 round-robin
    int staged = 0;         // backprojector variant: 1 = LDS-staged band windows
    int spitch = 0;         // rp == kFpStaged: the largest line pitch of the launch's jobs
};

// max_pitch, max_w: the largest line pitch (xp or tp) and band width of the jobs the
// forward projector will run on (0 = not known: the LDS-staged variant is not used).
LaunchCfg choose_launch(const tomo_ctx* ctx, long long total_rays, long long total_pixels,
                        int max_pitch = 0, int max_w = 0);
// As choose_launch, preferring an autotuned shape for (geometry, pixels, jobs).
LaunchCfg choose_launch_for(tomo_ctx* ctx, int gid, int jobs, long long total_rays,
                            long long total_pixels, int max_pitch = 0, int max_w = 0);
std::tuple<int, int, int> tune_key(int gid, int jobs, long long total_pixels);
void bp_tile(int ag, int ppt, int* th, int* tw);
size_t state_bytes(const Geom& g, const Plan& p);
tomo_status validate_params(tomo_ctx* ctx, const Geom& g, const roi_params& p);
hipEvent_t timing_event(tomo_ctx* ctx);
long long count_nnz(const Geom& g, const Rect& reg);
size_t step_size_scratch_bytes(tomo_ctx* ctx, int gid, const RoiState& st);
// The serving test executor (host-only contexts, which never solve): the request's
// step-size shape counts as computed from now on, as after a GPU preparation.
void step_size_assume_cached(tomo_ctx* ctx, int gid, const RoiState& st);
tomo_status step_size_for(tomo_ctx* ctx, int gid, RoiState& st, hipStream_t s, Staging& stg);
Job make_job(const Geom& g, const RoiState& st, int fp_mode, int bp_mode, int ntc);
// Work items; the device table pointers must already be known (items store them).
void fp_items(std::vector<Item>& out, int jj, const std::vector<AngFP>& afp, int seg, int rp,
              const AngFP* d_afp);
void bp_items(std::vector<Item>& out, int jj, int nr, int nc, int ag, int ppt,
              const AngBP* d_abp);
size_t count_fp_items(const std::vector<AngFP>& afp, int seg, int rp = 1);
size_t count_bp_items(int nr, int nc, int ag, int ppt);
void carve_state(const Geom& g, RoiState& st, char* blk);
tomo_status fbp_into(tomo_ctx* ctx, int gid, const float* sino, float* plain, float* xb, float* xt,
                     const Plan& P, hipStream_t s, std::vector<char*>& allocs, Staging& stg);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
struct Meta;
// Launches an iteration loop through the context's graph cache (see tomo_capi.cpp).
tomo_status run_loop(tomo_ctx* ctx, const std::vector<long long>& key, const Meta& m2,
                     const std::function<hipError_t(char*, hipStream_t)>& enqueue, hipStream_t s,
                     std::vector<char*>& allocs);

// Packs small host arrays for one upload into one device block.
struct Meta {
    std::vector<char> buf;
    size_t add(const void* p, size_t n) {
        const size_t off = align_up(buf.size(), 64);
        buf.resize(off + n);
        if (n) std::memcpy(buf.data() + off, p, n);
        return off;
    }
    size_t reserve(size_t n) {
        const size_t off = align_up(buf.size(), 64);
        buf.resize(off + n);
        return off;
    }
    void put(size_t off, const void* p, size_t n) {
        if (n) std::memcpy(buf.data() + off, p, n);
    }
};

}  // namespace tomo
