// Resident sinograms and the serving scheduler (continuous batching of ROI solves).
#pragma once

#include "tomo_runtime.h"

namespace tomo {

// A registered sinogram: the caller's data plus its exterior estimate and the
// residual r = p - W x_ext, computed once and reused by every local part
// (Section 3.3: precompute once, reuse across repeated local reconstructions).
struct SinoState {
    int gid = 0;
    const float* sino = nullptr;   // borrowed
    float* x_plain = nullptr;      // [n][n]
    float* xb = nullptr;           // padded [n][xp]
    float* xt = nullptr;           // padded transposed [n][tp]
    float* resid = nullptr;        // [n_angles][n_det]
    int xp = 0, tp = 0;
    char* block = nullptr;
    std::atomic<int> users{0};
};

// outs[i]: ROI i's crop, row pitch ldo (0: the ROI's width, i.e. contiguous).
// states[i] (optional, device): ROI i's iteration state, read when done > 0 (the
// state after `done` earlier iterations) and written after the solve.
tomo_status solve_batch(tomo_ctx* ctx, int gid, const float* sino, const float* x_ext_user,
                        const SinoState* reg, int count, const roi_params* params,
                        float* const* outs, hipStream_t s, int ldo = 0,
                        float* const* states = nullptr, int done = 0);

// Compute x_ext (Ram-Lak FBP) and r into a SinoState's buffers on stream s.
tomo_status build_resident(tomo_ctx* ctx, SinoState& S, hipStream_t s);

void serve_shutdown(tomo_ctx* ctx);
void serve_drain(tomo_ctx* ctx);   // until no request is queued or running
bool serve_is_fake(const tomo_ctx* ctx);   // serving through the host test executor

// Errors raised on the scheduler thread go to a thread-local buffer instead of
// the context's last-error string (which belongs to the caller's thread).
bool on_serve_thread();
void set_thread_error(const char* msg);

}  // namespace tomo
