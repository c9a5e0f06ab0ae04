// Serving: resident sinograms and a continuous-batching scheduler for ROI solves.
//
// Requests join a bounded host queue (roi_submit never blocks).  A scheduler
// thread owns one HIP stream; at every tick boundary it admits queued requests
// into free slots while their state fits in the workspace (the HBM budget),
// prepares them (exterior subtraction from the resident residual, step size),
// runs a few iterations of *all* admitted slots as one forward-projection and
// one backprojection launch per iteration, and retires finished slots (crop into
// the caller's buffer, ticket done).  A slot's arithmetic never depends on the
// other slots: its work items, reduction order and launch shape are fixed, so a
// result is bit-identical alone and in any mix.  Independent local parts are
// the paper's unit of parallel work (Section 5.6).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "tomo_runtime.h"
#include "tomo_serve.h"

namespace tomo {

namespace {
thread_local bool t_serve = false;
thread_local std::string t_err;

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Fixed launch shape for served slots (see the note at the top of the file).
// The backprojector variant (direct or LDS-staged) may change with the mix:
// for one group and pixel count per thread both give the same bits.
constexpr int kServeSeg = 1;   // forward projector: one segment per ray,
constexpr int kServeRP = 2;    // two rays per lane (the shape of large batches)
constexpr int kServeAG = 1;
constexpr int kServePPT = 2;
constexpr long long kServeStagedPixels = 1LL << 19;   // staged once the mix is this large
}  // namespace

bool on_serve_thread() { return t_serve; }
void set_thread_error(const char* msg) { t_err = msg; }

struct Request {
    uint64_t ticket = 0;
    int sino_id = 0;
    roi_params prm{};
    float* out = nullptr;
    double t_submit = 0.0;   // host clock (ms) at roi_submit
    double t_admit = 0.0;    // admitted and prepared
    double t_first = 0.0;    // its first iteration enqueued
};

struct Slot {
    Request req;
    RoiState st;
    SinoState* sino = nullptr;
    int it = 0;
    int parity0 = 0;
    std::vector<char*> allocs;
};

struct TicketInfo {
    int state = 0;   // 0 pending, 1 done, 2 failed
    float latency_ms = 0.f;
    // submit -> admitted, admitted -> first iteration, first iteration -> done
    // (negative until reached)
    float stage_ms[3] = {-1.f, -1.f, -1.f};
    std::string err;
};

struct ServeState {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, cv_idle;
    std::deque<Request> queue;
    size_t queue_cap = 8192;
    std::map<uint64_t, TicketInfo> tickets;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool busy = false;
    int max_slots = 32;
    int iters_per_tick = 4;
    hipStream_t stream = nullptr;
    Staging staging;
    long long step = 0;   // global iteration counter of the batch
    // Host-side test executor (host-only contexts): the scheduler runs its admission,
    // batching and retirement logic unchanged, but a tick launches nothing; it takes
    // fake_tick_us per iteration, or waits while fake_tick_us < 0 (a stalled
    // executor), and a retired request's output holds the number of iterations that
    // its slot ran.
    bool fake = false;
    int fake_tick_us = 0;
    std::condition_variable cv_fake;
};

// Workspace bytes of a resident sinogram: padded x_ext and its transpose, the plain
// x_ext, the residual and a flag word.
static size_t resident_bytes(const Geom& g, const Plan& P) {
    const size_t nb = (size_t)g.n * P.xp, nt = (size_t)g.n * P.tp, np = (size_t)g.n * g.n;
    const size_t nr = (size_t)g.na * g.nd;
    return (nb + nt + np + nr + 64) * sizeof(float) + 1280;
}

tomo_status build_resident(tomo_ctx* ctx, SinoState& S, hipStream_t s) {
    const Geom& g = ctx->geoms[S.gid];
    const Plan& P = g.full;
    S.xp = P.xp;
    S.tp = P.tp;
    const size_t nb = (size_t)g.n * P.xp, nt = (size_t)g.n * P.tp, np = (size_t)g.n * g.n;
    const size_t nr = (size_t)g.na * g.nd;
    S.block = ctx->arena.alloc(resident_bytes(g, P));
    if (!S.block) return fail(ctx, TOMO_ENOMEM, "workspace too small to register the sinogram");
    S.xb = (float*)S.block;
    S.xt = S.xb + align_up(nb, 64);
    S.x_plain = S.xt + align_up(nt, 64);
    S.resid = S.x_plain + align_up(np, 64);
    unsigned* d_bad = (unsigned*)(S.resid + align_up(nr, 64));   // non-finite input flag
    std::vector<char*> allocs;
    TOMO_HIP(ctx, launch_fill((float*)d_bad, 1, 0.f, s));
    TOMO_HIP(ctx, launch_check_finite(S.sino, nr, d_bad, s));
    TOMO_HIP(ctx, launch_fill(S.xb, (size_t)(S.resid - S.xb), 0.f, s));
    tomo_status st = fbp_into(ctx, S.gid, S.sino, S.x_plain, S.xb, S.xt, P, s, allocs, ctx->staging);
    if (st != TOMO_OK) {
        ctx->arena.free_after(allocs, s);
        return st;
    }
    // r = p - W x_ext over the whole detector
    const LaunchCfg L = choose_launch(ctx, (long long)g.na * g.nd, 0);
    std::vector<Item> items;
    Meta m;
    const size_t o_afp = m.add(P.afp.data(), P.afp.size() * sizeof(AngFP));
    const size_t o_job = m.reserve(sizeof(Job));
    const size_t o_it = m.reserve(count_fp_items(P.afp, L.seg, L.rp) * sizeof(Item));
    char* dm = ctx->arena.alloc(m.buf.size());
    if (!dm) {
        ctx->arena.free_after(allocs, s);
        return fail(ctx, TOMO_ENOMEM, "workspace too small for the residual tables");
    }
    allocs.push_back(dm);
    fp_items(items, 0, P.afp, L.seg, L.rp, (const AngFP*)(dm + o_afp));
    m.put(o_it, items.data(), items.size() * sizeof(Item));
    Job J;
    std::memset(&J, 0, sizeof J);
    J.nr = J.nc = g.n;
    J.xp = P.xp;
    J.tp = P.tp;
    J.n_angles = g.na;
    J.bpitch = P.bpitch;
    J.n_det = g.nd;
    J.fp_mode = FP_RESID;
    J.afp = (const AngFP*)(dm + o_afp);
    J.xb[0] = J.xb[1] = S.xb;
    J.xt = S.xt;
    J.gout = S.resid;
    J.gbase = S.sino;
    J.scale = -1.f;
    std::memcpy(m.buf.data() + o_job, &J, sizeof J);
    hipError_t e = ctx->staging.upload(dm, m.buf.data(), m.buf.size(), s);
    if (e == hipSuccess) e = launch_fill(S.resid, nr, 0.f, s);
    if (e == hipSuccess)
        e = launch_fp((const Job*)(dm + o_job), (const Item*)(dm + o_it), (int)items.size(), 0,
                      L.seg, s, L.cfp, L.rp);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ctx->arena.free_after(allocs, s);
    if (e != hipSuccess) return fail(ctx, TOMO_EHIP, "registering: %s", hipGetErrorString(e));
    unsigned bad = 0;
    TOMO_HIP(ctx, hipMemcpy(&bad, d_bad, sizeof bad, hipMemcpyDeviceToHost));
    if (bad) return fail(ctx, TOMO_EINVAL, "the sinogram holds NaN or infinite values");
    return TOMO_OK;
}

namespace {

// A slot's device tables (angle tables, and the job and items of its exterior
// subtraction), laid out for one upload.
struct SlotTables {
    Meta m;
    size_t o_afp = 0, o_abp = 0, o_job = 0, o_it = 0;
};

void slot_tables(const RoiState& r, SlotTables& T) {
    T.o_afp = T.m.add(r.plan.afp.data(), r.plan.afp.size() * sizeof(AngFP));
    T.o_abp = T.m.add(r.plan.abp.data(), r.plan.abp.size() * sizeof(AngBP));
    T.o_job = T.m.reserve(sizeof(Job));
    T.o_it = T.m.reserve(count_fp_items(r.plan.afp, kServeSeg, kServeRP) * sizeof(Item));
}

// A slot's share of the batch lists (its job, forward and backprojector items,
// and the alignment of the three arrays).
size_t slot_list_bytes(const RoiState& r) {
    return sizeof(Job) + 3 * 64 +
           (count_fp_items(r.plan.afp, kServeSeg, kServeRP) +
            count_bp_items(r.ext.rows, r.ext.cols, kServeAG, kServePPT)) *
               sizeof(Item);
}

// Prepare one admitted slot on the scheduler stream: tables (uploaded into `dm`,
// allocated at admission), b = r + W_L x_ext|L, step size, zeroed state.
tomo_status prepare_slot(tomo_ctx* ctx, ServeState& S, Slot& sl, SlotTables& T, char* dm) {
    const Geom& g = ctx->geoms[sl.sino->gid];
    RoiState& r = sl.st;
    hipStream_t s = S.stream;
    Meta& m = T.m;
    const size_t o_afp = T.o_afp, o_abp = T.o_abp, o_job = T.o_job, o_it = T.o_it;
    std::vector<Item> items;
    r.d_afp = (AngFP*)(dm + o_afp);
    r.d_abp = (AngBP*)(dm + o_abp);
    fp_items(items, 0, r.plan.afp, kServeSeg, kServeRP, r.d_afp);
    m.put(o_it, items.data(), items.size() * sizeof(Item));
    Job J = make_job(g, r, FP_BAND_FROM_GLOBAL, BP_STORE, 0);
    J.xb[1] = J.xb[0];
    J.gbase = sl.sino->resid;
    J.y = r.b;
    J.scale = 1.f;
    std::memcpy(m.buf.data() + o_job, &J, sizeof J);
    TOMO_HIP(ctx, S.staging.upload(dm, m.buf.data(), m.buf.size(), s));
    TOMO_HIP(ctx, launch_fill((float*)r.block, r.total_floats, 0.f, s));
    TOMO_HIP(ctx, launch_pad_copy(sl.sino->x_plain, g.n, r.ext.r0, r.ext.c0, r.ext.rows,
                                  r.ext.cols, r.xb0, r.plan.xp, r.xt, r.plan.tp, nullptr, 0, s));
    TOMO_HIP(ctx, launch_fp((const Job*)(dm + o_job), (const Item*)(dm + o_it), (int)items.size(),
                            0, kServeSeg, s, 1, kServeRP));
    tomo_status st = step_size_for(ctx, sl.sino->gid, r, s, S.staging);
    if (st != TOMO_OK) return st;
    TOMO_HIP(ctx, launch_fill((float*)r.block, r.state_floats, 0.f, s));
    return TOMO_OK;
}

void finish_ticket(ServeState& S, uint64_t t, int state, float lat, const std::string& err) {
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.tickets.find(t);
    if (it == S.tickets.end()) return;
    it->second.state = state;
    it->second.latency_ms = lat;
    it->second.err = err;
}

// Memory of retired work: after the stream's pending work (nothing is pending in the
// test executor).
void release(tomo_ctx* ctx, ServeState& S, const std::vector<char*>& ps) {
    if (S.fake) {
        for (char* p : ps)
            if (p) ctx->arena.free_now(p);
        return;
    }
    ctx->arena.free_after(ps, S.stream);
}

void record_stages(ServeState& S, const Request& q, double t_done) {
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.tickets.find(q.ticket);
    if (it == S.tickets.end()) return;
    it->second.stage_ms[0] = (float)(q.t_admit - q.t_submit);
    it->second.stage_ms[1] = (float)(q.t_first - q.t_admit);
    it->second.stage_ms[2] = (float)(t_done - q.t_first);
}

// One tick of the test executor: wait while stalled (or until shutdown), then take
// the configured time per iteration.
void fake_tick(ServeState& S, int iters) {
    int us = 0;
    {
        std::unique_lock<std::mutex> lk(S.mu);
        S.cv_fake.wait(lk, [&] { return S.stop || S.fake_tick_us >= 0; });
        us = std::max(S.fake_tick_us, 0);
    }
    if (us > 0) std::this_thread::sleep_for(std::chrono::microseconds((long long)us * iters));
}

void scheduler(tomo_ctx* ctx) {
    t_serve = true;
    ServeState& S = *ctx->serve;
    if (!S.fake) (void)hipSetDevice(ctx->device);
    std::vector<std::unique_ptr<Slot>> slots;
    char* d_lists = nullptr;
    size_t list_bytes = 0;   // the admitted slots' shares of the batch lists
    const Job* d_jobs = nullptr;
    const Item* d_fi = nullptr;
    const Item* d_bi = nullptr;
    int n_fi = 0, n_bi = 0;
    bool staged = false;
    bool changed = false;
    for (;;) {
        if (slots.empty() && d_lists) {   // idle: hold nothing beyond the registrations
            release(ctx, S, {d_lists});
            d_lists = nullptr;
        }
        // ---- admission ----
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.busy = !slots.empty() || !S.queue.empty();
            if (!S.busy) S.cv_idle.notify_all();
            S.cv.wait(lk, [&] { return S.stop || !S.queue.empty() || !slots.empty(); });
            if (S.stop && slots.empty()) {
                // fail whatever is still queued
                for (auto& q : S.queue) {
                    auto it = S.tickets.find(q.ticket);
                    if (it != S.tickets.end()) {
                        it->second.state = 2;
                        it->second.err = "context destroyed";
                    }
                    auto sit = ctx->sinos.find(q.sino_id);
                    if (sit != ctx->sinos.end()) sit->second->users--;
                }
                S.queue.clear();
                S.busy = false;
                S.cv_idle.notify_all();
                break;
            }
            S.busy = true;
        }
        for (;;) {
            Request req;
            {
                std::lock_guard<std::mutex> lk(S.mu);
                if (S.stop || S.queue.empty() || (int)slots.size() >= S.max_slots) break;
                req = S.queue.front();
            }
            auto sl = std::make_unique<Slot>();
            sl->req = req;
            {
                std::lock_guard<std::recursive_mutex> lk(ctx->mu);
                sl->sino = ctx->sinos.at(req.sino_id).get();
            }
            const Geom& g = ctx->geoms[sl->sino->gid];
            RoiState& r = sl->st;
            r.prm = req.prm;
            r.roi = Rect{req.prm.roi.row0, req.prm.roi.col0, req.prm.roi.rows, req.prm.roi.cols};
            r.ext = extend_rect(r.roi, req.prm.margin, g.n);
            r.plan = make_plan(g, r.ext, r.ext);
            // the slot's state, plus room for its step-size power iteration when
            // the step is not cached yet (probed now, released just before use)
            const size_t scratch = step_size_scratch_bytes(ctx, sl->sino->gid, r);
            char* blk = ctx->arena.alloc(state_bytes(g, r.plan), false);
            if (!blk && slots.empty()) blk = ctx->arena.alloc(state_bytes(g, r.plan), true);
            SlotTables T;
            slot_tables(r, T);
            char* tab = nullptr;
            if (blk) {
                tab = ctx->arena.alloc(T.m.buf.size(), false);
                if (!tab && slots.empty()) tab = ctx->arena.alloc(T.m.buf.size(), true);
                if (!tab) {
                    ctx->arena.free_now(blk);
                    blk = nullptr;
                }
            }
            char* probe = nullptr;
            if (blk && scratch) {
                probe = ctx->arena.alloc(scratch, false);
                if (!probe && slots.empty()) probe = ctx->arena.alloc(scratch, true);
                if (!probe) {
                    ctx->arena.free_now(tab);
                    ctx->arena.free_now(blk);
                    blk = nullptr;
                }
            }
            // the batch lists are rebuilt, with this slot in, after admission: while
            // other slots run, admit it only if they will fit next to everything held
            if (blk && !slots.empty() &&
                ctx->arena.largest_free() < list_bytes + slot_list_bytes(r) + 1024) {
                if (probe) ctx->arena.free_now(probe);
                ctx->arena.free_now(tab);
                ctx->arena.free_now(blk);
                blk = nullptr;
            }
            if (!blk) {
                if (slots.empty()) {   // cannot ever fit: fail it rather than stall
                    std::lock_guard<std::mutex> lk(S.mu);
                    S.queue.pop_front();
                    auto it = S.tickets.find(req.ticket);
                    if (it != S.tickets.end()) {
                        it->second.state = 2;
                        it->second.err = "request does not fit in the workspace";
                    }
                    sl->sino->users--;
                    continue;
                }
                break;   // wait for running slots to free memory
            }
            {
                std::lock_guard<std::mutex> lk(S.mu);
                S.queue.pop_front();
            }
            sl->allocs.push_back(blk);
            sl->allocs.push_back(tab);
            carve_state(g, r, blk);
            if (probe) ctx->arena.free_now(probe);
            t_err.clear();
            tomo_status st = TOMO_OK;
            if (S.fake)
                step_size_assume_cached(ctx, sl->sino->gid, r);
            else
                st = prepare_slot(ctx, S, *sl, T, tab);
            if (st != TOMO_OK) {
                finish_ticket(S, req.ticket, 2, 0.f, t_err);
                (void)hipStreamSynchronize(S.stream);
                release(ctx, S, sl->allocs);
                sl->sino->users--;
                continue;
            }
            sl->req.t_admit = now_ms();
            sl->parity0 = (int)((2 - (S.step & 1)) & 1);   // (step + parity0) even at it = 0
            list_bytes += slot_list_bytes(sl->st);
            slots.push_back(std::move(sl));
            changed = true;
        }
        if (slots.empty()) continue;
        // ---- batch lists (rebuilt when membership changes) ----
        if (changed) {
            std::vector<Job> jobs;
            std::vector<Item> fi, bi;
            int th, tw;
            bp_tile(kServeAG, kServePPT, &th, &tw);
            for (size_t q = 0; q < slots.size(); ++q) {
                Slot& sl = *slots[q];
                const Geom& g = ctx->geoms[sl.sino->gid];
                const bool cp = sl.st.prm.method == ROI_TV_NONNEG_CP;
                Job J = make_job(g, sl.st, cp ? FP_CP_DUAL : FP_SIRT, cp ? BP_CP : BP_SIRT,
                                 (sl.st.ext.cols + tw - 1) / tw);
                J.parity0 = sl.parity0;
                jobs.push_back(J);
                fp_items(fi, (int)q, sl.st.plan.afp, kServeSeg, kServeRP, sl.st.d_afp);
                bp_items(bi, (int)q, sl.st.ext.rows, sl.st.ext.cols, kServeAG, kServePPT,
                         sl.st.d_abp);
            }
            Meta m;
            const size_t o_j = m.add(jobs.data(), jobs.size() * sizeof(Job));
            const size_t o_f = m.add(fi.data(), fi.size() * sizeof(Item));
            const size_t o_b = m.add(bi.data(), bi.size() * sizeof(Item));
            if (d_lists) release(ctx, S, {d_lists});
            d_lists = ctx->arena.alloc(m.buf.size(), !S.fake);
            if (!d_lists ||
                (!S.fake &&
                 S.staging.upload(d_lists, m.buf.data(), m.buf.size(), S.stream) != hipSuccess)) {
                for (auto& sl : slots) {
                    finish_ticket(S, sl->req.ticket, 2, 0.f, "cannot upload the batch lists");
                    release(ctx, S, sl->allocs);
                    sl->sino->users--;
                }
                if (d_lists) release(ctx, S, {d_lists});
                d_lists = nullptr;
                slots.clear();
                list_bytes = 0;
                continue;
            }
            d_jobs = (const Job*)(d_lists + o_j);
            d_fi = (const Item*)(d_lists + o_f);
            d_bi = (const Item*)(d_lists + o_b);
            n_fi = (int)fi.size();
            n_bi = (int)bi.size();
            long long pix = 0;
            for (auto& sl : slots) pix += (long long)sl->st.ext.rows * sl->st.ext.cols;
            staged = pix >= kServeStagedPixels;
            changed = false;
        }
        // ---- one tick: the same few iterations for every admitted slot ----
        int tick = S.iters_per_tick;
        for (auto& sl : slots) tick = std::min(tick, sl->req.prm.iters - sl->it);
        hipError_t e = hipSuccess;
        TraceRange trace_tick("serve tick: %d slots x %d its", (int)slots.size(), tick);
        const double t_tick = now_ms();
        for (auto& sl : slots)
            if (sl->it == 0) sl->req.t_first = t_tick;
        if (S.fake) {
            fake_tick(S, tick);
            S.step += tick;
        }
        for (int t = 0; t < tick && e == hipSuccess && !S.fake; ++t) {
            const int stp = (int)(S.step & 0x3fffffff);
            // slots of uneven size: the forward projector's items dealt round-robin over
            // the XCDs, the backprojector's (equal tiles) in contiguous eighths
            e = launch_fp(d_jobs, d_fi, n_fi, stp, kServeSeg, S.stream, 0, kServeRP);
            if (e == hipSuccess)
                e = launch_bp(d_jobs, d_bi, n_bi, stp, kServeAG, kServePPT, S.stream, 1, staged);
            S.step++;
        }
        for (auto& sl : slots) sl->it += tick;
        // ---- retire finished slots ----
        std::vector<size_t> done;
        for (size_t q = 0; q < slots.size(); ++q)
            if (slots[q]->it >= slots[q]->req.prm.iters) done.push_back(q);
        for (size_t q : done) {
            const RoiState& r = slots[q]->st;
            if (S.fake) {
                std::fill(slots[q]->req.out, slots[q]->req.out + (size_t)r.roi.rows * r.roi.cols,
                          (float)slots[q]->it);
                continue;
            }
            if (e == hipSuccess)
                e = launch_crop(r.x, r.ext.cols, r.roi.r0 - r.ext.r0, r.roi.c0 - r.ext.c0,
                                r.roi.rows, r.roi.cols, slots[q]->req.out, r.roi.cols, S.stream);
        }
        if (e == hipSuccess && !S.fake) e = hipStreamSynchronize(S.stream);
        const double tnow = now_ms();
        if (e != hipSuccess) {
            for (auto& sl : slots) {
                finish_ticket(S, sl->req.ticket, 2, 0.f, hipGetErrorString(e));
                release(ctx, S, sl->allocs);
                sl->sino->users--;
            }
            slots.clear();
            list_bytes = 0;
            changed = true;
            continue;
        }
        for (auto qi = done.rbegin(); qi != done.rend(); ++qi) {
            Slot& sl = *slots[*qi];
            record_stages(S, sl.req, tnow);
            finish_ticket(S, sl.req.ticket, 1, (float)(tnow - sl.req.t_submit), "");
            release(ctx, S, sl.allocs);
            sl.sino->users--;
            list_bytes -= slot_list_bytes(sl.st);
            slots.erase(slots.begin() + (long)*qi);
            changed = true;
        }
    }
    if (d_lists) release(ctx, S, {d_lists});
    if (!S.fake) (void)hipStreamSynchronize(S.stream);
}

tomo_status ensure_serving(tomo_ctx* ctx) {
    if (ctx->serve && ctx->serve->th.joinable()) return TOMO_OK;
    if (!ctx->serve) ctx->serve = std::make_unique<ServeState>();
    ServeState& S = *ctx->serve;
    if (!S.stream && !S.fake)
        TOMO_HIP(ctx, hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking));
    S.stop = false;
    S.th = std::thread(scheduler, ctx);
    return TOMO_OK;
}

}  // namespace

void serve_shutdown(tomo_ctx* ctx) {
    if (!ctx->serve) return;
    ServeState& S = *ctx->serve;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
    }
    S.cv.notify_all();
    S.cv_fake.notify_all();
    if (S.th.joinable()) S.th.join();
    S.staging.destroy();
    if (S.stream) (void)hipStreamDestroy(S.stream);
    S.stream = nullptr;
}

bool serve_is_fake(const tomo_ctx* ctx) { return ctx->serve && ctx->serve->fake; }

void serve_drain(tomo_ctx* ctx) {
    if (!ctx->serve) return;
    ServeState& S = *ctx->serve;
    std::unique_lock<std::mutex> lk(S.mu);
    S.cv_idle.wait(lk, [&] { return !S.busy && S.queue.empty(); });
}

}  // namespace tomo

using namespace tomo;

tomo_ctx::tomo_ctx() = default;
tomo_ctx::~tomo_ctx() = default;

extern "C" {

static bool fake_serving(const tomo_ctx* ctx) { return serve_is_fake(ctx); }

// The test executor's registration: the same workspace share, the sinogram (host
// memory) checked on the host, no exterior estimate.
static tomo_status register_fake(tomo_ctx* ctx, SinoState& S) {
    const Geom& g = ctx->geoms[S.gid];
    const size_t nr = (size_t)g.na * g.nd;
    for (size_t i = 0; i < nr; ++i)
        if (!std::isfinite(S.sino[i]))
            return fail(ctx, TOMO_EINVAL, "the sinogram holds NaN or infinite values");
    S.xp = g.full.xp;
    S.tp = g.full.tp;
    S.block = ctx->arena.alloc(resident_bytes(g, g.full), false);
    if (!S.block) return fail(ctx, TOMO_ENOMEM, "workspace too small to register the sinogram");
    return TOMO_OK;
}

tomo_status tomo_register_sinogram(tomo_ctx* ctx, int32_t geom, const float* sino,
                                   int32_t* sino_id) {
    if (!ctx || !sino || !sino_id) return ctx ? fail(ctx, TOMO_EINVAL, "null pointer") : TOMO_EINVAL;
    if (ctx->host_only && !fake_serving(ctx))
        return fail(ctx, TOMO_ESTATE, "host-only context: no GPU calls");
    try {
        if (geom < 0 || geom >= (int)ctx->geoms.size())
            return fail(ctx, TOMO_ENOENT, "unknown geometry %d", geom);
        const bool fake = fake_serving(ctx);
        if (!fake) TOMO_HIP(ctx, hipSetDevice(ctx->device));
        auto S = std::make_unique<SinoState>();
        S->gid = geom;
        S->sino = sino;
        tomo_status st = fake ? register_fake(ctx, *S) : build_resident(ctx, *S, nullptr);
        if (st != TOMO_OK) {
            if (S->block && fake) ctx->arena.free_now(S->block);
            else if (S->block) ctx->arena.free_after({S->block}, nullptr);
            return st;
        }
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        const int id = ctx->next_sino++;
        ctx->sinos[id] = std::move(S);
        *sino_id = id;
        return TOMO_OK;
    } catch (...) {
        return fail(ctx, TOMO_ENOMEM, "host allocation failed");
    }
}

tomo_status tomo_unregister_sinogram(tomo_ctx* ctx, int32_t sino_id) {
    if (!ctx) return TOMO_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->sinos.find(sino_id);
    if (it == ctx->sinos.end()) return fail(ctx, TOMO_ENOENT, "unknown sinogram %d", sino_id);
    if (it->second->users.load() > 0)
        return fail(ctx, TOMO_EBUSY, "sinogram %d has %d live requests", sino_id,
                    it->second->users.load());
    if (fake_serving(ctx)) {
        ctx->arena.free_now(it->second->block);
    } else {
        (void)hipSetDevice(ctx->device);
        ctx->arena.free_after({it->second->block}, nullptr);
    }
    ctx->sinos.erase(it);
    return TOMO_OK;
}

tomo_status roi_submit(tomo_ctx* ctx, int32_t sino_id, const roi_params* params, float* out,
                       uint64_t* ticket) {
    if (!ctx || !params || !out || !ticket)
        return ctx ? fail(ctx, TOMO_EINVAL, "null pointer") : TOMO_EINVAL;
    if (ctx->host_only && !fake_serving(ctx))
        return fail(ctx, TOMO_ESTATE, "host-only context: no GPU calls");
    try {
        SinoState* sp = nullptr;
        {
            std::lock_guard<std::recursive_mutex> lk(ctx->mu);
            auto it = ctx->sinos.find(sino_id);
            if (it == ctx->sinos.end()) return fail(ctx, TOMO_ENOENT, "unknown sinogram %d", sino_id);
            sp = it->second.get();
        }
        const Geom& g = ctx->geoms[sp->gid];
        tomo_status st = validate_params(ctx, g, *params);
        if (st != TOMO_OK) return st;
        if (params->method >= ROI_LOCAL_SIRT)
            return fail(ctx, TOMO_EINVAL, "local-method requests go through roi_solve_local");
        const Rect roi{params->roi.row0, params->roi.col0, params->roi.rows, params->roi.cols};
        const Rect ext = extend_rect(roi, params->margin, g.n);
        RoiState probe;
        probe.prm = *params;
        probe.roi = roi;
        probe.ext = ext;
        probe.plan = make_plan(g, ext, ext);
        const size_t need = state_bytes(g, probe.plan) + step_size_scratch_bytes(ctx, sp->gid, probe);
        if (need + 64 * 1024 > ctx->arena.capacity())
            return fail(ctx, TOMO_ENOMEM, "request needs %zu bytes; the workspace holds %zu", need,
                        ctx->arena.capacity());
        st = ensure_serving(ctx);
        if (st != TOMO_OK) return st;
        ServeState& S = *ctx->serve;
        {
            std::lock_guard<std::mutex> lk(S.mu);
            if (S.queue.size() >= S.queue_cap) return fail(ctx, TOMO_EAGAIN, "request queue full");
            Request r;
            r.ticket = S.next_ticket++;
            r.sino_id = sino_id;
            r.prm = *params;
            r.out = out;
            r.t_submit = now_ms();
            S.tickets[r.ticket] = TicketInfo{};
            sp->users++;
            S.queue.push_back(r);
            *ticket = r.ticket;
        }
        S.cv.notify_all();
        return TOMO_OK;
    } catch (...) {
        return fail(ctx, TOMO_ENOMEM, "host allocation failed");
    }
}

tomo_status roi_poll(tomo_ctx* ctx, uint64_t ticket, int* done, float* latency_ms) {
    if (!ctx || !done) return ctx ? fail(ctx, TOMO_EINVAL, "null pointer") : TOMO_EINVAL;
    *done = 0;
    if (!ctx->serve) return fail(ctx, TOMO_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    ServeState& S = *ctx->serve;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.tickets.find(ticket);
    if (it == S.tickets.end())
        return fail(ctx, TOMO_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second.state == 0) return TOMO_OK;
    if (it->second.state == 2) {
        const std::string err = it->second.err;
        S.tickets.erase(it);
        return fail(ctx, TOMO_EHIP, "request failed: %s", err.c_str());
    }
    *done = 1;
    if (latency_ms) *latency_ms = it->second.latency_ms;
    S.tickets.erase(it);
    return TOMO_OK;
}

tomo_status roi_poll_stages(tomo_ctx* ctx, uint64_t ticket, int* done, float* stages_ms) {
    if (!ctx || !done || !stages_ms) return ctx ? fail(ctx, TOMO_EINVAL, "null pointer") : TOMO_EINVAL;
    *done = 0;
    for (int i = 0; i < 4; ++i) stages_ms[i] = -1.f;
    if (!ctx->serve) return fail(ctx, TOMO_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    ServeState& S = *ctx->serve;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.tickets.find(ticket);
    if (it == S.tickets.end())
        return fail(ctx, TOMO_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second.state == 0) return TOMO_OK;
    if (it->second.state == 2) {
        const std::string err = it->second.err;
        S.tickets.erase(it);
        return fail(ctx, TOMO_EHIP, "request failed: %s", err.c_str());
    }
    *done = 1;
    for (int i = 0; i < 3; ++i) stages_ms[i] = it->second.stage_ms[i];
    stages_ms[3] = it->second.latency_ms;
    S.tickets.erase(it);
    return TOMO_OK;
}

tomo_status tomo_serving_fake(tomo_ctx* ctx, size_t budget_bytes, int32_t tick_us) {
    if (!ctx) return TOMO_EINVAL;
    if (!ctx->host_only)
        return fail(ctx, TOMO_ESTATE, "the test executor runs on host-only contexts only");
    try {
        if (!ctx->serve) ctx->serve = std::make_unique<ServeState>();
        ServeState& S = *ctx->serve;
        if (budget_bytes) {
            if (S.fake) return fail(ctx, TOMO_ESTATE, "the test executor is already set up");
            if (budget_bytes < (1u << 20))
                return fail(ctx, TOMO_EINVAL, "the budget must be at least 1 MiB");
            // offsets only: no memory stands behind this range, and nothing reads it
            ctx->arena.init(reinterpret_cast<char*>((uintptr_t)1 << 40), budget_bytes);
            S.fake = true;
        } else if (!S.fake) {
            return fail(ctx, TOMO_ESTATE, "set the test executor up with a budget first");
        }
        {
            std::lock_guard<std::mutex> lk(S.mu);
            S.fake_tick_us = tick_us;
        }
        S.cv_fake.notify_all();
        return TOMO_OK;
    } catch (...) {
        return fail(ctx, TOMO_ENOMEM, "host allocation failed");
    }
}

tomo_status tomo_serving_config(tomo_ctx* ctx, int32_t max_slots, int32_t iters_per_tick) {
    if (!ctx) return TOMO_EINVAL;
    if (max_slots < 0 || iters_per_tick < 0 || max_slots > 4096 || iters_per_tick > 1000)
        return fail(ctx, TOMO_EINVAL, "serving knobs out of range");
    if (!ctx->serve) ctx->serve = std::make_unique<ServeState>();
    std::lock_guard<std::mutex> lk(ctx->serve->mu);
    if (max_slots) ctx->serve->max_slots = max_slots;
    if (iters_per_tick) ctx->serve->iters_per_tick = iters_per_tick;
    return TOMO_OK;
}

}  // extern "C"
