// The paper's own local method (Sections 3.1-3.3): the SIRT-approximating
// filters of Alg. 1, the filtered data C_{u_k} p shared by all local parts, the
// iterations of Alg. 2 (box prior) and Alg. 3 (FISTA-TV) batched over many ROIs
// the same way as the exterior-subtraction solvers, and the data preprocessing
// (disc subtraction, constant padding of truncated data).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "tomo_runtime.h"

using namespace tomo;

namespace {

// Zero lag of the filters per angle: the bin nearest the projection of the
// impulse pixel (n/2, n/2), decided in FP64 without contraction.
std::vector<int> filter_centres(const Geom& g) {
#pragma clang fp contract(off)
    const double xc = (double)(g.n / 2) - 0.5 * (double)(g.n - 1);
    const double yr = xc;
    std::vector<int> ctr(g.na);
    for (int a = 0; a < g.na; ++a) {
        const double px = xc * g.c[a];
        const double py = yr * g.s[a];
        const double t = px + py;
        const double u = (t - g.offset) / g.spacing;
        const double b = u + 0.5 * (double)(g.nd - 1);
        const double r = std::floor(b + 0.5);
        ctr[a] = (int)std::min(std::max(r, -2.0e9), 2.0e9);
    }
    return ctr;
}

// Device state of one local-method job: x, v (padded, ping-pong, and the
// transposed copy), the band (two-channel for the local methods) and, for
// FISTA-TV, the FGP input, x_s and the FGP duals p and r.
struct LocalBuf {
    float *x, *xb0, *xb1, *xt, *y;
    float *w = nullptr, *xs = nullptr, *fp = nullptr, *fr = nullptr;
};

size_t local_state_floats(const Geom& g, const Plan& p, bool two_channel, bool fista = false) {
    const size_t nr = p.reg.rows, nc = p.reg.cols;
    size_t f = align_up(nr * nc, 64) + 2 * align_up(nr * p.xp, 64) + align_up(nc * p.tp, 64) +
               align_up((two_channel ? 2 : 1) * (size_t)g.na * p.bpitch, 64);
    if (fista) f += 2 * align_up(nr * nc, 64) + 2 * align_up(2 * nr * nc, 64);
    return f;
}

LocalBuf carve_local(const Geom& g, const Plan& p, bool two_channel, float* f,
                     bool fista = false) {
    const size_t nr = p.reg.rows, nc = p.reg.cols;
    LocalBuf b;
    auto take = [&](size_t n) {
        float* q = f;
        f += align_up(n, 64);
        return q;
    };
    b.x = take(nr * nc);
    b.xb0 = take(nr * p.xp);
    b.xb1 = take(nr * p.xp);
    b.xt = take(nc * p.tp);
    b.y = take((two_channel ? 2 : 1) * (size_t)g.na * p.bpitch);
    if (fista) {
        b.w = take(nr * nc);
        b.xs = take(nr * nc);
        b.fp = take(2 * nr * nc);
        b.fr = take(2 * nr * nc);
    }
    return b;
}

// Momentum factors (t_{i} - 1) / t_{i+1} of the FISTA recursion
// t_{i+1} = (1 + sqrt(1 + 4 t_i^2)) / 2 from t_0 = 1, in FP64.
std::vector<float> fista_betas(int n) {
    std::vector<float> b(std::max(n, 1));
    double t = 1.0;
    for (int i = 0; i < n; ++i) {
        const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
        b[i] = (float)((t - 1.0) / tn);
        t = tn;
    }
    return b;
}

}  // namespace

tomo_status tomo_sirt_filters(tomo_ctx* ctx, int32_t geom, int32_t iters, float* filters,
                              void* hip_stream) {
    tomo_status st = need_gpu(ctx);
    if (st != TOMO_OK) return st;
    if (!filters || iters < 1) return fail(ctx, TOMO_EINVAL, "null filters or iters < 1");
    GUARD_BEGIN
    TraceRange trace("sirt filters: %d", iters);
    const Geom* gp;
    if ((st = get_geom(ctx, geom, &gp)) != TOMO_OK) return st;
    const Geom& g = *gp;
    hipStream_t s = (hipStream_t)hip_stream;
    const Rect full{0, 0, g.n, g.n};
    // The recursion is SIRT from the impulse with zero data and no box:
    // c <- c - alpha W^T W c, while the filter accumulates alpha W c.
    RoiState r;
    std::memset(&r.prm, 0, sizeof r.prm);
    r.prm.method = ROI_NONNEG_SIRT;
    r.prm.flags = ROI_FLAG_BOX;
    r.prm.box_lo = -INFINITY;
    r.prm.box_hi = INFINITY;
    r.roi = r.ext = full;
    r.plan = make_plan(g, full, full);
    const Plan& P = r.plan;
    LaunchCfg L = choose_launch(ctx, (long long)g.na * P.wmax, (long long)g.n * g.n);
    int th, tw;
    bp_tile(L.ag, L.ppt, &th, &tw);
    const size_t sfl = local_state_floats(g, P, false);

    std::vector<char*> allocs;
    auto cleanup = [&]() { ctx->arena.free_after(allocs, s); };
    Meta m;
    const size_t o_afp = m.add(P.afp.data(), P.afp.size() * sizeof(AngFP));
    const size_t o_abp = m.add(P.abp.data(), P.abp.size() * sizeof(AngBP));
    const size_t o_jobs = m.reserve(sizeof(Job) * iters);
    const size_t n_fi = count_fp_items(P.afp, L.seg, L.rp);
    const size_t n_bi = count_bp_items(g.n, g.n, L.ag, L.ppt);
    const size_t o_fi = m.reserve(n_fi * sizeof(Item));
    const size_t o_bi = m.reserve(n_bi * sizeof(Item));
    char* dm = ctx->arena.alloc(align_up(m.buf.size(), 256) + sfl * sizeof(float) + 256);
    if (!dm) return fail(ctx, TOMO_ENOMEM, "workspace too small for the filter recursion");
    allocs.push_back(dm);
    float* state = (float*)(dm + align_up(m.buf.size(), 256));
    const LocalBuf B = carve_local(g, P, false, state);
    r.d_afp = (AngFP*)(dm + o_afp);
    r.d_abp = (AngBP*)(dm + o_abp);
    r.x = B.x;
    r.xb0 = B.xb0;
    r.xb1 = B.xb1;
    r.xt = B.xt;
    r.y = B.y;
    std::vector<Item> fi, bi;
    fp_items(fi, 0, P.afp, L.seg, L.rp, r.d_afp);
    bp_items(bi, 0, g.n, g.n, L.ag, L.ppt, r.d_abp);
    m.put(o_fi, fi.data(), fi.size() * sizeof(Item));
    m.put(o_bi, bi.data(), bi.size() * sizeof(Item));
    const size_t plane = (size_t)g.na * g.nd;
    for (int k = 0; k < iters; ++k) {
        Job J = make_job(g, r, FP_FILTER, BP_SIRT, (g.n + tw - 1) / tw);
        J.gout = filters + (size_t)k * plane;
        J.gbase = filters + (size_t)(k > 0 ? k - 1 : 0) * plane;   // plane 0 starts at zero
        std::memcpy(m.buf.data() + o_jobs + k * sizeof(Job), &J, sizeof J);
    }
#define CK(expr)                                                                          \
    do {                                                                                  \
        hipError_t e__ = (expr);                                                          \
        if (e__ != hipSuccess) {                                                          \
            cleanup();                                                                    \
            return fail(ctx, TOMO_EHIP, "%s failed: %s", #expr, hipGetErrorString(e__));  \
        }                                                                                 \
    } while (0)
    CK(ctx->staging.upload(dm, m.buf.data(), m.buf.size(), s));
    CK(launch_fill(state, sfl, 0.f, s));
    CK(launch_fill(filters, (size_t)iters * plane, 0.f, s));
    // the impulse at pixel (n/2, n/2), in the plain, padded and transposed images
    const int ci = g.n / 2;
    CK(launch_fill(B.x + (size_t)ci * g.n + ci, 1, 1.f, s));
    CK(launch_fill(B.xb0 + (size_t)ci * P.xp + ci + kLpad, 1, 1.f, s));
    CK(launch_fill(B.xt + (size_t)ci * P.tp + ci + kLpad, 1, 1.f, s));
    const Job* d_jobs = (const Job*)(dm + o_jobs);
    for (int k = 0; k < iters; ++k) {
        CK(launch_fp(d_jobs + k, (const Item*)(dm + o_fi), (int)fi.size(), k, L.seg, s, L.cfp,
                     L.rp));
        if (k + 1 < iters)
            CK(launch_bp(d_jobs + k, (const Item*)(dm + o_bi), (int)bi.size(), k, L.ag, L.ppt, s,
                         L.cbp, L.staged));
    }
#undef CK
    cleanup();
    return TOMO_OK;
    GUARD_END(ctx)
}

tomo_status tomo_sirt_filter_sino(tomo_ctx* ctx, int32_t geom, const float* filters,
                                  int32_t count, const float* sino, float* out,
                                  void* hip_stream) {
    tomo_status st = need_gpu(ctx);
    if (st != TOMO_OK) return st;
    if (!filters || !sino || !out || count < 1)
        return fail(ctx, TOMO_EINVAL, "null pointer or count < 1");
    GUARD_BEGIN
    const Geom* gp;
    if ((st = get_geom(ctx, geom, &gp)) != TOMO_OK) return st;
    const Geom& g = *gp;
    if (g.nd > 8192) return fail(ctx, TOMO_EINVAL, "filtered data support at most 8192 bins");
    hipStream_t s = (hipStream_t)hip_stream;
    int lg = 2;
    while ((1 << lg) < 2 * g.nd - 1) ++lg;
    const int len = 1 << lg;
    std::vector<float> tw(2 * (size_t)len);
    for (int q = 0; q < len; ++q) {
        const double ang = 2.0 * M_PI * (double)q / (double)len;
        tw[2 * q] = (float)std::cos(ang);
        tw[2 * q + 1] = (float)-std::sin(ang);
    }
    const std::vector<int> ctr = filter_centres(g);
    Meta m;
    const size_t o_tw = m.add(tw.data(), tw.size() * sizeof(float));
    const size_t o_ctr = m.add(ctr.data(), ctr.size() * sizeof(int));
    const size_t spec_bytes = (size_t)g.na * len * 2 * sizeof(float);
    char* dm = ctx->arena.alloc(align_up(m.buf.size(), 256) + spec_bytes);
    if (!dm) return fail(ctx, TOMO_ENOMEM, "workspace too small for the data spectra");
    std::vector<char*> allocs{dm};
    float2* spec = (float2*)(dm + align_up(m.buf.size(), 256));
    hipError_t e = ctx->staging.upload(dm, m.buf.data(), m.buf.size(), s);
    if (e == hipSuccess)
        e = launch_spectra(sino, g.na, g.nd, lg, (const float2*)(dm + o_tw), spec, s);
    if (e == hipSuccess)
        e = launch_filter_conv(filters, count, g.na, g.nd, (const int*)(dm + o_ctr), lg,
                               (const float2*)(dm + o_tw), spec, out, s);
    ctx->arena.free_after(allocs, s);
    if (e != hipSuccess) return fail(ctx, TOMO_EHIP, "filtered data: %s", hipGetErrorString(e));
    return TOMO_OK;
    GUARD_END(ctx)
}

tomo_status roi_solve_local(tomo_ctx* ctx, int32_t geom, const float* filtered, int32_t planes,
                            int32_t count, const roi_params* params, float* const* outs,
                            void* hip_stream) {
    tomo_status st = need_gpu(ctx);
    if (st != TOMO_OK) return st;
    if (!filtered || !params || !outs || count < 1 || planes < 1)
        return fail(ctx, TOMO_EINVAL, "null pointer, count < 1 or planes < 1");
    GUARD_BEGIN
    TraceRange trace("roi_solve_local: %d ROIs", count);
    const Geom* gp;
    if ((st = get_geom(ctx, geom, &gp)) != TOMO_OK) return st;
    const Geom& g = *gp;
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<RoiState> R(count);
    std::vector<size_t> sfl(count);
    long long rays = 0, pix = 0;
    size_t state_total = 0;
    int max_nf = 0, max_iters = 0;
    for (int i = 0; i < count; ++i) {
        if ((st = validate_params(ctx, g, params[i])) != TOMO_OK) return st;
        if (params[i].method < ROI_LOCAL_SIRT)
            return fail(ctx, TOMO_EINVAL, "roi_solve_local takes the local methods only");
        if (params[i].iters > planes)
            return fail(ctx, TOMO_EINVAL, "ROI %d needs %d filtered planes, %d given", i,
                        params[i].iters, planes);
        if (!outs[i]) return fail(ctx, TOMO_EINVAL, "null output pointer for ROI %d", i);
        RoiState& r = R[i];
        r.prm = params[i];
        r.roi = Rect{params[i].roi.row0, params[i].roi.col0, params[i].roi.rows, params[i].roi.cols};
        r.ext = extend_rect(r.roi, params[i].margin, g.n);
        r.plan = make_plan(g, r.ext, r.ext);
        rays += (long long)g.na * r.plan.wmax;
        pix += (long long)r.ext.rows * r.ext.cols;
        const bool fista = params[i].method == ROI_LOCAL_FISTA_TV;
        const bool haar = params[i].method == ROI_LOCAL_FISTA_HAAR;
        sfl[i] = local_state_floats(g, r.plan, true, fista || haar);
        state_total += sfl[i] * sizeof(float);
        if (fista)
            max_nf = std::max(max_nf, params[i].inner_iters > 0 ? params[i].inner_iters : 100);
        max_iters = std::max(max_iters, params[i].iters);
    }
    // the regions' own projections may stage their lines in LDS
    int max_pitch = 0, max_w = 0;
    for (const RoiState& r : R) {
        max_pitch = std::max(max_pitch, std::max(r.plan.xp, r.plan.tp));
        max_w = std::max(max_w, r.plan.wmax);
    }
    LaunchCfg L = choose_launch_for(ctx, geom, count, rays, pix, max_pitch, max_w);
    int th, tw;
    bp_tile(L.ag, L.ppt, &th, &tw);

    std::vector<char*> allocs;
    auto cleanup = [&]() { ctx->arena.free_after(allocs, s); };
    Meta m;
    std::vector<size_t> o_afp(count), o_abp(count);
    for (int i = 0; i < count; ++i) {
        o_afp[i] = m.add(R[i].plan.afp.data(), R[i].plan.afp.size() * sizeof(AngFP));
        o_abp[i] = m.add(R[i].plan.abp.data(), R[i].plan.abp.size() * sizeof(AngBP));
    }
    const std::vector<float> b_in = fista_betas(max_nf), b_out = fista_betas(max_iters);
    const size_t o_bin = m.add(b_in.data(), b_in.size() * sizeof(float));
    const size_t o_bout = m.add(b_out.data(), b_out.size() * sizeof(float));
    char* dm = ctx->arena.alloc(align_up(m.buf.size(), 256) + state_total + 256);
    if (!dm)
        return fail(ctx, TOMO_ENOMEM, "workspace too small for %d local-method states", count);
    allocs.push_back(dm);
    float* state = (float*)(dm + align_up(m.buf.size(), 256));
    std::vector<LocalBuf> B(count);
    {
        float* f = state;
        for (int i = 0; i < count; ++i) {
            B[i] = carve_local(g, R[i].plan, true, f, R[i].prm.method >= ROI_LOCAL_FISTA_TV);
            f += sfl[i];
            RoiState& r = R[i];
            r.d_afp = (AngFP*)(dm + o_afp[i]);
            r.d_abp = (AngBP*)(dm + o_abp[i]);
            r.x = B[i].x;
            r.xb0 = B[i].xb0;
            r.xb1 = B[i].xb1;
            r.xt = B[i].xt;
            r.y = B[i].y;
        }
    }
    // ROIs by decreasing iteration count (the running ones form a prefix of the
    // work lists), larger regions first within a count.
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (R[a].prm.iters != R[b].prm.iters) return R[a].prm.iters > R[b].prm.iters;
        return (long long)R[a].ext.rows * R[a].ext.cols > (long long)R[b].ext.rows * R[b].ext.cols;
    });
    std::vector<Job> jobs(count);
    std::vector<Item> fi, bi, gi;
    std::vector<int> fi_end(count), bi_end(count), gi_end(count), nf_of(count, 0);
    // Haar prox items, one list per level count
    std::vector<Item> hi[kHaarMaxLevels + 1];
    std::vector<int> hi_end[kHaarMaxLevels + 1];
    for (auto& v : hi_end) v.assign(count, 0);
    std::vector<int> lv_of(count, 0);
    for (int q = 0; q < count; ++q) {
        RoiState& r = R[order[q]];
        const LocalBuf& lb = B[order[q]];
        const bool fista = r.prm.method == ROI_LOCAL_FISTA_TV;
        const bool haar = r.prm.method == ROI_LOCAL_FISTA_HAAR;
        Job J = make_job(g, r, FP_LOCAL, (fista || haar) ? BP_FISTA : BP_LOCAL,
                         (r.ext.cols + tw - 1) / tw);
        J.gbase = filtered;
        J.gstride = (int64_t)g.na * g.nd;
        J.dk0 = 0;
        J.z[0] = J.z[1] = nullptr;
        J.b = nullptr;
        J.part = nullptr;
        J.w = lb.w;
        J.xs = lb.xs;
        J.fp = lb.fp;
        J.fr = lb.fr;
        J.beta_in = (const float*)(dm + o_bin);
        J.beta_out = (const float*)(dm + o_bout);
        jobs[q] = J;
        fp_items(fi, q, r.plan.afp, L.seg, L.rp, r.d_afp);
        bp_items(bi, q, r.ext.rows, r.ext.cols, L.ag, L.ppt, r.d_abp);
        if (fista) {
            nf_of[q] = J.n_fgp;
            for (int a = 0; a < (r.ext.rows + kFgpTile - 1) / kFgpTile; ++a)
                for (int b = 0; b < (r.ext.cols + kFgpTile - 1) / kFgpTile; ++b)
                    gi.push_back(Item{q, a, b, 0, nullptr, 0});
        }
        if (haar) {
            const int L = J.levels, T = 1 << L;
            lv_of[q] = L;
            for (int a = 0; a < (r.ext.rows + T - 1) / T; ++a)
                for (int b = 0; b < (r.ext.cols + T - 1) / T; ++b)
                    hi[L].push_back(Item{q, a, b, 0, nullptr, 0});
        }
        fi_end[q] = (int)fi.size();
        bi_end[q] = (int)bi.size();
        gi_end[q] = (int)gi.size();
        for (int L = 1; L <= kHaarMaxLevels; ++L) hi_end[L][q] = (int)hi[L].size();
    }
    Meta m2;
    const size_t o_jobs = m2.add(jobs.data(), jobs.size() * sizeof(Job));
    const size_t o_fi = m2.add(fi.data(), fi.size() * sizeof(Item));
    const size_t o_bi = m2.add(bi.data(), bi.size() * sizeof(Item));
    const size_t o_gi = m2.add(gi.data(), gi.size() * sizeof(Item));
    size_t o_hi[kHaarMaxLevels + 1];
    for (int L = 1; L <= kHaarMaxLevels; ++L) o_hi[L] = m2.add(hi[L].data(), hi[L].size() * sizeof(Item));
    const int max_it = R[order[0]].prm.iters;
    const bool timed = ctx->timing_mode == 1;
    auto enqueue_loop = [&](char* base, hipStream_t sq) -> hipError_t {
        const Job* d_jobs = (const Job*)(base + o_jobs);
        const Item* d_fi = (const Item*)(base + o_fi);
        const Item* d_bi = (const Item*)(base + o_bi);
        const Item* d_gi = (const Item*)(base + o_gi);
        int active = count;
        for (int it = 0; it < max_it; ++it) {
            while (active > 0 && R[order[active - 1]].prm.iters <= it) --active;
            int nf = -1;   // FGP iterations of the running FISTA jobs (-1: none)
            bool any_haar = false;
            for (int q = 0; q < active; ++q) {
                if (R[order[q]].prm.method == ROI_LOCAL_FISTA_TV) nf = std::max(nf, nf_of[q]);
                if (R[order[q]].prm.method == ROI_LOCAL_FISTA_HAAR) any_haar = true;
            }
            hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
            hipError_t e;
            if (timed) {
                e0 = timing_event(ctx);
                e1 = timing_event(ctx);
                e2 = timing_event(ctx);
                if ((e = hipEventRecord(e0, sq)) != hipSuccess) return e;
            }
            if ((e = launch_fp(d_jobs, d_fi, fi_end[active - 1], it, L.seg, sq, L.cfp, L.rp,
                               L.spitch)) != hipSuccess)
                return e;
            if (timed && (e = hipEventRecord(e1, sq)) != hipSuccess) return e;
            if ((e = launch_bp(d_jobs, d_bi, bi_end[active - 1], it, L.ag, L.ppt, sq, L.cbp,
                               L.staged, 0, 1)) != hipSuccess)
                return e;
            if (timed) {
                if ((e = hipEventRecord(e2, sq)) != hipSuccess) return e;
                ctx->ev_pending.emplace_back(e0, e1, 0);
                ctx->ev_pending.emplace_back(e1, e2, 1);
            }
            if (nf >= 0) {   // FGP steps, kFgpSteps per launch; the last one finishes x^k
                const int nl = std::max(1, (nf + kFgpSteps - 1) / kFgpSteps);
                for (int l = 0; l < nl; ++l)
                    if ((e = launch_fgp(d_jobs, d_gi, gi_end[active - 1], it, l * kFgpSteps, sq)) !=
                        hipSuccess)
                        return e;
            }
            if (any_haar) {   // one tiled Haar prox launch per level count in use
                for (int L = 1; L <= kHaarMaxLevels; ++L)
                    if (hi_end[L][active - 1] > 0 &&
                        (e = launch_haar(d_jobs, (const Item*)(base + o_hi[L]),
                                         hi_end[L][active - 1], it, L, sq)) != hipSuccess)
                        return e;
            }
            if (nf >= 0 || any_haar) {
                if (timed) {
                    e3 = timing_event(ctx);
                    if ((e = hipEventRecord(e3, sq)) != hipSuccess) return e;
                    ctx->ev_pending.emplace_back(e2, e3, 2);
                }
            }
        }
        return hipSuccess;
    };
#define CK(expr)                                                                          \
    do {                                                                                  \
        hipError_t e__ = (expr);                                                          \
        if (e__ != hipSuccess) {                                                          \
            cleanup();                                                                    \
            return fail(ctx, TOMO_EHIP, "%s failed: %s", #expr, hipGetErrorString(e__));  \
        }                                                                                 \
    } while (0)
    CK(ctx->staging.upload(dm, m.buf.data(), m.buf.size(), s));
    CK(launch_fill(state, state_total / sizeof(float), 0.f, s));
    if (!timed) {
        std::vector<long long> key = {1,     max_it, L.seg, L.ag,  L.ppt, L.rp,
                                      L.staged, L.cfp, L.cbp, count, (long long)m2.buf.size()};
        for (int q = 0; q < count; ++q) {
            key.push_back(R[order[q]].prm.iters);
            key.push_back(fi_end[q]);
            key.push_back(bi_end[q]);
            key.push_back(gi_end[q]);
            key.push_back(nf_of[q]);
            key.push_back(lv_of[q]);
            key.push_back(R[order[q]].prm.method);
        }
        tomo_status rs = run_loop(ctx, key, m2, enqueue_loop, s, allocs);
        if (rs != TOMO_OK) {
            cleanup();
            return rs;
        }
    } else {
        char* dm2 = ctx->arena.alloc(m2.buf.size());
        if (!dm2) {
            cleanup();
            return fail(ctx, TOMO_ENOMEM, "workspace too small for the iteration tables");
        }
        allocs.push_back(dm2);
        CK(ctx->staging.upload(dm2, m2.buf.data(), m2.buf.size(), s));
        CK(enqueue_loop(dm2, s));
    }
    for (int i = 0; i < count; ++i) {
        const RoiState& r = R[i];
        CK(launch_crop(r.x, r.ext.cols, r.roi.r0 - r.ext.r0, r.roi.c0 - r.ext.c0, r.roi.rows,
                       r.roi.cols, outs[i], r.roi.cols, s));
    }
#undef CK
    cleanup();
    return TOMO_OK;
    GUARD_END(ctx)
}

tomo_status tomo_disc_subtract(tomo_ctx* ctx, int32_t geom, const float* sino, float* out,
                               float* value, void* hip_stream) {
    tomo_status st = need_gpu(ctx);
    if (st != TOMO_OK) return st;
    if (!sino || !out || !value) return fail(ctx, TOMO_EINVAL, "null pointer");
    GUARD_BEGIN
    const Geom* gp;
    if ((st = get_geom(ctx, geom, &gp)) != TOMO_OK) return st;
    const Geom& g = *gp;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t npix = (size_t)g.n * g.n, nsino = (size_t)g.na * g.nd;
    char* blk = ctx->arena.alloc(align_up(npix * sizeof(float), 256) +
                                 align_up(nsino * sizeof(float), 256) + 2 * g.na * sizeof(double));
    if (!blk) return fail(ctx, TOMO_ENOMEM, "workspace too small for the disc projection");
    std::vector<char*> allocs{blk};
    float* disc = (float*)blk;
    float* D = (float*)(blk + align_up(npix * sizeof(float), 256));
    double* sums = (double*)((char*)D + align_up(nsino * sizeof(float), 256));
    hipError_t e = launch_disc(disc, g.n, g.n, 0, 0, g.n, g.n, nullptr, 0, s);
    if (e != hipSuccess) {
        ctx->arena.free_after(allocs, s);
        return fail(ctx, TOMO_EHIP, "disc image: %s", hipGetErrorString(e));
    }
    // D = W disc through the library's own projection call
    st = tomo_fp(ctx, geom, tomo_rect{0, 0, g.n, g.n}, disc, D, 0, hip_stream);
    if (st == TOMO_OK) {
        e = launch_disc_value(sino, D, g.na, g.nd, sums, value, s);
        if (e == hipSuccess) e = launch_disc_apply(sino, D, nsino, value, out, s);
        if (e != hipSuccess) st = fail(ctx, TOMO_EHIP, "disc subtraction: %s", hipGetErrorString(e));
    }
    ctx->arena.free_after(allocs, s);
    return st;
    GUARD_END(ctx)
}

tomo_status tomo_disc_add(tomo_ctx* ctx, int32_t geom, tomo_rect region, const float* value,
                          float* img, void* hip_stream) {
    tomo_status st = need_gpu(ctx);
    if (st != TOMO_OK) return st;
    if (!value || !img) return fail(ctx, TOMO_EINVAL, "null pointer");
    GUARD_BEGIN
    const Geom* gp;
    if ((st = get_geom(ctx, geom, &gp)) != TOMO_OK) return st;
    const Geom& g = *gp;
    if (region.rows < 1 || region.cols < 1 || region.row0 < 0 || region.col0 < 0 ||
        region.row0 + region.rows > g.n || region.col0 + region.cols > g.n)
        return fail(ctx, TOMO_EINVAL, "region is empty or outside the grid");
    TOMO_HIP(ctx, launch_disc(img, region.cols, g.n, region.row0, region.col0, region.rows,
                              region.cols, value, 1, (hipStream_t)hip_stream));
    return TOMO_OK;
    GUARD_END(ctx)
}

tomo_status tomo_pad_truncated(tomo_ctx* ctx, int32_t geom, const float* trunc, int32_t first_bin,
                               int32_t n_bins, float* out, void* hip_stream) {
    tomo_status st = need_gpu(ctx);
    if (st != TOMO_OK) return st;
    if (!trunc || !out) return fail(ctx, TOMO_EINVAL, "null pointer");
    GUARD_BEGIN
    const Geom* gp;
    if ((st = get_geom(ctx, geom, &gp)) != TOMO_OK) return st;
    const Geom& g = *gp;
    if (n_bins < 1 || first_bin < 0 || first_bin + n_bins > g.nd)
        return fail(ctx, TOMO_EINVAL, "measured bins [%d, %d) outside the %d-bin detector",
                    first_bin, first_bin + n_bins, g.nd);
    TOMO_HIP(ctx, launch_pad_truncated(trunc, g.na, n_bins, first_bin, g.nd, out,
                                       (hipStream_t)hip_stream));
    return TOMO_OK;
    GUARD_END(ctx)
}
