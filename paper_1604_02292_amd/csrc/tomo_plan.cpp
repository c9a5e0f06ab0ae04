// Host-side planning: geometry tables, detector bands, the workspace arena and
// pinned staging for uploads.  No GPU kernels here.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "tomo_runtime.h"
#include "tomo_serve.h"

namespace tomo {

tomo_status fail(tomo_ctx* ctx, tomo_status st, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (on_serve_thread())
        set_thread_error(buf);
    else if (ctx)
        ctx->err = buf;
    return st;
}

static inline int round_up(int v, int a) { return (v + a - 1) / a * a; }

Rect extend_rect(const Rect& roi, int margin, int n) {
    // Section 3.3: pad the local part on each side, clipped to the grid.
    const int a0 = std::max(0, roi.r0 - margin), b0 = std::max(0, roi.c0 - margin);
    const int a1 = std::min(n, roi.r0 + roi.rows + margin);
    const int b1 = std::min(n, roi.c0 + roi.cols + margin);
    return Rect{a0, b0, a1 - a0, b1 - b0};
}

// Bins of angle k that pixels of rect b may reach: |s_i - t| < m for t between
// the extreme pixel-centre projections, widened by one bin on each side and not
// clipped to the detector (off-detector entries stay zero in band arrays).
void band_of(const Geom& g, const Rect& b, int k, int* i0, int* w) {
    const double h = (g.n - 1) / 2.0, hd = (g.nd - 1) / 2.0;
    const double xa = b.c0 - h, xb = b.c0 + b.cols - 1 - h;
    const double ya = b.r0 - h, yb = b.r0 + b.rows - 1 - h;
    const double c = g.c[k], s = g.s[k], m = g.m[k];
    const double t[4] = {xa * c + ya * s, xb * c + ya * s, xa * c + yb * s, xb * c + yb * s};
    const double tmin = std::min(std::min(t[0], t[1]), std::min(t[2], t[3]));
    const double tmax = std::max(std::max(t[0], t[1]), std::max(t[2], t[3]));
    const double ulo = (tmin - m - g.offset) / g.spacing + hd;
    const double uhi = (tmax + m - g.offset) / g.spacing + hd;
    const int lo = (int)std::floor(ulo) - 1;
    const int hi = (int)std::ceil(uhi) + 1;
    *i0 = lo;
    *w = hi - lo + 1;
}

Plan make_plan(const Geom& g, const Rect& reg, const Rect& bsrc) {
    Plan P;
    P.reg = reg;
    P.afp.resize(g.na);
    P.abp.resize(g.na);
    const double h = (g.n - 1) / 2.0, hd = (g.nd - 1) / 2.0;
    const double x0 = reg.c0 - h, y0 = reg.r0 - h;   // centre of the region's pixel (0, 0)
    const double sp = g.spacing;
    for (int k = 0; k < g.na; ++k) {
        int i0, w;
        band_of(g, bsrc, k, &i0, &w);
        const double c = g.c[k], s = g.s[k], m = g.m[k];
        const double D = ((i0 - hd) * sp + g.offset) - (x0 * c + y0 * s);
        AngFP& a = P.afp[k];
        std::memset(&a, 0, sizeof a);
        if (g.ystep[k]) {   // ray j meets row r at column (D + j sp - r s) / c
            a.a0 = D / c + kLpad;
            a.aj = sp / c;
            a.step = -s / c;
            a.tr = 0;
        } else {            // ray j meets column q at row (D + j sp - q c) / s
            a.a0 = D / s + kLpad;
            a.aj = sp / s;
            a.step = -c / s;
            a.tr = 1;
        }
        a.inv_m = (float)(1.0 / m);
        a.w = w;
        a.i0 = i0;
        a.bscale = (float)(sp / (m * m));
        AngBP& bp = P.abp[k];
        std::memset(&bp, 0, sizeof bp);
        bp.cud = c / sp;
        bp.sud = s / sp;
        bp.u0 = -D / sp + 1.0;
        bp.cu = (float)bp.cud;
        bp.su = (float)bp.sud;
        bp.r = (float)(m / sp);
        bp.rm1 = (float)(m / sp - 1.0);
        P.wmax = std::max(P.wmax, w);
    }
    // at least 64 entries: the backprojector stages 64-entry windows of each row
    P.bpitch = std::max(64, round_up(P.wmax + 3, 4));
    P.xp = round_up(reg.cols + kLpad + 2, 4);
    P.tp = round_up(reg.rows + kLpad + 2, 4);
    return P;
}

// ---------------------------------------------------------------------------
void Arena::init(char* base, size_t bytes) {
    std::lock_guard<std::recursive_mutex> lk(mu_);
    base_ = base;
    size_ = bytes;
    free_.clear();
    live_.clear();
    used_ = peak_ = 0;
    if (bytes) free_[0] = bytes;
}

size_t Arena::largest_free() const {
    size_t best = 0;
    for (auto& kv : free_) best = std::max(best, kv.second);
    return best;
}

char* Arena::alloc(size_t bytes, bool wait) {
    std::lock_guard<std::recursive_mutex> lk(mu_);
    bytes = ((std::max<size_t>(bytes, 1) + 255) / 256) * 256;
    for (int attempt = 0; attempt < 3; ++attempt) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            live_[off] = bytes;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return base_ + off;
        }
        if (attempt == 0)
            reclaim(false);
        else if (attempt == 1 && wait)
            reclaim(true);
        else
            break;
    }
    return nullptr;
}

void Arena::release_locked(size_t off) {
    auto it = live_.find(off);
    if (it == live_.end()) return;
    size_t len = it->second;
    live_.erase(it);
    used_ -= len;
    size_t start = off;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {
        len += nx->second;
        free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
            start = pv->first;
            len += pv->second;
            free_.erase(pv);
        }
    }
    free_[start] = len;
}

void Arena::free_now(char* p) {
    if (!p) return;
    std::lock_guard<std::recursive_mutex> lk(mu_);
    release_locked((size_t)(p - base_));
}

void Arena::free_after(std::vector<char*> ps, hipStream_t s) {
    std::lock_guard<std::recursive_mutex> lk(mu_);
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess) {
        // cannot order the free: wait for the stream instead
        if (ev) (void)hipEventDestroy(ev);
        (void)hipStreamSynchronize(s);
        for (char* p : ps)
            if (p) release_locked((size_t)(p - base_));
        return;
    }
    pending_.emplace_back(ev, std::move(ps));
}

void Arena::reclaim(bool wait) {
    std::lock_guard<std::recursive_mutex> lk(mu_);
    for (auto it = pending_.begin(); it != pending_.end();) {
        const hipError_t q = wait ? hipEventSynchronize(it->first) : hipEventQuery(it->first);
        if (q != hipSuccess) {
            ++it;
            continue;
        }
        for (char* p : it->second)
            if (p) release_locked((size_t)(p - base_));
        (void)hipEventDestroy(it->first);
        it = pending_.erase(it);
    }
}

// ---------------------------------------------------------------------------
hipError_t Staging::upload(void* dev, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (ev_live) {
        hipError_t e = hipEventSynchronize(ev);
        if (e != hipSuccess) return e;
        ev_live = false;
    }
    if (cap < bytes) {
        if (host) (void)hipHostFree(host);
        host = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(bytes, 1 << 20);
        hipError_t e = hipHostMalloc(&host, want, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        cap = want;
    }
    if (!ev) {
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    std::memcpy(host, src, bytes);
    hipError_t e = hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipEventRecord(ev, s);
    if (e != hipSuccess) return e;
    ev_live = true;
    return hipSuccess;
}

void Staging::destroy() {
    if (ev_live) (void)hipEventSynchronize(ev);
    if (ev) (void)hipEventDestroy(ev);
    if (host) (void)hipHostFree(host);
    host = nullptr;
    ev = nullptr;
    cap = 0;
    ev_live = false;
}

}  // namespace tomo
