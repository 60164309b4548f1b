// capi.hip -- host side of the C ABI declared in include/rdseg.h: argument
// validation, workspace layout, launch orchestration, batched plans with
// hipGraph capture, per-launch timing and the autotuner.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rdseg.h"
#include "rdseg_internal.h"

namespace rdseg {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

}  // namespace rdseg

using namespace rdseg;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sequential carve-out of a workspace.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t count) {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off = align_up(off + count * sizeof(T));
        return p;
    }
};

rdseg_status fail(rdseg_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

rdseg_status hip_status(int rc) { return rc ? RDSEG_ERR_HIP : RDSEG_OK; }

bool shape_ok(const rdseg_shape& s) {
    if (s.H < 1 || s.W < 1 || s.ld < s.W) return false;
    if ((int64_t)s.H * s.ld >= (int64_t)1 << 31) return false;
    return true;
}

rdseg_status check_shape(const rdseg_shape& s) {
    if (!shape_ok(s))
        return fail(RDSEG_ERR_SHAPE, "invalid shape: need H, W >= 1, ld >= W and H*ld < 2^31");
    return RDSEG_OK;
}

rdseg_status check_scalars(double lambda, double theta, double tau, double delta) {
    if (!(isfinite(lambda) && lambda >= 0)) return fail(RDSEG_ERR_ARG, "lambda must be finite and >= 0");
    if (!(isfinite(theta) && theta > 0)) return fail(RDSEG_ERR_ARG, "theta must be finite and > 0");
    if (!(isfinite(tau) && tau > 0)) return fail(RDSEG_ERR_ARG, "tau must be finite and > 0");
    if (isnan(delta)) return fail(RDSEG_ERR_ARG, "delta must not be NaN");
    return RDSEG_OK;
}

struct Geo {
    int64_t plane, tw, th, nt, strips, chunks;
};

Geo geo_of(const rdseg_shape& s) {
    Geo g;
    g.plane = (int64_t)s.H * s.ld;
    g.tw = (s.W + 7) / 8;
    g.th = (s.H + 7) / 8;
    g.nt = g.tw * g.th;
    g.strips = g.th * ((g.tw + 7) / 8);
    g.chunks = ((int64_t)s.H * s.W + 63) / 64;
    return g;
}

int64_t macro_count(const rdseg_shape& s, int bx, int by) {
    return (int64_t)((s.W + bx - 1) / bx) * ((s.H + by - 1) / by);
}

// Workspace of a single-image solve / active-set call.
struct SolveWs {
    float* c;
    float* st[3];
    uint64_t* masks;
    int64_t* npix;
    int32_t* flags;
    int32_t* offs;
    int32_t* part;
    int2* queue;
    int32_t* totals;   // [0] n_queue, [1] scratch total
    size_t bytes;
};

SolveWs carve_solve(void* base, const rdseg_shape& s) {
    Geo g = geo_of(s);
    Carver cv(base);
    SolveWs w;
    w.c = cv.take<float>(g.plane);
    for (int k = 0; k < 3; ++k) w.st[k] = cv.take<float>(g.plane);
    w.masks = cv.take<uint64_t>(g.nt);
    w.npix = cv.take<int64_t>(1);
    int64_t nflag = std::max<int64_t>(g.nt, g.chunks);
    w.flags = cv.take<int32_t>(nflag);
    w.offs = cv.take<int32_t>(nflag);
    w.part = cv.take<int32_t>(scan_partials(nflag));
    w.queue = cv.take<int2>(g.nt);
    w.totals = cv.take<int32_t>(4);
    w.bytes = cv.off;
    return w;
}

ImgDesc make_desc(const float* f, const rdseg_shape& s, double lambda, double theta,
                  double delta, float* u, float* v, float* p, float* c, float* const st1[3],
                  const float* u0, const float* p0, int bx, int by) {
    ImgDesc d;
    memset(&d, 0, sizeof(d));
    int64_t plane = (int64_t)s.H * s.ld;
    d.f = f;
    d.u = u;
    d.c = c;
    d.st[0][0] = v;
    d.st[0][1] = p;
    d.st[0][2] = p ? p + plane : nullptr;
    d.st[1][0] = st1[0];
    d.st[1][1] = st1[1];
    d.st[1][2] = st1[2];
    d.u0 = u0;
    d.p0x = p0;
    d.p0y = p0 ? p0 + plane : nullptr;
    d.H = s.H;
    d.W = s.W;
    d.ld = (int32_t)s.ld;
    d.tw = (s.W + 7) / 8;
    d.th = (s.H + 7) / 8;
    d.mw = (s.W + bx - 1) / bx;
    d.mh = (s.H + by - 1) / by;
    d.tl = (float)(theta * lambda);
    d.delta = delta;
    return d;
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

// ------------------------------------------------------------------ timing
struct TimingRec {
    hipEvent_t e0, e1;
    int nit;
    int64_t* npix_host;   // pinned slot filled by an async copy
};

struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<TimingRec> recs;
    std::vector<hipEvent_t> pool;
    int64_t* pinned = nullptr;
    size_t pinned_cap = 0, pinned_used = 0;
} g_timing;

hipEvent_t timing_event() {
    if (!g_timing.pool.empty()) {
        hipEvent_t e = g_timing.pool.back();
        g_timing.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int64_t* timing_slot() {
    if (!g_timing.pinned) {
        g_timing.pinned_cap = 1 << 16;
        if (hipHostMalloc((void**)&g_timing.pinned, g_timing.pinned_cap * sizeof(int64_t), 0) !=
            hipSuccess) {
            g_timing.pinned = nullptr;
            return nullptr;
        }
    }
    if (g_timing.pinned_used >= g_timing.pinned_cap) return nullptr;
    return g_timing.pinned + g_timing.pinned_used++;
}

// ------------------------------------------------------------------ tuning cache
struct TuneKey {
    int cls, qb;
    bool operator<(const TuneKey& o) const { return cls != o.cls ? cls < o.cls : qb < o.qb; }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

int size_class(const rdseg_shape& s) {
    int64_t n = (int64_t)s.H * s.W;
    int c = 0;
    while (n > 4096 && c < 12) { n >>= 2; ++c; }
    return c;
}

int q_bucket(double q) {
    if (q >= 0.5) return 4;
    if (q >= 0.2) return 3;
    if (q >= 0.05) return 2;
    if (q >= 0.01) return 1;
    return 0;
}

int heuristic_cfg(const rdseg_shape& s, double q) {
    int64_t n = (int64_t)s.H * s.W;
    if (n <= 128 * 128) return config_index(16, 16, 2);
    if (q >= 0.2) return config_index(64, 64, 4);
    if (q >= 0.03) return config_index(32, 32, 2);
    return config_index(16, 16, 1);
}

// ------------------------------------------------------------------ solve core
struct SolvePlanArgs {
    const ImgDesc* d0;
    const ImgDesc* descs;   // batched when non-NULL
    const int2* queue;
    const int32_t* n_queue;
    int64_t max_items;
    int ci;
    int iters;
    float theta, inv_theta, tau;
    int ckpt_every;
    float* tape;            // single image only
    const int64_t* npix;    // for timing
    hipStream_t st;
};

// Enqueue the launches of `iters` iterations; the final state lands in
// buffer 0 (the caller's v, p) and u is written by the last launch.
rdseg_status enqueue_iterations(const SolvePlanArgs& a) {
    if (a.iters <= 0) return RDSEG_OK;
    const int IT = config_at(a.ci).it;
    const int ce = (a.tape && a.ckpt_every > 0) ? a.ckpt_every : a.iters;
    // launch schedule: segments of ce iterations, each split into <= IT chunks
    std::vector<int> nits;
    std::vector<int> seg_start;   // launch index that starts each segment
    for (int k0 = 0; k0 < a.iters; k0 += ce) {
        int len = std::min(ce, a.iters - k0);
        seg_start.push_back((int)nits.size());
        for (int j = 0; j < len; j += IT) nits.push_back(std::min(IT, len - j));
    }
    const int L = (int)nits.size();
    size_t seg = 0;
    const int64_t plane = (int64_t)a.d0->H * a.d0->ld;
    for (int j = 0; j < L; ++j) {
        int in_buf = (L - j) % 2;
        if (a.tape && seg < seg_start.size() && seg_start[seg] == j) {
            int rc = launch_state_copy(*a.d0, in_buf, a.tape + (int64_t)seg * 3 * plane, true, a.st);
            if (rc) return RDSEG_ERR_HIP;
            ++seg;
        }
        TimingRec rec{};
        bool timed = false;
        if (g_timing.on) {
            std::lock_guard<std::mutex> lk(g_timing.mu);
            rec.e0 = timing_event();
            rec.e1 = timing_event();
            rec.nit = nits[j];
            rec.npix_host = nullptr;
            timed = rec.e0 && rec.e1;
            if (timed) (void)hipEventRecord(rec.e0, a.st);
        }
        int rc = launch_iterate(a.ci, a.d0, a.descs, a.descs != nullptr, a.queue, a.n_queue,
                                a.max_items, in_buf, nits[j], j == L - 1, a.theta, a.inv_theta,
                                a.tau, a.st);
        if (rc) return RDSEG_ERR_HIP;
        if (timed) {
            std::lock_guard<std::mutex> lk(g_timing.mu);
            (void)hipEventRecord(rec.e1, a.st);
            rec.npix_host = timing_slot();
            if (rec.npix_host && a.npix)
                (void)hipMemcpyAsync(rec.npix_host, a.npix, sizeof(int64_t), hipMemcpyDeviceToHost, a.st);
            g_timing.recs.push_back(rec);
        }
    }
    return RDSEG_OK;
}

// Choose the tile configuration for a single-image solve.
rdseg_status choose_cfg(const rdseg_params& prm, const rdseg_shape& s, const int64_t* npix_dev,
                        hipStream_t st, int* ci) {
    if (prm.tile_w > 0 && prm.tile_h > 0 && prm.iters_per_launch > 0) {
        *ci = config_index(prm.tile_w, prm.tile_h, prm.iters_per_launch);
        if (*ci < 0) return fail(RDSEG_ERR_ARG, "tile_w / tile_h / iters_per_launch is not a compiled configuration");
        return RDSEG_OK;
    }
    if (prm.tile_w || prm.tile_h || prm.iters_per_launch)
        return fail(RDSEG_ERR_ARG, "tile_w, tile_h and iters_per_launch must be all set or all 0");
    int64_t np = 0;
    if (hipMemcpyAsync(&np, npix_dev, sizeof(np), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(RDSEG_ERR_HIP, "reading the active-pixel count failed");
    double q = (double)np / ((double)s.H * s.W);
    TuneKey k{size_class(s), q_bucket(q)};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(k);
        if (it != g_tune.end()) {
            *ci = it->second;
            return RDSEG_OK;
        }
    }
    *ci = heuristic_cfg(s, q);
    return RDSEG_OK;
}

rdseg_status solve_impl(const float* f, rdseg_shape s, const rdseg_params* prm, const float* u0,
                        const float* p0, float* u, float* v, float* p, float* tape, void* ws,
                        size_t ws_bytes, hipStream_t st, int forced_ci) {
    if (!prm) return fail(RDSEG_ERR_ARG, "prm is NULL");
    rdseg_status r = check_shape(s);
    if (r) return r;
    r = check_scalars(prm->lambda, prm->theta, prm->tau, prm->delta);
    if (r) return r;
    if (!f || !u || !v || !p) return fail(RDSEG_ERR_ARG, "f, u, v and p must be non-NULL");
    if (prm->iters < 0) return fail(RDSEG_ERR_ARG, "iters must be >= 0");
    if (prm->ckpt_every < 0) return fail(RDSEG_ERR_ARG, "ckpt_every must be >= 0");
    if (prm->ckpt_every > 0 && !tape) return fail(RDSEG_ERR_TAPE, "ckpt_every > 0 needs a tape");
    const size_t plane_b = (size_t)s.H * s.ld * sizeof(float);
    if (ranges_overlap(u, plane_b, f, plane_b) || ranges_overlap(v, plane_b, f, plane_b) ||
        ranges_overlap(p, 2 * plane_b, f, plane_b) || ranges_overlap(u, plane_b, v, plane_b) ||
        ranges_overlap(u, plane_b, p, 2 * plane_b) || ranges_overlap(v, plane_b, p, 2 * plane_b))
        return fail(RDSEG_ERR_ARG, "u, v, p must not overlap f or each other");
    if ((u0 && u0 != u && ranges_overlap(u0, plane_b, u, plane_b)) ||
        (p0 && p0 != p && ranges_overlap(p0, 2 * plane_b, p, 2 * plane_b)))
        return fail(RDSEG_ERR_ARG, "u0 / p0 may equal u / p but must not partially overlap them");
    SolveWs need = carve_solve(nullptr, s);
    if (!ws || ws_bytes < need.bytes)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need.bytes) + " bytes");
    int ci = forced_ci;
    const bool explicit_cfg = prm->tile_w > 0 || prm->tile_h > 0 || prm->iters_per_launch > 0;
    if (ci < 0 && explicit_cfg) {
        r = choose_cfg(*prm, s, nullptr, st, &ci);   // validates before any launch
        if (r) return r;
    }
    SolveWs w = carve_solve(ws, s);
    Geo g = geo_of(s);

    // tile-configuration independent part of the descriptor first
    ImgDesc d = make_desc(f, s, prm->lambda, prm->theta, prm->delta, u, v, p, w.c, w.st, u0, p0, 8, 8);
    OffTables off{nullptr, nullptr, nullptr, nullptr};
    if (launch_tile_masks(&d, nullptr, off, 1, g.strips, w.masks, w.npix, st)) return RDSEG_ERR_HIP;
    if (ci < 0) {
        r = choose_cfg(*prm, s, w.npix, st, &ci);
        if (r) return r;
    }
    TileCfg cfg = config_at(ci);
    d = make_desc(f, s, prm->lambda, prm->theta, prm->delta, u, v, p, w.c, w.st, u0, p0, cfg.bx, cfg.by);
    if (launch_init(&d, nullptr, off, 1, s.H, st)) return RDSEG_ERR_HIP;
    int64_t nm = macro_count(s, cfg.bx, cfg.by);
    if (launch_macro_queue(&d, nullptr, off, 1, nm, cfg.bx, cfg.by, w.masks, w.flags, w.offs,
                           w.part, w.queue, w.totals, st))
        return RDSEG_ERR_HIP;
    SolvePlanArgs a;
    a.d0 = &d;
    a.descs = nullptr;
    a.queue = w.queue;
    a.n_queue = w.totals;
    a.max_items = nm;
    a.ci = ci;
    a.iters = prm->iters;
    a.theta = (float)prm->theta;
    a.inv_theta = (float)(1.0 / prm->theta);
    a.tau = (float)prm->tau;
    a.ckpt_every = prm->ckpt_every;
    a.tape = prm->ckpt_every > 0 ? tape : nullptr;
    a.npix = w.npix;
    a.st = st;
    return enqueue_iterations(a);
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* rdseg_status_string(rdseg_status st) {
    switch (st) {
        case RDSEG_OK: return "ok";
        case RDSEG_ERR_ARG: return "invalid argument";
        case RDSEG_ERR_SHAPE: return "invalid shape";
        case RDSEG_ERR_WORKSPACE: return "workspace too small";
        case RDSEG_ERR_HIP: return "HIP error";
        case RDSEG_ERR_TAPE: return "tape missing or inconsistent";
    }
    return "unknown status";
}

const char* rdseg_last_error(void) { return get_error(); }

size_t rdseg_workspace_size(const rdseg_shape* s, const rdseg_params* prm) {
    (void)prm;
    if (!s || !shape_ok(*s)) return 0;
    return carve_solve(nullptr, *s).bytes;
}

size_t rdseg_tape_size(const rdseg_shape* s, const rdseg_params* prm) {
    if (!s || !prm || !shape_ok(*s) || prm->ckpt_every <= 0 || prm->iters < 0) return 0;
    int64_t n = (prm->iters + prm->ckpt_every - 1) / prm->ckpt_every;
    return (size_t)n * 3 * (size_t)s->H * (size_t)s->ld * sizeof(float);
}

rdseg_status rdseg_active_set(const float* f, rdseg_shape s, double delta, int32_t* tile_ids,
                              uint64_t* tile_masks, int32_t* slot_map, int32_t* n_tiles,
                              int32_t* pixel_idx, int64_t* n_pixels, void* ws, size_t ws_bytes,
                              void* stream) {
    rdseg_status r = check_shape(s);
    if (r) return r;
    if (!f || !tile_ids || !tile_masks || !slot_map || !n_tiles)
        return fail(RDSEG_ERR_ARG, "f, tile_ids, tile_masks, slot_map and n_tiles must be non-NULL");
    if ((pixel_idx == nullptr) != (n_pixels == nullptr))
        return fail(RDSEG_ERR_ARG, "pixel_idx and n_pixels must be both NULL or both set");
    if (isnan(delta)) return fail(RDSEG_ERR_ARG, "delta must not be NaN");
    SolveWs need = carve_solve(nullptr, s);
    if (!ws || ws_bytes < need.bytes)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need.bytes) + " bytes");
    SolveWs w = carve_solve(ws, s);
    Geo g = geo_of(s);
    hipStream_t st = static_cast<hipStream_t>(stream);
    float* st1[3] = {nullptr, nullptr, nullptr};
    ImgDesc d = make_desc(f, s, 0.0, 1.0, delta, nullptr, nullptr, nullptr, nullptr, st1,
                          nullptr, nullptr, 8, 8);
    OffTables off{nullptr, nullptr, nullptr, nullptr};
    if (launch_tile_masks(&d, nullptr, off, 1, g.strips, w.masks, w.npix, st)) return RDSEG_ERR_HIP;
    if (launch_tile_list(w.masks, g.nt, w.flags, w.offs, w.part, n_tiles, tile_ids, tile_masks,
                         slot_map, st))
        return RDSEG_ERR_HIP;
    if (pixel_idx) {
        if (launch_pixel_list(f, s.H, s.W, (int)s.ld, delta, w.flags, w.offs, w.part,
                              w.totals + 1, pixel_idx, n_pixels, st))
            return RDSEG_ERR_HIP;
    }
    return RDSEG_OK;
}

rdseg_status rdseg_solve(const float* f, rdseg_shape s, const rdseg_params* prm, const float* u0,
                         const float* p0, float* u, float* v, float* p, float* tape, void* ws,
                         size_t ws_bytes, void* stream) {
    return solve_impl(f, s, prm, u0, p0, u, v, p, tape, ws, ws_bytes,
                      static_cast<hipStream_t>(stream), -1);
}

int32_t rdseg_config_count(void) { return config_count(); }

rdseg_status rdseg_config_get(int32_t i, int32_t* tile_w, int32_t* tile_h,
                              int32_t* iters_per_launch, int32_t* threads) {
    if (i < 0 || i >= config_count()) return fail(RDSEG_ERR_ARG, "configuration index out of range");
    TileCfg c = config_at(i);
    if (tile_w) *tile_w = c.bx;
    if (tile_h) *tile_h = c.by;
    if (iters_per_launch) *iters_per_launch = c.it;
    if (threads) *threads = c.nt;
    return RDSEG_OK;
}

rdseg_status rdseg_autotune(const float* f, rdseg_shape s, const rdseg_params* prm,
                            int32_t probe_iters, float* u, float* v, float* p, void* ws,
                            size_t ws_bytes, void* stream, int32_t* tile_w, int32_t* tile_h,
                            int32_t* iters_per_launch) {
    if (!prm) return fail(RDSEG_ERR_ARG, "prm is NULL");
    if (probe_iters < 1) return fail(RDSEG_ERR_ARG, "probe_iters must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    rdseg_params q = *prm;
    q.iters = probe_iters;
    q.ckpt_every = 0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RDSEG_ERR_HIP, "hipEventCreate failed");
    int best = -1;
    float best_ms = 0.0f;
    for (int ci = 0; ci < config_count(); ++ci) {
        // warm-up, then timed
        rdseg_status r = solve_impl(f, s, &q, nullptr, nullptr, u, v, p, nullptr, ws, ws_bytes, st, ci);
        if (r) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return r; }
        (void)hipEventRecord(e0, st);
        for (int rep = 0; rep < 3; ++rep) {
            r = solve_impl(f, s, &q, nullptr, nullptr, u, v, p, nullptr, ws, ws_bytes, st, ci);
            if (r) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return r; }
        }
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) {
            (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
            return fail(RDSEG_ERR_HIP, "autotune timing failed");
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (best < 0 || ms < best_ms) { best = ci; best_ms = ms; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // record under the problem's class and active-fraction bucket
    SolveWs w = carve_solve(ws, s);
    int64_t np = 0;
    if (hipMemcpy(&np, w.npix, sizeof(np), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(RDSEG_ERR_HIP, "reading the active-pixel count failed");
    double qf = (double)np / ((double)s.H * s.W);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[TuneKey{size_class(s), q_bucket(qf)}] = best;
    }
    TileCfg c = config_at(best);
    if (tile_w) *tile_w = c.bx;
    if (tile_h) *tile_h = c.by;
    if (iters_per_launch) *iters_per_launch = c.it;
    return RDSEG_OK;
}

rdseg_status rdseg_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.on = on != 0;
    return RDSEG_OK;
}

rdseg_status rdseg_timing_read(double* kernel_ms, int64_t* launches, double* alg_bytes,
                               int64_t* pixel_updates) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    double ms = 0.0, bytes = 0.0;
    int64_t upd = 0;
    for (auto& r : g_timing.recs) {
        if (hipEventSynchronize(r.e1) != hipSuccess) return fail(RDSEG_ERR_HIP, "event sync failed");
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, r.e0, r.e1);
        ms += t;
        int64_t np = r.npix_host ? *r.npix_host : 0;
        upd += np * r.nit;
        bytes += 28.0 * (double)np * r.nit;
        g_timing.pool.push_back(r.e0);
        g_timing.pool.push_back(r.e1);
    }
    if (kernel_ms) *kernel_ms = ms;
    if (launches) *launches = (int64_t)g_timing.recs.size();
    if (alg_bytes) *alg_bytes = bytes;
    if (pixel_updates) *pixel_updates = upd;
    g_timing.recs.clear();
    g_timing.pinned_used = 0;
    return RDSEG_OK;
}

}  // extern "C"
