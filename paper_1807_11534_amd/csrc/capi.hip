// capi.hip -- host side of the C ABI declared in include/rdseg.h: argument
// validation, workspace layout, launch orchestration, batched plans with
// hipGraph capture, per-launch timing and the autotuner.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <atomic>
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

// ceil(q n) without rounding error: with p = q n rounded and e = fma(q, n, -p)
// its exact residual (q n = p + e), the ceiling moves past p only when p is
// an integer and e > 0; a non-integer p lies within half an ulp of q n, never
// across an integer.
int64_t needed_count(double q, int64_t n) {
    if (!(q > 0.0) || n <= 0) return 0;
    if (q >= 1.0) return n;
    const double dn = (double)n;
    const double p = q * dn;
    const double e = fma(q, dn, -p);
    double c = ceil(p);
    if (c == p && e > 0.0) c += 1.0;
    return (int64_t)c;
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
    int32_t* tstate;
    int32_t* cflags;
    int2* cqueue;
    int32_t* totals;   // [0] n_queue, [1] scratch total, [2] n_closed
    int32_t* epoch;    // resident solve: per macro tile block counts, then a status word
    CompWs comp;       // small-component path
    size_t bytes;
};

SolveWs carve_solve(void* base, const rdseg_shape& s) {
    Geo g = geo_of(s);
    Carver cv(base);
    SolveWs w;
    w.c = cv.take<float>(g.plane);
    for (int k = 0; k < 3; ++k) w.st[k] = cv.take<float>(g.plane);
    w.masks = cv.take<uint64_t>(g.nt);
    w.npix = cv.take<int64_t>(2);   // [0] RD count, [1] status word (int32) of the last solve
    int64_t nflag = std::max<int64_t>(g.nt, g.chunks);
    w.flags = cv.take<int32_t>(nflag);
    w.offs = cv.take<int32_t>(nflag);
    w.part = cv.take<int32_t>(scan_partials(nflag));
    w.queue = cv.take<int2>(g.nt);
    w.tstate = cv.take<int32_t>(g.nt);
    w.cflags = cv.take<int32_t>(g.nt);
    w.cqueue = cv.take<int2>(g.nt);
    w.totals = cv.take<int32_t>(4);
    w.epoch = cv.take<int32_t>(g.nt + 1);
    w.comp.lab = cv.take<int32_t>(g.plane);
    w.comp.csize = cv.take<int32_t>(g.plane);
    w.comp.crank = cv.take<int32_t>(g.plane);
    w.comp.cslot = cv.take<int32_t>(g.plane);
    w.comp.lane_of = cv.take<int32_t>(g.plane);
    w.comp.wl_pix = cv.take<int32_t>(2 * g.plane + kCompLaneExtra);
    w.comp.ccount = cv.take<int32_t>(kCompCount);
    w.comp.npix_tile = cv.take<int64_t>(1);
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
    int nit;              // iterations covered by the bracketed launches
    int launches;         // launches bracketed
    int ci;
    int64_t* npix_host;   // pinned slot filled by an async copy
    bool resident;        // one launch of the resident kernel
};

std::atomic<bool> g_resident_on{true};
std::atomic<bool> g_components_on{true};
// form of the adjoint's reverse sweep: macro tile and steps per launch
std::atomic<int> g_adj_tile{32};
std::atomic<int> g_adj_steps{2};
// batched solves: 1 = every block in one persistent cooperative launch,
// 2 = one launch per block of iterations
std::atomic<int> g_batch_form{2};

struct Timing {
    std::mutex mu;
    bool on = false;
    TimingRec open{};
    bool has_open = false;
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
    int batched = 0;   // 1: a batched solve (cls from the batch's total pixel count)
    bool operator<(const TuneKey& o) const {
        if (batched != o.batched) return batched < o.batched;
        return cls != o.cls ? cls < o.cls : qb < o.qb;
    }
};
// configuration index and small-component choice (1 on, 2 off)
struct TuneVal {
    int ci, comps, resident;   // resident: 1 on-chip exchange allowed, 2 separate launches
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

int size_class_of(int64_t n) {
    int c = 0;
    while (n > 4096 && c < 12) { n >>= 2; ++c; }
    return c;
}

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

// The configuration for a problem class the tuning cache does not hold, from
// what the autotuner picked on measured workloads: deep launches on small
// tiles for thin bands and bands of up to half the image (few launches; the
// small tiles follow the band's shape), and for denser ones the 64x64 /
// 8-iteration form, resident where all its tiles fit on the chip (else 4
// iterations a launch, less halo recomputed).
int heuristic_cfg(const rdseg_shape& s, double q) {
    int64_t n = (int64_t)s.H * s.W;
    if (n <= 128 * 128) return config_index(16, 16, 2);
    if (q >= 0.5) {
        const int deep = config_index(64, 64, 8);
        return resident_fits(deep, macro_count(s, 64, 64)) ? deep : config_index(64, 64, 4);
    }
    if (q >= 0.01) return config_index(16, 16, 8);
    return config_index(8, 8, 32);
}

// ------------------------------------------------------------------ side stream
// Closed tiles are independent of every other RD pixel (no RD 4-neighbour
// outside the tile) and their pixels lie outside the queued macro tiles, so
// their all-iteration kernel can run beside the blocked launches: it is
// latency bound (one wave runs every iteration of its tile), the blocked
// launches are many short kernels, and the two write disjoint pixels.  The
// blocked kernel may read a closed tile's pixels as halo while they are being
// written, but those cells feed no RD pixel outside the tile (no RD
// 4-neighbour there; frozen cells contribute constants), so its results do
// not depend on what it reads.  One non-blocking stream per device, default
// priority, created on first use and kept for the process.
std::mutex g_side_mu;
std::map<int, hipStream_t> g_side;

hipStream_t side_stream() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_side_mu);
    auto it = g_side.find(dev);
    if (it != g_side.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    g_side[dev] = s;
    return s;
}

// Enqueue the closed-tile kernel after the work already on `st`, on the side
// stream when there is one (*join then receives the event that `st` must wait
// for before the solve's results are complete), else, and while `st` is being
// captured into a graph, on `st` itself.
template <class Launch>
rdseg_status closed_beside(hipStream_t st, hipEvent_t* join, Launch launch) {
    *join = nullptr;
    // under graph capture the fork and join make the kernel a parallel branch
    // of the captured graph
    hipStream_t side = side_stream();
    hipEvent_t fork = nullptr;
    if (!side || hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess)
        return launch(st) ? RDSEG_ERR_HIP : RDSEG_OK;
    if (hipEventCreateWithFlags(join, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(fork);
        *join = nullptr;
        return launch(st) ? RDSEG_ERR_HIP : RDSEG_OK;
    }
    rdseg_status r = RDSEG_OK;
    if (hipEventRecord(fork, st) != hipSuccess || hipStreamWaitEvent(side, fork, 0) != hipSuccess)
        r = fail(RDSEG_ERR_HIP, "forking the closed-tile stream failed");
    else if (launch(side))
        r = RDSEG_ERR_HIP;
    else if (hipEventRecord(*join, side) != hipSuccess)
        r = fail(RDSEG_ERR_HIP, "recording the closed-tile join failed");
    (void)hipEventDestroy(fork);
    if (r) {
        (void)hipEventDestroy(*join);
        *join = nullptr;
    }
    return r;
}

// Make `st` wait for the closed-tile kernel (no-op without a join event).
rdseg_status join_closed(hipStream_t st, hipEvent_t join) {
    if (!join) return RDSEG_OK;
    const hipError_t e = hipStreamWaitEvent(st, join, 0);
    (void)hipEventDestroy(join);
    return e == hipSuccess ? RDSEG_OK : fail(RDSEG_ERR_HIP, "joining the closed-tile stream failed");
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
    int inner = 1;                           // dual steps per outer iteration
    const struct StopSpec* stop = nullptr;   // convergence-driven solve (single image)
    int launches = 0;                        // out: number of launches enqueued
    int launches_per_check = 0;              // out (with stop)
    bool resident = false;                   // try the resident form first (single image)
    const int32_t* mflags = nullptr;         // resident: queued flag per macro tile
    int32_t* epoch = nullptr;                // resident: max_items int32 of workspace
    int32_t* status = nullptr;               // resident: the solve's status word
    bool epoch_cleared = false;              // resident: epoch words already zeroed
    const CompWs* comp = nullptr;            // resident: small components for idle workgroups
    const int64_t* comp_npix = nullptr;      // resident: full RD count (the labelling's)
    int64_t res_grid = 0;                    // resident: workgroups (0: max_items)
    bool no_alloc = false;                   // take no timing records (they create events)
};

// Stopping rule of a convergence-driven solve: change slots (one uint32
// float pattern per check, zeroed first), tolerance, check spacing.
struct StopSpec {
    double tol;
    int check_every;
    uint32_t* slots;
    int n_checks;
    int32_t* iters_done;
    bool poll;   // read the changes back chunk by chunk and stop enqueuing
};

// Host side of a polled convergence-driven solve: checks are read back in
// chunks of doubling length through a small pinned ring (two chunks in
// flight); the chunk after the current one is enqueued before the current
// one is waited for, so the device stays busy while the host decides.
constexpr int kPollMax = 1024;
std::mutex g_poll_mu;
float* g_poll_host = nullptr;   // 2 * kPollMax floats, pinned, kept for the process

// Small read-backs that a solve waits for (queue lengths, class counts): a
// one-wave kernel copies the values into pinned, host-coherent memory and then
// stores a sequence number there (system scope, after a system-scope fence),
// which the host spins on.  The wait therefore ends as soon as the values have
// landed, without a copy command or a wake-up of a blocked thread; after 2 ms
// of spinning it blocks on the stream instead (long work ahead on it, or an
// error, which the stream synchronisation then reports).
std::mutex g_rb_mu;
int32_t* g_rb_host = nullptr;   // kReadBack int32, pinned, kept for the process
int32_t g_rb_seq = 0;
constexpr int kReadBack = 64;   // the last word holds the sequence number
constexpr int kReadBackPieces = 4;

struct ReadBackArgs {
    const int32_t* src[kReadBackPieces];
    int n[kReadBackPieces];
    int k;
};

__global__ __launch_bounds__(64) void k_read_back(ReadBackArgs a, int32_t* host, int32_t seq) {
    int off = 0;
    for (int i = 0; i < a.k; ++i) {
        for (int j = threadIdx.x; j < a.n[i]; j += 64) host[off + j] = a.src[i][j];
        off += a.n[i];
    }
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(host + kReadBack - 1, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Copy n[i] int32 from each src[i] to dst[i] (k <= kReadBackPieces pieces,
// sum n < kReadBack) once the work enqueued on st before has written them.
rdseg_status read_back(int k, const int32_t* const* src, const int* n, int32_t* const* dst,
                       hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_rb_mu);
    if (!g_rb_host &&
        hipHostMalloc(reinterpret_cast<void**>(&g_rb_host), kReadBack * sizeof(int32_t),
                      hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable) !=
            hipSuccess) {
        g_rb_host = nullptr;
        return fail(RDSEG_ERR_HIP, "pinned host buffer for read-backs could not be allocated");
    }
    if (g_rb_seq == 0)   // a new buffer: no sequence number written yet
        __atomic_store_n(g_rb_host + kReadBack - 1, 0, __ATOMIC_RELEASE);
    if (k < 1 || k > kReadBackPieces) return fail(RDSEG_ERR_ARG, "read-back: 1 to 4 pieces");
    ReadBackArgs a{};
    a.k = k;
    int total = 0;
    for (int i = 0; i < k; ++i) {
        a.src[i] = src[i];
        a.n[i] = n[i];
        total += n[i];
    }
    if (total >= kReadBack) return fail(RDSEG_ERR_ARG, "read-back too large");
    int32_t* dev = nullptr;
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&dev), g_rb_host, 0) != hipSuccess)
        return fail(RDSEG_ERR_HIP, "mapping the read-back buffer failed");
    const int32_t seq = g_rb_seq = g_rb_seq == INT32_MAX ? 1 : g_rb_seq + 1;
    hipLaunchKernelGGL(k_read_back, dim3(1), dim3(64), 0, st, a, dev, seq);
    if (hipGetLastError() != hipSuccess) return fail(RDSEG_ERR_HIP, "reading back from the device failed");
    const auto t0 = std::chrono::steady_clock::now();
    int spins = 0;
    while (__atomic_load_n(g_rb_host + kReadBack - 1, __ATOMIC_ACQUIRE) != seq) {
        if ((++spins & 255) == 0 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
            if (hipStreamSynchronize(st) != hipSuccess)
                return fail(RDSEG_ERR_HIP, "reading back from the device failed");
            if (__atomic_load_n(g_rb_host + kReadBack - 1, __ATOMIC_ACQUIRE) != seq)
                return fail(RDSEG_ERR_HIP, "the read-back did not arrive");
            break;
        }
    }
    int off = 0;
    for (int i = 0; i < k; ++i) {
        memcpy(dst[i], g_rb_host + off, n[i] * sizeof(int32_t));
        off += n[i];
    }
    return RDSEG_OK;
}

struct Poller {
    const StopSpec& sp;
    hipStream_t st;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int c0[2] = {0, 0}, n[2] = {0, 0};
    bool busy[2] = {false, false};
    int k = 0;               // chunks issued
    int chunk_start = 0;     // first check of the open chunk
    int chunk_len = 2;
    bool stopped = false;
    bool ok = true;

    Poller(const StopSpec& s, hipStream_t stream) : sp(s), st(stream) {
        for (int r = 0; r < 2; ++r)
            if (hipEventCreateWithFlags(&ev[r], hipEventDisableTiming) != hipSuccess) ok = false;
    }
    ~Poller() {
        for (int r = 0; r < 2; ++r) {
            if (busy[r]) (void)hipEventSynchronize(ev[r]);
            if (ev[r]) (void)hipEventDestroy(ev[r]);
        }
    }
    int chunk_end() const { return std::min(chunk_start + chunk_len, sp.n_checks) - 1; }
    // wait for ring slot r and look for a change <= tol among its checks
    void settle(int r) {
        if (!busy[r]) return;
        if (hipEventSynchronize(ev[r]) != hipSuccess) ok = false;
        busy[r] = false;
        const float* h = g_poll_host + r * kPollMax;
        for (int i = 0; i < n[r]; ++i)
            if ((double)h[i] <= sp.tol) stopped = true;
    }
    // called after the launch that ends check c has been enqueued
    void after_check(int c) {
        if (c != chunk_end()) return;
        const int r = k & 1;
        settle(r);   // chunk k - 2, normally settled already
        c0[r] = chunk_start;
        n[r] = c - chunk_start + 1;
        if (hipMemcpyAsync(g_poll_host + r * kPollMax, sp.slots + c0[r], n[r] * sizeof(float),
                           hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipEventRecord(ev[r], st) != hipSuccess)
            ok = false;
        busy[r] = true;
        ++k;
        chunk_start = c + 1;
        chunk_len = std::min(chunk_len * 2, kPollMax);
        settle(r ^ 1);   // the previous chunk, while this one runs
    }
};

// Enqueue the launches of `iters` iterations; the final state lands in
// buffer 0 (the caller's v, p) and u is written by the last launch.
rdseg_status enqueue_iterations(SolvePlanArgs& a) {
    if (a.iters <= 0) return RDSEG_OK;
    const int IT = std::max(1, config_at(a.ci).it / a.inner);   // outer iterations per launch
    const bool stop = a.stop != nullptr;
    const int ce = stop ? a.stop->check_every
                        : ((a.tape && a.ckpt_every > 0) ? a.ckpt_every : a.iters);
    // launch schedule: segments of ce iterations (checkpoint spacing, or the
    // spacing of the stopping rule's checks), each split into <= IT chunks
    std::vector<int> nits;
    std::vector<int> seg_start;   // launch index that starts each segment
    std::vector<int> seg_of;      // segment of each launch
    for (int k0 = 0; k0 < a.iters; k0 += ce) {
        int len = std::min(ce, a.iters - k0);
        seg_start.push_back((int)nits.size());
        for (int j = 0; j < len; j += IT) {
            nits.push_back(std::min(IT, len - j));
            seg_of.push_back((int)seg_start.size() - 1);
        }
    }
    const int L = (int)nits.size();
    a.launches = L;
    a.launches_per_check = (ce + IT - 1) / IT;
    const bool timing_on = g_timing.on && !a.no_alloc;
    if (a.resident && !a.descs && !a.tape && !stop) {
        TimingRec rec{};
        const bool timed = timing_on;
        if (timed) {
            rec.e0 = timing_event();
            rec.e1 = timing_event();
        }
        const int rc = launch_resident(a.ci, *a.d0, a.queue, a.n_queue, a.mflags, a.epoch,
                                       a.status, a.max_items, L % 2, a.iters, IT,
                                       a.inner, a.theta, a.inv_theta, a.tau, a.st,
                                       timed ? rec.e0 : nullptr, a.comp, a.comp_npix,
                                       a.res_grid, a.epoch_cleared);
        if (rc > 0) return RDSEG_ERR_HIP;
        if (rc == 0) {
            a.launches = 1;
            if (timed && rec.e0 && rec.e1) {
                std::lock_guard<std::mutex> lk(g_timing.mu);
                (void)hipEventRecord(rec.e1, a.st);
                rec.nit = a.iters;
                rec.launches = 1;
                rec.ci = a.ci;
                rec.resident = true;
                rec.npix_host = timing_slot();
                if (rec.npix_host && a.npix)
                    (void)hipMemcpyAsync(rec.npix_host, a.npix, sizeof(int64_t),
                                         hipMemcpyDeviceToHost, a.st);
                g_timing.recs.push_back(rec);
            }
            return RDSEG_OK;
        }
        // rc < 0: not applicable, fall through to separate launches
        if (timed) {
            std::lock_guard<std::mutex> lk(g_timing.mu);
            if (rec.e0) g_timing.pool.push_back(rec.e0);
            if (rec.e1) g_timing.pool.push_back(rec.e1);
        }
    }
    size_t seg = 0;
    const int64_t plane = (int64_t)a.d0->H * a.d0->ld;
    std::unique_lock<std::mutex> poll_lock;
    Poller* poller = nullptr;
    if (stop && a.stop->poll && a.stop->n_checks > 0) {
        poll_lock = std::unique_lock<std::mutex>(g_poll_mu);
        if (!g_poll_host &&
            hipHostMalloc(reinterpret_cast<void**>(&g_poll_host), 2 * kPollMax * sizeof(float), 0) !=
                hipSuccess) {
            g_poll_host = nullptr;
            return fail(RDSEG_ERR_HIP, "pinned host buffer for polling could not be allocated");
        }
        poller = new Poller(*a.stop, a.st);
        if (!poller->ok) {
            delete poller;
            return fail(RDSEG_ERR_HIP, "event creation for polling failed");
        }
    }
    struct PollGuard {
        Poller*& p;
        ~PollGuard() { delete p; }
    } poll_guard{poller};
    for (int j = 0; j < L; ++j) {
        int in_buf = (L - j) % 2;
        if (a.tape && seg < seg_start.size() && seg_start[seg] == j) {
            int rc = launch_state_copy(*a.d0, in_buf, a.tape + (int64_t)seg * 3 * plane, a.st);
            if (rc) return RDSEG_ERR_HIP;
            ++seg;
        }
        // Timing brackets each run of back-to-back iteration launches (the whole
        // solve, or one checkpoint segment) with one event pair.
        const bool run_start = (j == 0) || (a.tape && seg_start.size() > seg - 1 && seg >= 1 &&
                                            seg_start[seg - 1] == j);
        const bool run_end = (j == L - 1) || (a.tape && seg < seg_start.size() && seg_start[seg] == j + 1);
        if (timing_on && run_start) {
            std::lock_guard<std::mutex> lk(g_timing.mu);
            TimingRec rec{};
            rec.e0 = timing_event();
            rec.e1 = timing_event();
            rec.nit = 0;
            rec.launches = 0;
            rec.ci = a.ci;
            rec.npix_host = nullptr;
            if (rec.e0 && rec.e1) {
                (void)hipEventRecord(rec.e0, a.st);
                g_timing.open = rec;
                g_timing.has_open = true;
            }
        }
        StopLaunch sl{};
        if (stop) {
            const int sg = seg_of[j];
            const bool seg_end = (j == L - 1) || seg_of[j + 1] != sg;
            sl.skip_slot = sg > 0 ? a.stop->slots + (sg - 1) : nullptr;
            sl.diff_slot = (seg_end && sg < a.stop->n_checks) ? a.stop->slots + sg : nullptr;
            sl.tol = a.stop->tol;
        }
        int rc = launch_iterate(a.ci, a.d0, a.descs, a.descs != nullptr, a.queue, a.n_queue,
                                a.max_items, in_buf, nits[j], stop || j == L - 1, a.theta,
                                a.inv_theta, a.tau, a.st, stop ? &sl : nullptr, a.inner);
        if (rc) return RDSEG_ERR_HIP;
        bool stop_now = false;
        if (poller && sl.diff_slot) {
            poller->after_check(seg_of[j]);
            if (!poller->ok) return fail(RDSEG_ERR_HIP, "reading back the changes failed");
            stop_now = poller->stopped;
        }
        if (timing_on) {
            std::lock_guard<std::mutex> lk(g_timing.mu);
            if (g_timing.has_open) {
                g_timing.open.nit += nits[j];
                g_timing.open.launches += 1;
                if (run_end || stop_now) {
                    TimingRec rec = g_timing.open;
                    g_timing.has_open = false;
                    (void)hipEventRecord(rec.e1, a.st);
                    rec.npix_host = timing_slot();
                    if (rec.npix_host && a.npix)
                        (void)hipMemcpyAsync(rec.npix_host, a.npix, sizeof(int64_t),
                                             hipMemcpyDeviceToHost, a.st);
                    g_timing.recs.push_back(rec);
                }
            }
        }
        if (stop_now) break;   // later launches would only skip; finalize reads the slots
    }
    return RDSEG_OK;
}

constexpr int kMaxInner = 16;   // deepest compiled halo

// The configuration with the tile of `ci` (or the nearest larger one) whose
// halo holds at least `inner` dual steps.
int deeper_cfg(int ci, int inner) {
    const TileCfg c = config_at(ci);
    int best = -1;
    for (int k = 0; k < config_count(); ++k) {
        const TileCfg e = config_at(k);
        if (e.it < inner) continue;
        const bool same = e.bx == c.bx && e.by == c.by;
        if (best < 0) { best = k; continue; }
        const TileCfg b = config_at(best);
        const bool best_same = b.bx == c.bx && b.by == c.by;
        if (same && !best_same) best = k;
        else if (same == best_same && e.it < b.it) best = k;
    }
    return best;
}

// Choose the tile configuration for a single-image solve.
rdseg_status choose_cfg(const rdseg_params& prm, const rdseg_shape& s, const int64_t* npix_dev,
                        hipStream_t st, int* ci, int* comps = nullptr,
                        int* resident = nullptr) {
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
            *ci = it->second.ci;
            if (comps) *comps = it->second.comps;
            if (resident) *resident = it->second.resident;
            return RDSEG_OK;
        }
    }
    *ci = heuristic_cfg(s, q);
    return RDSEG_OK;
}

rdseg_status solve_impl(const float* f, rdseg_shape s, const rdseg_params* prm, const float* u0,
                        const float* p0, float* u, float* v, float* p, float* tape, void* ws,
                        size_t ws_bytes, hipStream_t st, int forced_ci,
                        const StopSpec* stop = nullptr, bool no_alloc = false) {
    if (!prm) return fail(RDSEG_ERR_ARG, "prm is NULL");
    rdseg_status r = check_shape(s);
    if (r) return r;
    r = check_scalars(prm->lambda, prm->theta, prm->tau, prm->delta);
    if (r) return r;
    if (!f || !u || !v || !p) return fail(RDSEG_ERR_ARG, "f, u, v and p must be non-NULL");
    if (prm->iters < 0) return fail(RDSEG_ERR_ARG, "iters must be >= 0");
    if (prm->ckpt_every < 0) return fail(RDSEG_ERR_ARG, "ckpt_every must be >= 0");
    if (prm->ckpt_every > 0 && !tape) return fail(RDSEG_ERR_TAPE, "ckpt_every > 0 needs a tape");
    if (prm->inner < 0 || prm->inner > kMaxInner)
        return fail(RDSEG_ERR_ARG, "inner must lie in [0, 16]");
    if (prm->components < 0 || prm->components > 2)
        return fail(RDSEG_ERR_ARG, "components must be 0 (library's choice), 1 (on) or 2 (off)");
    if (prm->resident < 0 || prm->resident > 2)
        return fail(RDSEG_ERR_ARG, "resident must be 0 (library's choice), 1 (on-chip exchange) or 2 (separate launches)");
    const int inner = prm->inner > 1 ? prm->inner : 1;
    if (inner > 1 && prm->ckpt_every > 0)
        return fail(RDSEG_ERR_ARG, "checkpoints (for the adjoint) need inner = 1");
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
    if (ci >= 0 && config_at(ci).it < inner)
        return fail(RDSEG_ERR_ARG, "iters_per_launch (dual steps per launch) must be >= inner");
    SolveWs w = carve_solve(ws, s);
    Geo g = geo_of(s);

    // tile-configuration independent part of the descriptor first
    ImgDesc d = make_desc(f, s, prm->lambda, prm->theta, prm->delta, u, v, p, w.c, w.st, u0, p0, 8, 8);
    OffTables off{nullptr, nullptr, nullptr, nullptr};
    // initial state and tile masks in one pass; the RD count and the solve's
    // status word start at 0
    if (launch_prepare(&d, nullptr, off, 1, g.strips, w.masks, w.npix, st, 2))
        return RDSEG_ERR_HIP;
    int tuned_comps = 0, tuned_res = 0;
    if (ci < 0) {
        r = choose_cfg(*prm, s, w.npix, st, &ci, &tuned_comps, &tuned_res);
        if (r) return r;
        if (config_at(ci).it < inner) ci = deeper_cfg(ci, inner);
    }
    TileCfg cfg = config_at(ci);
    d = make_desc(f, s, prm->lambda, prm->theta, prm->delta, u, v, p, w.c, w.st, u0, p0, cfg.bx, cfg.by);
    int64_t nm = macro_count(s, cfg.bx, cfg.by);
    // Closed tiles run every iteration in one launch; a solve that writes a
    // checkpoint tape sends every tile through the blocked kernel instead.
    // The stopping rule needs every RD pixel's change at each check, so it
    // also keeps closed tiles in the blocked kernel.
    // Small RD components (<= 256 pixels) run whole in the component kernel
    // (which covers every closed tile as well: a closed tile's components are
    // inside it); not under the stopping rule, and index arithmetic in int32.
    // With a tape the component kernel writes its pixels' checkpoints (the
    // tile path's checkpoint copies take only the RD pixels left to it).
    const bool taped = prm->ckpt_every > 0 && tape;
    const int want_comps = prm->components ? prm->components : (tuned_comps ? tuned_comps : 1);
    const bool comps = want_comps == 1 && g_components_on.load() && prm->iters > 0 && !stop &&
                       g.plane <= ((int64_t)1 << 29);
    const bool use_closed = !taped && prm->iters > 0 && !stop && !comps;
    if (stop && stop->n_checks > 0 &&
        launch_fill(reinterpret_cast<float*>(stop->slots), 1, stop->n_checks, stop->n_checks,
                    0.0f, st))
        return RDSEG_ERR_HIP;
    if (comps && launch_components_prepare(d, w.comp, w.masks, w.npix, st)) return RDSEG_ERR_HIP;
    // The resident form keeps every queued macro tile on chip for the whole
    // solve; it needs all of them resident at once, so closed tiles then run
    // before it on the same stream instead of beside it.  When it may run,
    // the queue pass also zeroes its epoch words.
    bool resident = false;
    int64_t res_grid = 0;          // 0: one workgroup per macro tile of the image
    bool res_idle_comps = true;    // idle workgroups of the resident grid run the components
    const int want_res = prm->resident ? prm->resident : (tuned_res ? tuned_res : 1);
    // (the allocation-free form has no status word for the caller to read, so
    // it keeps to separate launches, whose waits cannot expire)
    bool eager = false;
    if (want_res == 1 && g_resident_on.load() && !stop && !taped && !no_alloc && prm->iters > 0 &&
        resident_available(ci)) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        eager = hipStreamIsCapturing(st, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone;
    }
    const bool epoch_cleared = eager;   // the resident form's epoch words zeroed ahead
    QueueScratch qs{w.cflags, w.tstate, w.flags, w.offs, w.part};
    if (epoch_cleared) qs.epoch = w.epoch;
    if (launch_macro_queue(&d, nullptr, off, 1, nm, cfg.bx, cfg.by, w.masks, qs, w.queue, w.totals,
                           g.nt, use_closed ? w.cqueue : nullptr, w.totals + 2, st))
        return RDSEG_ERR_HIP;
    if (eager) {
        if (resident_fits(ci, nm)) {
            resident = true;
        } else {
            // Finer tiles than fit on the chip all at once: the queue (the
            // band's tiles) may.  Read its length (synchronises).  The grid
            // is the co-resident capacity (the queued tiles, then idle
            // workgroups for the small components) when that leaves at least
            // half as many idle workgroups as tiles; otherwise just the
            // tiles, and the component kernel follows on the whole chip (a few
            // idle workgroups would hold every component chain).
            int32_t nq = 0;
            {
                const int32_t* src[1] = {w.totals};
                const int cnt[1] = {1};
                int32_t* dst[1] = {&nq};
                r = read_back(1, src, cnt, dst, st);
                if (r) return r;
            }
            const int64_t tiles = ((int64_t)nq + 7) / 8 * 8;
            const int64_t cap = resident_capacity(ci) / 8 * 8;
            if (nq > 0 && tiles <= cap) {
                resident = true;
                res_idle_comps = 2 * (cap - tiles) >= tiles;
                res_grid = res_idle_comps ? cap : tiles;
            }
        }
    }
    hipEvent_t join = nullptr;
    auto small = [&](hipStream_t cs) {
        return launch_components(d, w.comp, w.npix, prm->iters, inner, (float)prm->theta,
                                 (float)(1.0 / prm->theta), (float)prm->tau,
                                 taped ? tape : nullptr, taped ? prm->ckpt_every : 0, cs);
    };
    if (comps) {
        // resident: the idle workgroups of the resident kernel take the
        // components, and the component kernel follows it (below); without
        // allocation (no side stream, no events) it runs before the tiles
        if (!resident) {
            if (no_alloc) {
                if (small(st)) return RDSEG_ERR_HIP;
            } else {
                r = closed_beside(st, &join, small);
                if (r) return r;
            }
        }
    } else if (use_closed) {
        auto closed = [&](hipStream_t cs) {
            return launch_closed(&d, nullptr, false, w.cqueue, w.totals + 2, g.nt, prm->iters,
                                 (float)prm->theta, (float)(1.0 / prm->theta), (float)prm->tau,
                                 cs, inner);
        };
        if (resident || no_alloc) {
            if (closed(st)) return RDSEG_ERR_HIP;
        } else {
            r = closed_beside(st, &join, closed);
            if (r) return r;
        }
    }
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
    a.stop = stop;
    a.inner = inner;
    a.resident = resident;
    a.res_grid = res_grid;
    a.epoch_cleared = epoch_cleared;
    a.mflags = w.flags;
    a.epoch = w.epoch;
    a.status = reinterpret_cast<int32_t*>(w.npix + 1);
    a.no_alloc = no_alloc;
    if (comps) a.npix = w.comp.npix_tile;   // timing counts the tile path's pixels
    if (comps && resident && res_idle_comps) {
        a.comp = &w.comp;
        a.comp_npix = w.npix;
    }
    // A solve whose RD pixels all went to the component path leaves the tile
    // path nothing but launches on an empty queue (and, with a tape,
    // checkpoint copies of no pixel): read the queue length once
    // (synchronises the stream, the component kernel running on beside it;
    // not under graph capture, nor without allocation, nor for a resident
    // launch, which ends at once on an empty queue) and skip them.
    bool tiles_left = true;
    if (comps && (taped || (!resident && !no_alloc))) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone) {
            int32_t nq = 1;
            const int32_t* src[1] = {w.totals};
            const int cnt[1] = {1};
            int32_t* dst[1] = {&nq};
            r = read_back(1, src, cnt, dst, st);
            tiles_left = nq > 0;
        }
    }
    if (!r && tiles_left) r = enqueue_iterations(a);
    // after a resident launch: returns at once when its idle workgroups ran
    // the components, else runs them (serially, after the tiles)
    if (!r && comps && resident && small(st)) r = RDSEG_ERR_HIP;
    const rdseg_status rj = join_closed(st, join);
    if (r) return r;
    if (rj) return rj;
    if (!stop) return RDSEG_OK;
    return hip_status(launch_stop_finalize(d, stop->slots, stop->n_checks, stop->tol,
                                           stop->check_every, a.launches_per_check, a.launches,
                                           prm->iters, stop->iters_done, st));
}

// ------------------------------------------------------------------ batched
struct BatchLayout {
    std::vector<ImgDesc> descs;
    std::vector<int64_t> tabs;   // soff | toff | moff | roff, each n + 1
    int64_t strips = 0, tiles = 0, macros = 0, rows = 0;
    size_t bytes = 0;
    // device pointers (after carving)
    ImgDesc* d_descs = nullptr;
    int64_t* d_tabs = nullptr;
    uint64_t* masks = nullptr;
    int64_t* npix = nullptr;
    int64_t* npix_total = nullptr;
    int32_t* flags = nullptr;
    int32_t* offs = nullptr;
    int32_t* part = nullptr;
    int2* queue = nullptr;
    int32_t* tstate = nullptr;
    int32_t* cflags = nullptr;
    int2* cqueue = nullptr;
    int32_t* totals = nullptr;
};

rdseg_status validate_batch(const rdseg_image* imgs, int32_t n, double theta, double tau,
                            int32_t iters) {
    if (!imgs || n < 1) return fail(RDSEG_ERR_ARG, "imgs must hold n >= 1 images");
    if (iters < 0) return fail(RDSEG_ERR_ARG, "iters must be >= 0");
    for (int i = 0; i < n; ++i) {
        const rdseg_image& im = imgs[i];
        rdseg_status r = check_shape(im.s);
        if (r) return fail(r, "image " + std::to_string(i) + ": " + get_error());
        r = check_scalars(im.lambda, theta, tau, im.delta);
        if (r) return fail(r, "image " + std::to_string(i) + ": " + get_error());
        if (!im.f || !im.u || !im.v || !im.p)
            return fail(RDSEG_ERR_ARG, "image " + std::to_string(i) + ": f, u, v, p must be non-NULL");
        const size_t pb = (size_t)im.s.H * im.s.ld * sizeof(float);
        if (ranges_overlap(im.u, pb, im.f, pb) || ranges_overlap(im.v, pb, im.f, pb) ||
            ranges_overlap(im.p, 2 * pb, im.f, pb) || ranges_overlap(im.u, pb, im.v, pb) ||
            ranges_overlap(im.u, pb, im.p, 2 * pb) || ranges_overlap(im.v, pb, im.p, 2 * pb))
            return fail(RDSEG_ERR_ARG, "image " + std::to_string(i) + ": u, v, p must not overlap f or each other");
    }
    return RDSEG_OK;
}

int64_t batch_pixels(const rdseg_image* imgs, int32_t n) {
    int64_t px = 0;
    for (int i = 0; i < n; ++i) px += (int64_t)imgs[i].s.H * imgs[i].s.W;
    return px;
}

// Host-side layout of a batch; with base != NULL also fills device pointers.
BatchLayout layout_batch(const rdseg_image* imgs, int32_t n, int bx, int by, double theta,
                         void* base) {
    BatchLayout L;
    L.descs.resize(n);
    L.tabs.assign(4 * (size_t)(n + 1), 0);
    int64_t* soff = L.tabs.data();
    int64_t* toff = soff + (n + 1);
    int64_t* moff = toff + (n + 1);
    int64_t* roff = moff + (n + 1);
    Carver cv(base);
    L.d_descs = cv.take<ImgDesc>(n);
    L.d_tabs = cv.take<int64_t>(4 * (size_t)(n + 1));
    for (int i = 0; i < n; ++i) {
        const rdseg_image& im = imgs[i];
        Geo g = geo_of(im.s);
        soff[i + 1] = soff[i] + g.strips;
        toff[i + 1] = toff[i] + g.nt;
        moff[i + 1] = moff[i] + macro_count(im.s, bx, by);
        roff[i + 1] = roff[i] + im.s.H;
        float* c = cv.take<float>(g.plane);
        float* st1[3];
        for (int k = 0; k < 3; ++k) st1[k] = cv.take<float>(g.plane);
        ImgDesc d = make_desc(im.f, im.s, im.lambda, theta, im.delta, im.u, im.v, im.p, c, st1,
                              nullptr, nullptr, bx, by);
        d.toff = toff[i];
        d.soff = soff[i];
        d.moff = moff[i];
        d.roff = roff[i];
        L.descs[i] = d;
    }
    L.strips = soff[n];
    L.tiles = toff[n];
    L.macros = moff[n];
    L.rows = roff[n];
    L.masks = cv.take<uint64_t>(L.tiles);
    L.npix = cv.take<int64_t>(n);
    L.npix_total = cv.take<int64_t>(1);
    const int64_t nmax = std::max(L.macros, L.tiles);
    L.flags = cv.take<int32_t>(L.macros);
    L.offs = cv.take<int32_t>(nmax);
    L.part = cv.take<int32_t>(scan_partials(nmax));
    L.tstate = cv.take<int32_t>(L.tiles);
    L.cflags = cv.take<int32_t>(L.tiles);
    L.cqueue = cv.take<int2>(L.tiles);
    L.queue = cv.take<int2>(L.macros);
    L.totals = cv.take<int32_t>(8);   // [0] n_queue, [2] n_closed, [3] status, [4] barrier
    L.bytes = cv.off;
    return L;
}

OffTables tables_of(const BatchLayout& L, int n) {
    OffTables t;
    t.soff = L.d_tabs;
    t.toff = L.d_tabs + (n + 1);
    t.moff = L.d_tabs + 2 * (n + 1);
    t.roff = L.d_tabs + 3 * (n + 1);
    return t;
}

// Enqueue the whole batched solve (descriptors already resident).  persist:
// every block of iterations in one cooperative launch of the persistent
// kernel (grid-wide barriers), else one launch per block.
rdseg_status enqueue_batch(const BatchLayout& L, int n, int ci, int iters, double theta,
                           double tau, hipStream_t st, bool persist) {
    TileCfg cfg = config_at(ci);
    OffTables off = tables_of(L, n);
    const ImgDesc* d0 = &L.descs[0];   // unused by the batched kernels
    if (launch_prepare(d0, L.d_descs, off, n, L.strips, L.masks, L.npix, st)) return RDSEG_ERR_HIP;
    if (launch_sum_i64(L.npix, n, L.npix_total, st)) return RDSEG_ERR_HIP;
    QueueScratch qs{L.cflags, L.tstate, L.flags, L.offs, L.part};
    const bool use_closed = iters > 0;
    if (launch_macro_queue(d0, L.d_descs, off, n, L.macros, cfg.bx, cfg.by, L.masks, qs, L.queue,
                           L.totals, L.tiles, use_closed ? L.cqueue : nullptr, L.totals + 2, st))
        return RDSEG_ERR_HIP;
    hipEvent_t join = nullptr;
    if (use_closed) {
        rdseg_status r = closed_beside(st, &join, [&](hipStream_t cs) {
            return launch_closed(d0, L.d_descs, true, L.cqueue, L.totals + 2, L.tiles, iters,
                                 (float)theta, (float)(1.0 / theta), (float)tau, cs);
        });
        if (r) return r;
    }
    SolvePlanArgs a;
    a.d0 = d0;
    a.descs = L.d_descs;
    a.queue = L.queue;
    a.n_queue = L.totals;
    a.max_items = L.macros;
    a.ci = ci;
    a.iters = iters;
    a.theta = (float)theta;
    a.inv_theta = (float)(1.0 / theta);
    a.tau = (float)tau;
    a.ckpt_every = 0;
    a.tape = nullptr;
    a.npix = L.npix_total;
    a.st = st;
    rdseg_status r = RDSEG_OK;
    int rc = -1;
    if (persist && iters > 0) {
        // the solve's status word starts at 0
        if (launch_fill(reinterpret_cast<float*>(L.totals + 3), 1, 1, 1, 0.0f, st)) return RDSEG_ERR_HIP;
        const int IT = config_at(ci).it;
        rc = launch_iterate_persist(ci, d0, L.d_descs, L.queue, L.totals, iters, IT, a.theta,
                                    a.inv_theta, a.tau, L.totals + 4, L.totals + 3, st);
        if (rc > 0) r = RDSEG_ERR_HIP;
    }
    if (!r && rc < 0) r = enqueue_iterations(a);   // separate launches
    const rdseg_status rj = join_closed(st, join);
    return r ? r : rj;
}

// Upload a batch layout's descriptors and offset tables (synchronous).
rdseg_status upload_layout(const BatchLayout& L, int32_t n, hipStream_t st) {
    if (hipMemcpyAsync(L.d_descs, L.descs.data(), n * sizeof(ImgDesc), hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(L.d_tabs, L.tabs.data(), L.tabs.size() * sizeof(int64_t),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(RDSEG_ERR_HIP, "uploading batch descriptors failed");
    return RDSEG_OK;
}

// The batch's active fraction (RD pixels over all pixels): one pass of the
// initial-state kernel in `mem` (at least the 8x8 layout's bytes), read back.
rdseg_status batch_active_fraction(const rdseg_image* imgs, int32_t n, double theta, void* mem,
                                   hipStream_t st, double* q) {
    BatchLayout L = layout_batch(imgs, n, 8, 8, theta, mem);
    rdseg_status r = upload_layout(L, n, st);
    if (r) return r;
    const ImgDesc* d0 = &L.descs[0];
    if (launch_prepare(d0, L.d_descs, tables_of(L, n), n, L.strips, L.masks, L.npix, st) ||
        launch_sum_i64(L.npix, n, L.npix_total, st))
        return RDSEG_ERR_HIP;
    int64_t np = 0;
    if (hipMemcpyAsync(&np, L.npix_total, sizeof(np), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(RDSEG_ERR_HIP, "reading the batch's active-pixel count failed");
    *q = (double)np / (double)batch_pixels(imgs, n);
    return RDSEG_OK;
}

// Configuration and form of a batched solve.  Explicit tile / launch depth:
// that configuration, in the process-wide form (rdseg_set_batched_form).
// All 0: the tuning cache's entry for the batch's class (size class of its
// total pixel count, bucket of its active fraction), else 16x16 / 8 below
// half active and 64x64 / 8 above, in the process-wide form.
rdseg_status choose_batch(const rdseg_image* imgs, int32_t n, double theta, int32_t tile_w,
                          int32_t tile_h, int32_t ipl, void* mem, size_t mem_bytes,
                          hipStream_t st, int* ci, bool* persist) {
    *persist = g_batch_form.load() == 1;
    if (tile_w || tile_h || ipl) {
        *ci = config_index(tile_w, tile_h, ipl);
        if (*ci < 0)
            return fail(RDSEG_ERR_ARG, "tile_w / tile_h / iters_per_launch is not a compiled configuration");
        return RDSEG_OK;
    }
    if (!mem || mem_bytes < layout_batch(imgs, n, 8, 8, theta, nullptr).bytes)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small for the library's choice of configuration");
    double q = 0.0;
    rdseg_status r = batch_active_fraction(imgs, n, theta, mem, st, &q);
    if (r) return r;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(TuneKey{size_class_of(batch_pixels(imgs, n)), q_bucket(q), 1});
        if (it != g_tune.end()) {
            *ci = it->second.ci;
            *persist = it->second.resident == 1;
            return RDSEG_OK;
        }
    }
    *ci = q >= 0.5 ? config_index(64, 64, 8) : config_index(16, 16, 8);
    return RDSEG_OK;
}

// ------------------------------------------------------------------ backward
constexpr int kAdjTile = 32;        // macro tile of the reverse sweep
constexpr int kRecomputeTile = 16;  // macro tile of the segment recompute (8 steps a launch)

struct BackWs {
    float* c;
    float* seg;        // (ce - 1) slots of [3][H][ld]
    float* ab[6];      // pbx0, pby0, vb0, pbx1, pby1, vb1
    float* sacc;
    uint64_t* masks;
    int64_t* npix;
    int32_t* flags;
    int32_t* offs;
    int32_t* part;
    int2* queue;
    int32_t* tstate;
    int32_t* totals;
    int2* rqueue;      // the recompute's queue (its own macro tile)
    int32_t* rtotals;
    double* red;       // reduction partials
    double* out4;
    CompWs comp;       // small-component path
    size_t bytes;
};

BackWs carve_back(void* base, const rdseg_shape& s, int ce) {
    Geo g = geo_of(s);
    Carver cv(base);
    BackWs w;
    w.c = cv.take<float>(g.plane);
    w.seg = cv.take<float>((size_t)std::max(ce - 1, 0) * 3 * g.plane);
    for (int k = 0; k < 6; ++k) w.ab[k] = cv.take<float>(g.plane);
    w.sacc = cv.take<float>(g.plane);
    w.masks = cv.take<uint64_t>(g.nt);
    w.npix = cv.take<int64_t>(1);
    w.flags = cv.take<int32_t>(g.nt);
    w.offs = cv.take<int32_t>(g.nt);
    w.part = cv.take<int32_t>(scan_partials(g.nt));
    w.queue = cv.take<int2>(g.nt);
    w.tstate = cv.take<int32_t>(g.nt);
    w.totals = cv.take<int32_t>(4);
    w.rqueue = cv.take<int2>(g.nt);
    w.rtotals = cv.take<int32_t>(4);
    w.red = cv.take<double>(reduce_partials(s.H));
    w.out4 = cv.take<double>(4);
    w.comp.lab = cv.take<int32_t>(g.plane);
    w.comp.csize = cv.take<int32_t>(g.plane);
    w.comp.crank = cv.take<int32_t>(g.plane);
    w.comp.cslot = cv.take<int32_t>(g.plane);
    w.comp.lane_of = cv.take<int32_t>(g.plane);
    w.comp.wl_pix = cv.take<int32_t>(2 * g.plane + kCompLaneExtra);
    w.comp.ccount = cv.take<int32_t>(kCompCount);
    w.comp.npix_tile = cv.take<int64_t>(1);
    w.bytes = cv.off;
    return w;
}

size_t reduce_ws_bytes(const rdseg_shape& s) {
    Carver cv(nullptr);
    cv.take<double>(reduce_partials(s.H));
    cv.take<double>(4);
    return cv.off;
}

struct BatchPlan {
    std::vector<rdseg_image> imgs;
    double theta, tau;
    int32_t iters, ci;
    bool persist = false;
    bool library_choice = false;   // built with tile / launch depth left to the library
    void* mem = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

bool same_batch(const BatchPlan& P, const rdseg_image* imgs, int32_t n, double theta, double tau,
                int32_t iters, int ci) {
    if ((int32_t)P.imgs.size() != n || P.theta != theta || P.tau != tau || P.iters != iters ||
        P.ci != ci)
        return false;
    for (int i = 0; i < n; ++i) {
        const rdseg_image& a = P.imgs[i];
        const rdseg_image& b = imgs[i];
        if (a.f != b.f || a.u != b.u || a.v != b.v || a.p != b.p || a.s.H != b.s.H ||
            a.s.W != b.s.W || a.s.ld != b.s.ld || a.lambda != b.lambda ||
            memcmp(&a.delta, &b.delta, sizeof(double)) != 0)
            return false;
    }
    return true;
}

void plan_free(BatchPlan* P) {
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->mem) (void)hipFree(P->mem);
    delete P;
}

// ------------------------------------------------------------------ primal-dual
struct PdWs {
    SolveWs base;      // c, masks, scan scratch, queue (its state planes unused)
    float* ubar0;      // ubar of buffer 0 (the caller has no plane for it)
    float* st1[4];     // buffer 1: u, ubar, p_x, p_y
    size_t bytes;
};

PdWs carve_pd(void* base, const rdseg_shape& s) {
    PdWs w;
    w.base = carve_solve(base, s);
    Carver cv(base);
    cv.off = w.base.bytes;
    const int64_t plane = (int64_t)s.H * s.ld;
    w.ubar0 = cv.take<float>(plane);
    w.st1[0] = w.base.st[0];
    w.st1[1] = cv.take<float>(plane);
    w.st1[2] = w.base.st[1];
    w.st1[3] = w.base.st[2];
    w.bytes = cv.off;
    return w;
}

// ------------------------------------------------------------------ volumes
bool shape3_ok(const rdseg_shape3& s) {
    if (s.D < 1 || s.H < 1 || s.W < 1 || s.ld < s.W || s.lds < (int64_t)s.H * s.ld) return false;
    if ((int64_t)s.D * s.lds >= (int64_t)1 << 31) return false;
    return true;
}

struct VolWs {
    float* c;
    float* st[4];
    int32_t* flags;
    int64_t n_tiles;
    size_t bytes;
};

VolWs carve_vol(void* base, const rdseg_shape3& s) {
    int bx, by, bz;
    volume_tile(&bx, &by, &bz);
    const int64_t vol = (int64_t)s.D * s.lds;
    Carver cv(base);
    VolWs w;
    w.c = cv.take<float>(vol);
    for (int k = 0; k < 4; ++k) w.st[k] = cv.take<float>(vol);
    w.n_tiles = (int64_t)((s.W + bx - 1) / bx) * ((s.H + by - 1) / by) * ((s.D + bz - 1) / bz);
    w.flags = cv.take<int32_t>(w.n_tiles);
    w.bytes = cv.off;
    return w;
}

}  // namespace

// ------------------------------------------------------------------ tuning cache as text
namespace {

// Parser of the cache text: {"version": 1, "entries": [{"key": int, ...}, ...]}
// (whitespace anywhere between tokens; keys in any order; no other values).
struct CacheParser {
    const char* p;
    void ws() {
        while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r') ++p;
    }
    bool lit(char c) {
        ws();
        if (*p != c) return false;
        ++p;
        return true;
    }
    bool str(std::string& out) {
        ws();
        if (*p != '"') return false;
        ++p;
        out.clear();
        while (*p && *p != '"') {
            if (*p == '\\' || out.size() > 32) return false;
            out += *p++;
        }
        if (*p != '"') return false;
        ++p;
        return true;
    }
    bool integer(long& v) {
        ws();
        const char* q = p;
        if (*q == '-') ++q;
        if (*q < '0' || *q > '9') return false;
        char* end = nullptr;
        v = strtol(p, &end, 10);
        if (end == p || end - p > 10) return false;
        p = end;
        return true;
    }
};

bool parse_cache_text(const char* text, std::vector<std::pair<TuneKey, TuneVal>>& out,
                      std::string& why) {
    CacheParser ps{text};
    std::string key;
    long version = -1;
    bool have_entries = false;
    if (!ps.lit('{')) { why = "expected '{'"; return false; }
    if (ps.lit('}')) { why = "no \"entries\""; return false; }
    do {
        if (!ps.str(key) || !ps.lit(':')) { why = "expected a quoted key and ':'"; return false; }
        if (key == "version") {
            if (!ps.integer(version) || version != 1) { why = "version must be 1"; return false; }
        } else if (key == "entries") {
            have_entries = true;
            if (!ps.lit('[')) { why = "entries must be a list"; return false; }
            if (ps.lit(']')) continue;
            do {
                if (!ps.lit('{')) { why = "an entry must be an object"; return false; }
                const char* names[8] = {"size_class", "q_bucket", "tile_w", "tile_h",
                                        "iters_per_launch", "components", "resident", "batched"};
                long val[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                bool seen[8] = {false, false, false, false, false, false, false, false};
                do {
                    long x = 0;
                    if (!ps.str(key) || !ps.lit(':') || !ps.integer(x)) {
                        why = "an entry holds \"key\": integer pairs only";
                        return false;
                    }
                    int k = -1;
                    for (int j = 0; j < 8; ++j)
                        if (key == names[j]) k = j;
                    if (k < 0 || seen[k]) { why = "unknown or repeated key \"" + key + "\""; return false; }
                    seen[k] = true;
                    val[k] = x;
                } while (ps.lit(','));
                if (!ps.lit('}')) { why = "expected '}' after an entry"; return false; }
                for (int j = 0; j < 7; ++j)
                    if (!seen[j]) { why = std::string("entry without \"") + names[j] + "\""; return false; }
                if (val[0] < 0 || val[0] > 12 || val[1] < 0 || val[1] > 4) {
                    why = "size_class must lie in [0, 12] and q_bucket in [0, 4]";
                    return false;
                }
                if (val[5] != 1 && val[5] != 2) { why = "components must be 1 or 2"; return false; }
                if (val[6] != 1 && val[6] != 2) { why = "resident must be 1 or 2"; return false; }
                if (val[7] != 0 && val[7] != 1) { why = "batched must be 0 or 1"; return false; }
                if (val[2] < 1 || val[2] > 4096 || val[3] < 1 || val[3] > 4096 || val[4] < 1 ||
                    val[4] > 4096) {
                    why = "tile_w, tile_h and iters_per_launch out of range";
                    return false;
                }
                const int ci = config_index((int)val[2], (int)val[3], (int)val[4]);
                if (ci < 0) { why = "an entry names a configuration that is not compiled"; return false; }
                out.push_back({TuneKey{(int)val[0], (int)val[1], (int)val[7]},
                               TuneVal{ci, (int)val[5], (int)val[6]}});
            } while (ps.lit(','));
            if (!ps.lit(']')) { why = "expected ']' after the entries"; return false; }
        } else {
            why = "unknown key \"" + key + "\"";
            return false;
        }
    } while (ps.lit(','));
    if (!ps.lit('}')) { why = "expected '}'"; return false; }
    ps.ws();
    if (*ps.p) { why = "text after the closing '}'"; return false; }
    if (version != 1 || !have_entries) { why = "needs \"version\": 1 and \"entries\""; return false; }
    return true;
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
        case RDSEG_ERR_TIMEOUT: return "a bounded on-chip wait expired";
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

size_t rdseg_band_workspace_size(void) {
    Carver c(nullptr);
    c.take<uint32_t>(kBandHistBins);
    c.take<BandState>(1);
    return c.off;
}

rdseg_status rdseg_band_threshold(const float* f, rdseg_shape s, double q, double* delta_out,
                                  void* ws, size_t ws_bytes, void* stream) {
    rdseg_status r = check_shape(s);
    if (r) return r;
    if (!f || !delta_out) return fail(RDSEG_ERR_ARG, "f and delta_out must be non-NULL");
    if (!(q >= 0.0 && q <= 1.0)) return fail(RDSEG_ERR_ARG, "q must lie in [0, 1]");
    const size_t need = rdseg_band_workspace_size();
    if (!ws || ws_bytes < need)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    Carver c(ws);
    uint32_t* hist = c.take<uint32_t>(kBandHistBins);
    BandState* state = c.take<BandState>(1);
    const int64_t k = needed_count(q, (int64_t)s.H * s.W);
    return hip_status(launch_band_threshold(f, s.H, s.W, (int)s.ld, k, hist, state, delta_out,
                                            static_cast<hipStream_t>(stream)));
}

rdseg_status rdseg_solve(const float* f, rdseg_shape s, const rdseg_params* prm, const float* u0,
                         const float* p0, float* u, float* v, float* p, float* tape, void* ws,
                         size_t ws_bytes, void* stream) {
    return solve_impl(f, s, prm, u0, p0, u, v, p, tape, ws, ws_bytes,
                      static_cast<hipStream_t>(stream), -1);
}

// ------------------------------------------------------------------ allocation-free solve
// The workspace of rdseg_solve_noalloc: one array per GPU, held from the
// library's load until the process ends.  Its name is a host-side stand-in in
// host code; the device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[RDSEG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

rdseg_status scratch_of_current_device(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(RDSEG_ERR_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return fail(RDSEG_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(RDSEG_ERR_HIP, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                           hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return RDSEG_OK;
}
}  // namespace

rdseg_status rdseg_solve_noalloc(const float* f, rdseg_shape s, const rdseg_params* prm,
                                 const float* u0, const float* p0, float* u, float* v, float* p,
                                 void* stream) {
    if (!prm) return fail(RDSEG_ERR_ARG, "prm is NULL");
    rdseg_status r = check_shape(s);
    if (r) return r;
    if (prm->ckpt_every != 0)
        return fail(RDSEG_ERR_ARG, "rdseg_solve_noalloc writes no tape: ckpt_every must be 0");
    const size_t need = carve_solve(nullptr, s).bytes;
    if (need > RDSEG_NOALLOC_SCRATCH_BYTES)
        return fail(RDSEG_ERR_WORKSPACE,
                    "the image needs " + std::to_string(need) + " bytes of workspace, more than the " +
                        std::to_string((size_t)RDSEG_NOALLOC_SCRATCH_BYTES) +
                        " bytes of the allocation-free solve's scratch array (use rdseg_solve)");
    void* ws = nullptr;
    r = scratch_of_current_device(&ws);
    if (r) return r;
    return solve_impl(f, s, prm, u0, p0, u, v, p, nullptr, ws, RDSEG_NOALLOC_SCRATCH_BYTES,
                      static_cast<hipStream_t>(stream), -1, nullptr, true);
}

rdseg_status rdseg_solve_status(const rdseg_shape* s, const void* ws, size_t ws_bytes,
                                void* stream) {
    if (!s) return fail(RDSEG_ERR_ARG, "s is NULL");
    rdseg_status r = check_shape(*s);
    if (r) return r;
    const SolveWs need = carve_solve(nullptr, *s);
    if (!ws || ws_bytes < need.bytes)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need.bytes) + " bytes");
    const SolveWs w = carve_solve(const_cast<void*>(ws), *s);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int32_t word = 0;
    if (hipMemcpyAsync(&word, w.npix + 1, sizeof(word), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(RDSEG_ERR_HIP, "reading the solve's status word failed");
    if (word != 0)
        return fail(RDSEG_ERR_TIMEOUT,
                    "a wait of the resident solve for a neighbouring tile expired; u, v and p "
                    "hold NaN on the tiles that stopped");
    return RDSEG_OK;
}

rdseg_status rdseg_set_resident_wait(int64_t ticks) {
    set_resident_wait_ticks(ticks);
    return RDSEG_OK;
}

rdseg_status rdseg_solve_until(const float* f, rdseg_shape s, const rdseg_params* prm,
                               double tol, int32_t check_every, int32_t poll, const float* u0,
                               const float* p0,
                               float* u, float* v, float* p, int32_t* iters_done, float* diffs,
                               void* ws, size_t ws_bytes, void* stream) {
    if (!prm) return fail(RDSEG_ERR_ARG, "prm is NULL");
    if (isnan(tol)) return fail(RDSEG_ERR_ARG, "tol must not be NaN");
    if (check_every < 1) return fail(RDSEG_ERR_ARG, "check_every must be >= 1");
    if (prm->ckpt_every != 0)
        return fail(RDSEG_ERR_ARG, "a convergence-driven solve writes no checkpoints (ckpt_every must be 0)");
    if (!iters_done) return fail(RDSEG_ERR_ARG, "iters_done must be non-NULL");
    const int n_checks = prm->iters > 0 ? prm->iters / check_every : 0;
    if (n_checks > 0 && !diffs)
        return fail(RDSEG_ERR_ARG, "diffs must hold iters / check_every floats");
    StopSpec sp{tol, check_every, reinterpret_cast<uint32_t*>(diffs), n_checks, iters_done,
                poll != 0};
    return solve_impl(f, s, prm, u0, p0, u, v, p, nullptr, ws, ws_bytes,
                      static_cast<hipStream_t>(stream), -1, &sp);
}

size_t rdseg_pd_workspace_size(const rdseg_shape* s) {
    if (!s || !shape_ok(*s)) return 0;
    return carve_pd(nullptr, *s).bytes;
}

rdseg_status rdseg_solve_pd(const float* f, rdseg_shape s, const rdseg_pd_params* prm,
                            const float* u0, const float* p0, float* u, float* p, void* ws,
                            size_t ws_bytes, void* stream) {
    if (!prm) return fail(RDSEG_ERR_ARG, "prm is NULL");
    rdseg_status r = check_shape(s);
    if (r) return r;
    if (!(isfinite(prm->lambda) && prm->lambda >= 0)) return fail(RDSEG_ERR_ARG, "lambda must be finite and >= 0");
    if (!(isfinite(prm->tau) && prm->tau > 0)) return fail(RDSEG_ERR_ARG, "tau must be finite and > 0");
    if (!(isfinite(prm->sigma) && prm->sigma > 0)) return fail(RDSEG_ERR_ARG, "sigma must be finite and > 0");
    if (isnan(prm->delta)) return fail(RDSEG_ERR_ARG, "delta must not be NaN");
    if (prm->iters < 0) return fail(RDSEG_ERR_ARG, "iters must be >= 0");
    if (!f || !u || !p) return fail(RDSEG_ERR_ARG, "f, u and p must be non-NULL");
    const size_t pb = (size_t)s.H * s.ld * sizeof(float);
    if (ranges_overlap(u, pb, f, pb) || ranges_overlap(p, 2 * pb, f, pb) ||
        ranges_overlap(u, pb, p, 2 * pb))
        return fail(RDSEG_ERR_ARG, "u and p must not overlap f or each other");
    if ((u0 && u0 != u && ranges_overlap(u0, pb, u, pb)) ||
        (p0 && p0 != p && ranges_overlap(p0, 2 * pb, p, 2 * pb)))
        return fail(RDSEG_ERR_ARG, "u0 / p0 may equal u / p but must not partially overlap them");
    int ci = -1;
    if (prm->tile_w || prm->tile_h || prm->iters_per_launch) {
        ci = pd_config_index(prm->tile_w, prm->tile_h, prm->iters_per_launch);
        if (ci < 0) return fail(RDSEG_ERR_ARG, "tile_w / tile_h / iters_per_launch is not a compiled primal-dual configuration");
    }
    const PdWs need = carve_pd(nullptr, s);
    if (!ws || ws_bytes < need.bytes)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need.bytes) + " bytes");
    const PdWs w = carve_pd(ws, s);
    hipStream_t st = static_cast<hipStream_t>(stream);
    Geo g = geo_of(s);
    // tile masks and the macro queue come from the same compaction as rdseg_solve
    ImgDesc d = make_desc(f, s, prm->lambda, prm->tau, prm->delta, nullptr, nullptr, nullptr,
                          w.base.c, w.base.st, nullptr, nullptr, 8, 8);
    OffTables off{nullptr, nullptr, nullptr, nullptr};
    if (launch_tile_masks(&d, nullptr, off, 1, g.strips, w.base.masks, w.base.npix, st))
        return RDSEG_ERR_HIP;
    if (ci < 0) {
        // dense problems take the large tiles, sparse bands the small ones
        int64_t np = 0;
        if (hipMemcpyAsync(&np, w.base.npix, sizeof(np), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(RDSEG_ERR_HIP, "reading the active-pixel count failed");
        const double q = (double)np / ((double)s.H * s.W);
        ci = q > 0.3 ? pd_config_index(64, 64, 8) : pd_config_index(16, 16, 8);
    }
    const TileCfg cfg = pd_config_at(ci);
    d = make_desc(f, s, prm->lambda, prm->tau, prm->delta, nullptr, nullptr, nullptr, w.base.c,
                  w.base.st, nullptr, nullptr, cfg.bx, cfg.by);
    PdDesc pd{};
    pd.f = f;
    pd.c = w.base.c;
    const int64_t plane = (int64_t)s.H * s.ld;
    pd.st[0][0] = u;
    pd.st[0][1] = w.ubar0;
    pd.st[0][2] = p;
    pd.st[0][3] = p + plane;
    for (int k = 0; k < 4; ++k) pd.st[1][k] = w.st1[k];
    pd.u0 = u0;
    pd.p0x = p0;
    pd.p0y = p0 ? p0 + plane : nullptr;
    pd.H = s.H;
    pd.W = s.W;
    pd.ld = (int32_t)s.ld;
    pd.mw = d.mw;
    pd.tl = (float)(prm->tau * prm->lambda);
    pd.delta = prm->delta;
    if (launch_pd_init(pd, st)) return RDSEG_ERR_HIP;
    const int64_t nm = macro_count(s, cfg.bx, cfg.by);
    QueueScratch qs{nullptr, nullptr, w.base.flags, w.base.offs, w.base.part};
    if (launch_macro_queue(&d, nullptr, off, 1, nm, cfg.bx, cfg.by, w.base.masks, qs,
                           w.base.queue, w.base.totals, g.nt, nullptr, w.base.totals + 2, st))
        return RDSEG_ERR_HIP;
    const int L = (prm->iters + cfg.it - 1) / cfg.it;
    for (int j = 0; j < L; ++j) {
        const int nit = std::min(cfg.it, prm->iters - j * cfg.it);
        if (launch_pd_iterate(ci, pd, w.base.queue, w.base.totals, nm, (L - j) % 2, nit,
                              (float)prm->tau, (float)prm->sigma, st))
            return RDSEG_ERR_HIP;
    }
    return RDSEG_OK;
}

size_t rdseg_workspace_size3(const rdseg_shape3* s) {
    if (!s || !shape3_ok(*s)) return 0;
    return carve_vol(nullptr, *s).bytes;
}

rdseg_status rdseg_solve3d(const float* f, rdseg_shape3 s, const rdseg_params* prm,
                           const float* u0, const float* p0, float* u, float* v, float* p,
                           void* ws, size_t ws_bytes, void* stream) {
    if (!prm) return fail(RDSEG_ERR_ARG, "prm is NULL");
    if (!shape3_ok(s))
        return fail(RDSEG_ERR_SHAPE, "invalid volume shape: need D, H, W >= 1, ld >= W, lds >= H*ld and D*lds < 2^31");
    rdseg_status r = check_scalars(prm->lambda, prm->theta, prm->tau, prm->delta);
    if (r) return r;
    if (prm->iters < 0) return fail(RDSEG_ERR_ARG, "iters must be >= 0");
    if (prm->inner < 0 || prm->inner > kMaxInner) return fail(RDSEG_ERR_ARG, "inner must lie in [0, 16]");
    if (prm->tile_w || prm->tile_h || prm->iters_per_launch || prm->ckpt_every)
        return fail(RDSEG_ERR_ARG, "tile_w, tile_h, iters_per_launch and ckpt_every must be 0 for volumes");
    if (!f || !u || !v || !p) return fail(RDSEG_ERR_ARG, "f, u, v and p must be non-NULL");
    const int64_t vol = (int64_t)s.D * s.lds;
    const size_t vb = (size_t)vol * sizeof(float);
    if (ranges_overlap(u, vb, f, vb) || ranges_overlap(v, vb, f, vb) ||
        ranges_overlap(p, 3 * vb, f, vb) || ranges_overlap(u, vb, v, vb) ||
        ranges_overlap(u, vb, p, 3 * vb) || ranges_overlap(v, vb, p, 3 * vb))
        return fail(RDSEG_ERR_ARG, "u, v, p must not overlap f or each other");
    if ((u0 && u0 != u && ranges_overlap(u0, vb, u, vb)) ||
        (p0 && p0 != p && ranges_overlap(p0, 3 * vb, p, 3 * vb)))
        return fail(RDSEG_ERR_ARG, "u0 / p0 may equal u / p but must not partially overlap them");
    const VolWs need = carve_vol(nullptr, s);
    if (!ws || ws_bytes < need.bytes)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need.bytes) + " bytes");
    const VolWs w = carve_vol(ws, s);
    hipStream_t st = static_cast<hipStream_t>(stream);
    VolDesc d{};
    d.f = f;
    d.u = u;
    d.c = w.c;
    d.st[0][0] = v;
    for (int k = 0; k < 3; ++k) d.st[0][1 + k] = p + k * vol;
    for (int k = 0; k < 4; ++k) d.st[1][k] = w.st[k];
    d.u0 = u0;
    for (int k = 0; k < 3; ++k) d.p0[k] = p0 ? p0 + k * vol : nullptr;
    d.D = s.D;
    d.H = s.H;
    d.W = s.W;
    d.ld = (int32_t)s.ld;
    d.lds = (int32_t)s.lds;
    d.tl = (float)(prm->theta * prm->lambda);
    d.delta = prm->delta;
    if (launch_init3(d, st) || launch_tile_flags3(d, w.n_tiles, w.flags, st)) return RDSEG_ERR_HIP;
    const int inner = prm->inner > 1 ? prm->inner : 1;
    const int64_t L = (int64_t)prm->iters * inner;
    const float theta = (float)prm->theta, inv_theta = (float)(1.0 / prm->theta);
    const float tau = (float)prm->tau;
    // dual steps in pairs (one pass each), an odd last one alone; the last
    // launch writes buffer 0
    const int64_t n_launch = L / 2 + L % 2;
    for (int64_t j = 0, step = 0; j < n_launch; ++j) {
        const int in_buf = (int)((n_launch - j) % 2);
        const bool last = j == n_launch - 1;
        if (L - step >= 2) {
            const bool uv1 = (step + 1) % inner == 0, uv2 = (step + 2) % inner == 0;
            if (launch_iterate3x2(d, w.flags, w.n_tiles, in_buf, uv1, uv2, last, theta,
                                  inv_theta, tau, st))
                return RDSEG_ERR_HIP;
            step += 2;
        } else {
            const bool uv = (step + 1) % inner == 0;
            if (launch_iterate3(d, w.flags, w.n_tiles, in_buf, uv, last, theta, inv_theta, tau,
                                st))
                return RDSEG_ERR_HIP;
            step += 1;
        }
    }
    return RDSEG_OK;
}

size_t rdseg_metrics_workspace_size(void) { return align_up(metrics_partials_bytes()); }

rdseg_status rdseg_metrics(const float* u, const float* u_ref, rdseg_shape s, double eps,
                           double* out, void* ws, size_t ws_bytes, void* stream) {
    rdseg_status r = check_shape(s);
    if (r) return r;
    if (!u || !u_ref || !out) return fail(RDSEG_ERR_ARG, "u, u_ref and out must be non-NULL");
    if (isnan(eps)) return fail(RDSEG_ERR_ARG, "eps must not be NaN");
    const size_t need = rdseg_metrics_workspace_size();
    if (!ws || ws_bytes < need)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    return hip_status(launch_metrics(u, u_ref, s.H, s.W, (int)s.ld, eps, static_cast<double*>(ws),
                                     out, static_cast<hipStream_t>(stream)));
}

size_t rdseg_batched_workspace_size(const rdseg_image* imgs, int32_t n, int32_t tile_w,
                                    int32_t tile_h) {
    if (!imgs || n < 1) return 0;
    for (int i = 0; i < n; ++i)
        if (!shape_ok(imgs[i].s)) return 0;
    // the library's choice may pick any tile: the 8x8 layout is the largest
    int bx = tile_w > 0 ? tile_w : 8, by = tile_h > 0 ? tile_h : 8;
    if (bx % 8 || by % 8) return 0;
    return layout_batch(imgs, n, bx, by, 1.0, nullptr).bytes;
}

rdseg_status rdseg_solve_batched(const rdseg_image* imgs, int32_t n, double theta, double tau,
                                 int32_t iters, int32_t iters_per_launch, int32_t tile_w,
                                 int32_t tile_h, void** graph_plan, void* ws, size_t ws_bytes,
                                 void* stream) {
    rdseg_status r = validate_batch(imgs, n, theta, tau, iters);
    if (r) return r;
    const bool library_choice = tile_w == 0 && tile_h == 0 && iters_per_launch == 0;
    if (!library_choice && config_index(tile_w, tile_h, iters_per_launch) < 0)
        return fail(RDSEG_ERR_ARG, "tile_w / tile_h / iters_per_launch is not a compiled configuration");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int ci = -1;
    bool persist = false;

    if (!graph_plan) {
        // eager: caller workspace, descriptors uploaded synchronously
        r = choose_batch(imgs, n, theta, tile_w, tile_h, iters_per_launch, ws, ws_bytes, st, &ci,
                         &persist);
        if (r) return r;
        const TileCfg cfg = config_at(ci);
        BatchLayout need = layout_batch(imgs, n, cfg.bx, cfg.by, theta, nullptr);
        if (!ws || ws_bytes < need.bytes)
            return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need.bytes) + " bytes");
        BatchLayout L = layout_batch(imgs, n, cfg.bx, cfg.by, theta, ws);
        r = upload_layout(L, n, st);
        if (r) return r;
        return enqueue_batch(L, n, ci, iters, theta, tau, st, persist);
    }

    BatchPlan* P = static_cast<BatchPlan*>(*graph_plan);
    if (P) {
        const int want = library_choice ? P->ci : config_index(tile_w, tile_h, iters_per_launch);
        if (library_choice != P->library_choice || !same_batch(*P, imgs, n, theta, tau, iters, want))
            return fail(RDSEG_ERR_ARG, "plan was built for a different batch");
        if (hipGraphLaunch(P->exec, st) != hipSuccess) return fail(RDSEG_ERR_HIP, "hipGraphLaunch failed");
        return RDSEG_OK;
    }
    // build a plan: own workspace (the largest layout when the library
    // chooses the configuration), resident descriptors, captured graph
    P = new BatchPlan();
    P->imgs.assign(imgs, imgs + n);
    P->theta = theta;
    P->tau = tau;
    P->iters = iters;
    P->library_choice = library_choice;
    {
        const int bx = library_choice ? 8 : tile_w, by = library_choice ? 8 : tile_h;
        const size_t bytes = layout_batch(imgs, n, bx, by, theta, nullptr).bytes;
        if (hipMalloc(&P->mem, bytes) != hipSuccess) {
            plan_free(P);
            return fail(RDSEG_ERR_HIP, "hipMalloc of the plan workspace failed");
        }
        r = choose_batch(imgs, n, theta, tile_w, tile_h, iters_per_launch, P->mem, bytes, st, &ci,
                         &persist);
        if (r) {
            plan_free(P);
            return r;
        }
    }
    P->ci = ci;
    P->persist = persist;
    const TileCfg cfg = config_at(ci);
    BatchLayout L = layout_batch(imgs, n, cfg.bx, cfg.by, theta, P->mem);
    r = upload_layout(L, n, st);
    if (r) {
        plan_free(P);
        return r;
    }
    // occupancy queries outside the capture
    if (prepare_iterate(ci, true) || prepare_closed(true) ||
        (P->persist && prepare_iterate_persist(ci))) {
        plan_free(P);
        return RDSEG_ERR_HIP;
    }
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        plan_free(P);
        return fail(RDSEG_ERR_HIP, "hipStreamCreate failed");
    }
    bool timing_was = g_timing.on;
    g_timing.on = false;   // no events inside the captured graph
    r = RDSEG_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        r = fail(RDSEG_ERR_HIP, "hipStreamBeginCapture failed");
    } else {
        r = enqueue_batch(L, n, ci, iters, theta, tau, cap, P->persist);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cap, &g);
        if (r == RDSEG_OK && e != hipSuccess) r = fail(RDSEG_ERR_HIP, "hipStreamEndCapture failed");
        P->graph = g;
        if (r == RDSEG_OK && hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) != hipSuccess)
            r = fail(RDSEG_ERR_HIP, "hipGraphInstantiate failed");
    }
    g_timing.on = timing_was;
    (void)hipStreamDestroy(cap);
    if (r) {
        plan_free(P);
        return r;
    }
    *graph_plan = P;
    if (hipGraphLaunch(P->exec, st) != hipSuccess) return fail(RDSEG_ERR_HIP, "hipGraphLaunch failed");
    return RDSEG_OK;
}

rdseg_status rdseg_autotune_batched(const rdseg_image* imgs, int32_t n, double theta, double tau,
                                    int32_t probe_iters, int32_t fix_tile_w, int32_t fix_tile_h,
                                    int32_t fix_iters_per_launch, int32_t fix_form, void* ws,
                                    size_t ws_bytes, void* stream, int32_t* tile_w,
                                    int32_t* tile_h, int32_t* iters_per_launch, int32_t* form) {
    rdseg_status r = validate_batch(imgs, n, theta, tau, probe_iters);
    if (r) return r;
    if (probe_iters < 1) return fail(RDSEG_ERR_ARG, "probe_iters must be >= 1");
    if (fix_form < 0 || fix_form > 2)
        return fail(RDSEG_ERR_ARG, "form must be 0 (both are timed), 1 or 2");
    if (fix_tile_w < 0 || fix_tile_h < 0 || fix_iters_per_launch < 0)
        return fail(RDSEG_ERR_ARG, "fixed tile / launch depth must be >= 0");
    if (!ws || ws_bytes < layout_batch(imgs, n, 8, 8, theta, nullptr).bytes)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need rdseg_batched_workspace_size(imgs, n, 0, 0) bytes");
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto candidate = [&](int ci) {
        const TileCfg c = config_at(ci);
        return (fix_tile_w <= 0 || c.bx == fix_tile_w) && (fix_tile_h <= 0 || c.by == fix_tile_h) &&
               (fix_iters_per_launch <= 0 || c.it == fix_iters_per_launch);
    };
    {
        bool any = false;
        for (int ci = 0; ci < config_count(); ++ci) any = any || candidate(ci);
        if (!any)
            return fail(RDSEG_ERR_ARG, "no compiled configuration matches the fixed tile_w / tile_h / iters_per_launch");
    }
    const bool restricted = fix_tile_w > 0 || fix_tile_h > 0 || fix_iters_per_launch > 0 || fix_form != 0;
    const int f_lo = fix_form ? fix_form : 1, f_hi = fix_form ? fix_form : 2;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RDSEG_ERR_HIP, "hipEventCreate failed");
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(RDSEG_ERR_HIP, "hipStreamCreate failed");
    }
    const bool timing_was = g_timing.on;
    g_timing.on = false;
    // two rounds over all candidates, each timed over three graph replays
    // after a warm-up; the minimum per candidate damps clock and cache noise
    const int nc = config_count();
    std::vector<float> ms_min(2 * nc, -1.0f);   // [config][form - 1]
    for (int round = 0; round < 2 && !r; ++round) {
        for (int ci = 0; ci < nc && !r; ++ci) {
            if (!candidate(ci)) continue;
            const TileCfg cfg = config_at(ci);
            BatchLayout L = layout_batch(imgs, n, cfg.bx, cfg.by, theta, ws);
            r = upload_layout(L, n, st);
            if (r) break;
            if (prepare_iterate(ci, true) || prepare_closed(true) || prepare_iterate_persist(ci)) {
                r = RDSEG_ERR_HIP;
                break;
            }
            for (int fm = f_lo; fm <= f_hi && !r; ++fm) {
                // timed as it runs in a plan: the whole sequence captured in
                // a graph, replayed
                hipGraph_t g = nullptr;
                hipGraphExec_t ge = nullptr;
                if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                    r = fail(RDSEG_ERR_HIP, "hipStreamBeginCapture failed");
                    break;
                }
                r = enqueue_batch(L, n, ci, probe_iters, theta, tau, cap, fm == 1);
                const hipError_t ce = hipStreamEndCapture(cap, &g);
                if (!r && (ce != hipSuccess || hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess))
                    r = fail(RDSEG_ERR_HIP, "capturing a candidate of the batched autotune failed");
                if (!r && hipGraphLaunch(ge, st) != hipSuccess)
                    r = fail(RDSEG_ERR_HIP, "hipGraphLaunch failed");
                if (!r) {
                    (void)hipEventRecord(e0, st);
                    for (int rep = 0; rep < 3 && !r; ++rep)
                        if (hipGraphLaunch(ge, st) != hipSuccess)
                            r = fail(RDSEG_ERR_HIP, "hipGraphLaunch failed");
                    (void)hipEventRecord(e1, st);
                }
                if (!r && hipEventSynchronize(e1) != hipSuccess)
                    r = fail(RDSEG_ERR_HIP, "batched autotune timing failed");
                if (ge) (void)hipGraphExecDestroy(ge);
                if (g) (void)hipGraphDestroy(g);
                if (r) break;
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                float& m = ms_min[2 * ci + (fm - 1)];
                if (m < 0.0f || ms < m) m = ms;
            }
        }
    }
    g_timing.on = timing_was;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(cap);
    if (r) return r;
    int best = -1;
    for (int k = 0; k < 2 * nc; ++k)
        if (ms_min[k] >= 0.0f && (best < 0 || ms_min[k] < ms_min[best])) best = k;
    const int best_ci = best / 2, best_form = best % 2 + 1;
    if (!restricted) {
        double q = 0.0;
        r = batch_active_fraction(imgs, n, theta, ws, st, &q);
        if (r) return r;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[TuneKey{size_class_of(batch_pixels(imgs, n)), q_bucket(q), 1}] =
            TuneVal{best_ci, 2, best_form};
    }
    const TileCfg c = config_at(best_ci);
    if (tile_w) *tile_w = c.bx;
    if (tile_h) *tile_h = c.by;
    if (iters_per_launch) *iters_per_launch = c.it;
    if (form) *form = best_form;
    return RDSEG_OK;
}

rdseg_status rdseg_batched_lookup(const rdseg_image* imgs, int32_t n, double q, int32_t* tile_w,
                                  int32_t* tile_h, int32_t* iters_per_launch, int32_t* form,
                                  int32_t* cached) {
    if (!imgs || n < 1) return fail(RDSEG_ERR_ARG, "imgs must hold n >= 1 images");
    for (int i = 0; i < n; ++i) {
        const rdseg_status r = check_shape(imgs[i].s);
        if (r) return r;
    }
    if (!(q >= 0.0 && q <= 1.0)) return fail(RDSEG_ERR_ARG, "q must lie in [0, 1]");
    int ci = -1, fm = g_batch_form.load(), hit = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(TuneKey{size_class_of(batch_pixels(imgs, n)), q_bucket(q), 1});
        if (it != g_tune.end()) {
            ci = it->second.ci;
            fm = it->second.resident;
            hit = 1;
        }
    }
    if (ci < 0) ci = q >= 0.5 ? config_index(64, 64, 8) : config_index(16, 16, 8);
    const TileCfg c = config_at(ci);
    if (tile_w) *tile_w = c.bx;
    if (tile_h) *tile_h = c.by;
    if (iters_per_launch) *iters_per_launch = c.it;
    if (form) *form = fm;
    if (cached) *cached = hit;
    return RDSEG_OK;
}

rdseg_status rdseg_plan_destroy(void* plan) {
    plan_free(static_cast<BatchPlan*>(plan));
    return RDSEG_OK;
}

size_t rdseg_backward_workspace_size(const rdseg_shape* s, const rdseg_params* prm) {
    if (!s || !prm || !shape_ok(*s) || prm->ckpt_every <= 0) return 0;
    return carve_back(nullptr, *s, prm->ckpt_every).bytes;
}

rdseg_status rdseg_backward(const float* f, rdseg_shape s, const rdseg_params* prm,
                            const float* tape, const float* grad_u, const float* grad_v,
                            float* grad_f, double* grad_lambda, const rdseg_fit* fit,
                            double* grad_c1, double* grad_c2, double* grad_gamma, void* ws,
                            size_t ws_bytes, void* stream) {
    if (!prm) return fail(RDSEG_ERR_ARG, "prm is NULL");
    rdseg_status r = check_shape(s);
    if (r) return r;
    r = check_scalars(prm->lambda, prm->theta, prm->tau, prm->delta);
    if (r) return r;
    if (prm->iters < 0) return fail(RDSEG_ERR_ARG, "iters must be >= 0");
    if (!f || !grad_u || !grad_f || !grad_lambda)
        return fail(RDSEG_ERR_ARG, "f, grad_u, grad_f and grad_lambda must be non-NULL");
    if (!tape || prm->ckpt_every <= 0)
        return fail(RDSEG_ERR_TAPE, "backward needs the tape of a solve with ckpt_every > 0");
    if (prm->inner > 1) return fail(RDSEG_ERR_ARG, "the adjoint is available for inner = 1 only");
    if (fit && !fit->z) return fail(RDSEG_ERR_ARG, "fit->z must be non-NULL");
    const size_t pb = (size_t)s.H * s.ld * sizeof(float);
    if (ranges_overlap(grad_f, pb, f, pb) || ranges_overlap(grad_f, pb, grad_u, pb) ||
        (grad_v && ranges_overlap(grad_f, pb, grad_v, pb)))
        return fail(RDSEG_ERR_ARG, "grad_f must not overlap f, grad_u or grad_v");
    const int ce = prm->ckpt_every;
    BackWs need = carve_back(nullptr, s, ce);
    if (!ws || ws_bytes < need.bytes)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need.bytes) + " bytes");
    BackWs w = carve_back(ws, s, ce);
    hipStream_t st = static_cast<hipStream_t>(stream);
    Geo g = geo_of(s);
    float* nost[3] = {nullptr, nullptr, nullptr};
    ImgDesc d = make_desc(f, s, prm->lambda, prm->theta, prm->delta, nullptr, nullptr, nullptr,
                          w.c, nost, nullptr, nullptr, kAdjTile, kAdjTile);
    OffTables off{nullptr, nullptr, nullptr, nullptr};
    if (launch_init(&d, nullptr, off, 1, s.H, st)) return RDSEG_ERR_HIP;   // c only
    if (launch_tile_masks(&d, nullptr, off, 1, g.strips, w.masks, w.npix, st)) return RDSEG_ERR_HIP;
    const int K = prm->iters;
    // RD components of at most 256 pixels take the component reverse sweep
    // (every step in one launch); the tile path below covers the rest
    const bool comps = g_components_on.load() && prm->components != 2 && K > 0 &&
                       g.plane <= ((int64_t)1 << 29);
    if (comps && launch_components_prepare(d, w.comp, w.masks, w.npix, st)) return RDSEG_ERR_HIP;
    const int64_t nm = macro_count(s, kAdjTile, kAdjTile);
    QueueScratch qs{nullptr, nullptr, w.flags, w.offs, w.part};
    if (launch_macro_queue(&d, nullptr, off, 1, nm, kAdjTile, kAdjTile, w.masks, qs, w.queue,
                           w.totals, g.nt, nullptr, nullptr, st))
        return RDSEG_ERR_HIP;
    // the recompute's own queue, of its own macro tile
    ImgDesc dre = make_desc(f, s, prm->lambda, prm->theta, prm->delta, nullptr, nullptr, nullptr,
                            w.c, nost, nullptr, nullptr, kRecomputeTile, kRecomputeTile);
    const int64_t nmr = macro_count(s, kRecomputeTile, kRecomputeTile);
    if (launch_macro_queue(&dre, nullptr, off, 1, nmr, kRecomputeTile, kRecomputeTile, w.masks,
                           qs, w.rqueue, w.rtotals, g.nt, nullptr, nullptr, st))
        return RDSEG_ERR_HIP;
    if (launch_fill(w.sacc, s.H, s.W, (int)s.ld, 0.0f, st)) return RDSEG_ERR_HIP;
    const float theta = (float)prm->theta, inv_theta = (float)(1.0 / prm->theta);
    const float tau = (float)prm->tau;
    // with the component path on, skip the tile path when no macro tile is
    // left to it (one read of the queue length, which synchronises)
    int32_t n_tiles_left = 1;
    int32_t ccount[kCompCount] = {};
    int64_t comp_waves = -1, comp_jobs = -1;
    if (comps) {
        const int32_t* src[2] = {w.totals, w.comp.ccount};
        const int cnt[2] = {1, kCompCount};
        int32_t* dst[2] = {&n_tiles_left, ccount};
        const rdseg_status rb = read_back(2, src, cnt, dst, st);
        if (rb) return rb;
        // (meaningless, and unused on the device, if the labelling was skipped)
        comp_waves = component_waves_of(ccount);
        comp_jobs = component_group_jobs_of(ccount);
    }
    AdjBufs ab;
    ab.pbx[0] = w.ab[0]; ab.pby[0] = w.ab[1]; ab.vb[0] = w.ab[2];
    ab.pbx[1] = w.ab[3]; ab.pby[1] = w.ab[4]; ab.vb[1] = w.ab[5];
    ab.sacc = w.sacc;
    const int nseg = (K + ce - 1) / ce;
    const int64_t plane = g.plane;
    // the reverse kernel: its macro tile (16: the recompute's queue) and
    // steps per launch
    const int adj_tile = g_adj_tile.load();
    const int adj_ns = g_adj_steps.load();
    const int adj_ai = adj_config_find(adj_tile, adj_ns);
    if (adj_ai < 0) return fail(RDSEG_ERR_ARG, "no reverse kernel for the selected form");
    const bool adj_small = adj_tile == kRecomputeTile;
    // vbar^0 ends in buffer (number of reverse launches) % 2; the component
    // reverse writes its pixels' vbar^0 there too
    int final_buf = 0;
    for (int sg = 0; sg < nseg; ++sg) {
        const int len = std::min(ce, K - sg * ce);
        final_buf ^= ((len + adj_ns - 1) / adj_ns) & 1;
    }
    hipEvent_t join = nullptr;
    if (comps) {
        rdseg_status rc = closed_beside(st, &join, [&](hipStream_t cs) {
            return launch_adj_components(d, w.comp, w.npix, tape, w.seg, K, ce, grad_u, grad_v,
                                         ab.vb[final_buf], w.sacc, theta, inv_theta, tau, cs,
                                         comp_waves, comp_jobs);
        });
        if (rc) return rc;
    }
    int in_buf = 0;
    for (int sg = n_tiles_left > 0 ? nseg - 1 : -1; sg >= 0; --sg) {
        const int k0 = sg * ce;
        const int len = std::min(ce, K - k0);
        auto slot = [&](int j) -> float* {
            return j == 0 ? const_cast<float*>(tape) + (int64_t)sg * 3 * plane
                          : w.seg + (int64_t)(j - 1) * 3 * plane;
        };
        // recompute the forward states k0+1 .. k0+len-1 of this segment: up
        // to 8 steps a launch, each step's state written to its slot
        for (int j = 0; j + 1 < len; j += 8) {
            const int nit = std::min(8, len - 1 - j);
            ImgDesc dr = dre;
            dr.st[1][0] = slot(j); dr.st[1][1] = slot(j) + plane; dr.st[1][2] = slot(j) + 2 * plane;
            float* last = slot(j + nit);
            dr.st[0][0] = last; dr.st[0][1] = last + plane; dr.st[0][2] = last + 2 * plane;
            if (launch_recompute(dr, w.rqueue, w.rtotals, nmr, 1, nit, theta, inv_theta, tau,
                                 slot(j + 1), 3 * plane, plane, st))
                return RDSEG_ERR_HIP;
        }
        // reverse sweep, up to adj_ns steps a launch
        for (int k = k0 + len; k >= k0 + 1;) {
            const int ns = std::min(adj_ns, k - k0);
            AdjSlots sl;
            sl.plane = plane;
            for (int i = 0; i < kAdjMaxSteps; ++i) sl.s[i] = i < ns ? slot(k - 1 - i - k0) : nullptr;
            const bool first = (k == K);
            if (launch_adj_block(adj_ai, adj_small ? dre : d, sl, ns, ab, in_buf, first, grad_v,
                                 first ? grad_u : nullptr, adj_small ? w.rqueue : w.queue,
                                 adj_small ? w.rtotals : w.totals, adj_small ? nmr : nm, theta,
                                 tau, st))
                return RDSEG_ERR_HIP;
            in_buf = 1 - in_buf;
            k -= ns;
        }
    }
    if (n_tiles_left == 0) in_buf = final_buf;   // where the skipped launches would have left vbar
    {
        const rdseg_status rj = join_closed(st, join);
        if (rj) return rj;
    }
    if (comps && launch_components_restore(d, w.comp, w.npix, st)) return RDSEG_ERR_HIP;
    const float* vb0 = ab.vb[in_buf];
    if (K == 0) {
        if (grad_v) {
            vb0 = grad_v;
        } else {
            if (launch_fill(ab.vb[0], s.H, s.W, (int)s.ld, 0.0f, st)) return RDSEG_ERR_HIP;
            vb0 = ab.vb[0];
        }
    }
    if (launch_adj_final(d, w.sacc, vb0, grad_f, prm->lambda, prm->theta, fit ? fit->z : nullptr,
                         fit ? fit->P : nullptr, fit ? fit->c1 : 0.0, fit ? fit->c2 : 0.0, w.red,
                         reduce_partials(s.H), w.out4, st))
        return RDSEG_ERR_HIP;
    if (launch_scatter_scalars(w.out4, grad_lambda, fit ? grad_c1 : nullptr, fit ? grad_c2 : nullptr,
                               fit ? grad_gamma : nullptr, st))
        return RDSEG_ERR_HIP;
    return RDSEG_OK;
}

rdseg_status rdseg_fit_forward(const rdseg_fit* fit, rdseg_shape s, float* f, void* stream) {
    rdseg_status r = check_shape(s);
    if (r) return r;
    if (!fit || !fit->z || !f) return fail(RDSEG_ERR_ARG, "fit, fit->z and f must be non-NULL");
    if (!(isfinite(fit->c1) && isfinite(fit->c2) && isfinite(fit->gamma)))
        return fail(RDSEG_ERR_ARG, "c1, c2, gamma must be finite");
    const size_t pb = (size_t)s.H * s.ld * sizeof(float);
    if (ranges_overlap(f, pb, fit->z, pb) || (fit->P && ranges_overlap(f, pb, fit->P, pb)))
        return fail(RDSEG_ERR_ARG, "f must not overlap z or P");
    if (launch_fit_forward(fit->z, fit->P, fit->c1, fit->c2, fit->gamma, s.H, s.W, (int)s.ld, f,
                           static_cast<hipStream_t>(stream)))
        return RDSEG_ERR_HIP;
    return RDSEG_OK;
}

size_t rdseg_reduce_workspace_size(const rdseg_shape* s) {
    if (!s || !shape_ok(*s)) return 0;
    return reduce_ws_bytes(*s);
}

rdseg_status rdseg_fit_backward(const rdseg_fit* fit, rdseg_shape s, const float* grad_f,
                                double* grad_c1, double* grad_c2, double* grad_gamma, void* ws,
                                size_t ws_bytes, void* stream) {
    rdseg_status r = check_shape(s);
    if (r) return r;
    if (!fit || !fit->z || !grad_f) return fail(RDSEG_ERR_ARG, "fit, fit->z and grad_f must be non-NULL");
    if (!(isfinite(fit->c1) && isfinite(fit->c2)))
        return fail(RDSEG_ERR_ARG, "c1, c2 must be finite");
    size_t need = reduce_ws_bytes(s);
    if (!ws || ws_bytes < need)
        return fail(RDSEG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    Carver cv(ws);
    double* red = cv.take<double>(reduce_partials(s.H));
    double* out = cv.take<double>(4);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (launch_fit_backward(fit->z, fit->P, grad_f, fit->c1, fit->c2, s.H, s.W, (int)s.ld, red,
                            reduce_partials(s.H), out, st))
        return RDSEG_ERR_HIP;
    if (launch_scatter_scalars(out, grad_c1, grad_c2, grad_gamma, nullptr, st)) return RDSEG_ERR_HIP;
    return RDSEG_OK;
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
                            int32_t* iters_per_launch, int32_t* components, int32_t* resident) {
    if (!prm) return fail(RDSEG_ERR_ARG, "prm is NULL");
    if (probe_iters < 1) return fail(RDSEG_ERR_ARG, "probe_iters must be >= 1");
    if (prm->components < 0 || prm->components > 2)
        return fail(RDSEG_ERR_ARG, "components must be 0 (library's choice), 1 (on) or 2 (off)");
    if (prm->resident < 0 || prm->resident > 2)
        return fail(RDSEG_ERR_ARG, "resident must be 0 (library's choice), 1 (on-chip exchange) or 2 (separate launches)");
    {
        const rdseg_status rs = check_shape(s);
        if (rs) return rs;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    rdseg_params q = *prm;
    q.iters = probe_iters;
    q.ckpt_every = 0;
    hipEvent_t e0, e1;
    const int inner = prm->inner > 1 ? prm->inner : 1;
    // a nonzero tile_w / tile_h / iters_per_launch / components / resident in
    // prm fixes that parameter: only candidates that match it take part
    auto candidate = [&](int ci) {
        const TileCfg c = config_at(ci);
        return c.it >= inner && (prm->tile_w <= 0 || c.bx == prm->tile_w) &&
               (prm->tile_h <= 0 || c.by == prm->tile_h) &&
               (prm->iters_per_launch <= 0 || c.it == prm->iters_per_launch);
    };
    const bool restricted = prm->tile_w > 0 || prm->tile_h > 0 || prm->iters_per_launch > 0 ||
                            prm->components != 0 || prm->resident != 0;
    {
        bool any = false;
        for (int ci = 0; ci < config_count(); ++ci) any = any || candidate(ci);
        if (!any)
            return fail(RDSEG_ERR_ARG, "no compiled configuration matches the fixed tile_w / tile_h / iters_per_launch");
    }
    const int comp_lo = prm->components ? prm->components : 1;
    const int comp_hi = prm->components ? prm->components : 2;
    // the barrier between blocks of iterations: on-chip exchange (resident
    // form, where the configuration has one: a solve uses it when the image's
    // tiles, or else the queued ones, fit on the chip) or kernel boundaries
    // (what a configuration without that form runs, and is recorded as)
    auto res_range = [&](int ci, int& lo, int& hi) {
        const bool capable = resident_available(ci);
        lo = prm->resident ? prm->resident : (capable ? 1 : 2);
        hi = prm->resident ? prm->resident : 2;
    };
    q.tile_w = q.tile_h = q.iters_per_launch = 0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RDSEG_ERR_HIP, "hipEventCreate failed");
    // two rounds over all candidates, each timed over three solves after a
    // warm-up; the minimum per candidate damps clock and cache noise
    const int n = config_count();
    std::vector<float> ms_min(4 * n, -1.0f);   // [config][components - 1][resident - 1]
    for (int round = 0; round < 2; ++round) {
        for (int ci = 0; ci < n; ++ci) {
            if (!candidate(ci)) continue;
            int res_lo = 1, res_hi = 1;
            res_range(ci, res_lo, res_hi);
            for (int cm = comp_lo; cm <= comp_hi; ++cm)
            for (int rk = res_lo; rk <= res_hi; ++rk) {
                q.components = cm;
                q.resident = rk;
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
                float& m = ms_min[4 * ci + 2 * (cm - 1) + (rk - 1)];
                if (m < 0.0f || ms < m) m = ms;
            }
        }
    }
    int best = -1;
    float best_ms = 0.0f;
    for (int k = 0; k < 4 * n; ++k)
        if (ms_min[k] >= 0.0f && (best < 0 || ms_min[k] < best_ms)) { best = k; best_ms = ms_min[k]; }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int best_ci = best / 4, best_comps = (best / 2) % 2 + 1, best_res = best % 2 + 1;
    // record under the problem's class and active-fraction bucket (a search
    // over a restricted set does not speak for the class)
    if (!restricted) {
        SolveWs w = carve_solve(ws, s);
        int64_t np = 0;
        if (hipMemcpy(&np, w.npix, sizeof(np), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(RDSEG_ERR_HIP, "reading the active-pixel count failed");
        double qf = (double)np / ((double)s.H * s.W);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[TuneKey{size_class(s), q_bucket(qf)}] = TuneVal{best_ci, best_comps, best_res};
    }
    TileCfg c = config_at(best_ci);
    if (tile_w) *tile_w = c.bx;
    if (tile_h) *tile_h = c.by;
    if (iters_per_launch) *iters_per_launch = c.it;
    if (components) *components = best_comps;
    if (resident) *resident = best_res;
    return RDSEG_OK;
}

rdseg_status rdseg_tune_cache_export(char* buf, size_t cap, size_t* len) {
    if (!len) return fail(RDSEG_ERR_ARG, "len is NULL");
    std::string t = "{\"version\": 1, \"entries\": [";
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        bool first = true;
        for (const auto& kv : g_tune) {
            const TileCfg c = config_at(kv.second.ci);
            char e[256];
            snprintf(e, sizeof(e),
                     "%s\n  {\"size_class\": %d, \"q_bucket\": %d, \"tile_w\": %d, \"tile_h\": %d, "
                     "\"iters_per_launch\": %d, \"components\": %d, \"resident\": %d%s}",
                     first ? "" : ",", kv.first.cls, kv.first.qb, c.bx, c.by, c.it,
                     kv.second.comps, kv.second.resident,
                     kv.first.batched ? ", \"batched\": 1" : "");
            t += e;
            first = false;
        }
    }
    t += "]}\n";
    *len = t.size() + 1;
    if (cap < t.size() + 1 || !buf)
        return fail(RDSEG_ERR_ARG, "buffer too small: need " + std::to_string(t.size() + 1) + " bytes");
    memcpy(buf, t.c_str(), t.size() + 1);
    return RDSEG_OK;
}

rdseg_status rdseg_tune_lookup(const rdseg_shape* s, double q, int32_t* tile_w, int32_t* tile_h,
                               int32_t* iters_per_launch, int32_t* components,
                               int32_t* resident, int32_t* cached) {
    if (!s) return fail(RDSEG_ERR_ARG, "s is NULL");
    rdseg_status r = check_shape(*s);
    if (r) return r;
    if (!(q >= 0.0 && q <= 1.0)) return fail(RDSEG_ERR_ARG, "q must lie in [0, 1]");
    int ci = -1, cm = 0, rk = 0, hit = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(TuneKey{size_class(*s), q_bucket(q)});
        if (it != g_tune.end()) {
            ci = it->second.ci;
            cm = it->second.comps;
            rk = it->second.resident;
            hit = 1;
        }
    }
    if (ci < 0) ci = heuristic_cfg(*s, q);
    const TileCfg c = config_at(ci);
    if (tile_w) *tile_w = c.bx;
    if (tile_h) *tile_h = c.by;
    if (iters_per_launch) *iters_per_launch = c.it;
    if (components) *components = cm;
    if (resident) *resident = rk;
    if (cached) *cached = hit;
    return RDSEG_OK;
}

rdseg_status rdseg_tune_cache_import(const char* json) {
    if (!json) return fail(RDSEG_ERR_ARG, "json is NULL");
    std::vector<std::pair<TuneKey, TuneVal>> entries;
    std::string why;
    if (!parse_cache_text(json, entries, why)) return fail(RDSEG_ERR_ARG, "tuning cache text: " + why);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& e : entries) g_tune[e.first] = e.second;
    return RDSEG_OK;
}

rdseg_status rdseg_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return RDSEG_OK;
}

rdseg_status rdseg_set_resident(int32_t on) {
    g_resident_on.store(on != 0);
    return RDSEG_OK;
}

rdseg_status rdseg_set_batched_form(int32_t form) {
    if (form != 1 && form != 2)
        return fail(RDSEG_ERR_ARG, "form must be 1 (one persistent launch) or 2 (separate launches)");
    g_batch_form.store(form);
    return RDSEG_OK;
}

rdseg_status rdseg_set_adjoint_form(int32_t tile, int32_t steps) {
    if (tile == 0) tile = 32;
    if (steps == 0) steps = 2;
    if (adj_config_find(tile, steps) < 0)
        return fail(RDSEG_ERR_ARG, "no reverse kernel for tile " + std::to_string(tile) +
                                       " and " + std::to_string(steps) + " steps a launch");
    g_adj_tile.store(tile);
    g_adj_steps.store(steps);
    return RDSEG_OK;
}

rdseg_status rdseg_set_components(int32_t on) {
    g_components_on.store(on != 0);
    return RDSEG_OK;
}

rdseg_status rdseg_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.on = on != 0;
    return RDSEG_OK;
}

rdseg_status rdseg_timing_read(int32_t config, double* kernel_ms, int64_t* launches,
                               double* alg_bytes, int64_t* pixel_updates) {
    return rdseg_timing_read_form(config, -1, kernel_ms, launches, alg_bytes, pixel_updates);
}

rdseg_status rdseg_timing_read_form(int32_t config, int32_t form, double* kernel_ms,
                                    int64_t* launches, double* alg_bytes,
                                    int64_t* pixel_updates) {
    if (form < -1 || form > 1) return fail(RDSEG_ERR_ARG, "form must be -1, 0 or 1");
    std::lock_guard<std::mutex> lk(g_timing.mu);
    double ms = 0.0, bytes = 0.0;
    int64_t upd = 0, n = 0;
    for (auto& r : g_timing.recs) {
        if (config >= 0 && r.ci != config) continue;
        if (form >= 0 && (int)r.resident != form) continue;
        if (hipEventSynchronize(r.e1) != hipSuccess) return fail(RDSEG_ERR_HIP, "event sync failed");
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, r.e0, r.e1);
        ms += t;
        int64_t np = r.npix_host ? *r.npix_host : 0;
        upd += np * r.nit;
        bytes += 28.0 * (double)np * r.nit;
        n += r.launches;
    }
    if (kernel_ms) *kernel_ms = ms;
    if (launches) *launches = n;
    if (alg_bytes) *alg_bytes = bytes;
    if (pixel_updates) *pixel_updates = upd;
    return RDSEG_OK;
}

rdseg_status rdseg_release(void) {
    rdseg_status r = RDSEG_OK;
    {
        std::lock_guard<std::mutex> lk(g_side_mu);
        for (auto& kv : g_side) {
            int cur = 0;
            if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(kv.first) != hipSuccess ||
                hipStreamSynchronize(kv.second) != hipSuccess ||
                hipStreamDestroy(kv.second) != hipSuccess)
                r = fail(RDSEG_ERR_HIP, "releasing a side stream failed");
            (void)hipSetDevice(cur);
        }
        g_side.clear();
    }
    {
        std::lock_guard<std::mutex> lk(g_timing.mu);
        for (auto& rec : g_timing.recs) {
            (void)hipEventSynchronize(rec.e1);
            g_timing.pool.push_back(rec.e0);
            g_timing.pool.push_back(rec.e1);
        }
        g_timing.recs.clear();
        if (g_timing.has_open) {
            g_timing.pool.push_back(g_timing.open.e0);
            g_timing.pool.push_back(g_timing.open.e1);
            g_timing.has_open = false;
        }
        for (hipEvent_t e : g_timing.pool)
            if (e && hipEventDestroy(e) != hipSuccess) r = fail(RDSEG_ERR_HIP, "releasing an event failed");
        g_timing.pool.clear();
        if (g_timing.pinned && hipHostFree(g_timing.pinned) != hipSuccess)
            r = fail(RDSEG_ERR_HIP, "releasing the pinned timing buffer failed");
        g_timing.pinned = nullptr;
        g_timing.pinned_cap = g_timing.pinned_used = 0;
    }
    {
        std::lock_guard<std::mutex> lk(g_poll_mu);
        if (g_poll_host && hipHostFree(g_poll_host) != hipSuccess)
            r = fail(RDSEG_ERR_HIP, "releasing the pinned polling buffer failed");
        g_poll_host = nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(g_rb_mu);
        if (g_rb_host && hipHostFree(g_rb_host) != hipSuccess)
            r = fail(RDSEG_ERR_HIP, "releasing the pinned read-back buffer failed");
        g_rb_host = nullptr;
        g_rb_seq = 0;
    }
    return r;
}

rdseg_status rdseg_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    for (auto& r : g_timing.recs) {
        if (hipEventSynchronize(r.e1) != hipSuccess) return fail(RDSEG_ERR_HIP, "event sync failed");
        g_timing.pool.push_back(r.e0);
        g_timing.pool.push_back(r.e1);
    }
    g_timing.recs.clear();
    g_timing.pinned_used = 0;
    return RDSEG_OK;
}

}  // extern "C"
