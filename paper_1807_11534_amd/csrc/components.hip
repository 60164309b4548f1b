// components.hip -- small RD components solved whole, one lane per pixel.
//
// An RD pixel interacts only with the RD pixels of its own 4-connected
// component: the dual step reads w at x + e and the divergence p at x - e,
// and at frozen neighbours both are constants (w = -H(-f)/theta, p = 0).  A
// component of at most 64 pixels can therefore run every iteration inside one
// wave, one pixel per lane, its neighbours' values fetched from other lanes
// (ds_bpermute) and its frozen neighbours entering as constants; one of 65-256
// pixels in a group of 128 or 256 threads of a workgroup (values exchanged
// through LDS).  Below the percolation threshold of the band most RD pixels
// sit in such components; the tile path then only has to cover the large
// ones.
//
// Steps (single image; skipped on the device when more than 55 % of the
// pixels are RD, where one component spans the image):
//   k_cc_init      labels: the first pixel of its horizontal RD run within
//                  the wave's 64 pixels on RD, -1 elsewhere; counters cleared
//   k_cc_union     lock-free union of runs, right across a wave boundary and
//                  down (the larger root is linked below the smaller one with
//                  atomicMin)
//   k_cc_flatten   every RD pixel points at its root; component sizes (one
//                  atomic per root and wave) and each pixel's rank in its
//                  component
//   k_cc_class     each small component (<= 256 pixels) takes a slot in the
//                  class of its size rounded up to a power of two
//   k_cc_assign    each of its pixels takes a lane: waves of a class k <= 6
//                  hold 64 / 2^k components of 2^k lanes, classes 7 and 8 a
//                  group of 2^k lanes a component (the lanes no pixel takes
//                  are marked -1 by the components' first pixels); the pixel
//                  is then frozen for the tile path (c = +inf, its tile-mask
//                  bit cleared; the tile path's RD count is the full count
//                  less these pixels)
//   k_components   every iteration of the groups, then of the packed waves
// Lane order within a component depends on atomics, but no result does: each
// pixel's arithmetic reads exact neighbour values, with the per-pixel
// functions of the other kernels, so results are bitwise equal to theirs.
#include <atomic>
#include <algorithm>

#include "components_device.h"

namespace rdseg {

namespace {

__device__ __forceinline__ int size_class(int s) {   // ceil(log2(s)), s in [1, 64]
    return s <= 1 ? 0 : 32 - __clz(s - 1);
}

__device__ __forceinline__ int cc_find(int32_t* lab, int x) {
    while (true) {
        const int p = __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == x) return x;
        const int gp = __hip_atomic_load(lab + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (gp != p)   // path halving: gp is an ancestor of x as well
            __hip_atomic_store(lab + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

// Root of x without writing (for the flattening pass, whose only stores must
// be roots: a path-halving store there could overwrite a finished root with
// an intermediate ancestor).
__device__ __forceinline__ int cc_root(const int32_t* lab, int x) {
    while (true) {
        const int p = __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == x) return x;
        x = p;
    }
}

__device__ __forceinline__ void cc_unite(int32_t* lab, int a, int b) {
    while (true) {
        a = cc_find(lab, a);
        b = cc_find(lab, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(lab + a, b);   // a was a root: link it below b
        if (old == a) return;
        a = old;   // a was linked meanwhile: continue from its new parent
    }
}

// The grid-stride loops below run 256-thread workgroups over consecutive pixel
// indices, so every wave holds 64 consecutive indices starting at a multiple
// of 64 (a "segment"; lane = index mod 64).

__global__ __launch_bounds__(256) void k_cc_init(ImgDesc d, CompWs w, const int64_t* npix) {
    if (blockIdx.x == 0 && threadIdx.x == 0) w.npix_tile[0] = npix[0];
    if (cc_skip(npix, d)) return;
    const int64_t plane = (int64_t)d.H * d.ld;
    const int l = threadIdx.x & 63;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < plane;
         g += (int64_t)gridDim.x * 256) {
        const int y = (int)(g / d.ld), x = (int)(g - (int64_t)y * d.ld);
        const bool act = x < d.W && c_active(d.c[g]);
        // A horizontal run of RD pixels inside the segment (a run also starts
        // at x = 0) is linked to its first pixel at once, so the union pass
        // only joins runs.
        const uint64_t gap = __ballot(!act);
        const uint64_t row0 = __ballot(act && x == 0);
        const uint64_t gb = gap & ((1ull << l) - 1);         // lanes below l
        int start = gb ? 64 - __clzll(gb) : 0;                // past the last gap
        const uint64_t rb = row0 & ((2ull << l) - 1);         // lanes up to l
        if (rb) start = max(start, 63 - __clzll(rb));
        w.lab[g] = act ? (int32_t)(g - (l - start)) : -1;
        if (act) {   // read at roots only
            w.csize[g] = 0;
            w.cslot[g] = 0;
        }
        w.lane_of[g] = -1;
        if (g < kCompCount) w.ccount[g] = 0;
    }
}

// Joins of runs: across a segment boundary on the right, and down, where a
// vertical pair of RD pixels has no vertical RD pair directly to its left
// (that pair, or the first one of the stretch, already joins the two runs:
// consecutive RD pixels of a row are linked by their run or by a boundary
// join).
__global__ __launch_bounds__(256) void k_cc_union(ImgDesc d, CompWs w, const int64_t* npix) {
    if (cc_skip(npix, d)) return;
    const int64_t plane = (int64_t)d.H * d.ld;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < plane;
         g += (int64_t)gridDim.x * 256) {
        const int y = (int)(g / d.ld), x = (int)(g - (int64_t)y * d.ld);
        if (x >= d.W || !c_active(d.c[g])) continue;
        if ((g & 63) == 63 && x + 1 < d.W && c_active(d.c[g + 1]))
            cc_unite(w.lab, (int)g, (int)g + 1);
        if (y + 1 < d.H && c_active(d.c[g + d.ld])) {
            const bool left_pair = x > 0 && c_active(d.c[g - 1]) && c_active(d.c[g - 1 + d.ld]);
            if (!left_pair) cc_unite(w.lab, (int)g, (int)g + d.ld);
        }
    }
}

__global__ __launch_bounds__(256) void k_cc_flatten(ImgDesc d, CompWs w, const int64_t* npix) {
    if (cc_skip(npix, d)) return;
    const int64_t plane = (int64_t)d.H * d.ld;
    const int l = threadIdx.x & 63;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < plane;
         g += (int64_t)gridDim.x * 256) {
        const bool act = w.lab[g] >= 0;
        int r = -1;
        if (act) {
            r = cc_root(w.lab, (int)g);
            __hip_atomic_store(w.lab + g, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // Sizes are exact up to kCompMax + 1; beyond that only "large"
        // matters.  cslot[r] (cleared by the init pass, written for small
        // roots only by the class pass) flags a root that has passed
        // kCompMax, so the pixels of large components stop adding to one
        // contended counter (a stale read only costs an extra add).  The
        // lanes of a wave that share a root add their count with one atomic,
        // and each takes the count before it as its rank in the component
        // (crank[g]: distinct, in [0, size) for every pixel of a small
        // component, whose pixels are all counted).
        bool want = act && !w.cslot[r];
        while (true) {
            const uint64_t m = __ballot(want);
            if (!m) break;
            const int leader = __ffsll((unsigned long long)m) - 1;
            const int r0 = __shfl(r, leader);
            const bool same = want && r == r0;
            const uint64_t sm = __ballot(same);
            int old = 0;
            if (l == leader) {
                const int cnt = __popcll(sm);
                old = atomicAdd(w.csize + r0, cnt);
                if (old + cnt > kCompMax) w.cslot[r0] = 1;
            }
            old = __shfl(old, leader);
            if (same) {
                w.crank[g] = old + __popcll(sm & ((1ull << l) - 1));
                want = false;
            }
        }
    }
}

// Slots within the size classes: each workgroup counts its small roots per
// class in LDS, takes one block of slots per class with a single global
// atomic, and hands them out in the order of its local counting.
__global__ __launch_bounds__(256) void k_cc_class(ImgDesc d, CompWs w, const int64_t* npix) {
    __shared__ int sCount[kCompClasses], sBase[kCompClasses];
    if (cc_skip(npix, d)) return;   // uniform: npix is not changed by this pass
    const int t = threadIdx.x;
    if (t < kCompClasses) sCount[t] = 0;
    __syncthreads();
    const int64_t plane = (int64_t)d.H * d.ld;
    const int64_t per_wg = (plane + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * per_wg;
    const int64_t g1 = min(plane, g0 + per_wg);
    const int l = t & 63;
    // four pixels a thread per round, their loads issued together
    for (int64_t gb = g0; gb < g1; gb += 1024) {
        int lv[4], sz[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = gb + t + i * 256;
            lv[i] = g < g1 ? w.lab[g] : -1;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = gb + t + i * 256;
            sz[i] = (g < g1 && lv[i] == (int32_t)g) ? w.csize[g] : 0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = gb + t + i * 256;
            // size class of a small root
            const int k = (sz[i] >= 1 && sz[i] <= kCompMax) ? size_class(sz[i]) : -1;
            // local slots: one LDS atomic per class and wave, lanes in order
            for (int c = 0; c < kCompClasses; ++c) {
                const uint64_t m = __ballot(k == c);
                if (!m) continue;   // uniform
                const int leader = __ffsll((unsigned long long)m) - 1;
                int base = 0;
                if (l == leader) base = atomicAdd(&sCount[c], __popcll(m));
                base = __shfl(base, leader);
                if (k == c) w.cslot[g] = base + __popcll(m & ((1ull << l) - 1));
            }
        }
    }
    __syncthreads();
    if (t < kCompClasses) sBase[t] = sCount[t] ? atomicAdd(w.ccount + t, sCount[t]) : 0;
    __syncthreads();
    for (int64_t gb = g0; gb < g1; gb += 1024) {
        int lv[4], sz[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = gb + t + i * 256;
            lv[i] = g < g1 ? w.lab[g] : -1;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = gb + t + i * 256;
            sz[i] = (g < g1 && lv[i] == (int32_t)g) ? w.csize[g] : 0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = gb + t + i * 256;
            if (sz[i] >= 1 && sz[i] <= kCompMax) w.cslot[g] += sBase[size_class(sz[i])];
        }
    }
}

__global__ __launch_bounds__(256) void k_cc_assign(ImgDesc d, CompWs w, uint64_t* masks,
                                                   const int64_t* npix) {
    __shared__ int sFrozen;
    __shared__ int sCB[kCompClasses];   // class_base of each class
    if (cc_skip(npix, d)) return;   // uniform: npix is not changed by this pass
    if (threadIdx.x == 0) sFrozen = 0;
    if (threadIdx.x < kCompClasses) sCB[threadIdx.x] = class_base(w.ccount, threadIdx.x);
    __syncthreads();
    const int64_t plane = (int64_t)d.H * d.ld;
    int frozen = 0;
    const int l = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * 256;
    // four pixels a thread per round (each wave still 64 consecutive pixels
    // for each of them), their loads issued together
    for (int64_t gb = (int64_t)blockIdx.x * 256 + threadIdx.x; gb < plane; gb += 4 * stride) {
        int rr[4], sz[4], sl[4], rk[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = gb + i * stride;
            rr[i] = g < plane ? w.lab[g] : -1;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = gb + i * stride;
            const bool ok = rr[i] >= 0 && rr[i] < plane;
            sz[i] = ok ? w.csize[rr[i]] : 0;
            sl[i] = ok ? w.cslot[rr[i]] : -1;
            rk[i] = ok ? w.crank[g] : 0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = gb + i * stride;
            if (g - threadIdx.x + (threadIdx.x & ~63) >= plane) break;   // uniform per wave
            const int y = (int)(g / d.ld), x = (int)(g - (int64_t)y * d.ld);
            const int s = sz[i];
            bool frz = false;
            if (g < plane && s >= 1 && s <= kCompMax) {
                const int k = size_class(s);
                const int slot = sl[i];
                const int rank = rk[i];
                int L;
                if (k < kWaveClasses) {   // 64 / 2^k components packed into a wave
                    const int per = kSmallMax >> k;
                    const int wave = sCB[k] + slot / per;
                    L = wave * 64 + (slot % per) * (1 << k) + rank;
                } else {                  // one component a group of 2^k lanes
                    L = sCB[k] * 64 + slot * (1 << k) + rank;
                }
                // never false for a well-formed labelling (see kCompLaneExtra);
                // a guard against writing outside the lane table
                if (slot >= 0 && rank < s && L >= 0 && L < 2 * plane + kCompLaneExtra) {
                    w.lane_of[g] = L;
                    w.wl_pix[L] = (int32_t)g;
                    d.c[g] = __builtin_inff();   // frozen for the tile path from here on
                    frz = true;
                    ++frozen;
                    // The component's first pixel marks the lanes no pixel
                    // takes: the rest of its 2^k lanes and, for the last
                    // component of a wave class, the free slots after it in
                    // its wave (every lane the component passes read lies in
                    // some class's slot, so all of them are written)
                    if (rank == 0) {
                        const int64_t top = 2 * plane + kCompLaneExtra;
                        for (int j = s; j < (1 << k); ++j)
                            if (L + j < top) w.wl_pix[L + j] = -1;
                        if (k < kWaveClasses && slot == w.ccount[k] - 1) {
                            const int per = kSmallMax >> k;
                            const int64_t w0 = (int64_t)(sCB[k] + slot / per) * 64;
                            for (int j = (slot % per + 1) << k; j < 64; ++j)
                                if (w0 + j < top) w.wl_pix[w0 + j] = -1;
                        }
                    }
                }
            }
            // Tile-mask bits of the frozen pixels: the lanes of one 8x8 tile
            // row are consecutive in the wave (they start where x mod 8 = 0,
            // or at lane 0), so the first of them clears all their bits with
            // one atomic.
            const uint64_t fm = __ballot(frz);
            if (fm && g < plane && ((x & 7) == 0 || l == 0) && x < d.W) {
                const int glen = min(min(8 - (x & 7), 64 - l), d.W - x);
                const uint64_t bits = (fm >> l) & ((1ull << glen) - 1);
                if (bits) {
                    const int64_t T = (int64_t)(y >> 3) * d.tw + (x >> 3);
                    atomicAnd((unsigned long long*)(masks + T), ~(bits << (8 * (y & 7) + (x & 7))));
                }
            }
        }
    }
    if (frozen) atomicAdd(&sFrozen, frozen);
    __syncthreads();
    if (threadIdx.x == 0 && sFrozen)
        atomicAdd((unsigned long long*)w.npix_tile, (unsigned long long)(-(long long)sFrozen));
}

// Every iteration of the component path (unless the resident kernel's idle
// workgroups already ran them: ccount[kCompFlag] set): first the group
// classes (jobs of a whole workgroup), then the packed one-wave classes.
__global__ __launch_bounds__(256) void k_components(ImgDesc d, CompWs w, const int64_t* npix,
                                                    int iters, int inner, float theta,
                                                    float inv_theta, float tau,
                                                    float* __restrict__ tape, int ce) {
    __shared__ float xbuf[1024];
    if (cc_skip(npix, d) || w.ccount[kCompFlag]) return;
    component_groups(d, w, iters, inner, theta, inv_theta, tau, tape, ce, blockIdx.x,
                     gridDim.x, xbuf);
    component_waves(d, w, iters, inner, theta, inv_theta, tau, tape, ce,
                    blockIdx.x * 4 + (threadIdx.x >> 6), gridDim.x * 4);
}

// Reverse sweep of the small components, every segment in one launch: per
// segment (last first) each lane loads its pixel's checkpoint from the tape,
// recomputes the segment's forward states (the arithmetic of one k_iterate
// iteration) and then runs the segment's reverse steps with the arithmetic of
// the tile path's reverse kernel (k_adj_block), neighbour values from other
// lanes and frozen neighbours as constants (w right / below; p, ubar, gbar
// and wbar are 0 there).  Where
// the segment fits a workgroup's LDS (one wave per workgroup, lane-major):
// lds_mode 2 (ce x 1536 bytes) keeps each forward step's dual-update outputs
// (p, g, m) and u, so the reverse steps recompute nothing; lds_mode 1
// ((ce - 1) x 768 bytes) keeps the states and the reverse recomputes each
// step's dual update from them; lds_mode 0 keeps the states in the per-pixel
// slots of seg that the tile path uses.  The adjoint state (pbar, vbar) and
// the clamp-adjoint sum stay in registers; the sum goes to sacc and vbar^0 to
// vb_out at the end.  Results are bitwise those of the tile path.
//
// REG (a separate instantiation, so that its registers do not weigh on the
// LDS forms): no LDS at all, for many waves.  A first forward pass over the
// segment keeps a checkpoint every kSubLen states in registers; then per
// sub-segment (last first) a second forward pass from its checkpoint keeps
// the dual-update outputs and u of its at most kSubLen steps in registers and
// the reverse steps read them.  The occupancy follows the registers instead
// of 22 KB of LDS per wave.  The same forward and reverse arithmetic, so
// bitwise the other forms.
constexpr int kSubLen = 8;   // steps per sub-segment
constexpr int kSubMax = 5;   // sub-segments per segment: ckpt_every <= 40

template <bool G> struct XOf { using type = WaveX; };
template <> struct XOf<true> { using type = GroupX; };

template <bool REG, bool GRP>
__global__ __launch_bounds__(256) void k_adj_components_t(
    ImgDesc d, CompWs w, const int64_t* npix, const float* __restrict__ tape,
    float* __restrict__ seg, int K, int ce, const float* __restrict__ grad_u,
    const float* __restrict__ grad_v, float* __restrict__ vb_out, float* __restrict__ sacc,
    float theta, float inv_theta, float tau, int lds_mode) {
    extern __shared__ float s_states[];
    __shared__ float xbuf[GRP ? 1024 : 1];
    if (cc_skip(npix, d)) return;
    const int64_t plane = (int64_t)d.H * d.ld;
    // GRP: the group classes, one job (two components of class 7 or one of
    // class 8) per 256-thread workgroup, the register form or the per-pixel
    // slots; else the packed one-wave classes
    if (GRP && lds_mode != 0) lds_mode = 0;
    const int nwork = GRP ? group_jobs(w.ccount)
                          : (int)min((int64_t)class_base(w.ccount, kWaveClasses),
                                     (2 * plane + kCompLaneExtra) / 64);
    const int lane = GRP ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    // lds_mode 4: two waves per workgroup on the same packed wave, one running
    // the reverse of segment sg while the other runs the forward of segment
    // sg - 1 into the other of two buffers [ce][6][64]
    const bool duo = !GRP && lds_mode == 4;
    const bool fwd_wave = duo && (threadIdx.x >> 6) == 1;
    const int wpb = (duo || GRP) ? 1 : (int)(blockDim.x >> 6);
    const int wslot = (duo || GRP) ? 0 : (int)(threadIdx.x >> 6);
    // LDS per wave: lds_mode 1 holds states [ce - 1][3][64], lds_mode 2 the
    // dual-update outputs and u [ce][6][64]; lds_mode 0 uses seg instead
    const int per_wave = lds_mode == 2 ? ce * 384 : (lds_mode == 1 ? (ce - 1) * 192 : 0);
    float* __restrict__ my_states = s_states + wslot * per_wave + lane;
    typename XOf<GRP>::type xc;
    if constexpr (GRP) {
        xc.buf = xbuf;
        xc.par = 0;
        xc.t = (int)threadIdx.x;
    }
    for (int item = blockIdx.x * wpb + wslot; item < nwork;
         item += gridDim.x * wpb) {   // uniform per wave (per workgroup with lds_mode 4 or GRP)
        int g, base;
        if constexpr (GRP) {
            int ln;
            group_lane(w.ccount, item, lane, ln, base);
            g = (ln >= 0 && ln < 2 * plane + kCompLaneExtra) ? w.wl_pix[ln] : -1;
        } else {
            g = w.wl_pix[item * 64 + lane];
            base = item * 64;
        }
        const bool mine = g >= 0 && g < plane;
        const int gg = mine ? g : 0;
        const int y = gg / d.ld, x = gg - y * d.ld;
        const float c = mine ? c_of(d.f[gg], d.delta, d.tl) : __builtin_inff();
        uint32_t fl = mine ? (CF_ACT | CF_OUT) : 0u;
        if (mine && x == d.W - 1) fl |= CF_LASTC;
        if (mine && y == d.H - 1) fl |= CF_LASTR;
        const bool lastc = (fl & CF_LASTC) != 0, lastr = (fl & CF_LASTR) != 0;
        int nR = -1, nD = -1, nL = -1, nU = -1;
        float wR = 0.0f, wD = 0.0f;
        if (mine) {
            if (x + 1 < d.W) {
                const int L = w.lane_of[gg + 1];
                if (L >= 0) nR = L - base;
                else wR = w_of(0.0f, heav_from_c(c_of(d.f[gg + 1], d.delta, d.tl)), inv_theta, false);
            } else {
                wR = w_of(0.0f, 0.0f, inv_theta, false);
            }
            if (y + 1 < d.H) {
                const int L = w.lane_of[gg + d.ld];
                if (L >= 0) nD = L - base;
                else wD = w_of(0.0f, heav_from_c(c_of(d.f[gg + d.ld], d.delta, d.tl)), inv_theta, false);
            } else {
                wD = w_of(0.0f, 0.0f, inv_theta, false);
            }
            if (x > 0) {
                const int L = w.lane_of[gg - 1];
                if (L >= 0) nL = L - base;
            }
            if (y > 0) {
                const int L = w.lane_of[gg - d.ld];
                if (L >= 0) nU = L - base;
            }
        }
        // exchange indices (a lane reads itself when the neighbour is frozen)
        const int iR = nR >= 0 ? nR : lane, iD = nD >= 0 ? nD : lane;
        const int iL = nL >= 0 ? nL : lane, iU = nU >= 0 ? nU : lane;
        // x - 1 and y - 1 neighbours of (a, b), x + 1 and y + 1 neighbours of
        // a, of quantities that are 0 at frozen cells; every lane calls them
        // together
        auto left_up = [&](float a, float b, float& l, float& u) {
            float tl, tu;
            xc.two(a, iL, b, iU, tl, tu);
            l = nL >= 0 ? tl : 0.0f;
            u = nU >= 0 ? tu : 0.0f;
        };
        auto right_down0 = [&](float a, float& r, float& dn) {
            float tr, td;
            xc.same2(a, iR, iD, tr, td);
            r = nR >= 0 ? tr : 0.0f;
            dn = nD >= 0 ? td : 0.0f;
        };

        float pbx = 0.0f, pby = 0.0f;
        float vb = (mine && grad_v) ? grad_v[gg] : 0.0f;
        float S = 0.0f;
        // one reverse step k from the dual update of step k (p^k, g, m of
        // state k - 1) and u^k: the arithmetic of k_adj_block
        auto reverse_step = [&](int k, float opx, float opy, float ogx, float ogy, float om,
                                float u) {
            const float sarg = u - c;
            const float sb = (mine && sarg > 0.0f && sarg < 1.0f) ? vb : 0.0f;
            float ub = sb;
            if (k == K && grad_u && mine) ub += grad_u[gg];
            ub = mine ? ub : 0.0f;
            // pbt = pbar^k + theta grad(ubar); gbar
            float ubr, ubd;
            right_down0(ub, ubr, ubd);
            const float gux = lastc ? 0.0f : (ubr - ub);
            const float guy = lastr ? 0.0f : (ubd - ub);
            const float ptx = mine ? fmaf(theta, gux, pbx) : 0.0f;
            const float pty = mine ? fmaf(theta, guy, pby) : 0.0f;
            const float nn = __builtin_amdgcn_sqrtf(fmaf(ogx, ogx, ogy * ogy));
            const float inv_n = nn > 0.0f ? __builtin_amdgcn_rcpf(nn) : 0.0f;
            const float tm = tau * om;
            const float dot = fmaf(opx, ptx, opy * pty);
            const float k2 = tm * dot * inv_n;
            float gbx = fmaf(tm, ptx, -k2 * ogx);
            float gby = fmaf(tm, pty, -k2 * ogy);
            gbx = (mine && !lastc) ? gbx : 0.0f;
            gby = (mine && !lastr) ? gby : 0.0f;
            // wbar = -div gbar; pbar^(k-1), vbar^(k-1)
            float gbl, gbu;
            left_up(gbx, gby, gbl, gbu);
            const float dg = div_p(gbx, gbl, gby, gbu);
            const float wb = mine ? -dg : 0.0f;
            float wbr, wbd;
            right_down0(wb, wbr, wbd);
            const float gwx = lastc ? 0.0f : (wbr - wb);
            const float gwy = lastr ? 0.0f : (wbd - wb);
            pbx = lastc ? 0.0f : fmaf(om, ptx, -gwx);
            pby = lastr ? 0.0f : fmaf(om, pty, -gwy);
            vb = fmaf(-wb, inv_theta, ub);
            S += sb;
        };
        // one forward step from state (v, px, py): the dual update and u
        auto forward_step = [&](float v, float px, float py, DualOut& o, float& u) {
            float pl, pu;
            left_up(px, py, pl, pu);
            const float dd = div_p(px, pl, py, pu);
            const float wv = w_of(dd, v, inv_theta, mine);
            float wr, wd;
            xc.same2(wv, iR, iD, wr, wd);
            o = dual_update(px, py, wv, nR >= 0 ? wr : wR, nD >= 0 ? wd : wD, fl, tau);
            float ol, ou;
            left_up(o.px, o.py, ol, ou);
            u = u_step(v, div_p(o.px, ol, o.py, ou), theta);
        };
        const int nseg = (K + ce - 1) / ce;
        if constexpr (REG) {
            for (int sg = nseg - 1; sg >= 0; --sg) {
                const int k0 = sg * ce;
                const int len = min(ce, K - k0);
                const int nb = (len + kSubLen - 1) / kSubLen;
                float cpv[kSubMax], cpx[kSubMax], cpy[kSubMax];
                {
                    float v = 0.0f, px = 0.0f, py = 0.0f;   // the checkpoint, state k0
                    if (mine) {
                        const float* __restrict__ s0 = tape + (int64_t)sg * 3 * plane;
                        v = s0[gg];
                        px = s0[plane + gg];
                        py = s0[2 * plane + gg];
                    }
#pragma unroll
                    for (int b = 0; b < kSubMax; ++b) {
                        cpv[b] = v;
                        cpx[b] = px;
                        cpy[b] = py;
                        if (b + 1 < nb) {   // uniform
                            for (int j = 0; j < kSubLen; ++j) {
                                DualOut o;
                                float u;
                                forward_step(v, px, py, o, u);
                                px = o.px;
                                py = o.py;
                                v = v_step(u, c);
                            }
                        }
                    }
                }
                for (int b = nb - 1; b >= 0; --b) {
                    const int j0 = b * kSubLen;
                    const int sl = min(kSubLen, len - j0);
                    float v = cpv[0], px = cpx[0], py = cpy[0];
#pragma unroll
                    for (int q = 1; q < kSubMax; ++q) {
                        if (q == b) {
                            v = cpv[q];
                            px = cpx[q];
                            py = cpy[q];
                        }
                    }
                    float opx[kSubLen], opy[kSubLen], ogx[kSubLen], ogy[kSubLen], om[kSubLen],
                        ou[kSubLen];
#pragma unroll
                    for (int i = 0; i < kSubLen; ++i) {
                        opx[i] = 0.0f; opy[i] = 0.0f; ogx[i] = 0.0f; ogy[i] = 0.0f;
                        om[i] = 0.0f; ou[i] = 0.0f;
                        if (i < sl) {   // uniform
                            DualOut o;
                            float u;
                            forward_step(v, px, py, o, u);
                            opx[i] = o.px; opy[i] = o.py; ogx[i] = o.gx; ogy[i] = o.gy;
                            om[i] = o.m; ou[i] = u;
                            px = o.px;
                            py = o.py;
                            v = v_step(u, c);
                        }
                    }
#pragma unroll
                    for (int i = kSubLen - 1; i >= 0; --i)
                        if (i < sl) reverse_step(k0 + j0 + i + 1, opx[i], opy[i], ogx[i], ogy[i],
                                                 om[i], ou[i]);
                }
            }
        } else if (duo) {
            auto fwd_store = [&](float* __restrict__ base, int j, float& v, float& px, float& py) {
                DualOut o;
                float u;
                forward_step(v, px, py, o, u);
                float* __restrict__ sj = base + j * 384;
                sj[0] = o.px;
                sj[64] = o.py;
                sj[128] = o.gx;
                sj[192] = o.gy;
                sj[256] = o.m;
                sj[320] = u;
                px = o.px;
                py = o.py;
                v = v_step(u, c);
            };
            auto fwd_segment = [&](int sg, float* __restrict__ base) {
                float v = 0.0f, px = 0.0f, py = 0.0f;
                if (mine) {
                    const float* __restrict__ s0 = tape + (int64_t)sg * 3 * plane;
                    v = s0[gg];
                    px = s0[plane + gg];
                    py = s0[2 * plane + gg];
                }
                const int len = min(ce, K - sg * ce);
                for (int j = 0; j < len; ++j) fwd_store(base, j, v, px, py);
            };
            float* const bufs[2] = {s_states + lane, s_states + ce * 384 + lane};
            if (fwd_wave) fwd_segment(nseg - 1, bufs[(nseg - 1) & 1]);
            __syncthreads();
            for (int sg = nseg - 1; sg >= 0; --sg) {
                if (fwd_wave) {
                    if (sg > 0) fwd_segment(sg - 1, bufs[(sg - 1) & 1]);
                } else {
                    const int k0 = sg * ce;
                    const int len = min(ce, K - k0);
                    const float* __restrict__ cur = bufs[sg & 1];
                    for (int i = 0; i < len; ++i) {
                        const float* __restrict__ sj = cur + (len - 1 - i) * 384;
                        reverse_step(k0 + len - i, sj[0], sj[64], sj[128], sj[192], sj[256],
                                     sj[320]);
                    }
                }
                __syncthreads();
            }
        } else {
            for (int sg = nseg - 1; sg >= 0; --sg) {
                const int k0 = sg * ce;
                const int len = min(ce, K - k0);
                const float* __restrict__ s0 = tape + (int64_t)sg * 3 * plane;
                float cv = 0.0f, cpx = 0.0f, cpy = 0.0f;   // the checkpoint, state k0
                if (mine) {
                    cv = s0[gg];
                    cpx = s0[plane + gg];
                    cpy = s0[2 * plane + gg];
                }
                if (lds_mode == 2) {
                    // forward over all len steps, keeping what the reverse reads:
                    // slot j = p^(k0+j+1), g, m and u^(k0+j+1) of the step from state k0 + j
                    float v = cv, px = cpx, py = cpy;
                    for (int j = 0; j < len; ++j) {
                        DualOut o;
                        float u;
                        forward_step(v, px, py, o, u);
                        float* __restrict__ sj = my_states + j * 384;
                        sj[0] = o.px;
                        sj[64] = o.py;
                        sj[128] = o.gx;
                        sj[192] = o.gy;
                        sj[256] = o.m;
                        sj[320] = u;
                        px = o.px;
                        py = o.py;
                        v = v_step(u, c);
                    }
                    for (int k = k0 + len; k >= k0 + 1; --k) {
                        const float* __restrict__ sj = my_states + (k - 1 - k0) * 384;
                        reverse_step(k, sj[0], sj[64], sj[128], sj[192], sj[256], sj[320]);
                    }
                    continue;
                }
                // forward: the states k0 + 1 .. k0 + len - 1 of this segment
                {
                    float v = cv, px = cpx, py = cpy;
                    for (int j = 1; j < len; ++j) {
                        DualOut o;
                        float u;
                        forward_step(v, px, py, o, u);
                        px = o.px;
                        py = o.py;
                        v = v_step(u, c);
                        if (lds_mode == 1) {
                            float* __restrict__ sj = my_states + (j - 1) * 192;
                            sj[0] = v;
                            sj[64] = px;
                            sj[128] = py;
                        } else if (mine) {
                            float* __restrict__ sj = seg + (int64_t)(j - 1) * 3 * plane;
                            sj[gg] = v;
                            sj[plane + gg] = px;
                            sj[2 * plane + gg] = py;
                        }
                    }
                }
                // reverse: steps k0 + len .. k0 + 1 from the states k - 1
                for (int k = k0 + len; k >= k0 + 1; --k) {
                    const int j = k - 1 - k0;
                    float sv = 0.0f, spx = 0.0f, spy = 0.0f;
                    if (j == 0) {
                        sv = cv;
                        spx = cpx;
                        spy = cpy;
                    } else if (lds_mode == 1) {
                        const float* __restrict__ sj = my_states + (j - 1) * 192;
                        sv = mine ? sj[0] : 0.0f;
                        spx = mine ? sj[64] : 0.0f;
                        spy = mine ? sj[128] : 0.0f;
                    } else if (mine) {
                        const float* __restrict__ sj = seg + (int64_t)(j - 1) * 3 * plane;
                        sv = sj[gg];
                        spx = sj[plane + gg];
                        spy = sj[2 * plane + gg];
                    }
                    // w from p^(k-1), v^(k-1); the dual update gives p^k, g and m; u^k
                    DualOut o;
                    float u;
                    forward_step(sv, spx, spy, o, u);
                    reverse_step(k, o.px, o.py, o.gx, o.gy, o.m, u);
                }
            }
        }
        if (mine && !fwd_wave) {
            sacc[gg] = S;
            vb_out[gg] = vb;
        }
        if constexpr (GRP) __syncthreads();   // the exchange buffers are reused by the next job
    }
}

// c of the small-component pixels back to theta lambda f (after the solve's
// tile path, for passes that test RD through c).
__global__ __launch_bounds__(256) void k_cc_restore(ImgDesc d, CompWs w, const int64_t* npix) {
    if (cc_skip(npix, d)) return;
    const int64_t plane = (int64_t)d.H * d.ld;
    const int64_t lanes =
        min((int64_t)class_base(w.ccount, kCompClasses) * 64, 2 * plane + kCompLaneExtra);
    for (int64_t L = (int64_t)blockIdx.x * 256 + threadIdx.x; L < lanes;
         L += (int64_t)gridDim.x * 256) {
        const int g = w.wl_pix[L];
        if (g >= 0 && g < plane) d.c[g] = c_of(d.f[g], d.delta, d.tl);
    }
}

unsigned grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

int g_comp_grid = 0;
int g_adj_comp_grid = 0;
// LDS forms of the component reverse sweep: ce x 1536 or (ce - 1) x 768 bytes
// per wave, at most the default 64 KiB of a workgroup; the grid for the last
// size used
constexpr int kAdjLdsMax = 65536;
std::atomic<int> g_adj_lds_limit{0};   // the device's largest workgroup allocation

}  // namespace

int launch_components_prepare(const ImgDesc& d, const CompWs& w, uint64_t* masks,
                              const int64_t* npix, hipStream_t st) {
    const unsigned grid = grid_for((int64_t)d.H * d.ld);
    hipLaunchKernelGGL(k_cc_init, dim3(grid), dim3(256), 0, st, d, w, (const int64_t*)npix);
    hipLaunchKernelGGL(k_cc_union, dim3(grid), dim3(256), 0, st, d, w, (const int64_t*)npix);
    hipLaunchKernelGGL(k_cc_flatten, dim3(grid), dim3(256), 0, st, d, w, (const int64_t*)npix);
    // the class and assignment passes end with per-workgroup atomics on a few
    // shared counters (class counts, the tile path's RD count): fewer, larger
    // workgroups keep that contention small
    hipLaunchKernelGGL(k_cc_class, dim3(std::min(grid, 1024u)), dim3(256), 0, st, d, w,
                       (const int64_t*)npix);
    hipLaunchKernelGGL(k_cc_assign, dim3(std::min(grid, 1024u)), dim3(256), 0, st, d, w, masks,
                       (const int64_t*)npix);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_components(const ImgDesc& d, const CompWs& w, const int64_t* npix, int iters,
                      int inner, float theta, float inv_theta, float tau, float* tape, int ce,
                      hipStream_t st) {
    if (tape && (ce <= 0 || inner != 1)) {
        set_error("component checkpoints need ckpt_every > 0 and inner = 1");
        return 3;
    }
    if (g_comp_grid == 0) {
        g_comp_grid = persistent_blocks(reinterpret_cast<const void*>(k_components), 256, 0);
        if (g_comp_grid <= 0) {
            g_comp_grid = 0;
            set_error("occupancy query failed for the component kernel");
            return 4;
        }
    }
    hipLaunchKernelGGL(k_components, dim3((unsigned)g_comp_grid), dim3(256), 0, st, d, w, npix,
                       iters, inner, theta, inv_theta, tau, tape, ce);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int64_t component_waves_of(const int32_t* ccount_host) {
    int64_t b = 0;
    for (int j = 0; j < kWaveClasses; ++j) {
        const int per = kSmallMax >> j;
        b += ((int64_t)ccount_host[j] + per - 1) / per;
    }
    return b;
}

int64_t component_group_jobs_of(const int32_t* ccount_host) {
    return ((int64_t)ccount_host[7] + 1) / 2 + ccount_host[8];
}

int launch_adj_components(const ImgDesc& d, const CompWs& w, const int64_t* npix,
                          const float* tape, float* seg, int K, int ce, const float* grad_u,
                          const float* grad_v, float* vb_out, float* sacc, float theta,
                          float inv_theta, float tau, hipStream_t st, int64_t nwaves_hint,
                          int64_t group_jobs) {
    // The group classes (components of 65-256 pixels): one job a 256-thread
    // workgroup, the register form where ckpt_every allows, else the
    // per-pixel slots of seg.
    if (group_jobs != 0) {
        const bool reg = ce <= kSubLen * kSubMax;
        static std::atomic<int> cap_reg{0}, cap_slots{0};
        std::atomic<int>& cap = reg ? cap_reg : cap_slots;
        const void* gfn = reg ? reinterpret_cast<const void*>(k_adj_components_t<true, true>)
                              : reinterpret_cast<const void*>(k_adj_components_t<false, true>);
        int grid = cap.load(std::memory_order_relaxed);
        if (grid == 0) {
            grid = persistent_blocks(gfn, 256, 0);
            if (grid <= 0) {
                set_error("occupancy query failed for the component adjoint kernel");
                return 4;
            }
            cap.store(grid, std::memory_order_relaxed);
        }
        if (group_jobs > 0 && group_jobs < grid) grid = (int)group_jobs;
        if (reg)
            hipLaunchKernelGGL((k_adj_components_t<true, true>), dim3((unsigned)grid), dim3(256), 0,
                               st, d, w, npix, tape, seg, K, ce, grad_u, grad_v, vb_out, sacc,
                               theta, inv_theta, tau, 0);
        else
            hipLaunchKernelGGL((k_adj_components_t<false, true>), dim3((unsigned)grid), dim3(256),
                               0, st, d, w, npix, tape, seg, K, ce, grad_u, grad_v, vb_out, sacc,
                               theta, inv_theta, tau, 0);
        RDSEG_HIP_CHECK(hipGetLastError());
    }
    // The kept dual-update outputs (modes 2, 4) shorten every reverse step but
    // take twice the LDS of the states (mode 1), so fewer waves run at once:
    // they are used when all the component waves fit on the chip together.
    // Mode 4 adds a second wave per workgroup that runs the next segment's
    // forward beside the current reverse (two buffers; a workgroup allocation
    // above the default 64 KiB where the device offers one).
    const size_t rich = (size_t)ce * 384 * sizeof(float);
    const size_t lean = (size_t)(ce - 1) * 192 * sizeof(float);
    const bool lean_ok = ce > 1 && lean <= (size_t)kAdjLdsMax;
    int lds_limit = g_adj_lds_limit.load(std::memory_order_relaxed);
    if (lds_limit == 0) {
        int dev = 0, v = 0;
        lds_limit = kAdjLdsMax;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                hipSuccess &&
            v > kAdjLdsMax)
            lds_limit = v;
        g_adj_lds_limit.store(lds_limit, std::memory_order_relaxed);
    }
    const void* fn = reinterpret_cast<const void*>(k_adj_components_t<false, false>);
    auto cap_of = [&](int threads, size_t bytes) {
        return bytes > (size_t)lds_limit ? 0 : persistent_blocks(fn, threads, bytes);
    };
    const bool few = nwaves_hint >= 0;
    int mode = lean_ok ? 1 : 0;
    if (rich <= (size_t)kAdjLdsMax) {
        const int cap = cap_of(64, rich);
        if (!lean_ok || (few && cap > 0 && nwaves_hint <= cap)) mode = 2;
    }
    if (mode == 2 && few && K > ce) {
        const int cap = cap_of(128, 2 * rich);
        if (cap > 0 && nwaves_hint <= cap) mode = 4;
    }
    if (mode == 4 && 2 * rich > (size_t)kAdjLdsMax &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(2 * rich)) !=
            hipSuccess) {
        (void)hipGetLastError();
        mode = 2;   // the larger allocation is not available: one wave, one buffer
    }
    // many waves: the register form (no LDS, occupancy by registers) in place
    // of the states in LDS (22 KB a wave at ckpt_every = 30: seven waves a CU)
    if (mode == 1 && ce <= kSubLen * kSubMax) {
        static std::atomic<int> reg_grid{0};
        const void* rfn = reinterpret_cast<const void*>(k_adj_components_t<true, false>);
        int grid = reg_grid.load(std::memory_order_relaxed);
        if (grid == 0) {
            grid = persistent_blocks(rfn, 256, 0);
            if (grid <= 0) {
                set_error("occupancy query failed for the component adjoint kernel");
                return 4;
            }
            reg_grid.store(grid, std::memory_order_relaxed);
        }
        hipLaunchKernelGGL((k_adj_components_t<true, false>), dim3((unsigned)grid), dim3(256), 0, st, d,
                           w, npix, tape, seg, K, ce, grad_u, grad_v, vb_out, sacc, theta,
                           inv_theta, tau, 0);
        RDSEG_HIP_CHECK(hipGetLastError());
        return 0;
    }
    if (mode > 0) {
        const int threads = mode == 4 ? 128 : 64;
        const size_t lds = mode == 4 ? 2 * rich : (mode == 2 ? rich : lean);
        const int grid = persistent_blocks(fn, threads, lds);
        if (grid <= 0) {
            set_error("occupancy query failed for the component adjoint kernel");
            return 4;
        }
        hipLaunchKernelGGL((k_adj_components_t<false, false>), dim3((unsigned)grid), dim3(threads), lds, st, d, w,
                           npix, tape, seg, K, ce, grad_u, grad_v, vb_out, sacc, theta,
                           inv_theta, tau, mode);
        RDSEG_HIP_CHECK(hipGetLastError());
        return 0;
    }
    if (g_adj_comp_grid == 0) {
        g_adj_comp_grid = persistent_blocks(fn, 256, 0);
        if (g_adj_comp_grid <= 0) {
            g_adj_comp_grid = 0;
            set_error("occupancy query failed for the component adjoint kernel");
            return 4;
        }
    }
    hipLaunchKernelGGL((k_adj_components_t<false, false>), dim3((unsigned)g_adj_comp_grid), dim3(256), 0, st, d, w,
                       npix, tape, seg, K, ce, grad_u, grad_v, vb_out, sacc, theta, inv_theta,
                       tau, 0);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_components_restore(const ImgDesc& d, const CompWs& w, const int64_t* npix,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_cc_restore, dim3(grid_for(2 * (int64_t)d.H * d.ld)), dim3(256), 0, st, d,
                       w, npix);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace rdseg
