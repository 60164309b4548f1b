// components_device.h -- the small-component solve as a device function,
// shared by the component kernel and the idle workgroups of the resident
// kernel.
//
// An RD pixel interacts only with the RD pixels of its own 4-connected
// component (Sec. 3: the frozen pixels' values never change): the dual step
// reads w at x + e and the divergence p at x - e, and at frozen neighbours
// both are constants (w = -H(-f)/theta, p = 0).  A component of at most 64
// pixels therefore runs every iteration inside one wave, one pixel per lane,
// its neighbours' values fetched from other lanes (ds_bpermute) and its frozen
// neighbours entering as constants; one of 65-256 pixels runs in a group of
// 128 or 256 lanes of a workgroup, its neighbours' values exchanged through
// LDS between workgroup barriers.  The per-pixel functions are those of
// rdseg_device.h, so results are bitwise those of the tile kernels.
#pragma once

#include "rdseg_internal.h"

namespace rdseg {

constexpr int kSmallMax = 64;    // largest component of the one-wave classes
constexpr int kCompMax = 256;    // largest component of the component path
constexpr int kWaveClasses = 7;  // classes 0..6: padded sizes 1 .. 64, packed into waves
// Classes 7 and 8 (padded sizes 128, 256): one component a group of 128 or
// 256 lanes.  Lanes used: a component of class k >= 1 has more than 2^(k-1)
// pixels and takes 2^k lanes, so all classes together take fewer than twice
// the pixels plus a partly filled last wave per class: wl_pix holds
// 2 * plane + kCompLaneExtra.

__device__ __forceinline__ bool cc_skip(const int64_t* npix, const ImgDesc& d) {
    return 100 * npix[0] > 55 * (int64_t)d.H * d.W;
}

// 64-lane units taken by the classes below k: packed waves for the one-wave
// classes, 2^(k - 6) units a component above
__device__ __forceinline__ int class_base(const int32_t* ccount, int k) {
    int b = 0;
    for (int j = 0; j < k; ++j) {
        if (j < kWaveClasses) {
            const int per = kSmallMax >> j;
            b += (ccount[j] + per - 1) / per;
        } else {
            b += ccount[j] << (j - 6);
        }
    }
    return b;
}

// Neighbour exchange of the component solve.  Indices are a lane of the wave
// (WaveX: ds_bpermute) or a thread of the workgroup (GroupX: a value written
// to LDS, a barrier, the neighbour's value read; two buffers alternate, so one
// barrier per exchange suffices).  Every call is made by all lanes together.
struct WaveX {
    __device__ __forceinline__ float get(int idx, float a) const {
        return __int_as_float(__builtin_amdgcn_ds_bpermute(4 * idx, __float_as_int(a)));
    }
    // a read at i1 and at i2
    __device__ __forceinline__ void same2(float a, int i1, int i2, float& r1, float& r2) {
        r1 = get(i1, a);
        r2 = get(i2, a);
    }
    // a read at i1, b at i2
    __device__ __forceinline__ void two(float a, int i1, float b, int i2, float& r1, float& r2) {
        r1 = get(i1, a);
        r2 = get(i2, b);
    }
};

struct GroupX {
    float* buf;   // LDS of this 256-thread slice: 2 buffers x 2 values x 256
    int par;
    int t;        // the thread's index in its slice
    __device__ __forceinline__ void same2(float a, int i1, int i2, float& r1, float& r2) {
        float* b = buf + par * 512;
        b[t] = a;
        __syncthreads();
        r1 = b[i1];
        r2 = b[i2];
        par ^= 1;
    }
    __device__ __forceinline__ void two(float a, int i1, float bb, int i2, float& r1, float& r2) {
        float* b = buf + par * 512;
        b[t] = a;
        b[256 + t] = bb;
        __syncthreads();
        r1 = b[i1];
        r2 = b[256 + i2];
        par ^= 1;
    }
};

// One component's pixel on this lane for every iteration.  g: its pixel (or
// < 0: an empty lane); self: this lane's exchange index; base: the packed
// lane (lane_of value) whose exchange index is 0.  The u-step / v-step / dual
// step are those of k_iterate; x +/- 1 and y +/- 1 neighbours come from their
// lanes, frozen neighbours as constants (w right and below, p = 0 left and
// above).  Reads the start state from buffer 0 and leaves the final one
// there; writes u.  With a tape (inner = 1, ce > 0) the state before iteration
// k goes to slot k / ce whenever ce divides k.
template <class X>
__device__ __forceinline__ void component_chain(const ImgDesc& d, const CompWs& w, X& xc, int g,
                                                int self, int base, int iters, int inner,
                                                float theta, float inv_theta, float tau,
                                                float* __restrict__ tape, int ce) {
    const int64_t plane = (int64_t)d.H * d.ld;
    const bool mine = g >= 0 && g < plane;
    const int gg = mine ? g : 0;
    const int y = gg / d.ld, x = gg - y * d.ld;
    // this pixel: RD by construction; its state from buffer 0
    const float fv = mine ? d.f[gg] : 0.0f;
    const float c = mine ? c_of(fv, d.delta, d.tl) : __builtin_inff();
    float v = 0.0f, px = 0.0f, py = 0.0f;
    if (mine) {
        v = d.st[0][0][gg];
        px = d.st[0][1][gg];
        py = d.st[0][2][gg];
    }
    uint32_t fl = mine ? (CF_ACT | CF_OUT) : 0u;
    if (mine && x == d.W - 1) fl |= CF_LASTC;
    if (mine && y == d.H - 1) fl |= CF_LASTR;
    // neighbour lanes (same component), or -1 with a frozen constant
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
    const int iR = nR >= 0 ? nR : self, iD = nD >= 0 ? nD : self;
    const int iL = nL >= 0 ? nL : self, iU = nU >= 0 ? nU : self;
    float pxl, pyu;
    xc.two(px, iL, py, iU, pxl, pyu);
    float dd = div_p(px, nL >= 0 ? pxl : 0.0f, py, nU >= 0 ? pyu : 0.0f);
    float wv = w_of(dd, v, inv_theta, mine);
    const int steps = iters * inner;
    int left = inner;
    // checkpoints (inner = 1): the state before iteration k goes to tape
    // slot k / ce whenever ce divides k
    int to_ckpt = 0, slot = 0;
    for (int it = 0; it < steps; ++it) {
        if (tape && to_ckpt-- == 0) {
            to_ckpt = ce - 1;
            if (mine) {
                float* __restrict__ t = tape + (int64_t)slot * 3 * plane;
                t[gg] = v;
                t[plane + gg] = px;
                t[2 * plane + gg] = py;
            }
            ++slot;
        }
        float wr, wd;
        xc.same2(wv, iR, iD, wr, wd);
        const DualOut o = dual_update(px, py, wv, nR >= 0 ? wr : wR, nD >= 0 ? wd : wD, fl, tau);
        px = o.px;
        py = o.py;
        xc.two(px, iL, py, iU, pxl, pyu);
        dd = div_p(px, nL >= 0 ? pxl : 0.0f, py, nU >= 0 ? pyu : 0.0f);
        const bool last = (it == steps - 1);
        const bool outer_end = --left == 0;
        if (outer_end) {
            left = inner;
            const float u = u_step(v, dd, theta);
            v = v_step(u, c);
            if (last) {
                if (mine) d.u[gg] = u;
                break;
            }
        }
        wv = w_of(dd, v, inv_theta, mine);
    }
    if (mine) {
        d.st[0][0][gg] = v;
        d.st[0][1][gg] = px;
        d.st[0][2][gg] = py;
    }
}

// Waves of the packed one-wave classes taken by one caller: wave0, wave0 +
// stride, ... (uniform per wave); wave = packed group of components, lane =
// one pixel (or empty).
__device__ __forceinline__ void component_waves(const ImgDesc& d, const CompWs& w, int iters,
                                                int inner, float theta, float inv_theta,
                                                float tau, float* __restrict__ tape, int ce,
                                                int wave0, int stride) {
    const int64_t plane = (int64_t)d.H * d.ld;
    const int nwaves = (int)min((int64_t)class_base(w.ccount, kWaveClasses),
                                (2 * plane + kCompLaneExtra) / 64);
    const int lane = threadIdx.x & 63;
    WaveX xc;
    for (int wave = wave0; wave < nwaves; wave += stride)   // uniform per wave
        component_chain(d, w, xc, w.wl_pix[wave * 64 + lane], lane, wave * 64, iters, inner,
                        theta, inv_theta, tau, tape, ce);
}

// The group classes' jobs of a 256-thread workgroup: job j is two components
// of class 7 (128 lanes each) for j < ceil(ccount[7] / 2), else one of class
// 8.  For thread t it gives the packed lane of its pixel (wl_pix index; -1: no
// component) and the packed lane of the workgroup's thread 0 (exchange index
// = packed lane - that).
__device__ __forceinline__ int group_jobs(const int32_t* ccount) {
    return (ccount[7] + 1) / 2 + ccount[8];
}
__device__ __forceinline__ void group_lane(const int32_t* ccount, int job, int t, int& lane,
                                           int& base) {
    const int j7 = (ccount[7] + 1) / 2;
    if (job < j7) {
        const int comp = 2 * job + (t >> 7);
        const int first = class_base(ccount, 7) * 64 + 2 * job * 128;
        lane = comp < ccount[7] ? first + t : -1;
        base = first;
    } else {
        const int first = class_base(ccount, 8) * 64 + (job - j7) * 256;
        lane = first + t;
        base = first;
    }
}

// Jobs of the group classes taken by the 256-thread slices of one workgroup
// (blockDim.x a multiple of 256, xbuf 1024 floats a slice): workgroup wg of
// n_wg takes jobs (wg + r n_wg) slices + slice, r = 0, 1, ..., the same
// number of rounds in every slice (a slice past the last job runs an empty
// chain), so the slices pass the same workgroup barriers.
__device__ __forceinline__ void component_groups(const ImgDesc& d, const CompWs& w, int iters,
                                                 int inner, float theta, float inv_theta,
                                                 float tau, float* __restrict__ tape, int ce,
                                                 int wg, int n_wg, float* xbuf) {
    const int64_t plane = (int64_t)d.H * d.ld;
    const int njobs = group_jobs(w.ccount);
    const int64_t lanes = 2 * plane + kCompLaneExtra;
    const int slices = (int)(blockDim.x >> 8);
    const int slice = (int)(threadIdx.x >> 8);
    const int t = (int)(threadIdx.x & 255);
    const int per_round = n_wg * slices;
    const int rounds = (njobs + per_round - 1) / per_round;
    GroupX xc{xbuf + slice * 1024, 0, t};
    for (int r = 0; r < rounds; ++r) {   // uniform per workgroup
        const int job = (wg + r * n_wg) * slices + slice;
        int lane = -1, base = 0;
        if (job < njobs) group_lane(w.ccount, job, t, lane, base);
        const int g = (lane >= 0 && lane < lanes) ? w.wl_pix[lane] : -1;
        component_chain(d, w, xc, g, t, base, iters, inner, theta, inv_theta, tau, tape, ce);
        __syncthreads();   // the exchange buffers are reused by the next job
    }
}

}  // namespace rdseg
