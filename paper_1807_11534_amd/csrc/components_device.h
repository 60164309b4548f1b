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
// neighbours entering as constants.  The per-pixel functions are those of
// rdseg_device.h, so results are bitwise those of the tile kernels.
#pragma once

#include "rdseg_internal.h"

namespace rdseg {

constexpr int kSmallMax = 64;
constexpr int kClasses = 7;   // padded sizes 1, 2, 4, ..., 64
// Lanes used: a component of class k >= 1 has more than 2^(k-1) pixels and
// takes 2^k lanes, so all classes together take fewer than twice the pixels
// plus a partly filled last wave per class: wl_pix holds 2 * plane + kWlExtra.
constexpr int kWlExtra = kClasses * 64;

__device__ __forceinline__ bool cc_skip(const int64_t* npix, const ImgDesc& d) {
    return 100 * npix[0] > 55 * (int64_t)d.H * d.W;
}

// waves taken by the classes below k
__device__ __forceinline__ int class_base(const int32_t* ccount, int k) {
    int b = 0;
    for (int j = 0; j < k; ++j) {
        const int per = kSmallMax >> j;
        b += (ccount[j] + per - 1) / per;
    }
    return b;
}

// Waves of the packed components taken by one caller: wave0, wave0 + stride,
// ... (uniform per wave).  Every iteration of each: wave = packed group, lane =
// one pixel (or empty).  The u-step / v-step / dual step are those of
// k_iterate; x +/- 1 and y +/- 1 neighbours come from their lanes, frozen
// neighbours as constants (w right and below, p = 0 left and above).  Reads
// the start state from buffer 0 and leaves the final one there; writes u.
// With a tape (inner = 1, ce > 0) the state before iteration k goes to slot
// k / ce whenever ce divides k.
__device__ __forceinline__ void component_waves(const ImgDesc& d, const CompWs& w, int iters,
                                                int inner, float theta, float inv_theta,
                                                float tau, float* __restrict__ tape, int ce,
                                                int wave0, int stride) {
    const int64_t plane = (int64_t)d.H * d.ld;
    const int nwaves = (int)min((int64_t)class_base(w.ccount, kClasses),
                                (2 * plane + kWlExtra) / 64);
    const int lane = threadIdx.x & 63;
    for (int wave = wave0; wave < nwaves; wave += stride) {   // uniform per wave
        const int g = w.wl_pix[wave * 64 + lane];
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
                if (L >= 0) nR = L & 63;
                else wR = w_of(0.0f, heav_from_c(c_of(d.f[gg + 1], d.delta, d.tl)), inv_theta, false);
            } else {
                wR = w_of(0.0f, 0.0f, inv_theta, false);
            }
            if (y + 1 < d.H) {
                const int L = w.lane_of[gg + d.ld];
                if (L >= 0) nD = L & 63;
                else wD = w_of(0.0f, heav_from_c(c_of(d.f[gg + d.ld], d.delta, d.tl)), inv_theta, false);
            } else {
                wD = w_of(0.0f, 0.0f, inv_theta, false);
            }
            if (x > 0) {
                const int L = w.lane_of[gg - 1];
                if (L >= 0) nL = L & 63;
            }
            if (y > 0) {
                const int L = w.lane_of[gg - d.ld];
                if (L >= 0) nU = L & 63;
            }
        }
        // bpermute addresses (a lane reads itself when the neighbour is frozen)
        const int aR = 4 * (nR >= 0 ? nR : lane), aD = 4 * (nD >= 0 ? nD : lane);
        const int aL = 4 * (nL >= 0 ? nL : lane), aU = 4 * (nU >= 0 ? nU : lane);
        auto from = [](int addr, float a) {
            return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(a)));
        };
        float pxl = from(aL, px), pyu = from(aU, py);
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
            const float wr = from(aR, wv), wd = from(aD, wv);
            const DualOut o = dual_update(px, py, wv, nR >= 0 ? wr : wR, nD >= 0 ? wd : wD, fl, tau);
            px = o.px;
            py = o.py;
            pxl = from(aL, px);
            pyu = from(aU, py);
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
}

}  // namespace rdseg
