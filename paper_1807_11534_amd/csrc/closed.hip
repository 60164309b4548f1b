// closed.hip -- every iteration of the closed 8x8 tiles in one launch.
//
// A tile is closed when none of its RD pixels has an RD 4-neighbour outside
// it (the work lists flag such tiles in macro tiles that hold no open tile).
// Its RD pixels then see nothing of the rest of the image but the constants of
// frozen neighbours, so one wave can run all of its iterations alone.
#include <atomic>
#include "rdseg_internal.h"

namespace rdseg {

namespace {

// Every iteration of one closed 8x8 tile per wave (64-thread workgroup), one
// pixel per lane (lane = 8 y + x).  A closed tile's RD pixels have no RD
// 4-neighbour outside the tile, so the only values they read from outside are
// the constants of frozen neighbours (p = 0, w = -H(-f)/theta): two per-lane
// constants (w right of x = 7 and below y = 7) stand for the ring.  (An RD
// pixel of the ring belongs to another component and is never read by this
// tile's RD pixels; it is held as a frozen cell.)  Neighbours inside the tile
// come from other lanes: x +/- 1 by DPP row shifts, y +/- 1 by wave shuffles,
// so the iterations run without LDS or barriers and each costs a short chain
// of cross-lane moves and arithmetic.  The per-pixel arithmetic is that of
// k_iterate, so results are bitwise equal.
__device__ __forceinline__ float lane_next(float a) {   // lane + 1 within a row of 16
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), 0x101, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_prev(float a) {   // lane - 1 within a row of 16
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), 0x111, 0xf, 0xf, false));
}

template <bool BATCHED>
__global__ __launch_bounds__(64) void k_closed(ImgDesc d0, const ImgDesc* __restrict__ descs,
                                               const int2* __restrict__ cqueue,
                                               const int32_t* __restrict__ n_closed, int iters,
                                               int inner, float theta, float inv_theta,
                                               float tau) {
    const int lane = threadIdx.x;
    const int x = lane & 7, y = lane >> 3;
    const int n = *n_closed;
    for (int item = blockIdx.x; item < n; item += gridDim.x) {
        const int2 q = cqueue[item];
        const ImgDesc& d = BATCHED ? descs[q.x] : d0;
        const int ty = q.y / d.tw;
        const int tx = q.y - ty * d.tw;
        const int gx = tx * 8 + x, gy = ty * 8 + y;
        const bool inb = gx < d.W && gy < d.H;
        const int g = gy * d.ld + gx;
        // a batch keeps no c plane: c from f (the function that fills it)
        auto c_at = [&](int gg) { return BATCHED ? c_of(d.f[gg], d.delta, d.tl) : d.c[gg]; };
        const float c = inb ? c_at(g) : __builtin_inff();
        const bool act = c_active(c);
        float v = heav_from_c(c), px = 0.0f, py = 0.0f;
        if (act) {
            v = d.st[0][0][g];
            px = d.st[0][1][g];
            py = d.st[0][2][g];
        }
        uint32_t fl = act ? (CF_ACT | CF_OUT) : 0u;
        if (gx == d.W - 1) fl |= CF_LASTC;
        if (gy == d.H - 1) fl |= CF_LASTR;
        // w of the ring cells right of x = 7 and below y = 7 (frozen)
        float wR = 0.0f, wD = 0.0f;
        if (x == 7) {
            float cr = (gx + 1 < d.W && gy < d.H) ? c_at(g + 1) : __builtin_inff();
            if (c_active(cr)) cr = __builtin_inff();
            wR = w_of(0.0f, heav_from_c(cr), inv_theta, false);
        }
        if (y == 7) {
            float cd = (gx < d.W && gy + 1 < d.H) ? c_at(g + d.ld) : __builtin_inff();
            if (c_active(cd)) cd = __builtin_inff();
            wD = w_of(0.0f, heav_from_c(cd), inv_theta, false);
        }
        float pxl = lane_prev(px), pyu = __shfl_up(py, 8);
        float dd = div_p(px, x == 0 ? 0.0f : pxl, py, y == 0 ? 0.0f : pyu);
        float w = w_of(dd, v, inv_theta, act);
        const int steps = iters * inner;
        int left = inner;   // dual steps left in the current outer iteration
        for (int it = 0; it < steps; ++it) {
            const float wr = lane_next(w), wd = __shfl_down(w, 8);
            const DualOut o = dual_update(px, py, w, x == 7 ? wR : wr, y == 7 ? wD : wd, fl, tau);
            px = o.px;
            py = o.py;
            pxl = lane_prev(px);
            pyu = __shfl_up(py, 8);
            dd = div_p(px, x == 0 ? 0.0f : pxl, py, y == 0 ? 0.0f : pyu);
            const bool last = (it == steps - 1);
            const bool outer_end = --left == 0;
            if (outer_end) {
                left = inner;
                const float u = u_step(v, dd, theta);
                v = v_step(u, c);
                if (last) {
                    if (fl & CF_OUT) d.u[g] = u;
                    break;
                }
            }
            w = w_of(dd, v, inv_theta, act);
        }
        if (fl & CF_OUT) {
            d.st[0][0][g] = v;
            d.st[0][1][g] = px;
            d.st[0][2][g] = py;
        }
    }
}

}  // namespace

// occupancy-derived grid sizes, filled on first use (any host thread)
std::atomic<int> g_closed_grid[2];

int prepare_closed(bool batched) {
    const void* fn = batched ? reinterpret_cast<const void*>(k_closed<true>)
                             : reinterpret_cast<const void*>(k_closed<false>);
    std::atomic<int>& cached = g_closed_grid[batched ? 1 : 0];
    if (cached.load(std::memory_order_relaxed) == 0) {
        const int b = persistent_blocks(fn, 64, 0);
        if (b <= 0) {
            set_error("occupancy query failed for the closed-tile kernel");
            return 4;
        }
        cached.store(b, std::memory_order_relaxed);
    }
    return 0;
}

int launch_closed(const ImgDesc* d0, const ImgDesc* descs, bool batched, const int2* cqueue,
                  const int32_t* n_closed, int64_t max_items, int iters, float theta,
                  float inv_theta, float tau, hipStream_t st, int inner) {
    if (prepare_closed(batched)) return 4;
    int64_t g = g_closed_grid[batched ? 1 : 0].load(std::memory_order_relaxed);
    if (max_items < g) g = max_items;
    if (g < 1) g = 1;
    if (batched)
        hipLaunchKernelGGL(k_closed<true>, dim3((unsigned)g), dim3(64), 0, st, *d0, descs, cqueue,
                           n_closed, iters, inner, theta, inv_theta, tau);
    else
        hipLaunchKernelGGL(k_closed<false>, dim3((unsigned)g), dim3(64), 0, st, *d0, descs, cqueue,
                           n_closed, iters, inner, theta, inv_theta, tau);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace rdseg
