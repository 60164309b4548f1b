// iterate.hip -- initial state and the temporally blocked restricted iteration.
//
// The iteration kernel processes one macro tile (BX x BY pixels) of the
// compacted queue at a time.  It loads the macro tile plus a halo of IT + 1
// pixels on the left / top and IT on the right / bottom into LDS (p) and
// registers (v, c, flags), runs `nit` <= IT outer iterations entirely on chip,
// and writes back the macro tile's RD pixels.  Per iteration two barriers
// separate
//   phase B (dual step, reads w at x, x + e_x, x + e_y; writes p), and
//   phase A (u-step and v-step from div p at x, x - e_x, x - e_y; writes the
//           next w),
// so every on-chip value depends on cells at most one step away per phase.
// After n iterations p is exact n cells inside the loaded region on every
// side and v one more on the left / top, which is why that halo suffices;
// garbage computed at the region's border never reaches the macro tile.
//
// State is double-buffered in HBM (launch reads buffer `in_buf`, writes the
// other), so tiles never read a neighbour's halo while it is being written.
// Pixels off RD are never read from or written to the state buffers: their
// values (v = H(-f), p = 0) come from c = -/+inf.
#include <atomic>
#include "components_device.h"

namespace rdseg {

namespace {

__device__ __forceinline__ int find_image(const int64_t* off, int n, int64_t g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <bool BATCHED>
__global__ __launch_bounds__(256) void k_init(ImgDesc d0, const ImgDesc* __restrict__ descs,
                                              OffTables off, int n_img, int64_t n_rows) {
    for (int64_t R = blockIdx.x; R < n_rows; R += gridDim.x) {
        int img = BATCHED ? find_image(off.roff, n_img, R) : 0;
        const ImgDesc& d = BATCHED ? descs[img] : d0;
        int y = (int)(R - (BATCHED ? off.roff[img] : 0));
        for (int x = threadIdx.x; x < d.W; x += blockDim.x) {
            int g = y * d.ld + x;
            float fv = d.f[g];
            float c = c_of(fv, d.delta, d.tl);
            bool act = c_active(c);
            float h = (fv < 0.0f) ? 1.0f : 0.0f;
            float u0 = act ? (d.u0 ? d.u0[g] : h) : h;
            float v0 = v_step(u0, c);
            float px = (act && x < d.W - 1 && d.p0x) ? d.p0x[g] : 0.0f;
            float py = (act && y < d.H - 1 && d.p0y) ? d.p0y[g] : 0.0f;
            d.c[g] = c;
            if (!d.u) continue;   // c-only mode (used by the adjoint)
            d.u[g] = u0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                d.st[b][0][g] = v0;
                d.st[b][1][g] = px;
                d.st[b][2][g] = py;
            }
        }
    }
}

// The on-chip iterations.  Slot j of a thread is region cell t + j * NT in
// MODE_DENSE (every region cell, with per-cell selects for cells off RD and on
// the last column / row), MODE_DENSE_IN (the same for a region that holds no
// cell of the last column / row: the dual step runs select-free with a step of
// 0 on cells off RD, which leaves their p = 0 exactly) and MODE_FAST (every
// region cell is inside the grid, in RD and away from the last column / row:
// no selects), and the j-th entry
// of the block's ascending list of RD cells in MODE_COMPACT (idx[j] < 0: empty
// slot); there cells off RD are never visited: their p = 0 and
// w = -H(-f)/theta were stored in LDS when the region was loaded.
// STOP: ru holds u of the previous iteration on CF_OUT cells; with `check`,
// the last iteration folds max(|u - u_prev|, |v - v_prev|) of those cells into
// dmax (bit patterns of non-negative floats order like their values).
enum { MODE_DENSE = 0, MODE_FAST = 1, MODE_COMPACT = 2, MODE_DENSE_IN = 3 };

// TAPE: after outer iteration s of the call, the state (v, p_x, p_y) of the
// tile's RD cells is also written to tape + s * tape_step (planes tape_plane
// apart): the adjoint's recompute of a checkpoint segment.
template <int BX, int BY, int IT, int NT, int MODE, bool STOP, bool TAPE = false>
__device__ __forceinline__ void run_iterations(float* __restrict__ sPX, float* __restrict__ sPY,
                                               float* __restrict__ sW, const int* idx, float* rv,
                                               float* rpx, float* rpy, const float* rc,
                                               const uint32_t* fl, const int* gi,
                                               float* __restrict__ U, int nit, int write_u,
                                               float theta, float inv_theta, float tau, float* ru,
                                               bool check, uint32_t& dmax, int inner,
                                               float* __restrict__ tape = nullptr,
                                               int64_t tape_step = 0, int64_t tape_plane = 0) {
    constexpr int RX = BX + 2 * IT + 1;
    constexpr int RY = BY + 2 * IT + 1;
    constexpr int RC = RX * RY;
    constexpr int CPT = (RC + NT - 1) / NT;
    constexpr int PAD = RX + 1;
    const int t = threadIdx.x;
    // prologue: w from the loaded state
    {
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = MODE == MODE_COMPACT ? idx[j] : t + j * NT;
            if (MODE == MODE_COMPACT ? (i >= 0) : (i < RC)) {
                float dd = div_p(rpx[j], sPX[PAD + i - 1], rpy[j], sPY[PAD + i - RX]);
                sW[PAD + i] = w_of(dd, rv[j], inv_theta,
                                   (MODE == MODE_DENSE || MODE == MODE_DENSE_IN) ? (fl[j] & CF_ACT) != 0 : true);
            }
        }
    }
    __syncthreads();
    // nit outer iterations of `inner` dual steps each; between the dual steps
    // of one outer iteration phase A only refreshes w = div p - v/theta
    const int steps = nit * inner;
    int left = inner;   // dual steps left in the current outer iteration
    for (int it = 0; it < steps; ++it) {
        // phase B: dual step
        {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int i = MODE == MODE_COMPACT ? idx[j] : t + j * NT;
                if (MODE == MODE_COMPACT ? (i >= 0) : (i < RC)) {
                    const float wc = sW[PAD + i];
                    float npx, npy;
                    if (MODE == MODE_FAST || MODE == MODE_DENSE_IN) {
                        const float tc = (MODE == MODE_FAST || (fl[j] & CF_ACT)) ? tau : 0.0f;
                        const float gx = sW[PAD + i + 1] - wc;
                        const float gy = sW[PAD + i + RX] - wc;
                        const float nn = __builtin_amdgcn_sqrtf(fmaf(gx, gx, gy * gy));
                        const float m = __builtin_amdgcn_rcpf(fmaf(tc, nn, 1.0f));
                        npx = fmaf(tc, gx, rpx[j]) * m;
                        npy = fmaf(tc, gy, rpy[j]) * m;
                    } else {
                        DualOut o = dual_update(rpx[j], rpy[j], wc, sW[PAD + i + 1],
                                                sW[PAD + i + RX], fl[j], tau);
                        npx = o.px;
                        npy = o.py;
                    }
                    rpx[j] = npx;
                    rpy[j] = npy;
                    sPX[PAD + i] = npx;
                    sPY[PAD + i] = npy;
                }
            }
        }
        __syncthreads();
        // phase A: u-step, v-step, next w (w alone inside an outer iteration)
        const bool last = (it == steps - 1);
        if (--left > 0) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int i = MODE == MODE_COMPACT ? idx[j] : t + j * NT;
                if (MODE == MODE_COMPACT ? (i >= 0) : (i < RC)) {
                    float dd = div_p(rpx[j], sPX[PAD + i - 1], rpy[j], sPY[PAD + i - RX]);
                    sW[PAD + i] = w_of(dd, rv[j], inv_theta,
                                       (MODE == MODE_DENSE || MODE == MODE_DENSE_IN) ? (fl[j] & CF_ACT) != 0 : true);
                }
            }
        } else {
            left = inner;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int i = MODE == MODE_COMPACT ? idx[j] : t + j * NT;
                if (MODE == MODE_COMPACT ? (i >= 0) : (i < RC)) {
                    float dd = div_p(rpx[j], sPX[PAD + i - 1], rpy[j], sPY[PAD + i - RX]);
                    float u = u_step(rv[j], dd, theta);
                    const float vn = v_step(u, rc[j]);
                    if (STOP) {
                        if (last && check && (fl[j] & CF_OUT)) {
                            const uint32_t a = __float_as_uint(fabsf(u - ru[j]));
                            const uint32_t b = __float_as_uint(fabsf(vn - rv[j]));
                            dmax = max(dmax, max(a, b));
                        }
                        ru[j] = u;
                    }
                    rv[j] = vn;
                    if (TAPE && (fl[j] & CF_OUT)) {
                        float* __restrict__ ts = tape + (int64_t)(it / inner) * tape_step + gi[j];
                        ts[0] = vn;
                        ts[tape_plane] = rpx[j];
                        ts[2 * tape_plane] = rpy[j];
                    }
                    if (last) {
                        if (write_u && (fl[j] & CF_OUT)) U[gi[j]] = u;
                    } else {
                        sW[PAD + i] = w_of(dd, rv[j], inv_theta,
                                           (MODE == MODE_DENSE || MODE == MODE_DENSE_IN) ? (fl[j] & CF_ACT) != 0 : true);
                    }
                }
            }
        }
        if (!last) __syncthreads();
    }
}

// Per-cell flags of region cell (rx, ry) at grid position (gx, gy).
template <int BX, int BY, int IT>
__device__ __forceinline__ uint32_t cell_flags(bool act, int rx, int ry, int gx, int gy, int W,
                                               int H) {
    constexpr int H0 = IT + 1;
    uint32_t f = act ? CF_ACT : 0u;
    if (gx == W - 1) f |= CF_LASTC;
    if (gy == H - 1) f |= CF_LASTR;
    const bool interior = rx >= H0 && rx < H0 + BX && ry >= H0 && ry < H0 + BY;
    if (interior && act) f |= CF_OUT;
    return f;
}

// FAST_OK: whether this instantiation carries the select-free variant for
// tiles that lie inside the grid and inside RD (worth it for large tiles, where
// such tiles dominate).  COMPACT_OK (the smaller tiles, chosen for sparse
// bands): a tile whose region is less than 40 % RD runs on its compacted RD
// cells (the 64-wide tiles serve dense images and skip this machinery, which
// costs them a few per cent of LDS traffic and barriers): wave ballots of
// the RD flags, a scan of the per-wave counts and a scatter give the ascending
// list of RD cells, and the threads take the listed cells in order, so the
// work per iteration follows the number of RD cells.  Listed cells are
// gathered from LDS (scattered addresses, bank conflicts), which costs about
// 2.4x a dense cell, so denser tiles run every region cell with selects.  The
// arithmetic per cell is the same in every variant, so the results do not
// depend on which one ran.
//
// STOP (single image, convergence-driven solve): a launch whose skip_slot
// already holds a change <= tol does nothing (the solve has converged at an
// earlier check; slots of checks that never ran stay 0); otherwise u of the
// previous iteration is loaded with the state, and with diff_slot non-NULL the
// last iteration's max(|u - u_prev|, |v - v_prev|) over RD is reduced into
// *diff_slot (one atomicMax per wave).
// One launch's work (the kernel below; the persistent form runs it once per
// block of iterations).
template <int BX, int BY, int IT, int NT, bool BATCHED, bool STOP, bool FAST_OK, bool COMPACT_OK,
          bool TAPE = false>
__device__ __forceinline__ void iterate_pass(ImgDesc d0, const ImgDesc* __restrict__ descs,
                                             const int2* __restrict__ queue,
                                             const int32_t* __restrict__ n_queue, int in_buf,
                                             int nit, int write_u, float theta, float inv_theta,
                                             float tau, const uint32_t* __restrict__ skip_slot,
                                             uint32_t* __restrict__ diff_slot, double tol,
                                             int inner, float* __restrict__ tape = nullptr,
                                             int64_t tape_step = 0, int64_t tape_plane = 0) {
    if (STOP && skip_slot && (double)__uint_as_float(*skip_slot) <= tol) return;
    constexpr int RX = BX + 2 * IT + 1;
    constexpr int RY = BY + 2 * IT + 1;
    constexpr int RC = RX * RY;
    constexpr int CPT = (RC + NT - 1) / NT;
    constexpr int PAD = RX + 1;
    constexpr int LS = RC + 2 * PAD;
    constexpr int H0 = IT + 1;   // left / top halo
    constexpr int NW = NT / 64;  // waves per workgroup
    constexpr int NCNT = CPT * NW;
    static_assert(NT % 64 == 0 && NCNT <= 128, "the count scan covers at most 128 entries");
    static_assert(RC < 32768, "region index must fit the 16-bit cell list");
    __shared__ float sPX[LS];
    __shared__ float sPY[LS];
    __shared__ float sW[LS];
    __shared__ float sC[COMPACT_OK ? RC : 1];
    __shared__ uint16_t sList[COMPACT_OK ? RC : 1];
    __shared__ int sCnt[COMPACT_OK ? NCNT + 1 : 1];

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = t >> 6;
    for (int k = t; k < PAD; k += NT) {
        sPX[k] = 0.0f; sPY[k] = 0.0f; sW[k] = 0.0f;
        sPX[PAD + RC + k] = 0.0f; sPY[PAD + RC + k] = 0.0f; sW[PAD + RC + k] = 0.0f;
    }

    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of the ascending queue so that neighbouring macro tiles
    // (which re-read each other's halos) share that XCD's L2.
    const int nq = *n_queue;
    const int per = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7;
    const int rank = blockIdx.x >> 3;
    const int chunk = (nq + 7) >> 3;
    const int q0 = xcd * chunk;
    const int q1 = min(nq, q0 + chunk);
    const int out_buf = 1 - in_buf;
    const bool check = STOP && diff_slot != nullptr;
    uint32_t dmax = 0u;

    for (int item = q0 + rank; item < q1; item += per) {
        const int2 q = queue[item];
        const ImgDesc& d = BATCHED ? descs[q.x] : d0;
        const int my = q.y / d.mw;
        const int mx = q.y - my * d.mw;
        const int ox = mx * BX - H0;
        const int oy = my * BY - H0;
        const int W = d.W, H = d.H, ld = d.ld;
        const float* __restrict__ C = d.c;
        const float* __restrict__ Vi = d.st[in_buf][0];
        const float* __restrict__ PXi = d.st[in_buf][1];
        const float* __restrict__ PYi = d.st[in_buf][2];

        float rv[CPT], rpx[CPT], rpy[CPT], rc[CPT];
        float ru[STOP ? CPT : 1];
        uint32_t fl[CPT];
        int gi[CPT];
        int idx[CPT];
        uint64_t amask[CPT];

        __syncthreads();   // LDS of the previous item fully consumed
        int plain = 1;     // every cell inside the grid, in RD, off the last column / row
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            rv[j] = 0.0f; rpx[j] = 0.0f; rpy[j] = 0.0f; rc[j] = __builtin_inff();
            fl[j] = 0u; gi[j] = 0;
            bool act = false;
            if (i < RC) {
                const int ry = i / RX;
                const int rx = i - ry * RX;
                const int gx = ox + rx, gy = oy + ry;
                const bool inb = (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H;
                const int g = gy * ld + gx;
                gi[j] = g;
                // all loads of the cell are issued together (one memory round
                // trip); state read off RD is discarded by the selects below
                float c = __builtin_inff(), v = 0.0f, px = 0.0f, py = 0.0f, uo = 0.0f;
                if (inb) {
                    // a batch keeps no c plane: c from f (the same function
                    // that fills the plane of a single image)
                    c = BATCHED ? c_of(d.f[g], d.delta, d.tl) : C[g];
                    v = Vi[g];
                    px = PXi[g];
                    py = PYi[g];
                    if (STOP) uo = d.u[g];
                }
                act = c_active(c);
                rc[j] = c;
                rv[j] = act ? v : heav_from_c(c);
                rpx[j] = act ? px : 0.0f;
                rpy[j] = act ? py : 0.0f;
                const uint32_t f = cell_flags<BX, BY, IT>(act, rx, ry, gx, gy, W, H);
                fl[j] = f;
                if (STOP) ru[j] = (f & CF_OUT) ? uo : 0.0f;
                plain &= (act && !(f & (CF_LASTC | CF_LASTR))) ? 1 : 0;
                sPX[PAD + i] = rpx[j];
                sPY[PAD + i] = rpy[j];
                if (COMPACT_OK) {
                    // RD cells park v here until the prologue writes their w;
                    // other cells hold their constant w = -H(-f)/theta
                    sW[PAD + i] = act ? rv[j] : w_of(0.0f, rv[j], inv_theta, false);
                    sC[i] = c;
                }
            }
            if (COMPACT_OK) amask[j] = __ballot(act);
        }
        bool fast = false;
        if (FAST_OK) fast = __syncthreads_and(plain) != 0;
        else __syncthreads();
        // does the region reach the grid's last column or row?
        const bool edge = ox + RX >= W || oy + RY >= H;
        if (fast) {
            run_iterations<BX, BY, IT, NT, MODE_FAST, STOP, TAPE>(sPX, sPY, sW, idx, rv, rpx, rpy, rc,
                                                            fl, gi, d.u, nit, write_u, theta,
                                                            inv_theta, tau, ru, check, dmax, inner, tape, tape_step, tape_plane);
        } else if (!COMPACT_OK) {
            if (edge)
                run_iterations<BX, BY, IT, NT, MODE_DENSE, STOP, TAPE>(sPX, sPY, sW, idx, rv, rpx, rpy,
                                                                 rc, fl, gi, d.u, nit, write_u,
                                                                 theta, inv_theta, tau, ru,
                                                                 check, dmax, inner, tape, tape_step, tape_plane);
            else
                run_iterations<BX, BY, IT, NT, MODE_DENSE_IN, STOP, TAPE>(sPX, sPY, sW, idx, rv, rpx,
                                                                    rpy, rc, fl, gi, d.u, nit,
                                                                    write_u, theta, inv_theta,
                                                                    tau, ru, check, dmax, inner, tape, tape_step, tape_plane);
        } else {
            // count the RD cells of the region (ascending list offsets)
            if (lane == 0) {
#pragma unroll
                for (int j = 0; j < CPT; ++j) sCnt[j * NW + wv] = __popcll(amask[j]);
            }
            __syncthreads();
            if (wv == 0) {   // exclusive scan of the NCNT counts, two per lane
                const int e0 = 2 * lane < NCNT ? sCnt[2 * lane] : 0;
                const int e1 = 2 * lane + 1 < NCNT ? sCnt[2 * lane + 1] : 0;
                const int s = e0 + e1;
                int incl = s;
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(incl, o);
                    if (lane >= o) incl += y;
                }
                const int excl = incl - s;
                if (2 * lane < NCNT) sCnt[2 * lane] = excl;
                if (2 * lane + 1 < NCNT) sCnt[2 * lane + 1] = excl + e0;
                if (lane == 63) sCnt[NCNT] = incl;
            }
            __syncthreads();
            const int n_act = sCnt[NCNT];
            if (5 * n_act >= 2 * RC) {   // dense enough: every region cell
                if (edge)
                    run_iterations<BX, BY, IT, NT, MODE_DENSE, STOP, TAPE>(sPX, sPY, sW, idx, rv, rpx,
                                                                     rpy, rc, fl, gi, d.u, nit,
                                                                     write_u, theta, inv_theta,
                                                                     tau, ru, check, dmax, inner, tape, tape_step, tape_plane);
                else
                    run_iterations<BX, BY, IT, NT, MODE_DENSE_IN, STOP, TAPE>(
                        sPX, sPY, sW, idx, rv, rpx, rpy, rc, fl, gi, d.u, nit, write_u, theta,
                        inv_theta, tau, ru, check, dmax, inner, tape, tape_step, tape_plane);
            } else {
                const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
                for (int j = 0; j < CPT; ++j) {
                    if ((amask[j] >> lane) & 1ull)
                        sList[sCnt[j * NW + wv] + __popcll(amask[j] & below)] =
                            (uint16_t)(t + j * NT);
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < CPT; ++j) {
                    const int k = t + j * NT;
                    idx[j] = -1;
                    fl[j] = 0u;
                    if (k < n_act) {
                        const int i = sList[k];
                        const int ry = i / RX;
                        const int rx = i - ry * RX;
                        const int gx = ox + rx, gy = oy + ry;
                        const int g = gy * ld + gx;
                        idx[j] = i;
                        gi[j] = g;
                        rv[j] = sW[PAD + i];
                        rpx[j] = sPX[PAD + i];
                        rpy[j] = sPY[PAD + i];
                        rc[j] = sC[i];
                        const uint32_t f = cell_flags<BX, BY, IT>(true, rx, ry, gx, gy, W, H);
                        fl[j] = f;
                        if (STOP) ru[j] = (f & CF_OUT) ? d.u[g] : 0.0f;
                    }
                }
                __syncthreads();   // parked v read before the prologue overwrites it
                run_iterations<BX, BY, IT, NT, MODE_COMPACT, STOP, TAPE>(sPX, sPY, sW, idx, rv, rpx, rpy,
                                                                   rc, fl, gi, d.u, nit, write_u,
                                                                   theta, inv_theta, tau, ru,
                                                                   check, dmax, inner, tape, tape_step, tape_plane);
            }
        }
        float* __restrict__ Vo = d.st[out_buf][0];
        float* __restrict__ PXo = d.st[out_buf][1];
        float* __restrict__ PYo = d.st[out_buf][2];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if (fl[j] & CF_OUT) {
                Vo[gi[j]] = rv[j];
                PXo[gi[j]] = rpx[j];
                PYo[gi[j]] = rpy[j];
            }
        }
    }
    if (check) {
        for (int o = 32; o > 0; o >>= 1) dmax = max(dmax, (uint32_t)__shfl_xor((int)dmax, o));
        if ((threadIdx.x & 63) == 0 && dmax) atomicMax(diff_slot, dmax);
    }
}

template <int BX, int BY, int IT, int NT, bool BATCHED, bool STOP, bool FAST_OK = (BX >= 64),
          bool COMPACT_OK = (BX < 64)>
__global__ __launch_bounds__(NT) void k_iterate(ImgDesc d0, const ImgDesc* __restrict__ descs,
                                                const int2* __restrict__ queue,
                                                const int32_t* __restrict__ n_queue, int in_buf,
                                                int nit, int write_u, float theta,
                                                float inv_theta, float tau,
                                                const uint32_t* __restrict__ skip_slot,
                                                uint32_t* __restrict__ diff_slot, double tol,
                                                int inner) {
    iterate_pass<BX, BY, IT, NT, BATCHED, STOP, FAST_OK, COMPACT_OK>(
        d0, descs, queue, n_queue, in_buf, nit, write_u, theta, inv_theta, tau, skip_slot,
        diff_slot, tol, inner);
}

// The adjoint's recompute of a checkpoint segment: `nit` outer iterations of
// the single-image blocked kernel from state buffer in_buf, with the state
// after each iteration s written to tape + s * tape_step (the segment's slots)
// for the queued tiles' RD pixels; the arithmetic and buffer parities of
// k_iterate, so the states are bitwise those of single-step launches.
template <int BX, int BY, int IT, int NT>
__global__ __launch_bounds__(NT) void k_recompute(ImgDesc d0, const int2* __restrict__ queue,
                                                  const int32_t* __restrict__ n_queue,
                                                  int in_buf, int nit, float theta,
                                                  float inv_theta, float tau,
                                                  float* __restrict__ tape, int64_t tape_step,
                                                  int64_t tape_plane) {
    iterate_pass<BX, BY, IT, NT, false, false, (BX >= 64), (BX < 64), true>(
        d0, nullptr, queue, n_queue, in_buf, nit, 0, theta, inv_theta, tau, nullptr, nullptr,
        0.0, 1, tape, tape_step, tape_plane);
}

// Grid-wide barrier of a cooperative launch: every workgroup adds one to
// *bar (a counter that starts at 0 and only grows), then waits until it reads
// gen * gridDim.x.  Every thread first waits until its own stores have
// completed (s_waitcnt 0: the workgroup barrier alone does not wait for
// them, and a store that reaches the XCD's L2 after thread 0's write-back
// would stay there, unseen by the other XCDs); then thread 0's release fence
// writes the L2 back before the arrival, and its acquire fence after the wait
// invalidates it, so the state buffers written before the barrier are ordered
// against the loads after it, as at a kernel boundary.  The wait is bounded
// (wait_ticks of the 100 MHz wall clock; < 0 gives up at once): on expiry the
// workgroup sets *status and returns false.
__device__ __forceinline__ bool grid_barrier(int32_t* bar, int gen, int64_t wait_ticks,
                                             int32_t* status) {
    __shared__ int sOk;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t target = gen * (int32_t)gridDim.x;
        const uint64_t t0 = wall_clock64();
        int ok = 1;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (wait_ticks < 0 || wall_clock64() - t0 > (uint64_t)wait_ticks) {
                ok = 0;
                __hip_atomic_store(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        sOk = ok;
    }
    __syncthreads();
    return sOk != 0;
}

// The macro tiles a workgroup takes in iterate_pass (the same XCD-chunked
// split of the queue) marked as failed: NaN in u, v and p of every pixel of
// the tile.
template <int BX, int BY, int NT>
__device__ void mark_failed_tiles(const ImgDesc* __restrict__ descs,
                                  const int2* __restrict__ queue,
                                  const int32_t* __restrict__ n_queue) {
    const int nq = *n_queue;
    const int per = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7;
    const int rank = blockIdx.x >> 3;
    const int chunk = (nq + 7) >> 3;
    const int q0 = xcd * chunk;
    const int q1 = min(nq, q0 + chunk);
    const float nan = __builtin_nanf("");
    for (int item = q0 + rank; item < q1; item += per) {
        const int2 q = queue[item];
        const ImgDesc& d = descs[q.x];
        const int my = q.y / d.mw;
        const int mx = q.y - my * d.mw;
        for (int k = threadIdx.x; k < BX * BY; k += NT) {
            const int x = mx * BX + k % BX, y = my * BY + k / BX;
            if (x >= d.W || y >= d.H) continue;
            const int64_t g = (int64_t)y * d.ld + x;
            d.u[g] = nan;
            d.st[0][0][g] = nan;
            d.st[0][1][g] = nan;
            d.st[0][2][g] = nan;
        }
    }
}

// Persistent form of the batched iteration: one cooperative launch runs every
// block of `per` outer iterations over the global (image, macro tile) queue,
// exactly the work and buffer parities of the L = ceil(iters / per) separate
// launches, with a grid-wide barrier in place of each kernel boundary (so the
// results are bitwise those of the separate launches).  An empty queue ends
// the launch at once.  A barrier whose wait expires stops the workgroup: the
// solve's status word is set and the workgroup writes NaN into u, v and p of
// its macro tiles, so that the incomplete result cannot pass for a solution
// (the other workgroups' waits then expire too, or they read those NaN in
// their halos).
template <int BX, int BY, int IT, int NT>
__global__ __launch_bounds__(NT) void k_iterate_persist(ImgDesc d0,
                                                        const ImgDesc* __restrict__ descs,
                                                        const int2* __restrict__ queue,
                                                        const int32_t* __restrict__ n_queue,
                                                        int iters, int per, float theta,
                                                        float inv_theta, float tau,
                                                        int32_t* __restrict__ bar,
                                                        int32_t* __restrict__ status,
                                                        int64_t wait_ticks) {
    if (*n_queue == 0) return;   // the same value for every workgroup
    const int L = (iters + per - 1) / per;
    for (int j = 0; j < L; ++j) {
        const int nit = min(per, iters - j * per);
        iterate_pass<BX, BY, IT, NT, true, false, (BX >= 64), (BX < 64)>(
            d0, descs, queue, n_queue, (L - j) & 1, nit, j == L - 1 ? 1 : 0, theta, inv_theta,
            tau, nullptr, nullptr, 0.0, 1);
        if (j < L - 1 && !grid_barrier(bar, j + 1, wait_ticks, status)) {
            mark_failed_tiles<BX, BY, NT>(descs, queue, n_queue);
            return;
        }
    }
}

// Resident variant of the blocked iteration (single image, no checkpoint
// tape, no stopping rule), for images whose queued macro tiles fit on the
// chip at once (a cooperative launch guarantees that every workgroup is
// resident).  Each workgroup loads its macro tile's region once and keeps it
// in registers and LDS for the whole solve: after every block of `per` outer
// iterations it writes the frame of its macro tile that the neighbours' halos
// cover (the IT + 1 outermost rows and columns; everything at the last block)
// to the state buffer the equivalent separate launch would write, publishes
// the block count in epoch[m], waits until each of its up to 8 queued
// neighbours has published the same count, and reloads only its halo ring
// from that buffer.  Values and buffer parities are those of the separate
// launches, so the results are bitwise equal.  A neighbour that is not queued
// holds no open RD tile; its pixels belong to other components than this
// tile's RD pixels, so they are not waited for.
//
// Ordering without cache-wide fences: frame values are written and the ring
// is read with device-scope atomic stores and loads, which the hardware keeps
// coherent across the XCDs' L2 caches (they do not stay in, or hit stale
// lines of, one XCD's L2).  Each thread waits for its frame stores to complete
// (s_waitcnt 0) before the barrier after which thread 0 stores the count, and
// the ring loads are issued only after the waiting lanes have read the
// neighbours' counts and the workgroup has passed a barrier.  (Release and
// acquire fences at device scope would write back and invalidate the whole
// L2 of the XCD at every block, which costs more than a separate launch.)
// This ordering rests on gfx950's memory system (device-scope atomics bypass
// the non-coherent L2 lines; s_waitcnt 0 covers the completion of stores), not
// on the HIP memory model alone, so the kernel is built for gfx950 only.
//
// Every wait is bounded in time (wait_ticks of the 100 MHz wall clock; < 0:
// each wait gives up at once, a failure the host can force to test this
// path).  On expiry the workgroup sets *status, publishes the epoch value -1
// and stops: it writes NaN for u, v and p of its tile and publishes nothing
// more.  A neighbour waiting for it sees -1 and stops the same way, so every
// tile that would have read a frame computed from a stale ring holds NaN,
// every other tile holds its exact result, and a solve can never hang.
#if !defined(__gfx950__) && defined(__HIP_DEVICE_COMPILE__)
#error "k_resident's cross-workgroup ordering is written for gfx950"
#endif
constexpr int32_t kEpochFailed = -1;

template <int BX, int BY, int IT, int NT>
__global__ __launch_bounds__(NT) void k_resident(ImgDesc d, const int2* __restrict__ queue,
                                                 const int32_t* __restrict__ n_queue,
                                                 const int32_t* __restrict__ mflags,
                                                 int32_t* __restrict__ epoch,
                                                 int32_t* __restrict__ status, int in_buf,
                                                 int iters, int per, int inner, float theta,
                                                 float inv_theta, float tau, CompWs cw,
                                                 const int64_t* __restrict__ cnpix, int citers,
                                                 int64_t wait_ticks) {
    constexpr int RX = BX + 2 * IT + 1;
    constexpr int RY = BY + 2 * IT + 1;
    constexpr int RC = RX * RY;
    constexpr int CPT = (RC + NT - 1) / NT;
    constexpr int PAD = RX + 1;
    constexpr int LS = RC + 2 * PAD;
    constexpr int H0 = IT + 1;
    __shared__ float sPX[LS];
    __shared__ float sPY[LS];
    __shared__ float sW[LS];
    __shared__ int sFail;
    __shared__ float sGrp[NT / 256 * 1024];   // idle workgroups: the group classes' exchange
    static_assert(NT % 256 == 0, "idle workgroups run the group classes in 256-thread slices");

    const int t = threadIdx.x;
    // the same XCD-contiguous assignment of queue items as the launched kernel
    const int nq = *n_queue;
    const int xcd = blockIdx.x & 7;
    const int rank = blockIdx.x >> 3;
    const int chunk = (nq + 7) >> 3;
    const int item = xcd * chunk + rank;
    if (rank >= chunk || item >= nq) {   // no tile for this workgroup
        // With citers > 0 the idle workgroups (the grid holds one per macro
        // tile of the image, or the queued tiles and some more, the queue only
        // the tiles left to the tile path) run the component path's
        // iterations beside the tiles, the group classes in 256-thread slices
        // and then the packed waves, and flag that they did (ccount[kCompFlag],
        // cleared by the labelling).  Workgroup ids among the idle ones: XCD
        // by XCD, ranks past that XCD's tiles.
        if (citers > 0 && !cc_skip(cnpix, d)) {
            const int per_x = (int)gridDim.x >> 3;
            auto tiles_of = [&](int x) { return max(0, min(chunk, nq - x * chunk)); };
            int gid = rank - tiles_of(xcd);
            for (int x = 0; x < xcd; ++x) gid += per_x - tiles_of(x);
            const int idle = (int)gridDim.x - nq;
            if (gid == 0 && t == 0) cw.ccount[kCompFlag] = 1;
            component_groups(d, cw, citers, inner, theta, inv_theta, tau, nullptr, 0, gid, idle,
                             sGrp);
            component_waves(d, cw, citers, inner, theta, inv_theta, tau, nullptr, 0,
                            gid * (NT / 64) + (t >> 6), idle * (NT / 64));
        }
        return;   // the whole workgroup leaves together
    }

    for (int k = t; k < PAD; k += NT) {
        sPX[k] = 0.0f; sPY[k] = 0.0f; sW[k] = 0.0f;
        sPX[PAD + RC + k] = 0.0f; sPY[PAD + RC + k] = 0.0f; sW[PAD + RC + k] = 0.0f;
    }
    if (t == 0) sFail = 0;
    const int2 q = queue[item];
    const int m = q.y;
    const int my = m / d.mw;
    const int mx = m - my * d.mw;
    const int ox = mx * BX - H0;
    const int oy = my * BY - H0;
    const int W = d.W, H = d.H, ld = d.ld;

    float rv[CPT], rpx[CPT], rpy[CPT], rc[CPT];
    float ru[1];
    uint32_t fl[CPT];
    int gi[CPT];
    int idx[CPT];
    uint32_t ring = 0u;   // bit j: slot j is a halo cell inside the grid
    uint32_t frame = 0u;  // bit j: slot j is an RD cell of the macro tile a neighbour reads
    int plain = 1;
    {
        const float* __restrict__ Vi = d.st[in_buf][0];
        const float* __restrict__ PXi = d.st[in_buf][1];
        const float* __restrict__ PYi = d.st[in_buf][2];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            rv[j] = 0.0f; rpx[j] = 0.0f; rpy[j] = 0.0f; rc[j] = __builtin_inff();
            fl[j] = 0u; gi[j] = 0; idx[j] = i;
            if (i < RC) {
                const int ry = i / RX;
                const int rx = i - ry * RX;
                const int gx = ox + rx, gy = oy + ry;
                const bool inb = (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H;
                const int g = gy * ld + gx;
                gi[j] = g;
                float c = __builtin_inff(), v = 0.0f, px = 0.0f, py = 0.0f;
                if (inb) {
                    c = d.c[g];
                    v = Vi[g];
                    px = PXi[g];
                    py = PYi[g];
                }
                const bool act = c_active(c);
                rc[j] = c;
                rv[j] = act ? v : heav_from_c(c);
                rpx[j] = act ? px : 0.0f;
                rpy[j] = act ? py : 0.0f;
                const uint32_t f = cell_flags<BX, BY, IT>(act, rx, ry, gx, gy, W, H);
                fl[j] = f;
                plain &= (act && !(f & (CF_LASTC | CF_LASTR))) ? 1 : 0;
                const int xi = rx - H0, yi = ry - H0;
                const bool interior = xi >= 0 && xi < BX && yi >= 0 && yi < BY;
                if (!interior && inb) ring |= 1u << j;
                if ((f & CF_OUT) && (xi <= IT || xi >= BX - IT - 1 || yi <= IT || yi >= BY - IT - 1))
                    frame |= 1u << j;
                sPX[PAD + i] = rpx[j];
                sPY[PAD + i] = rpy[j];
            }
        }
    }
    const bool fast = __syncthreads_and(plain) != 0;
    const bool edge = ox + RX >= W || oy + RY >= H;
    uint32_t dmax = 0u;
    const int nb = (iters + per - 1) / per;
    for (int b = 0; b < nb; ++b) {
        const int nit = min(per, iters - b * per);
        const bool lastb = b == nb - 1;
        const int wu = lastb ? 1 : 0;
        if (fast)
            run_iterations<BX, BY, IT, NT, MODE_FAST, false>(sPX, sPY, sW, idx, rv, rpx, rpy, rc,
                                                             fl, gi, d.u, nit, wu, theta,
                                                             inv_theta, tau, ru, false, dmax,
                                                             inner);
        else if (edge)
            run_iterations<BX, BY, IT, NT, MODE_DENSE, false>(sPX, sPY, sW, idx, rv, rpx, rpy,
                                                              rc, fl, gi, d.u, nit, wu, theta,
                                                              inv_theta, tau, ru, false, dmax,
                                                              inner);
        else
            run_iterations<BX, BY, IT, NT, MODE_DENSE_IN, false>(sPX, sPY, sW, idx, rv, rpx,
                                                                 rpy, rc, fl, gi, d.u, nit, wu,
                                                                 theta, inv_theta, tau, ru,
                                                                 false, dmax, inner);
        const int xb = (in_buf + b + 1) & 1;   // the buffer launch b would write
        float* __restrict__ Vo = d.st[xb][0];
        float* __restrict__ PXo = d.st[xb][1];
        float* __restrict__ PYo = d.st[xb][2];
        if (lastb) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                if (fl[j] & CF_OUT) {
                    Vo[gi[j]] = rv[j];
                    PXo[gi[j]] = rpx[j];
                    PYo[gi[j]] = rpy[j];
                }
            }
            break;
        }
        // The frame goes out as device-coherent stores (they do not stay in
        // this XCD's L2); once every thread has seen its stores complete, the
        // barrier lets thread 0 publish the block count.
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if ((frame >> j) & 1u) {
                __hip_atomic_store(Vo + gi[j], rv[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(PXo + gi[j], rpx[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(PYo + gi[j], rpy[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (t == 0) __hip_atomic_store(epoch + m, b + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t < 9 && t != 4) {
            const int nx = mx + (t % 3) - 1, ny = my + (t / 3) - 1;
            if (nx >= 0 && nx < d.mw && ny >= 0 && ny < d.mh && mflags[ny * d.mw + nx]) {
                const int32_t* e = epoch + ny * d.mw + nx;
                const uint64_t t0 = wall_clock64();
                while (true) {
                    const int32_t seen = __hip_atomic_load(e, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                    // a host-forced failure (wait_ticks < 0) gives up before
                    // looking at the count, so every tile with a queued
                    // neighbour stops at its first exchange
                    if (wait_ticks >= 0 && seen >= b + 1) break;
                    if (seen == kEpochFailed || wait_ticks < 0 ||
                        wall_clock64() - t0 > (uint64_t)wait_ticks) {
                        sFail = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
        }
        __syncthreads();
        if (sFail) {   // uniform: set before the barrier, read after it
            if (t == 0) {
                __hip_atomic_store(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(epoch + m, kEpochFailed, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            break;
        }
        // the halo ring from the neighbours' frames, as device-coherent loads
        // issued after the counts were seen
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if ((ring >> j) & 1u) {
                const int i = t + j * NT;
                const bool act = (fl[j] & CF_ACT) != 0;
                const float v = __hip_atomic_load(Vo + gi[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const float px = __hip_atomic_load(PXo + gi[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const float py = __hip_atomic_load(PYo + gi[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                rv[j] = act ? v : heav_from_c(rc[j]);
                rpx[j] = act ? px : 0.0f;
                rpy[j] = act ? py : 0.0f;
                sPX[PAD + i] = rpx[j];
                sPY[PAD + i] = rpy[j];
            }
        }
        __syncthreads();
    }
    if (sFail) {
        // the buffer the last block writes (the caller's v, p)
        const int xf = (in_buf + nb) & 1;
        const float nan = __builtin_nanf("");
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if (fl[j] & CF_OUT) {
                d.u[gi[j]] = nan;
                d.st[xf][0][gi[j]] = nan;
                d.st[xf][1][gi[j]] = nan;
                d.st[xf][2][gi[j]] = nan;
            }
        }
    }
}

// (v, p_x, p_y) of the RD pixels from state buffer `buf` into a full-grid
// slot [3][H][ld].  VEC: ld is a multiple of 4 and every plane 16-byte
// aligned; each lane takes 4 pixels of a row (a row's last group may reach
// into the row padding, which is read but never written).
template <bool VEC>
__global__ __launch_bounds__(256) void k_state_copy(ImgDesc d, int buf, float* __restrict__ slot) {
    const int64_t plane = (int64_t)d.H * d.ld;
    const int W = d.W, ld = d.ld;
    const int gpr = VEC ? (W + 3) >> 2 : W;   // groups per row
    const int64_t ng = (int64_t)gpr * d.H;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < ng;
         q += (int64_t)gridDim.x * 256) {
        const int y = (int)(q / gpr);
        const int x = (int)(q - (int64_t)y * gpr) * (VEC ? 4 : 1);
        const int64_t g = (int64_t)y * ld + x;
        if (VEC) {
            const float4 c = *reinterpret_cast<const float4*>(d.c + g);
            const float cc[4] = {c.x, c.y, c.z, c.w};
            bool act[4];
            bool all = x + 3 < W;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                act[e] = x + e < W && c_active(cc[e]);
                all = all && act[e];
            }
            if (!(act[0] || act[1] || act[2] || act[3])) continue;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float4 v = *reinterpret_cast<const float4*>(d.st[buf][k] + g);
                float* o = slot + k * plane + g;
                if (all) {
                    *reinterpret_cast<float4*>(o) = v;
                } else {
                    if (act[0]) o[0] = v.x;
                    if (act[1]) o[1] = v.y;
                    if (act[2]) o[2] = v.z;
                    if (act[3]) o[3] = v.w;
                }
            }
        } else {
            if (!c_active(d.c[g])) continue;
#pragma unroll
            for (int k = 0; k < 3; ++k) slot[k * plane + g] = d.st[buf][k][g];
        }
    }
}

// ---------------------------------------------------------------- config table
using IterFn = void (*)(ImgDesc, const ImgDesc*, const int2*, const int32_t*, int, int, int,
                        float, float, float, const uint32_t*, uint32_t*, double, int);

using PersistFn = void (*)(ImgDesc, const ImgDesc*, const int2*, const int32_t*, int, int,
                           float, float, float, int32_t*, int32_t*, int64_t);

struct CfgEntry {
    TileCfg cfg;
    IterFn fn[3];   // single image, batched, single image with the stopping rule
    PersistFn pfn;  // batched, every block in one cooperative launch
};

#define RDSEG_CFG(bx, by, it, nt)                                                         \
    CfgEntry{TileCfg{bx, by, it, nt},                                                     \
             {k_iterate<bx, by, it, nt, false, false>, k_iterate<bx, by, it, nt, true, false>, \
              k_iterate<bx, by, it, nt, false, true>},                                    \
             k_iterate_persist<bx, by, it, nt>}

const CfgEntry kCfgs[] = {
    RDSEG_CFG(8, 8, 1, 64),
    RDSEG_CFG(8, 8, 4, 128),
    RDSEG_CFG(8, 8, 8, 256),
    RDSEG_CFG(8, 8, 16, 512),
    RDSEG_CFG(8, 8, 32, 512),
    RDSEG_CFG(16, 16, 1, 128),
    RDSEG_CFG(16, 16, 2, 128),
    RDSEG_CFG(16, 16, 4, 256),
    RDSEG_CFG(16, 16, 8, 512),
    RDSEG_CFG(16, 16, 16, 512),
    RDSEG_CFG(32, 16, 2, 256),
    RDSEG_CFG(32, 32, 2, 256),
    RDSEG_CFG(32, 32, 4, 256),
    RDSEG_CFG(32, 32, 8, 512),
    RDSEG_CFG(64, 32, 2, 256),
    RDSEG_CFG(64, 32, 4, 512),
    RDSEG_CFG(64, 64, 2, 512),
    RDSEG_CFG(64, 64, 4, 512),
    RDSEG_CFG(64, 64, 8, 1024),
};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);

// occupancy-derived grid sizes, filled on first use (any host thread)
std::atomic<int> g_grid_cache[kNumCfgs][3];
std::atomic<int> g_persist_cap[kNumCfgs];

using ResFn = void (*)(ImgDesc, const int2*, const int32_t*, const int32_t*, int32_t*, int32_t*,
                       int, int, int, int, float, float, float, CompWs, const int64_t*, int,
                       int64_t);

struct ResEntry {
    int bx, by, it, nt;
    ResFn fn;
};

#define RDSEG_RES(bx, by, it, nt) ResEntry{bx, by, it, nt, k_resident<bx, by, it, nt>}

const ResEntry kRes[] = {
    RDSEG_RES(16, 16, 8, 512),
    RDSEG_RES(32, 32, 8, 512),
    RDSEG_RES(64, 32, 4, 512),
    RDSEG_RES(64, 64, 8, 1024),
};
constexpr int kNumRes = sizeof(kRes) / sizeof(kRes[0]);
std::atomic<int> g_res_cap[kNumRes];   // co-resident workgroups; -1: none

int resident_entry(int ci) {
    const TileCfg c = kCfgs[ci].cfg;
    for (int r = 0; r < kNumRes; ++r)
        if (kRes[r].bx == c.bx && kRes[r].by == c.by && kRes[r].it == c.it && kRes[r].nt == c.nt)
            return r;
    return -1;
}

}  // namespace

int config_count() { return kNumCfgs; }

TileCfg config_at(int i) { return kCfgs[i].cfg; }

int config_index(int bx, int by, int it) {
    for (int i = 0; i < kNumCfgs; ++i)
        if (kCfgs[i].cfg.bx == bx && kCfgs[i].cfg.by == by && kCfgs[i].cfg.it == it) return i;
    return -1;
}

int persistent_blocks(const void* kernel, int threads, size_t dyn_lds) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, dyn_lds) != hipSuccess)
        return 0;
    if (per < 1) per = 1;
    return per * ncu;
}

// Workgroups of a cooperative launch (every workgroup must be resident at
// once): the occupancy query's count, but at most 24 waves (6 a SIMD) and 16
// workgroups per CU.  The query allows up to 8 waves a SIMD; measured on
// gfx950, persistent grids sized to 7 or 8 waves a SIMD did not all become
// resident (their grid barriers' bounded waits expired), while grids of up
// to 6 waves a SIMD always did.
int cooperative_blocks(const void* kernel, int threads, size_t dyn_lds) {
    constexpr int kWavesPerCu = 24, kGroupsPerCu = 16;
    const int total = persistent_blocks(kernel, threads, dyn_lds);
    int dev = 0, ncu = 0;
    if (total <= 0 || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
        return 0;
    const int waves = (threads + 63) / 64;
    int per = total / ncu;
    per = std::min(per, std::max(1, kWavesPerCu / waves));
    per = std::min(per, kGroupsPerCu);
    return per * ncu;
}

namespace {
// 1 s of the 100 MHz wall clock per wait, unless the host set another bound
constexpr int64_t kResidentWaitTicks = 100000000;
std::atomic<int64_t> g_wait_ticks{kResidentWaitTicks};
}  // namespace

void set_resident_wait_ticks(int64_t ticks) {
    g_wait_ticks.store(ticks == 0 ? kResidentWaitTicks : ticks, std::memory_order_relaxed);
}

int64_t resident_wait_ticks() { return g_wait_ticks.load(std::memory_order_relaxed); }

int resident_capacity(int ci) {
    const int r = resident_entry(ci);
    if (r < 0) return 0;
    int cap = g_res_cap[r].load(std::memory_order_relaxed);
    if (cap == 0) {
        cap = cooperative_blocks(reinterpret_cast<const void*>(kRes[r].fn), kRes[r].nt, 0);
        if (cap <= 0) cap = -1;
        g_res_cap[r].store(cap, std::memory_order_relaxed);
    }
    return cap > 0 ? cap : 0;
}

bool resident_available(int ci) { return resident_entry(ci) >= 0; }

bool resident_fits(int ci, int64_t max_items) {
    if (max_items < 1) return false;
    const int cap = resident_capacity(ci);
    return cap > 0 && ((max_items + 7) / 8) * 8 <= cap;
}

int launch_resident(int ci, const ImgDesc& d, const int2* queue, const int32_t* n_queue,
                    const int32_t* mflags, int32_t* epoch, int32_t* status, int64_t max_items,
                    int in_buf, int iters, int per, int inner, float theta, float inv_theta,
                    float tau, hipStream_t st, hipEvent_t before, const CompWs* comp,
                    const int64_t* comp_npix, int64_t n_grid, bool epoch_cleared) {
    const int r = resident_entry(ci);
    if (n_grid <= 0) n_grid = max_items;
    if (r < 0 || !resident_fits(ci, n_grid)) return -1;
    // epoch[0 .. max_items) starts at 0 (*status was cleared with the RD count;
    // epoch_cleared: the caller enqueued that fill already)
    if (!epoch_cleared &&
        launch_fill(reinterpret_cast<float*>(epoch), 1, (int)max_items, (int)max_items, 0.0f, st))
        return 1;
    if (before) (void)hipEventRecord(before, st);
    const unsigned grid = (unsigned)(((n_grid + 7) / 8) * 8);
    ImgDesc dd = d;
    CompWs cw{};
    if (comp) cw = *comp;
    const int64_t* cnpix = comp ? comp_npix : nullptr;
    int citers = comp ? iters : 0;
    int64_t wait = resident_wait_ticks();
    void* args[] = {&dd,    &queue, &n_queue,   &mflags, &epoch, &status, &in_buf, &iters,
                    &per,   &inner, &theta,     &inv_theta, &tau, &cw,     &cnpix,  &citers,
                    &wait};
    const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kRes[r].fn),
                                                    dim3(grid), dim3(kRes[r].nt), args, 0, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return -1;   // not launched: the caller falls back to separate launches
    }
    return 0;
}

int launch_init(const ImgDesc* d0, const ImgDesc* descs, OffTables off, int n_img,
                int64_t n_rows, hipStream_t st) {
    unsigned grid = (unsigned)(n_rows < 65536 ? n_rows : 65536);
    if (descs)
        hipLaunchKernelGGL(k_init<true>, dim3(grid), dim3(256), 0, st, *d0, descs, off, n_img,
                           n_rows);
    else
        hipLaunchKernelGGL(k_init<false>, dim3(grid), dim3(256), 0, st, *d0, descs, off, n_img,
                           n_rows);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int prepare_iterate(int ci, bool batched, bool stop) {
    const CfgEntry& e = kCfgs[ci];
    const int kind = stop ? 2 : (batched ? 1 : 0);
    IterFn fn = e.fn[kind];
    std::atomic<int>& cached = g_grid_cache[ci][kind];
    if (cached.load(std::memory_order_relaxed) == 0) {
        const int b = persistent_blocks(reinterpret_cast<const void*>(fn), e.cfg.nt, 0);
        if (b <= 0) {
            set_error("occupancy query failed for the iteration kernel");
            return 4;
        }
        cached.store(b, std::memory_order_relaxed);
    }
    return 0;
}

int launch_iterate(int ci, const ImgDesc* d0, const ImgDesc* descs, bool batched,
                   const int2* queue, const int32_t* n_queue, int64_t max_items, int in_buf,
                   int nit, bool write_u, float theta, float inv_theta, float tau,
                   hipStream_t st, const StopLaunch* stop, int inner) {
    const CfgEntry& e = kCfgs[ci];
    if (stop && batched) {
        set_error("the stopping rule is available for single-image solves only");
        return 1;
    }
    const int kind = stop ? 2 : (batched ? 1 : 0);
    IterFn fn = e.fn[kind];
    if (prepare_iterate(ci, batched, stop != nullptr)) return 4;
    int64_t g = g_grid_cache[ci][kind].load(std::memory_order_relaxed);
    if (max_items < g) g = max_items;
    g = ((g + 7) / 8) * 8;
    if (g < 8) g = 8;
    hipLaunchKernelGGL(fn, dim3((unsigned)g), dim3(e.cfg.nt), 0, st, *d0, descs, queue, n_queue,
                       in_buf, nit, write_u ? 1 : 0, theta, inv_theta, tau,
                       stop ? stop->skip_slot : nullptr, stop ? stop->diff_slot : nullptr,
                       stop ? stop->tol : 0.0, inner);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_recompute(const ImgDesc& d, const int2* queue, const int32_t* n_queue,
                     int64_t max_items, int in_buf, int nit, float theta, float inv_theta,
                     float tau, float* tape, int64_t tape_step, int64_t tape_plane,
                     hipStream_t st) {
    constexpr int BX = 16, BY = 16, IT = 8, NT = 512;
    if (nit < 1 || nit > IT) {
        set_error("recompute: 1 <= nit <= 8");
        return 1;
    }
    static std::atomic<int> cap{0};
    int g = cap.load(std::memory_order_relaxed);
    if (g == 0) {
        g = persistent_blocks(reinterpret_cast<const void*>(k_recompute<BX, BY, IT, NT>), NT, 0);
        if (g <= 0) {
            set_error("occupancy query failed for the recompute kernel");
            return 4;
        }
        cap.store(g, std::memory_order_relaxed);
    }
    int64_t grid = g;
    if (max_items < grid) grid = max_items;
    grid = ((grid + 7) / 8) * 8;
    if (grid < 8) grid = 8;
    hipLaunchKernelGGL((k_recompute<BX, BY, IT, NT>), dim3((unsigned)grid), dim3(NT), 0, st, d,
                       queue, n_queue, in_buf, nit, theta, inv_theta, tau, tape, tape_step,
                       tape_plane);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int prepare_iterate_persist(int ci) {
    const CfgEntry& e = kCfgs[ci];
    int cap = g_persist_cap[ci].load(std::memory_order_relaxed);
    if (cap == 0) {
        cap = cooperative_blocks(reinterpret_cast<const void*>(e.pfn), e.cfg.nt, 0);
        if (cap <= 0) cap = -1;
        g_persist_cap[ci].store(cap, std::memory_order_relaxed);
    }
    return 0;
}

int launch_iterate_persist(int ci, const ImgDesc* d0, const ImgDesc* descs, const int2* queue,
                           const int32_t* n_queue, int iters, int per, float theta,
                           float inv_theta, float tau, int32_t* bar, int32_t* status,
                           hipStream_t st) {
    const CfgEntry& e = kCfgs[ci];
    prepare_iterate_persist(ci);
    const int cap = g_persist_cap[ci].load(std::memory_order_relaxed);
    const int grid = cap > 0 ? cap / 8 * 8 : 0;
    if (grid < 8) return -1;
    // the barrier counter starts at 0 (a fill kernel: no memset node in a graph)
    if (launch_fill(reinterpret_cast<float*>(bar), 1, 1, 1, 0.0f, st)) return 1;
    ImgDesc dd = *d0;
    int64_t wait = resident_wait_ticks();
    void* args[] = {&dd,    &descs, &queue, &n_queue, &iters, &per, &theta,
                    &inv_theta, &tau, &bar, &status, &wait};
    const hipError_t err = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(e.pfn),
                                                      dim3(grid), dim3(e.cfg.nt), args, 0, st);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return 0;
}

namespace {

__global__ __launch_bounds__(256) void k_stop_decide(const uint32_t* __restrict__ slots,
                                                     int n_checks, double tol, int check_every,
                                                     int iters, int32_t* __restrict__ iters_done) {
    __shared__ int smin[256];
    const int t = threadIdx.x;
    int best = n_checks;
    for (int c = t; c < n_checks; c += 256) {
        if ((double)__uint_as_float(slots[c]) <= tol) {
            best = c;   // ascending per thread: the first hit is its minimum
            break;
        }
    }
    smin[t] = best;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) smin[t] = min(smin[t], smin[t + o]);
        __syncthreads();
    }
    if (t == 0) *iters_done = smin[0] < n_checks ? (smin[0] + 1) * check_every : iters;
}

__global__ __launch_bounds__(256) void k_stop_copy(ImgDesc d, const int32_t* __restrict__ iters_done,
                                                   int check_every, int launches_per_check,
                                                   int n_launches, int iters) {
    const int done = *iters_done;
    if (done >= iters) return;   // ran to the end: the last launch wrote buffer 0
    const int c = done / check_every - 1;
    const int j = (c + 1) * launches_per_check - 1;
    if (1 - (n_launches - j) % 2 == 0) return;
    for (int y = blockIdx.x; y < d.H; y += gridDim.x) {
        for (int x = threadIdx.x; x < d.W; x += blockDim.x) {
            const int g = y * d.ld + x;
            if (!c_active(d.c[g])) continue;
#pragma unroll
            for (int k = 0; k < 3; ++k) d.st[0][k][g] = d.st[1][k][g];
        }
    }
}

}  // namespace

int launch_stop_finalize(const ImgDesc& d, const uint32_t* slots, int n_checks, double tol,
                         int check_every, int launches_per_check, int n_launches, int iters,
                         int32_t* iters_done, hipStream_t st) {
    hipLaunchKernelGGL(k_stop_decide, dim3(1), dim3(256), 0, st, slots, n_checks, tol,
                       check_every, iters, iters_done);
    RDSEG_HIP_CHECK(hipGetLastError());
    const unsigned grid = (unsigned)(d.H < 4096 ? d.H : 4096);
    hipLaunchKernelGGL(k_stop_copy, dim3(grid), dim3(256), 0, st, d, (const int32_t*)iters_done,
                       check_every, launches_per_check, n_launches, iters);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_state_copy(const ImgDesc& d, int buf, float* slot, hipStream_t st) {
    auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    const bool vec = (d.ld & 3) == 0 && al16(d.c) && al16(slot) && al16(d.st[buf][0]) &&
                     al16(d.st[buf][1]) && al16(d.st[buf][2]);
    const int64_t groups = (int64_t)d.H * (vec ? (d.W + 3) / 4 : d.W);
    int64_t grid = (groups + 255) / 256;
    if (grid > 8192) grid = 8192;
    if (grid < 1) grid = 1;
    if (vec)
        hipLaunchKernelGGL(k_state_copy<true>, dim3((unsigned)grid), dim3(256), 0, st, d, buf, slot);
    else
        hipLaunchKernelGGL(k_state_copy<false>, dim3((unsigned)grid), dim3(256), 0, st, d, buf, slot);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace rdseg
