// adjoint.hip -- reverse mode of the unrolled restricted iteration, the fitting
// terms of Sec. 1 (eq. CV / eq. DS) and fixed-order FP64 reductions.
//
// One reverse step k works on the queued macro tiles.  From
// the stored state (p^{k-1}, v^{k-1}) it recomputes w, g = grad w, m =
// 1/(1 + tau|g|), p^k and the clamp argument s = u^k - theta lambda f, then
// applies, on RD only (RD and u0 = H(-f) are held fixed):
//   sbar  = vbar^k [0 < s < 1]                  (clamp)
//   ubar  = sbar (+ dL/du at the last iteration)
//   pbt   = pbar^k + theta grad(ubar)           (u = v - theta div p, div = -grad^T)
//   gbar  = tau m pbt - tau m (p^k . pbt) g/|g| (normalised dual update)
//   wbar  = -div gbar                           (g = grad w)
//   vbar^{k-1} = ubar - wbar / theta,  pbar^{k-1} = m pbt - grad(wbar)
// The x component on the last column and the y component on the last row are
// constants (zero) and get no adjoint.  The sum of sbar over iterations is
// accumulated per pixel; dL/df = -theta lambda * that sum and dL/dlambda =
// -theta sum f * that sum.  Six LDS phases separated by barriers per step;
// each step's halo is 3 pixels on every side (each phase reaches one cell
// further), and a launch runs up to NS steps on a halo of 3 NS.
#include <atomic>
#include "rdseg_internal.h"

namespace rdseg {

namespace {

constexpr int RED_T = 256;

// The ns reverse steps of one macro tile.  Dense: slot j of a thread is
// region cell t + j NT.  COMPACT: slot j is idx[j], an RD cell of the region
// (-1: none); the cells off RD are never visited, their LDS entries hold
// constants written when the region was set up (p, ubar, gbar, wbar 0 and
// w = -H(-f)/theta), exactly what the dense steps would store there, so both
// give the same bits.  sA / sB: p^{k-1}, then p^k, then gbar; sW: w; sZ:
// ubar, then wbar.
template <int BX, int BY, int NS, int NT, bool COMPACT, int CPT>
__device__ __forceinline__ void adj_steps(
    float* __restrict__ sA, float* __restrict__ sB, float* __restrict__ sW,
    float* __restrict__ sZ, const int* idx, const float* rc, const uint32_t* fl, const int* gi,
    float* rpbx, float* rpby, float* rvb, float* racc, const AdjSlots& sl, int ns, bool first,
    const float* __restrict__ grad_u, float theta, float inv_theta, float tau) {
    constexpr int HL = 3 * NS;
    constexpr int RX = BX + 2 * HL;
    constexpr int RY = BY + 2 * HL;
    constexpr int RC = RX * RY;
    constexpr int PAD = RX + 1;
    const int t = threadIdx.x;
    const int64_t plane = sl.plane;
#define ADJ_CELL(j) const int i = COMPACT ? idx[j] : t + (j) * NT; \
                    const bool live = COMPACT ? (i >= 0) : (i < RC)
    for (int s = 0; s < ns; ++s) {
        const float* __restrict__ sv = sl.s[s];
        const bool last = s == ns - 1;
        float rv[CPT], rnx[CPT], rny[CPT], rgx[CPT], rgy[CPT], rm[CPT], rsb[CPT], rub[CPT];
        // P0: the state (p^{k-1}, v^{k-1}) of this step
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            ADJ_CELL(j);
            rv[j] = 0.0f;
            if (live) {
                float px0 = 0.0f, py0 = 0.0f;
                if (COMPACT || (fl[j] & CF_ACT)) {
                    const int g = gi[j];
                    rv[j] = sv[g];
                    px0 = sv[plane + g];
                    py0 = sv[2 * plane + g];
                } else {
                    rv[j] = heav_from_c(rc[j]);
                }
                sA[PAD + i] = px0;
                sB[PAD + i] = py0;
            }
        }
        __syncthreads();
        // P1: w from p^{k-1}, v^{k-1}
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            ADJ_CELL(j);
            if (live) {
                float dd = div_p(sA[PAD + i], sA[PAD + i - 1], sB[PAD + i], sB[PAD + i - RX]);
                sW[PAD + i] = w_of(dd, rv[j], inv_theta, (fl[j] & CF_ACT) != 0);
            }
        }
        __syncthreads();
        // P2: dual update -> p^k, keep g and m
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            ADJ_CELL(j);
            if (live) {
                DualOut o = dual_update(sA[PAD + i], sB[PAD + i], sW[PAD + i], sW[PAD + i + 1],
                                        sW[PAD + i + RX], fl[j], tau);
                rnx[j] = o.px;
                rny[j] = o.py;
                rgx[j] = o.gx;
                rgy[j] = o.gy;
                rm[j] = o.m;
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            ADJ_CELL(j);
            if (live) {
                sA[PAD + i] = rnx[j];
                sB[PAD + i] = rny[j];
            }
        }
        __syncthreads();
        // P3: u^k, s, clamp adjoint, ubar (dL/du enters at the last iteration)
        const float* __restrict__ gu = (first && s == 0) ? grad_u : nullptr;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            ADJ_CELL(j);
            if (live) {
                float d1 = div_p(rnx[j], sA[PAD + i - 1], rny[j], sB[PAD + i - RX]);
                float u = u_step(rv[j], d1, theta);
                float sv1 = u - rc[j];
                const bool act = (fl[j] & CF_ACT) != 0;
                float sb = (act && sv1 > 0.0f && sv1 < 1.0f) ? rvb[j] : 0.0f;
                float ub = sb;
                if (gu && act) ub += gu[gi[j]];
                ub = act ? ub : 0.0f;
                rsb[j] = sb;
                rub[j] = ub;
                sZ[PAD + i] = ub;
            }
        }
        __syncthreads();
        // P4: pbt = pbar^k + theta grad(ubar); gbar
        float rptx[CPT], rpty[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            ADJ_CELL(j);
            rptx[j] = 0.0f; rpty[j] = 0.0f;
            if (live) {
                const uint32_t f = fl[j];
                const bool act = (f & CF_ACT) != 0;
                float uc = sZ[PAD + i];
                float gux = (f & CF_LASTC) ? 0.0f : (sZ[PAD + i + 1] - uc);
                float guy = (f & CF_LASTR) ? 0.0f : (sZ[PAD + i + RX] - uc);
                float ptx = act ? fmaf(theta, gux, rpbx[j]) : 0.0f;
                float pty = act ? fmaf(theta, guy, rpby[j]) : 0.0f;
                rptx[j] = ptx;
                rpty[j] = pty;
                float nn = __builtin_amdgcn_sqrtf(fmaf(rgx[j], rgx[j], rgy[j] * rgy[j]));
                float inv_n = nn > 0.0f ? __builtin_amdgcn_rcpf(nn) : 0.0f;
                float tm = tau * rm[j];
                float dot = fmaf(rnx[j], ptx, rny[j] * pty);
                float k2 = tm * dot * inv_n;
                float gbx = fmaf(tm, ptx, -k2 * rgx[j]);
                float gby = fmaf(tm, pty, -k2 * rgy[j]);
                gbx = (act && !(f & CF_LASTC)) ? gbx : 0.0f;
                gby = (act && !(f & CF_LASTR)) ? gby : 0.0f;
                sA[PAD + i] = gbx;
                sB[PAD + i] = gby;
            }
        }
        __syncthreads();
        // P5: wbar = -div gbar
        float rwb[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            ADJ_CELL(j);
            rwb[j] = 0.0f;
            if (live) {
                const bool act = (fl[j] & CF_ACT) != 0;
                float dg = div_p(sA[PAD + i], sA[PAD + i - 1], sB[PAD + i], sB[PAD + i - RX]);
                rwb[j] = act ? -dg : 0.0f;
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            ADJ_CELL(j);
            if (live) sZ[PAD + i] = rwb[j];
        }
        __syncthreads();
        // P6: pbar^{k-1}, vbar^{k-1}: kept for the next step, written
        // after the last
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            ADJ_CELL(j);
            const uint32_t f = fl[j];
            if (live && (f & CF_ACT) && (!last || (f & CF_OUT))) {
                float wc = rwb[j];
                float gwx = (f & CF_LASTC) ? 0.0f : (sZ[PAD + i + 1] - wc);
                float gwy = (f & CF_LASTR) ? 0.0f : (sZ[PAD + i + RX] - wc);
                float pbx = (f & CF_LASTC) ? 0.0f : fmaf(rm[j], rptx[j], -gwx);
                float pby = (f & CF_LASTR) ? 0.0f : fmaf(rm[j], rpty[j], -gwy);
                float vb = fmaf(-wc, inv_theta, rub[j]);
                rpbx[j] = pbx;
                rpby[j] = pby;
                rvb[j] = vb;
                if (f & CF_OUT) racc[j] += rsb[j];
            }
        }
    }
#undef ADJ_CELL
}

// One macro tile's reverse steps on CPT slots per thread (cells as in
// adj_steps): the adjoint state entering the first step and the
// clamp-adjoint sum are read, the steps run, and the interior RD cells'
// (pbar, vbar) and sum are written.
template <int BX, int BY, int NS, int NT, bool COMPACT, int CPT>
__device__ __forceinline__ void adj_item(
    float* __restrict__ sA, float* __restrict__ sB, float* __restrict__ sW,
    float* __restrict__ sZ, const int* idx, const float* rc, const uint32_t* fl, const int* gi,
    const AdjSlots& sl, int ns, bool first, const float* __restrict__ pbx_in,
    const float* __restrict__ pby_in, const float* __restrict__ vb_in,
    float* __restrict__ pbx_out, float* __restrict__ pby_out, float* __restrict__ vb_out,
    float* __restrict__ sacc, const float* __restrict__ grad_v,
    const float* __restrict__ grad_u, float theta, float inv_theta, float tau) {
    float rpbx[CPT], rpby[CPT], rvb[CPT], racc[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        rpbx[j] = 0.0f; rpby[j] = 0.0f; rvb[j] = 0.0f; racc[j] = 0.0f;
        if (fl[j] & CF_ACT) {
            const int g = gi[j];
            if (first) {
                rvb[j] = grad_v ? grad_v[g] : 0.0f;
            } else {
                rpbx[j] = pbx_in[g];
                rpby[j] = pby_in[g];
                rvb[j] = vb_in[g];
            }
            if (fl[j] & CF_OUT) racc[j] = sacc[g];
        }
    }
    adj_steps<BX, BY, NS, NT, COMPACT, CPT>(sA, sB, sW, sZ, idx, rc, fl, gi, rpbx, rpby, rvb, racc,
                                            sl, ns, first, grad_u, theta, inv_theta, tau);
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        if (fl[j] & CF_OUT) {
            const int g = gi[j];
            pbx_out[g] = rpbx[j];
            pby_out[g] = rpby[j];
            vb_out[g] = rvb[j];
            sacc[g] = racc[j];
        }
    }
}

// NS reverse steps per launch (k, k - 1, ..., k - ns + 1, ns <= NS): the
// halo is 3 NS pixels, every step reaches 3 cells further in, the adjoint
// state (pbar, vbar) and the clamp-adjoint sum stay in registers between the
// steps and only the state of each step (its slot) is read per step.  Cells
// nearer the region's edge than 3 (s + 1) after step s hold values that no
// cell further in reads.  Each cell's arithmetic and the order of the sums are
// those of one step per launch, so the result does not depend on NS.  A
// region less than 40 % RD runs on its compacted RD cells.  Workgroups take
// the queue in 8 contiguous runs, one per XCD (neighbouring tiles share that
// XCD's L2); the grid is a multiple of 8.
template <int BX, int BY, int NS, int NT>
__global__ __launch_bounds__(NT, NT >= 512 ? 4 : 1) void k_adj_block(
    ImgDesc d, AdjSlots sl, int ns, const float* __restrict__ pbx_in,
    const float* __restrict__ pby_in, const float* __restrict__ vb_in,
    float* __restrict__ pbx_out, float* __restrict__ pby_out, float* __restrict__ vb_out,
    float* __restrict__ sacc, int first, const float* __restrict__ grad_v,
    const float* __restrict__ grad_u, const int2* __restrict__ queue,
    const int32_t* __restrict__ n_queue, float theta, float inv_theta, float tau) {
    constexpr int HL = 3 * NS;
    constexpr int RX = BX + 2 * HL;
    constexpr int RY = BY + 2 * HL;
    constexpr int RC = RX * RY;
    constexpr int CPT = (RC + NT - 1) / NT;
    constexpr int PAD = RX + 1;
    constexpr int LS = RC + 2 * PAD;
    constexpr int NW = NT / 64;
    constexpr int NCNT = CPT * NW;
    constexpr int CPTC = (2 * RC + 5 * NT - 1) / (5 * NT);   // compact slots: < 40 % of RC
    static_assert(NT % 64 == 0 && NCNT <= 128, "the count scan covers at most 128 entries");
    static_assert(RC < 32768, "region index must fit the 16-bit cell list");
    __shared__ float sA[LS];
    __shared__ float sB[LS];
    __shared__ float sW[LS];
    __shared__ float sZ[LS];
    __shared__ uint16_t sList[RC];
    __shared__ int sCnt[NCNT + 1];

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = t >> 6;
    for (int k = t; k < PAD; k += NT) {
        sA[k] = 0.0f; sB[k] = 0.0f; sW[k] = 0.0f; sZ[k] = 0.0f;
        sA[PAD + RC + k] = 0.0f; sB[PAD + RC + k] = 0.0f; sW[PAD + RC + k] = 0.0f;
        sZ[PAD + RC + k] = 0.0f;
    }
    const int nq = *n_queue;
    const int per = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7;
    const int rank = blockIdx.x >> 3;
    const int chunk = (nq + 7) >> 3;
    const int q0 = xcd * chunk;
    const int q1 = min(nq, q0 + chunk);
    const int W = d.W, H = d.H, ld = d.ld;
    const bool fst = first != 0;
    for (int item = q0 + rank; item < q1; item += per) {
        const int2 q = queue[item];
        const int my = q.y / d.mw;
        const int mx = q.y - my * d.mw;
        const int ox = mx * BX - HL;
        const int oy = my * BY - HL;

        float rc[CPT];
        uint32_t fl[CPT];
        int gi[CPT];
        uint64_t amask[CPT];

        __syncthreads();   // LDS of the previous item fully consumed
        // region set-up: c, flags and the constants of the cells off RD (RD
        // cells park c in sZ until the first ubar overwrites it)
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            rc[j] = __builtin_inff(); fl[j] = 0u; gi[j] = 0;
            bool act = false;
            if (i < RC) {
                const int ry = i / RX;
                const int rx = i - ry * RX;
                const int gx = ox + rx, gy = oy + ry;
                const bool inb = (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H;
                const int g = gy * ld + gx;
                gi[j] = g;
                const float c = inb ? d.c[g] : __builtin_inff();
                act = c_active(c);
                rc[j] = c;
                const bool interior = rx >= HL && rx < HL + BX && ry >= HL && ry < HL + BY;
                uint32_t f = act ? CF_ACT : 0u;
                if (gx == W - 1) f |= CF_LASTC;
                if (gy == H - 1) f |= CF_LASTR;
                if (interior && act) f |= CF_OUT;
                fl[j] = f;
                sA[PAD + i] = 0.0f;
                sB[PAD + i] = 0.0f;
                sW[PAD + i] = w_of(0.0f, heav_from_c(c), inv_theta, false);
                sZ[PAD + i] = act ? c : 0.0f;
            }
            amask[j] = __ballot(act);
        }
        // count the RD cells of the region (ascending list offsets)
        if (lane == 0) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) sCnt[j * NW + wv] = __popcll(amask[j]);
        }
        __syncthreads();
        if (wv == 0) {   // exclusive scan of the NCNT counts, two per lane
            const int e0 = 2 * lane < NCNT ? sCnt[2 * lane] : 0;
            const int e1 = 2 * lane + 1 < NCNT ? sCnt[2 * lane + 1] : 0;
            const int sm = e0 + e1;
            int incl = sm;
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            const int excl = incl - sm;
            if (2 * lane < NCNT) sCnt[2 * lane] = excl;
            if (2 * lane + 1 < NCNT) sCnt[2 * lane + 1] = excl + e0;
            if (lane == 63) sCnt[NCNT] = incl;
        }
        __syncthreads();
        const int n_act = sCnt[NCNT];
        if (5 * n_act < 2 * RC) {
            // compact: the list of the region's RD cells, CPTC slots a thread
            const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                if ((amask[j] >> lane) & 1ull)
                    sList[sCnt[j * NW + wv] + __popcll(amask[j] & below)] = (uint16_t)(t + j * NT);
            }
            __syncthreads();
            float cc[CPTC];
            uint32_t cf[CPTC];
            int cg[CPTC], ci[CPTC];
#pragma unroll
            for (int j = 0; j < CPTC; ++j) {
                const int k = t + j * NT;
                ci[j] = -1; cf[j] = 0u; cg[j] = 0; cc[j] = 0.0f;
                if (k < n_act) {
                    const int i = sList[k];
                    const int ry = i / RX;
                    const int rx = i - ry * RX;
                    const int gx = ox + rx, gy = oy + ry;
                    ci[j] = i;
                    cg[j] = gy * ld + gx;
                    cc[j] = sZ[PAD + i];
                    const bool interior = rx >= HL && rx < HL + BX && ry >= HL && ry < HL + BY;
                    uint32_t f = CF_ACT;
                    if (gx == W - 1) f |= CF_LASTC;
                    if (gy == H - 1) f |= CF_LASTR;
                    if (interior) f |= CF_OUT;
                    cf[j] = f;
                }
            }
            adj_item<BX, BY, NS, NT, true, CPTC>(sA, sB, sW, sZ, ci, cc, cf, cg, sl, ns, fst,
                                                 pbx_in, pby_in, vb_in, pbx_out, pby_out, vb_out,
                                                 sacc, grad_v, grad_u, theta, inv_theta, tau);
        } else {
            adj_item<BX, BY, NS, NT, false, CPT>(sA, sB, sW, sZ, nullptr, rc, fl, gi, sl, ns, fst,
                                                 pbx_in, pby_in, vb_in, pbx_out, pby_out, vb_out,
                                                 sacc, grad_v, grad_u, theta, inv_theta, tau);
        }
    }
}

__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ p, int H, int W, int ld,
                                                  float v) {
    for (int y = blockIdx.x; y < H; y += gridDim.x)
        for (int x = threadIdx.x; x < W; x += blockDim.x) p[y * ld + x] = v;
}

// Per-block FP64 partial sums over rows assigned in a fixed pattern; the
// block tree is fixed too, so the result does not depend on timing.
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double* __restrict__ out) {
    __shared__ double s[NV][RED_T];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = RED_T / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
#pragma unroll
            for (int k = 0; k < NV; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = s[k][0];
    }
}

// grad_f, and per-block partials of (lambda, c1, c2, gamma) adjoints.
__global__ __launch_bounds__(RED_T) void k_adj_final(
    ImgDesc d, const float* __restrict__ sacc, const float* __restrict__ vb0,
    float* __restrict__ grad_f, double lambda, double theta, const float* __restrict__ z,
    const float* __restrict__ P, double c1, double c2, double* __restrict__ partials) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double tl = theta * lambda;
    for (int y = blockIdx.x; y < d.H; y += gridDim.x) {
        for (int x = threadIdx.x; x < d.W; x += RED_T) {
            const int g = y * d.ld + x;
            const float c = d.c[g];
            double gf = 0.0;
            if (c_active(c)) {
                const float h = d.f[g] < 0.0f ? 1.0f : 0.0f;
                const float s0 = h - c;   // clamp argument of v0 with u0 = H(-f)
                double S = (double)sacc[g];
                if (s0 > 0.0f && s0 < 1.0f) S += (double)vb0[g];
                gf = -tl * S;
                acc[0] += -theta * (double)d.f[g] * S;
                if (z) {
                    const double zz = (double)z[g];
                    acc[1] += gf * (-2.0 * (zz - c1));
                    acc[2] += gf * (2.0 * (zz - c2));
                    if (P) acc[3] += gf * (double)P[g];
                }
            }
            grad_f[g] = (float)gf;
        }
    }
    block_reduce_store<4>(acc, partials + 4 * (int64_t)blockIdx.x);
}

__global__ __launch_bounds__(RED_T) void k_reduce_partials(const double* __restrict__ part,
                                                           int nblk, int nv,
                                                           double* __restrict__ out) {
    // one wave per value: lane l sums blocks l, l + 64, ... in order (their
    // loads independent of each other), then a fixed xor tree over the lanes;
    // the order is the same on every call
    const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (k >= nv) return;   // uniform per wave
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += part[(int64_t)b * 4 + k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) out[k] = s;
}

__global__ __launch_bounds__(256) void k_fit_fwd(const float* __restrict__ z,
                                                 const float* __restrict__ P, double c1,
                                                 double c2, double gamma, int H, int W, int ld,
                                                 float* __restrict__ f) {
    for (int y = blockIdx.x; y < H; y += gridDim.x)
        for (int x = threadIdx.x; x < W; x += blockDim.x) {
            const int g = y * ld + x;
            const double zz = (double)z[g];
            const double a = zz - c1, b = zz - c2;
            double v = a * a - b * b;
            if (P) v += gamma * (double)P[g];
            f[g] = (float)v;
        }
}

__global__ __launch_bounds__(RED_T) void k_fit_bwd(const float* __restrict__ z,
                                                   const float* __restrict__ P,
                                                   const float* __restrict__ gf, double c1,
                                                   double c2, int H, int W, int ld,
                                                   double* __restrict__ partials) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int y = blockIdx.x; y < H; y += gridDim.x)
        for (int x = threadIdx.x; x < W; x += RED_T) {
            const int g = y * ld + x;
            const double zz = (double)z[g];
            const double b = (double)gf[g];
            acc[0] += b * (-2.0 * (zz - c1));
            acc[1] += b * (2.0 * (zz - c2));
            if (P) acc[2] += b * (double)P[g];
        }
    block_reduce_store<4>(acc, partials + 4 * (int64_t)blockIdx.x);
}

__global__ void k_scatter_scalars(const double* __restrict__ src, double* a, double* b,
                                  double* c, double* d) {
    if (threadIdx.x == 0) {
        if (a) *a = src[0];
        if (b) *b = src[1];
        if (c) *c = src[2];
        if (d) *d = src[3];
    }
}

using AdjFn = void (*)(ImgDesc, AdjSlots, int, const float*, const float*, const float*, float*,
                       float*, float*, float*, int, const float*, const float*, const int2*,
                       const int32_t*, float, float, float);

struct AdjEntry {
    int bx, by, ns, nt;
    AdjFn fn;
};

const AdjEntry kAdj[] = {
    {32, 32, 1, 256, k_adj_block<32, 32, 1, 256>},
    {16, 16, 2, 256, k_adj_block<16, 16, 2, 256>},
    {16, 16, 4, 512, k_adj_block<16, 16, 4, 512>},
    {32, 32, 2, 512, k_adj_block<32, 32, 2, 512>},
    {32, 32, 4, 1024, k_adj_block<32, 32, 4, 1024>},
};
// occupancy-derived grid sizes, filled on first use (any host thread)
std::atomic<int> g_adj_grid[sizeof(kAdj) / sizeof(kAdj[0])];

inline unsigned red_blocks(int H) { return (unsigned)(H < 1024 ? H : 1024); }

}  // namespace

int adj_config_count() { return (int)(sizeof(kAdj) / sizeof(kAdj[0])); }

int64_t reduce_partials(int H) { return (int64_t)red_blocks(H) * 4; }

int adj_config_find(int tile, int ns) {
    for (int i = 0; i < adj_config_count(); ++i)
        if (kAdj[i].bx == tile && kAdj[i].by == tile && kAdj[i].ns == ns) return i;
    return -1;
}

int adj_config_steps(int ai) { return kAdj[ai].ns; }

int adj_config_tile(int ai) { return kAdj[ai].bx; }

int launch_adj_block(int ai, const ImgDesc& d, const AdjSlots& sl, int ns, const AdjBufs& ab,
                     int in_buf, bool first, const float* grad_v, const float* grad_u,
                     const int2* queue, const int32_t* n_queue, int64_t max_items, float theta,
                     float tau, hipStream_t st) {
    if (ai < 0 || ai >= adj_config_count() || ns < 1 || ns > kAdj[ai].ns ||
        d.mw != (d.W + kAdj[ai].bx - 1) / kAdj[ai].bx) {
        set_error("adjoint launch: no kernel for this tile size and step count");
        return 1;
    }
    int64_t g = g_adj_grid[ai].load(std::memory_order_relaxed);
    if (g == 0) {
        const int b = persistent_blocks(reinterpret_cast<const void*>(kAdj[ai].fn), kAdj[ai].nt, 0);
        if (b <= 0) {
            set_error("occupancy query failed for the adjoint kernel");
            return 4;
        }
        g_adj_grid[ai].store(b, std::memory_order_relaxed);
        g = b;
    }
    if (max_items < g) g = max_items;
    g = ((g + 7) / 8) * 8;   // the kernel splits the queue into 8 runs
    if (g < 8) g = 8;
    const int out = 1 - in_buf;
    hipLaunchKernelGGL(kAdj[ai].fn, dim3((unsigned)g), dim3(kAdj[ai].nt), 0, st, d, sl, ns,
                       ab.pbx[in_buf], ab.pby[in_buf], ab.vb[in_buf], ab.pbx[out], ab.pby[out],
                       ab.vb[out], ab.sacc, first ? 1 : 0, grad_v, grad_u, queue, n_queue, theta,
                       1.0f / theta, tau);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_fill(float* p, int H, int W, int ld, float v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_f32, dim3(red_blocks(H)), dim3(256), 0, st, p, H, W, ld, v);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_adj_final(const ImgDesc& d, const float* sacc, const float* vb0, float* grad_f,
                     double lambda, double theta, const float* z, const float* P, double c1,
                     double c2, double* partials, int64_t n_part, double* out4,
                     hipStream_t st) {
    unsigned nb = red_blocks(d.H);
    if ((int64_t)nb * 4 > n_part) {
        set_error("reduction scratch too small");
        return 3;
    }
    hipLaunchKernelGGL(k_adj_final, dim3(nb), dim3(RED_T), 0, st, d, sacc, vb0, grad_f, lambda,
                       theta, z, P, c1, c2, partials);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(RED_T), 0, st, partials, (int)nb, 4, out4);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_scatter_scalars(const double* src, double* a, double* b, double* c, double* d,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_scalars, dim3(1), dim3(64), 0, st, src, a, b, c, d);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_fit_forward(const float* z, const float* P, double c1, double c2, double gamma,
                       int H, int W, int ld, float* f, hipStream_t st) {
    hipLaunchKernelGGL(k_fit_fwd, dim3(red_blocks(H)), dim3(256), 0, st, z, P, c1, c2, gamma, H,
                       W, ld, f);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_fit_backward(const float* z, const float* P, const float* grad_f, double c1,
                        double c2, int H, int W, int ld, double* partials, int64_t n_part,
                        double* out3, hipStream_t st) {
    unsigned nb = red_blocks(H);
    if ((int64_t)nb * 4 > n_part) {
        set_error("reduction scratch too small");
        return 3;
    }
    hipLaunchKernelGGL(k_fit_bwd, dim3(nb), dim3(RED_T), 0, st, z, P, grad_f, c1, c2, H, W, ld,
                       partials);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(RED_T), 0, st, partials, (int)nb, 3, out3);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace rdseg
