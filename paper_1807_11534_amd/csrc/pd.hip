// pd.hip -- the restricted domain carried over to another solver (the
// conclusion, Sec. 5, proposes it): the first-order primal-dual iteration of
// Chambolle and Pock for eq. CR, min over u in [0,1] of TV(u) + lambda <f, u>,
// restricted as in Sec. 3 (u = H(-f), p = 0 off RD).  Per pixel of RD
//   a    = p + sigma grad ubar               (forward differences)
//   p    = a / max(1, |a|)
//   u'   = clamp(u + tau div p - tau lambda f, 0, 1)
//   ubar = 2 u' - u,  u = u'
// Off RD the library stores c = -/+inf in place of tau lambda f, so the clamp
// returns H(-f) there and ubar = H(-f) too, with no branch.
//
// The kernel has the structure of the dual solver's blocked kernel: one
// workgroup per queued macro tile, the tile plus a halo of IT + 1 (left/top)
// and IT (right/bottom) in LDS (p, ubar) and registers (u, c, flags), IT
// iterations on chip with two barriers each (phase B: the p step from ubar at
// x, x+e_x, x+e_y; phase A: the u step from div p at x, x-e_x, x-e_y), so each
// phase reaches one cell further and the halo covers IT iterations.
#include "rdseg_internal.h"

namespace rdseg {

namespace {

__device__ __forceinline__ void pd_dual(float& px, float& py, float ubc, float ubr, float ubd,
                                        uint32_t fl, float sigma) {
    const float gx = (fl & CF_LASTC) ? 0.0f : (ubr - ubc);
    const float gy = (fl & CF_LASTR) ? 0.0f : (ubd - ubc);
    const float ax = fmaf(sigma, gx, px);
    const float ay = fmaf(sigma, gy, py);
    const float n = __builtin_amdgcn_sqrtf(fmaf(ax, ax, ay * ay));
    const float r = __builtin_amdgcn_rcpf(fmaxf(n, 1.0f));
    const bool act = (fl & CF_ACT) != 0;
    px = act ? ax * r : 0.0f;
    py = act ? ay * r : 0.0f;
}

__global__ __launch_bounds__(256) void k_pd_init(PdDesc d, int64_t n_rows) {
    for (int64_t R = blockIdx.x; R < n_rows; R += gridDim.x) {
        const int y = (int)R;
        for (int x = threadIdx.x; x < d.W; x += blockDim.x) {
            const int g = y * d.ld + x;
            const float fv = d.f[g];
            const float c = c_of(fv, d.delta, d.tl);
            const bool act = c_active(c);
            const float h = (fv < 0.0f) ? 1.0f : 0.0f;
            const float u0 = act ? (d.u0 ? d.u0[g] : h) : h;
            const float px = (act && x < d.W - 1 && d.p0x) ? d.p0x[g] : 0.0f;
            const float py = (act && y < d.H - 1 && d.p0y) ? d.p0y[g] : 0.0f;
            d.c[g] = c;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                d.st[b][0][g] = u0;
                d.st[b][1][g] = u0;   // ubar starts at u
                d.st[b][2][g] = px;
                d.st[b][3][g] = py;
            }
        }
    }
}

template <int BX, int BY, int IT, int NT>
__global__ __launch_bounds__(NT) void k_pd_iterate(PdDesc d, const int2* __restrict__ queue,
                                                   const int32_t* __restrict__ n_queue,
                                                   int in_buf, int nit, float tau, float sigma) {
    constexpr int RX = BX + 2 * IT + 1;
    constexpr int RY = BY + 2 * IT + 1;
    constexpr int RC = RX * RY;
    constexpr int CPT = (RC + NT - 1) / NT;
    constexpr int PAD = RX + 1;
    constexpr int LS = RC + 2 * PAD;
    constexpr int H0 = IT + 1;
    __shared__ float sPX[LS], sPY[LS], sUB[LS];

    const int t = threadIdx.x;
    for (int k = t; k < PAD; k += NT) {
        sPX[k] = 0.0f; sPY[k] = 0.0f; sUB[k] = 0.0f;
        sPX[PAD + RC + k] = 0.0f; sPY[PAD + RC + k] = 0.0f; sUB[PAD + RC + k] = 0.0f;
    }
    // contiguous queue chunk per XCD (workgroups go round-robin over 8 XCDs)
    const int nq = *n_queue;
    const int per = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7;
    const int rank = blockIdx.x >> 3;
    const int chunk = (nq + 7) >> 3;
    const int q0 = xcd * chunk;
    const int q1 = min(nq, q0 + chunk);
    const float* __restrict__ Ui = d.st[in_buf][0];
    const float* __restrict__ UBi = d.st[in_buf][1];
    const float* __restrict__ PXi = d.st[in_buf][2];
    const float* __restrict__ PYi = d.st[in_buf][3];
    float* __restrict__ Uo = d.st[1 - in_buf][0];
    float* __restrict__ UBo = d.st[1 - in_buf][1];
    float* __restrict__ PXo = d.st[1 - in_buf][2];
    float* __restrict__ PYo = d.st[1 - in_buf][3];

    for (int item = q0 + rank; item < q1; item += per) {
        const int2 q = queue[item];
        const int my = q.y / d.mw;
        const int mx = q.y - my * d.mw;
        const int ox = mx * BX - H0, oy = my * BY - H0;
        float ru[CPT], rub[CPT], rpx[CPT], rpy[CPT], rc[CPT];
        uint32_t fl[CPT];
        int gi[CPT];
        __syncthreads();   // LDS of the previous item consumed
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            ru[j] = 0.0f; rub[j] = 0.0f; rpx[j] = 0.0f; rpy[j] = 0.0f;
            rc[j] = __builtin_inff(); fl[j] = 0u; gi[j] = 0;
            if (i < RC) {
                const int ry = i / RX, rx = i - ry * RX;
                const int gx = ox + rx, gy = oy + ry;
                const bool inb = (unsigned)gx < (unsigned)d.W && (unsigned)gy < (unsigned)d.H;
                const int g = gy * d.ld + gx;
                gi[j] = g;
                float c = __builtin_inff(), u = 0.0f, ub = 0.0f, px = 0.0f, py = 0.0f;
                if (inb) {   // issued together; state off RD is discarded
                    c = d.c[g];
                    u = Ui[g];
                    ub = UBi[g];
                    px = PXi[g];
                    py = PYi[g];
                }
                const bool act = c_active(c);
                const float h = heav_from_c(c);
                rc[j] = c;
                ru[j] = act ? u : h;
                rub[j] = act ? ub : h;
                rpx[j] = act ? px : 0.0f;
                rpy[j] = act ? py : 0.0f;
                uint32_t f = act ? CF_ACT : 0u;
                if (gx == d.W - 1) f |= CF_LASTC;
                if (gy == d.H - 1) f |= CF_LASTR;
                const bool interior = rx >= H0 && rx < H0 + BX && ry >= H0 && ry < H0 + BY;
                if (interior && act) f |= CF_OUT;
                fl[j] = f;
                sPX[PAD + i] = rpx[j];
                sPY[PAD + i] = rpy[j];
                sUB[PAD + i] = rub[j];
            }
        }
        __syncthreads();
        for (int it = 0; it < nit; ++it) {
            // phase B: projected ascent on p from grad ubar
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int i = t + j * NT;
                if (i < RC) {
                    pd_dual(rpx[j], rpy[j], rub[j], sUB[PAD + i + 1], sUB[PAD + i + RX], fl[j],
                            sigma);
                    sPX[PAD + i] = rpx[j];
                    sPY[PAD + i] = rpy[j];
                }
            }
            __syncthreads();
            // phase A: clamped descent on u from div p, then the extrapolation
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int i = t + j * NT;
                if (i < RC) {
                    const float dd = div_p(rpx[j], sPX[PAD + i - 1], rpy[j], sPY[PAD + i - RX]);
                    const float un = clamp01(fmaf(tau, dd, ru[j]) - rc[j]);
                    rub[j] = fmaf(2.0f, un, -ru[j]);
                    ru[j] = un;
                    sUB[PAD + i] = rub[j];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if (fl[j] & CF_OUT) {
                Uo[gi[j]] = ru[j];
                UBo[gi[j]] = rub[j];
                PXo[gi[j]] = rpx[j];
                PYo[gi[j]] = rpy[j];
            }
        }
    }
}

using PdFn = void (*)(PdDesc, const int2*, const int32_t*, int, int, float, float);

struct PdCfgEntry {
    TileCfg cfg;
    PdFn fn;
};

#define RDSEG_PD_CFG(bx, by, it, nt) PdCfgEntry{TileCfg{bx, by, it, nt}, k_pd_iterate<bx, by, it, nt>}

const PdCfgEntry kPdCfgs[] = {
    RDSEG_PD_CFG(8, 8, 16, 512),
    RDSEG_PD_CFG(16, 16, 8, 512),
    RDSEG_PD_CFG(32, 32, 4, 256),
    RDSEG_PD_CFG(64, 64, 8, 1024),
};
constexpr int kNumPdCfgs = sizeof(kPdCfgs) / sizeof(kPdCfgs[0]);
int g_pd_grid[kNumPdCfgs];

}  // namespace

int pd_config_count() { return kNumPdCfgs; }
TileCfg pd_config_at(int i) { return kPdCfgs[i].cfg; }
int pd_config_index(int bx, int by, int it) {
    for (int i = 0; i < kNumPdCfgs; ++i)
        if (kPdCfgs[i].cfg.bx == bx && kPdCfgs[i].cfg.by == by && kPdCfgs[i].cfg.it == it) return i;
    return -1;
}

int launch_pd_init(const PdDesc& d, hipStream_t st) {
    const unsigned grid = (unsigned)(d.H < 65536 ? d.H : 65536);
    hipLaunchKernelGGL(k_pd_init, dim3(grid), dim3(256), 0, st, d, (int64_t)d.H);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_pd_iterate(int ci, const PdDesc& d, const int2* queue, const int32_t* n_queue,
                      int64_t max_items, int in_buf, int nit, float tau, float sigma,
                      hipStream_t st) {
    const PdCfgEntry& e = kPdCfgs[ci];
    int& cached = g_pd_grid[ci];
    if (cached == 0) {
        cached = persistent_blocks(reinterpret_cast<const void*>(e.fn), e.cfg.nt, 0);
        if (cached <= 0) {
            cached = 0;
            set_error("occupancy query failed for the primal-dual kernel");
            return 4;
        }
    }
    int64_t g = cached;
    if (max_items < g) g = max_items;
    g = ((g + 7) / 8) * 8;
    if (g < 8) g = 8;
    hipLaunchKernelGGL(e.fn, dim3((unsigned)g), dim3(e.cfg.nt), 0, st, d, queue, n_queue, in_buf,
                       nit, tau, sigma);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace rdseg
