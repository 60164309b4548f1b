/*
 * rdseg_oracle.c -- plain, slow, single-threaded FP64 reference of the
 * restricted-domain dual method for two-phase segmentation
 * (Spencer, "A Restricted-Domain Dual Formulation for Two-Phase Image
 * Segmentation", arXiv 1807.11534).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * What it computes (paper section / equation in brackets):
 *   - restricted domain RD = {x : -q < f(x) < q}, Fg = {f <= -q}, Bg = {f >= q}
 *     [Sec. 3, definition of Fg/Bg/RD]; q is called `delta` here;
 *   - initial indicator u0 = H(-f), Heaviside with H(0) = 0 [Sec. 1];
 *   - the alternating dual iteration of Sec. 2.1 [u-step u = v - theta div p,
 *     Chambolle's semi-implicit fixed point for p, v-step clamp] restricted to
 *     RD as in Sec. 3 [u = 1 on Fg, 0 on Bg; p = 0 off RD; v = 1 / 0 on Fg/Bg];
 *   - the discrete gradient (forward differences, zero on the last column /
 *     row) and divergence (its negative adjoint), which the paper takes from
 *     Chambolle (2004) [end of Sec. 2.1];
 *   - reverse-mode (adjoint) and tangent-linear derivatives of the unrolled
 *     iteration with respect to f and lambda, and the fitting terms of
 *     Sec. 1 [eq. CV, eq. DS] with their derivatives.
 *
 * Readings of points the paper leaves open:
 *   - w = div p - v/theta is set to -h/theta at frozen pixels (div p taken as
 *     0 there), h = H(-f): the exact Chambolle step of the dual of the u
 *     sub-problem restricted to RD with u = h held on Fg and Bg;
 *   - one dual step per outer iteration by default (`inner` > 1 repeats it);
 *   - Jacobi update: every right-hand side uses iterate k;
 *   - v0 = clamp(u0 - theta lambda f, 0, 1), then each outer iteration does
 *     (p, u, v) in that order;
 *   - a caller's u0 / p0 is ignored on frozen pixels.
 *
 * Layout: row-major [H][W], index y*W + x, x contiguous.  f arrives as FP32
 * (held exactly in FP64); every other field is FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_MEM 2

static double clamp01(double s) { return s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s); }

/* Restricted-domain membership [Sec. 3]: strict band |f| < delta, compared in
 * FP64.  NaN compares false, so NaN pixels are frozen. */
static int in_rd(float fv, double delta) { return fabs((double)fv) < delta; }

/* Heaviside of -f [Sec. 1], with H(0) = 0: 1 (foreground) iff f < 0. */
static double heav_neg(float fv) { return ((double)fv < 0.0) ? 1.0 : 0.0; }

/* ------------------------------------------------------------------------ */
/* Active set as 8x8 tiles and as an ascending pixel list.                   */
/* tile id t = ty * ceil(W/8) + tx; mask bit b = (y mod 8) * 8 + (x mod 8);   */
/* slot_map[t] = position of t in the tile list, or -1; pixel id = y*W + x.   */
/* Any output pointer may be NULL.                                            */
/* ------------------------------------------------------------------------ */
int orc_active_set(const float* f, int H, int W, double delta,
                   int32_t* tile_ids, uint64_t* masks, int32_t* slot_map,
                   int32_t* n_tiles, int32_t* pix, int64_t* n_pix)
{
    if (!f || H < 1 || W < 1 || isnan(delta)) return ORC_ERR_ARG;
    int TW = (W + 7) / 8, TH = (H + 7) / 8;
    int32_t nt = 0;
    for (int ty = 0; ty < TH; ++ty) {
        for (int tx = 0; tx < TW; ++tx) {
            uint64_t m = 0;
            for (int r = 0; r < 8; ++r) {
                for (int c = 0; c < 8; ++c) {
                    int y = ty * 8 + r, x = tx * 8 + c;
                    if (y < H && x < W && in_rd(f[(size_t)y * W + x], delta))
                        m |= (uint64_t)1 << (r * 8 + c);
                }
            }
            int t = ty * TW + tx;
            if (m) {
                if (tile_ids) tile_ids[nt] = t;
                if (masks) masks[nt] = m;
                if (slot_map) slot_map[t] = nt;
                ++nt;
            } else if (slot_map) {
                slot_map[t] = -1;
            }
        }
    }
    if (n_tiles) *n_tiles = nt;
    int64_t np = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            if (in_rd(f[(size_t)y * W + x], delta)) {
                if (pix) pix[np] = (int32_t)((size_t)y * W + x);
                ++np;
            }
    if (n_pix) *n_pix = np;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Discrete operators of Chambolle (2004), cited at the end of Sec. 2.1.     */
/* ------------------------------------------------------------------------ */

/* Forward-difference gradient; the x component is 0 on the last column and
 * the y component is 0 on the last row. */
void orc_grad(const double* u, int H, int W, double* gx, double* gy)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            gx[i] = (x < W - 1) ? u[i + 1] - u[i] : 0.0;
            gy[i] = (y < H - 1) ? u[i + W] - u[i] : 0.0;
        }
}

/* Divergence, defined so that div = -grad^T: backward differences in which
 * the component on the first column / row enters alone and the one on the
 * last column / row is not used. */
void orc_div(const double* px, const double* py, int H, int W, double* d)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            double dx = 0.0, dy = 0.0;
            if (x < W - 1) dx += px[i];
            if (x > 0) dx -= px[i - 1];
            if (y < H - 1) dy += py[i];
            if (y > 0) dy -= py[i - W];
            d[i] = dx + dy;
        }
}

/* ------------------------------------------------------------------------ */
/* Work buffers                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int H, W;
    size_t N;
    unsigned char* A;  /* restricted-domain indicator */
    double* h;         /* H(-f) */
    double* fd;        /* f as double */
    double *d, *w, *gx, *gy, *qx, *qy;
} orc_ctx;

static void ctx_free(orc_ctx* c)
{
    free(c->A); free(c->h); free(c->fd); free(c->d); free(c->w);
    free(c->gx); free(c->gy); free(c->qx); free(c->qy);
}

static int ctx_init(orc_ctx* c, const float* f, int H, int W, double delta)
{
    memset(c, 0, sizeof(*c));
    c->H = H; c->W = W; c->N = (size_t)H * W;
    size_t N = c->N;
    c->A = (unsigned char*)malloc(N);
    c->h = (double*)malloc(N * sizeof(double));
    c->fd = (double*)malloc(N * sizeof(double));
    c->d = (double*)malloc(N * sizeof(double));
    c->w = (double*)malloc(N * sizeof(double));
    c->gx = (double*)malloc(N * sizeof(double));
    c->gy = (double*)malloc(N * sizeof(double));
    c->qx = (double*)malloc(N * sizeof(double));
    c->qy = (double*)malloc(N * sizeof(double));
    if (!c->A || !c->h || !c->fd || !c->d || !c->w || !c->gx || !c->gy || !c->qx || !c->qy) {
        ctx_free(c);
        return ORC_ERR_MEM;
    }
    for (size_t i = 0; i < N; ++i) {
        c->A[i] = (unsigned char)in_rd(f[i], delta);
        c->h[i] = heav_neg(f[i]);
        c->fd[i] = (double)f[i];
    }
    return ORC_OK;
}

/* Initial state [Sec. 1: u0 = H(-f); Sec. 3: rho0 = 0, frozen values]. */
static void init_state(const orc_ctx* c, double lambda, double theta,
                       const double* u0, const double* p0x, const double* p0y,
                       double* u, double* v, double* px, double* py)
{
    int H = c->H, W = c->W;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            if (c->A[i]) {
                u[i] = u0 ? u0[i] : c->h[i];
                v[i] = clamp01(u[i] - theta * lambda * c->fd[i]);
                px[i] = (p0x && x < W - 1) ? p0x[i] : 0.0;
                py[i] = (p0y && y < H - 1) ? p0y[i] : 0.0;
            } else {
                u[i] = c->h[i];
                v[i] = c->h[i];
                px[i] = 0.0;
                py[i] = 0.0;
            }
        }
}

/* One Chambolle fixed-point step for p with v held fixed, on RD only
 * [Sec. 3: rho^{n+1} = (rho^n + tau grad(div rho^n - v/theta)) /
 *                      (1 + tau |grad(div rho^n - v/theta)|)].
 * w = div p - v/theta on RD and -h/theta off RD; p stays 0 off RD. */
static void dual_step(orc_ctx* c, double theta, double tau, const double* v,
                      double* px, double* py)
{
    size_t N = c->N;
    orc_div(px, py, c->H, c->W, c->d);
    for (size_t i = 0; i < N; ++i)
        c->w[i] = c->A[i] ? c->d[i] - v[i] / theta : -c->h[i] / theta;
    orc_grad(c->w, c->H, c->W, c->gx, c->gy);
    for (size_t i = 0; i < N; ++i) {
        if (c->A[i]) {
            double n = sqrt(c->gx[i] * c->gx[i] + c->gy[i] * c->gy[i]);
            c->qx[i] = (px[i] + tau * c->gx[i]) / (1.0 + tau * n);
            c->qy[i] = (py[i] + tau * c->gy[i]) / (1.0 + tau * n);
        } else {
            c->qx[i] = 0.0;
            c->qy[i] = 0.0;
        }
    }
    memcpy(px, c->qx, N * sizeof(double));
    memcpy(py, c->qy, N * sizeof(double));
}

/* u-step then v-step on RD [Sec. 3: u = v - theta div rho on RD;
 * v = min(max(u - theta lambda f, 0), 1) on RD]. */
static void uv_step(orc_ctx* c, double lambda, double theta,
                    const double* px, const double* py, double* u, double* v)
{
    size_t N = c->N;
    orc_div(px, py, c->H, c->W, c->d);
    for (size_t i = 0; i < N; ++i)
        if (c->A[i]) u[i] = v[i] - theta * c->d[i];
    for (size_t i = 0; i < N; ++i)
        if (c->A[i]) v[i] = clamp01(u[i] - theta * lambda * c->fd[i]);
}

/* Full restricted solve: init, then `iters` outer iterations, each made of
 * `inner` dual steps followed by the u-step and the v-step.
 * u0, p0x, p0y may be NULL (defaults H(-f) and 0).  Outputs are full grids;
 * frozen pixels hold u = v = H(-f), p = 0. */
int orc_solve(const float* f, int H, int W, double lambda, double theta, double tau,
              double delta, int iters, int inner,
              const double* u0, const double* p0x, const double* p0y,
              double* u, double* v, double* px, double* py)
{
    if (!f || !u || !v || !px || !py || H < 1 || W < 1 || iters < 0 || inner < 1 ||
        !(theta > 0) || !(tau > 0) || !(lambda >= 0) || isnan(delta))
        return ORC_ERR_ARG;
    orc_ctx c;
    if (ctx_init(&c, f, H, W, delta)) return ORC_ERR_MEM;
    init_state(&c, lambda, theta, u0, p0x, p0y, u, v, px, py);
    for (int k = 0; k < iters; ++k) {
        for (int j = 0; j < inner; ++j) dual_step(&c, theta, tau, v, px, py);
        uv_step(&c, lambda, theta, px, py, u, v);
    }
    ctx_free(&c);
    return ORC_OK;
}

/* `n` dual steps with v held fixed (the inner problem alone). */
int orc_dual_steps(const float* f, int H, int W, double theta, double tau, double delta,
                   const double* v, int n, double* px, double* py)
{
    if (!f || !v || !px || !py || H < 1 || W < 1 || n < 0 || !(theta > 0) || !(tau > 0) ||
        isnan(delta))
        return ORC_ERR_ARG;
    orc_ctx c;
    if (ctx_init(&c, f, H, W, delta)) return ORC_ERR_MEM;
    for (int j = 0; j < n; ++j) dual_step(&c, theta, tau, v, px, py);
    ctx_free(&c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Derivatives of the unrolled solve (default start: u0 = H(-f), p0 = 0).    */
/* The domain RD and u0 depend on f only through comparisons, so they are    */
/* held fixed (their derivative is zero almost everywhere).  The clamp has   */
/* derivative 1 strictly inside (0, 1) and 0 elsewhere; d|g|/dg = g/|g| and  */
/* 0 at g = 0.                                                                */
/* ------------------------------------------------------------------------ */

/* Reverse mode.  ubar: adjoint of the final u; vbar (nullable): adjoint of
 * the final v.  Outputs fbar [H][W] and *lambar.  Memory: stores p and v for
 * every iterate, 3 * (iters + 1) * H * W doubles. */
int orc_reverse(const float* f, int H, int W, double lambda, double theta, double tau,
                double delta, int iters, const double* ubar, const double* vbar,
                double* fbar, double* lambar)
{
    if (!f || !ubar || !fbar || !lambar || H < 1 || W < 1 || iters < 0 ||
        !(theta > 0) || !(tau > 0) || !(lambda >= 0) || isnan(delta))
        return ORC_ERR_ARG;
    orc_ctx c;
    if (ctx_init(&c, f, H, W, delta)) return ORC_ERR_MEM;
    size_t N = c.N;
    size_t K1 = (size_t)iters + 1;
    double* Px = (double*)malloc(K1 * N * sizeof(double));
    double* Py = (double*)malloc(K1 * N * sizeof(double));
    double* V = (double*)malloc(K1 * N * sizeof(double));
    double* u = (double*)malloc(N * sizeof(double));
    double* u0 = (double*)malloc(N * sizeof(double));
    double* S = (double*)calloc(N, sizeof(double));     /* sum of clamp adjoints */
    double* pbx = (double*)calloc(N, sizeof(double));
    double* pby = (double*)calloc(N, sizeof(double));
    double* vb = (double*)calloc(N, sizeof(double));
    double* ub = (double*)malloc(N * sizeof(double));
    double* tx = (double*)malloc(N * sizeof(double));
    double* ty = (double*)malloc(N * sizeof(double));
    double* wb = (double*)malloc(N * sizeof(double));
    double* nx = (double*)malloc(N * sizeof(double));  /* new p^k (recomputed) */
    double* ny = (double*)malloc(N * sizeof(double));
    double* gxs = (double*)malloc(N * sizeof(double));
    double* gys = (double*)malloc(N * sizeof(double));
    if (!Px || !Py || !V || !u || !u0 || !S || !pbx || !pby || !vb || !ub || !tx || !ty ||
        !wb || !nx || !ny || !gxs || !gys) {
        free(Px); free(Py); free(V); free(u); free(u0); free(S); free(pbx); free(pby);
        free(vb); free(ub); free(tx); free(ty); free(wb); free(nx); free(ny); free(gxs);
        free(gys);
        ctx_free(&c);
        return ORC_ERR_MEM;
    }
    /* forward sweep, storing every (p^k, v^k) */
    init_state(&c, lambda, theta, NULL, NULL, NULL, u, V, Px, Py);
    memcpy(u0, u, N * sizeof(double));
    for (int k = 0; k < iters; ++k) {
        double* px = Px + (size_t)(k + 1) * N;
        double* py = Py + (size_t)(k + 1) * N;
        double* v = V + (size_t)(k + 1) * N;
        memcpy(px, Px + (size_t)k * N, N * sizeof(double));
        memcpy(py, Py + (size_t)k * N, N * sizeof(double));
        memcpy(v, V + (size_t)k * N, N * sizeof(double));
        dual_step(&c, theta, tau, v, px, py);
        uv_step(&c, lambda, theta, px, py, u, v);
    }
    /* adjoint of the final state */
    for (size_t i = 0; i < N; ++i) vb[i] = (vbar && c.A[i]) ? vbar[i] : 0.0;
    /* reverse sweep */
    for (int k = iters; k >= 1; --k) {
        const double* pxo = Px + (size_t)(k - 1) * N;   /* p^{k-1} */
        const double* pyo = Py + (size_t)(k - 1) * N;
        const double* vo = V + (size_t)(k - 1) * N;     /* v^{k-1} */
        const double* pxn = Px + (size_t)k * N;         /* p^k */
        const double* pyn = Py + (size_t)k * N;
        /* recompute g at step k */
        orc_div(pxo, pyo, H, W, c.d);
        for (size_t i = 0; i < N; ++i)
            c.w[i] = c.A[i] ? c.d[i] - vo[i] / theta : -c.h[i] / theta;
        orc_grad(c.w, H, W, gxs, gys);
        /* u^k and the clamp argument s^k */
        orc_div(pxn, pyn, H, W, c.d);
        for (size_t i = 0; i < N; ++i) {
            if (c.A[i]) {
                double uk = vo[i] - theta * c.d[i];
                double s = uk - theta * lambda * c.fd[i];
                double sb = (s > 0.0 && s < 1.0) ? vb[i] : 0.0;
                S[i] += sb;
                ub[i] = sb + (k == iters ? ubar[i] : 0.0);
            } else {
                ub[i] = 0.0;
            }
        }
        /* u^k = v^{k-1} - theta div p^k:  vbar^{k-1} = ubar;  pbar^k += theta grad(ubar) */
        orc_grad(ub, H, W, tx, ty);
        for (size_t i = 0; i < N; ++i) {
            if (c.A[i]) {
                pbx[i] += theta * tx[i];
                pby[i] += theta * ty[i];
            } else {
                pbx[i] = 0.0;
                pby[i] = 0.0;
            }
            vb[i] = ub[i];
        }
        /* p^k = (p^{k-1} + tau g) / (1 + tau |g|) on RD */
        for (size_t i = 0; i < N; ++i) {
            int x = (int)(i % (size_t)W), y = (int)(i / (size_t)W);
            if (c.A[i]) {
                double gx = gxs[i], gy = gys[i];
                double n = sqrt(gx * gx + gy * gy);
                double m = 1.0 / (1.0 + tau * n);
                double dot = pxn[i] * pbx[i] + pyn[i] * pby[i];
                double hx = n > 0.0 ? gx / n : 0.0, hy = n > 0.0 ? gy / n : 0.0;
                double gbx = tau * m * pbx[i] - tau * m * dot * hx;
                double gby = tau * m * pby[i] - tau * m * dot * hy;
                nx[i] = (x < W - 1) ? gbx : 0.0;   /* reuse nx/ny as gbar */
                ny[i] = (y < H - 1) ? gby : 0.0;
                pbx[i] = (x < W - 1) ? m * pbx[i] : 0.0;
                pby[i] = (y < H - 1) ? m * pby[i] : 0.0;
            } else {
                nx[i] = ny[i] = 0.0;
                pbx[i] = pby[i] = 0.0;
            }
        }
        /* g = grad w:  wbar = grad^T gbar = -div gbar */
        orc_div(nx, ny, H, W, wb);
        for (size_t i = 0; i < N; ++i) wb[i] = c.A[i] ? -wb[i] : 0.0;
        /* w = div p^{k-1} - v^{k-1}/theta on RD */
        for (size_t i = 0; i < N; ++i)
            if (c.A[i]) vb[i] += -wb[i] / theta;
        orc_grad(wb, H, W, tx, ty);   /* div^T = -grad */
        for (size_t i = 0; i < N; ++i) {
            int x = (int)(i % (size_t)W), y = (int)(i / (size_t)W);
            if (c.A[i]) {
                if (x < W - 1) pbx[i] += -tx[i];
                if (y < H - 1) pby[i] += -ty[i];
            }
        }
    }
    /* v^0 = clamp(u^0 - theta lambda f) on RD, with u^0 held fixed */
    for (size_t i = 0; i < N; ++i) {
        if (c.A[i]) {
            double s = u0[i] - theta * lambda * c.fd[i];
            if (s > 0.0 && s < 1.0) S[i] += vb[i];
        }
    }
    double lb = 0.0;
    for (size_t i = 0; i < N; ++i) {
        fbar[i] = c.A[i] ? -theta * lambda * S[i] : 0.0;
        lb += c.A[i] ? -theta * c.fd[i] * S[i] : 0.0;
    }
    *lambar = lb;
    free(Px); free(Py); free(V); free(u); free(u0); free(S); free(pbx); free(pby);
    free(vb); free(ub); free(tx); free(ty); free(wb); free(nx); free(ny); free(gxs);
    free(gys);
    ctx_free(&c);
    return ORC_OK;
}

/* Tangent-linear (forward mode): directional derivative of the final (u, v)
 * along (df, dlam), default start. */
int orc_tangent(const float* f, int H, int W, double lambda, double theta, double tau,
                double delta, int iters, const double* df, double dlam,
                double* du, double* dv)
{
    if (!f || !df || !du || !dv || H < 1 || W < 1 || iters < 0 ||
        !(theta > 0) || !(tau > 0) || !(lambda >= 0) || isnan(delta))
        return ORC_ERR_ARG;
    orc_ctx c;
    if (ctx_init(&c, f, H, W, delta)) return ORC_ERR_MEM;
    size_t N = c.N;
    double* u = (double*)malloc(N * sizeof(double));
    double* v = (double*)malloc(N * sizeof(double));
    double* px = (double*)malloc(N * sizeof(double));
    double* py = (double*)malloc(N * sizeof(double));
    double* dpx = (double*)calloc(N, sizeof(double));
    double* dpy = (double*)calloc(N, sizeof(double));
    double* dw = (double*)malloc(N * sizeof(double));
    double* dgx = (double*)malloc(N * sizeof(double));
    double* dgy = (double*)malloc(N * sizeof(double));
    double* dd = (double*)malloc(N * sizeof(double));
    double* dc = (double*)malloc(N * sizeof(double));
    if (!u || !v || !px || !py || !dpx || !dpy || !dw || !dgx || !dgy || !dd || !dc) {
        free(u); free(v); free(px); free(py); free(dpx); free(dpy); free(dw); free(dgx);
        free(dgy); free(dd); free(dc);
        ctx_free(&c);
        return ORC_ERR_MEM;
    }
    init_state(&c, lambda, theta, NULL, NULL, NULL, u, v, px, py);
    for (size_t i = 0; i < N; ++i) {
        /* c = theta lambda f  =>  dc = theta (dlam f + lambda df) */
        dc[i] = c.A[i] ? theta * (dlam * c.fd[i] + lambda * df[i]) : 0.0;
        double s = u[i] - theta * lambda * c.fd[i];
        dv[i] = (c.A[i] && s > 0.0 && s < 1.0) ? -dc[i] : 0.0;
        du[i] = 0.0;
    }
    for (int k = 0; k < iters; ++k) {
        /* primal g and its tangent, both from iterate k */
        orc_div(px, py, H, W, c.d);
        for (size_t i = 0; i < N; ++i)
            c.w[i] = c.A[i] ? c.d[i] - v[i] / theta : -c.h[i] / theta;
        orc_grad(c.w, H, W, c.gx, c.gy);
        orc_div(dpx, dpy, H, W, dd);
        for (size_t i = 0; i < N; ++i) dw[i] = c.A[i] ? dd[i] - dv[i] / theta : 0.0;
        orc_grad(dw, H, W, dgx, dgy);
        for (size_t i = 0; i < N; ++i) {
            if (c.A[i]) {
                double gx = c.gx[i], gy = c.gy[i];
                double n = sqrt(gx * gx + gy * gy);
                double m = 1.0 / (1.0 + tau * n);
                double dn = n > 0.0 ? (gx * dgx[i] + gy * dgy[i]) / n : 0.0;
                double dm = -tau * m * m * dn;
                double ax = px[i] + tau * gx, ay = py[i] + tau * gy;
                double nxv = ax * m, nyv = ay * m;
                double dnx = (dpx[i] + tau * dgx[i]) * m + ax * dm;
                double dny = (dpy[i] + tau * dgy[i]) * m + ay * dm;
                c.qx[i] = nxv; c.qy[i] = nyv;
                dgx[i] = dnx; dgy[i] = dny;   /* reuse as new dp */
            } else {
                c.qx[i] = c.qy[i] = 0.0;
                dgx[i] = dgy[i] = 0.0;
            }
        }
        memcpy(px, c.qx, N * sizeof(double));
        memcpy(py, c.qy, N * sizeof(double));
        memcpy(dpx, dgx, N * sizeof(double));
        memcpy(dpy, dgy, N * sizeof(double));
        /* u-step and v-step with tangents */
        orc_div(px, py, H, W, c.d);
        orc_div(dpx, dpy, H, W, dd);
        for (size_t i = 0; i < N; ++i) {
            if (c.A[i]) {
                double un = v[i] - theta * c.d[i];
                double dun = dv[i] - theta * dd[i];
                double s = un - theta * lambda * c.fd[i];
                u[i] = un;
                du[i] = dun;
                v[i] = clamp01(s);
                dv[i] = (s > 0.0 && s < 1.0) ? dun - dc[i] : 0.0;
            }
        }
    }
    free(u); free(v); free(px); free(py); free(dpx); free(dpy); free(dw); free(dgx);
    free(dgy); free(dd); free(dc);
    ctx_free(&c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Fitting terms [Sec. 1, eq. CV and eq. DS]:                                */
/*   f = (z - c1)^2 - (z - c2)^2 + gamma P   (P may be NULL: eq. CV)         */
/* and the vector-Jacobian product of f with respect to (c1, c2, gamma).     */
/* ------------------------------------------------------------------------ */
void orc_fit_term(const float* z, const float* P, size_t n, double c1, double c2,
                  double gamma, double* f)
{
    for (size_t i = 0; i < n; ++i) {
        double zi = (double)z[i];
        double a = zi - c1, b = zi - c2;
        f[i] = a * a - b * b + (P ? gamma * (double)P[i] : 0.0);
    }
}

void orc_fit_vjp(const float* z, const float* P, size_t n, double c1, double c2,
                 const double* fbar, double* c1bar, double* c2bar, double* gbar)
{
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double zi = (double)z[i];
        s1 += fbar[i] * (-2.0 * (zi - c1));
        s2 += fbar[i] * (2.0 * (zi - c2));
        if (P) s3 += fbar[i] * (double)P[i];
    }
    *c1bar = s1;
    *c2bar = s2;
    *gbar = s3;
}

/* ------------------------------------------------------------------------ */
/* Band threshold from a target fraction [Sec. 3: q-hat starts at 0 and is   */
/* raised until the fraction of nodes in RD = {|f| < q-hat} reaches q].      */
/* Reading: q-hat is the smallest double with #{|f| < q-hat} >= q N, N = all */
/* nodes.  With a_k the k-th smallest |f| and k = ceil(q N) (exact), that is */
/* 0 for k = 0 and the next double above a_k otherwise.  NaN and infinite    */
/* |f| never enter RD; when fewer than k values are finite no q-hat reaches  */
/* q and the result is +inf (RD = every finite node).                        */
/* ------------------------------------------------------------------------ */

/* ceil(q * n) in exact integer arithmetic: q = M 2^E with M a 53-bit integer. */
int64_t orc_count_needed(double q, int64_t n)
{
    if (!(q > 0.0) || n <= 0) return 0;
    if (q >= 1.0) return n;
    int e;
    double m = frexp(q, &e);                  /* q = m 2^e, 0.5 <= m < 1 */
    uint64_t M = (uint64_t)ldexp(m, 53);      /* exact: q = M 2^(e - 53) */
    int s = 53 - e;                           /* q n = M n / 2^s, s >= 53 */
    unsigned __int128 prod = (unsigned __int128)M * (unsigned __int128)(uint64_t)n;
    if (s >= 127) return prod > 0 ? 1 : 0;    /* 0 < q n < 1 */
    unsigned __int128 one = 1;
    unsigned __int128 k = (prod + ((one << s) - 1)) >> s;
    return (int64_t)k;
}

static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

int orc_band_threshold(const float* f, int H, int W, double q, double* qhat)
{
    if (!f || !qhat || H < 1 || W < 1 || isnan(q) || q < 0.0 || q > 1.0) return ORC_ERR_ARG;
    size_t N = (size_t)H * W;
    int64_t k = orc_count_needed(q, (int64_t)N);
    if (k == 0) { *qhat = 0.0; return ORC_OK; }
    double* a = (double*)malloc(N * sizeof(double));
    if (!a) return ORC_ERR_MEM;
    size_t nf = 0;
    for (size_t i = 0; i < N; ++i) {
        double v = fabs((double)f[i]);
        if (isfinite(v)) a[nf++] = v;
    }
    if ((size_t)k > nf) {
        *qhat = INFINITY;
    } else {
        qsort(a, nf, sizeof(double), cmp_double);
        *qhat = nextafter(a[k - 1], INFINITY);
    }
    free(a);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Convergence-driven solve [Sec. 4: iterate until the larger of the norms   */
/* of u^l - u^(l-1) and v^l - v^(l-1) is at most a tolerance].               */
/* Readings: the norm is the maximum norm over all nodes (frozen nodes never */
/* change); the criterion is evaluated at every iteration l that is a        */
/* multiple of check_every; the solve stops at the first such l that meets   */
/* it, or after max_iters.  diffs (nullable) receives the measured value at  */
/* each evaluated l, in order; *iters_done the number of iterations run.     */
/* Each iteration takes `inner` dual steps, as in orc_solve.                 */
/* ------------------------------------------------------------------------ */
int orc_solve_until(const float* f, int H, int W, double lambda, double theta, double tau,
                    double delta, int max_iters, double tol, int check_every,
                    const double* u0, const double* p0x, const double* p0y,
                    double* u, double* v, double* px, double* py,
                    int* iters_done, double* diffs, int inner)
{
    if (!f || !u || !v || !px || !py || !iters_done || H < 1 || W < 1 || max_iters < 0 ||
        check_every < 1 || inner < 1 || !(theta > 0) || !(tau > 0) || !(lambda >= 0) ||
        isnan(delta) || isnan(tol))
        return ORC_ERR_ARG;
    orc_ctx c;
    if (ctx_init(&c, f, H, W, delta)) return ORC_ERR_MEM;
    size_t N = c.N;
    double* uprev = (double*)malloc(N * sizeof(double));
    double* vprev = (double*)malloc(N * sizeof(double));
    if (!uprev || !vprev) { free(uprev); free(vprev); ctx_free(&c); return ORC_ERR_MEM; }
    init_state(&c, lambda, theta, u0, p0x, p0y, u, v, px, py);
    int done = 0, n_checks = 0;
    for (int l = 1; l <= max_iters; ++l) {
        memcpy(uprev, u, N * sizeof(double));
        memcpy(vprev, v, N * sizeof(double));
        for (int j = 0; j < inner; ++j) dual_step(&c, theta, tau, v, px, py);
        uv_step(&c, lambda, theta, px, py, u, v);
        done = l;
        if (l % check_every == 0) {
            double d = 0.0;
            for (size_t i = 0; i < N; ++i) {
                double du = fabs(u[i] - uprev[i]), dv = fabs(v[i] - vprev[i]);
                if (du > d) d = du;
                if (dv > d) d = dv;
            }
            if (diffs) diffs[n_checks] = d;
            ++n_checks;
            if (d <= tol) break;
        }
    }
    *iters_done = done;
    free(uprev); free(vprev);
    ctx_free(&c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Evaluation measures [Sec. 4]: thresholded labels GT = (u_gt > eps) and    */
/* Omega = (u > eps); E1 = N(GT and Omega) / N(GT or Omega) (Tanimoto), E2 = */
/* the integral of (u - u_gt)^2, here a plain sum over nodes (unit cell).    */
/* Returns the two counts and E2; E1 with an empty union is taken as 1.      */
/* ------------------------------------------------------------------------ */
void orc_metrics(const double* u, const double* ugt, size_t n, double eps,
                 int64_t* n_inter, int64_t* n_union, double* e2)
{
    int64_t a = 0, b = 0;
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) {
        int g = ugt[i] > eps, o = u[i] > eps;
        a += (g && o);
        b += (g || o);
        double d = u[i] - ugt[i];
        s += d * d;
    }
    *n_inter = a;
    *n_union = b;
    *e2 = s;
}

/* ------------------------------------------------------------------------ */
/* Volumes (the conclusion, Sec. 5, names 3-D problems as an extension of    */
/* interest; the method carries over with a third axis).  Layout             */
/* [D][H][W], index (z*H + y)*W + x.  Gradient: forward differences along    */
/* x, y and z with a zero component on the last plane of each axis;          */
/* divergence: its negative adjoint.  The restricted iteration is the one of */
/* orc_solve with the 3-vector p and |g| the Euclidean norm of the 3-vector. */
/* ------------------------------------------------------------------------ */
void orc_grad3(const double* u, int D, int H, int W, double* gx, double* gy, double* gz)
{
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t i = ((size_t)z * H + y) * W + x;
                gx[i] = x < W - 1 ? u[i + 1] - u[i] : 0.0;
                gy[i] = y < H - 1 ? u[i + W] - u[i] : 0.0;
                gz[i] = z < D - 1 ? u[i + (size_t)H * W] - u[i] : 0.0;
            }
}

void orc_div3(const double* px, const double* py, const double* pz, int D, int H, int W,
              double* d)
{
    size_t S = (size_t)H * W;
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t i = ((size_t)z * H + y) * W + x;
                double a = (x < W - 1 ? px[i] : 0.0) - (x > 0 ? px[i - 1] : 0.0);
                double b = (y < H - 1 ? py[i] : 0.0) - (y > 0 ? py[i - W] : 0.0);
                double c = (z < D - 1 ? pz[i] : 0.0) - (z > 0 ? pz[i - S] : 0.0);
                d[i] = a + b + c;
            }
}

/* Restricted solve on a volume: init as orc_solve (u0 = H(-f) or the        */
/* caller's, v0 = clamp(u0 - theta lambda f), p0 = 0 or the caller's with the */
/* last-plane components zero), then iters x (inner dual steps, u-step,      */
/* v-step) on RD = {|f| < delta}; frozen voxels hold u = v = H(-f), p = 0.    */
int orc_solve3(const float* f, int D, int H, int W, double lambda, double theta, double tau,
               double delta, int iters, int inner, const double* u0, const double* p0x,
               const double* p0y, const double* p0z, double* u, double* v, double* px,
               double* py, double* pz)
{
    if (!f || !u || !v || !px || !py || !pz || D < 1 || H < 1 || W < 1 || iters < 0 ||
        inner < 1 || !(theta > 0) || !(tau > 0) || !(lambda >= 0) || isnan(delta))
        return ORC_ERR_ARG;
    size_t N = (size_t)D * H * W;
    unsigned char* A = (unsigned char*)malloc(N);
    double* h = (double*)malloc(N * sizeof(double));
    double* d = (double*)malloc(N * sizeof(double));
    double* w = (double*)malloc(N * sizeof(double));
    double* gx = (double*)malloc(N * sizeof(double));
    double* gy = (double*)malloc(N * sizeof(double));
    double* gz = (double*)malloc(N * sizeof(double));
    if (!A || !h || !d || !w || !gx || !gy || !gz) {
        free(A); free(h); free(d); free(w); free(gx); free(gy); free(gz);
        return ORC_ERR_MEM;
    }
    for (size_t i = 0; i < N; ++i) {
        A[i] = (unsigned char)in_rd(f[i], delta);
        h[i] = heav_neg(f[i]);
    }
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t i = ((size_t)z * H + y) * W + x;
                if (A[i]) {
                    u[i] = u0 ? u0[i] : h[i];
                    v[i] = clamp01(u[i] - theta * lambda * (double)f[i]);
                    px[i] = (p0x && x < W - 1) ? p0x[i] : 0.0;
                    py[i] = (p0y && y < H - 1) ? p0y[i] : 0.0;
                    pz[i] = (p0z && z < D - 1) ? p0z[i] : 0.0;
                } else {
                    u[i] = v[i] = h[i];
                    px[i] = py[i] = pz[i] = 0.0;
                }
            }
    for (int k = 0; k < iters; ++k) {
        for (int j = 0; j < inner; ++j) {
            /* dual step with v held: w = div p - v/theta on RD, -h/theta off RD */
            orc_div3(px, py, pz, D, H, W, d);
            for (size_t i = 0; i < N; ++i) w[i] = A[i] ? d[i] - v[i] / theta : -h[i] / theta;
            orc_grad3(w, D, H, W, gx, gy, gz);
            for (size_t i = 0; i < N; ++i) {
                if (!A[i]) continue;
                double n = sqrt(gx[i] * gx[i] + gy[i] * gy[i] + gz[i] * gz[i]);
                px[i] = (px[i] + tau * gx[i]) / (1.0 + tau * n);
                py[i] = (py[i] + tau * gy[i]) / (1.0 + tau * n);
                pz[i] = (pz[i] + tau * gz[i]) / (1.0 + tau * n);
            }
        }
        /* u-step, then v-step, on RD */
        orc_div3(px, py, pz, D, H, W, d);
        for (size_t i = 0; i < N; ++i)
            if (A[i]) u[i] = v[i] - theta * d[i];
        for (size_t i = 0; i < N; ++i)
            if (A[i]) v[i] = clamp01(u[i] - theta * lambda * (double)f[i]);
    }
    free(A); free(h); free(d); free(w); free(gx); free(gy); free(gz);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The restriction applied to another solver (Sec. 5 proposes carrying the   */
/* restricted domain over to other methods): the first-order primal-dual     */
/* iteration of Chambolle and Pock for eq. CR itself,                        */
/*     min over u in [0,1] of  TV(u) + lambda <f, u>,                         */
/* restricted as in Sec. 3: u = H(-f) on Fg and Bg, p = 0 there, the TV terms */
/* of the pixels of RD.  Per iteration, on RD:                               */
/*     p <- (p + sigma grad ubar) / max(1, |p + sigma grad ubar|)             */
/*     u_new = clamp(u + tau div p - tau lambda f, 0, 1)                      */
/*     ubar  = 2 u_new - u                                                   */
/* with ubar = u = H(-f) off RD; sigma tau <= 1/8 for convergence.           */
/* Start: u0 (or H(-f)), ubar0 = u0, p0 (or 0).  Outputs u, p.               */
/* ------------------------------------------------------------------------ */
int orc_solve_pd(const float* f, int H, int W, double lambda, double tau, double sigma,
                 double delta, int iters, const double* u0, const double* p0x,
                 const double* p0y, double* u, double* px, double* py)
{
    if (!f || !u || !px || !py || H < 1 || W < 1 || iters < 0 || !(tau > 0) || !(sigma > 0) ||
        !(lambda >= 0) || isnan(delta))
        return ORC_ERR_ARG;
    orc_ctx c;
    if (ctx_init(&c, f, H, W, delta)) return ORC_ERR_MEM;
    size_t N = c.N;
    double* ub = (double*)malloc(N * sizeof(double));
    if (!ub) { ctx_free(&c); return ORC_ERR_MEM; }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            if (c.A[i]) {
                u[i] = u0 ? u0[i] : c.h[i];
                px[i] = (p0x && x < W - 1) ? p0x[i] : 0.0;
                py[i] = (p0y && y < H - 1) ? p0y[i] : 0.0;
            } else {
                u[i] = c.h[i];
                px[i] = py[i] = 0.0;
            }
            ub[i] = u[i];
        }
    for (int k = 0; k < iters; ++k) {
        orc_grad(ub, H, W, c.gx, c.gy);
        for (size_t i = 0; i < N; ++i) {
            if (!c.A[i]) continue;
            double ax = px[i] + sigma * c.gx[i], ay = py[i] + sigma * c.gy[i];
            double n = sqrt(ax * ax + ay * ay);
            double s = n > 1.0 ? n : 1.0;
            px[i] = ax / s;
            py[i] = ay / s;
        }
        orc_div(px, py, H, W, c.d);
        for (size_t i = 0; i < N; ++i) {
            if (!c.A[i]) continue;
            double un = clamp01(u[i] + tau * c.d[i] - tau * lambda * c.fd[i]);
            ub[i] = 2.0 * un - u[i];
            u[i] = un;
        }
    }
    free(ub);
    ctx_free(&c);
    return ORC_OK;
}
