// volume.hip -- the restricted iteration on volumes [D][H][W] (7-point
// stencil; the conclusion, Sec. 5, names 3-D problems as the extension of
// interest).  Per voxel the arithmetic is that of the images with a third
// gradient / divergence component, in the same operation order, so a volume of
// identical slices reproduces the image solve bit for bit.
//
// One launch runs one dual step (plus, at the end of an outer iteration, the
// u-step and v-step) with one workgroup per 32 x 16 column tile and chunk of 32
// planes, streamed along z (see k_stream3): the x-y halo is two voxels on the
// low side and one on the high side, the z neighbours pass from one plane to
// the next in registers.  Deeper temporal blocking would multiply the halo
// volume, so the kernel streams its 36 bytes per voxel of RD (read c, v, p:
// 20; write v, p: 16) from HBM; frozen voxels cost their 4-byte c alone.
// Tiles without a voxel of RD return at once (flags computed once per solve).
#include <algorithm>

#include "rdseg_internal.h"

namespace rdseg {

namespace {

__device__ __forceinline__ float div_p3(float pxc, float pxl, float pyc, float pyu, float pzc,
                                        float pzd) {
    return div_p(pxc, pxl, pyc, pyu) + (pzc - pzd);
}

__global__ __launch_bounds__(256) void k_init3(VolDesc d) {
    const int64_t rows = (int64_t)d.D * d.H;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int z = (int)(r / d.H), y = (int)(r - (int64_t)z * d.H);
        for (int x = threadIdx.x; x < d.W; x += blockDim.x) {
            const int g = z * d.lds + y * d.ld + x;
            const float fv = d.f[g];
            const float c = c_of(fv, d.delta, d.tl);
            const bool act = c_active(c);
            const float h = (fv < 0.0f) ? 1.0f : 0.0f;
            const float u0 = act ? (d.u0 ? d.u0[g] : h) : h;
            const float v0 = v_step(u0, c);
            const float px = (act && x < d.W - 1 && d.p0[0]) ? d.p0[0][g] : 0.0f;
            const float py = (act && y < d.H - 1 && d.p0[1]) ? d.p0[1][g] : 0.0f;
            const float pz = (act && z < d.D - 1 && d.p0[2]) ? d.p0[2][g] : 0.0f;
            d.c[g] = c;
            d.u[g] = u0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                d.st[b][0][g] = v0;
                d.st[b][1][g] = px;
                d.st[b][2][g] = py;
                d.st[b][3][g] = pz;
            }
        }
    }
}

// flags[t] = 1 when tile t (of size BX x BY x BZ) holds a voxel of RD.
__global__ __launch_bounds__(256) void k_tile_flags3(VolDesc d, int bx, int by, int bz,
                                                     int32_t* __restrict__ flags) {
    const int ntx = (d.W + bx - 1) / bx, nty = (d.H + by - 1) / by;
    const int t = blockIdx.x;
    const int tz = t / (ntx * nty), r = t - tz * ntx * nty;
    const int ty = r / ntx, tx = r - ty * ntx;
    int any = 0;
    for (int k = threadIdx.x; k < bx * by * bz; k += blockDim.x) {
        const int z = tz * bz + k / (bx * by);
        const int rem = k % (bx * by);
        const int y = ty * by + rem / bx, x = tx * bx + rem % bx;
        if (x < d.W && y < d.H && z < d.D && c_active(d.c[z * d.lds + y * d.ld + x])) any = 1;
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) flags[t] = any;
}

// One dual step (and, at the end of an outer iteration, the u/v step) on a
// BX x BY column tile over ZC planes, streamed plane by plane.  Step s loads
// plane s, forms w(s), then finishes plane s - 1: its dual step (w of planes
// s - 1 and s), then its u/v step (the new p of planes s - 1 and s - 2).  The
// z neighbours travel in registers from one step to the next; only the x-y
// neighbours go through LDS, so the halo is x-y only (2 low, 1 high) and the
// z halo is the two planes below the chunk and one above.
template <int BX, int BY, int ZC, int NT>
__global__ __launch_bounds__(NT) void k_stream3(VolDesc d, const int32_t* __restrict__ flags,
                                                int in_buf, int uv, int write_u, float theta,
                                                float inv_theta, float tau) {
    constexpr int RX = BX + 3, RY = BY + 3, RS = RX * RY;   // plane region
    constexpr int CPT = (RS + NT - 1) / NT;
    constexpr int PAD = RX + 1;
    constexpr int LS = RS + 2 * PAD;
    constexpr uint32_t XY_IN = 32u, XY_OUT = 64u;   // in the grid / in the tile
    __shared__ float sPX[LS], sPY[LS];    // old p of plane s (x-y divergence of w(s))
    __shared__ float sW[2][LS];           // w of planes s - 1 and s
    __shared__ float sNX[LS], sNY[LS];    // new p of plane s - 1

    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of tiles so that x and y neighbours, which fetch each
    // other's halo lines, share that XCD's L2.
    const int ntx = (d.W + BX - 1) / BX, nty = (d.H + BY - 1) / BY;
    const int ntz = (d.D + ZC - 1) / ZC;
    const int n_tiles = ntx * nty * ntz;
    const int per_xcd = (n_tiles + 7) >> 3;
    const int tb = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (tb >= n_tiles || !flags[tb]) return;
    const int tz = tb / (ntx * nty), rt = tb - tz * ntx * nty;
    const int ty = rt / ntx, tx = rt - ty * ntx;
    const int ox = tx * BX - 2, oy = ty * BY - 2;
    const int z0 = tz * ZC, z1 = min(z0 + ZC, d.D);
    const int t = threadIdx.x;
    for (int k = t; k < PAD; k += NT) {
        sPX[k] = 0.0f; sPY[k] = 0.0f; sW[0][k] = 0.0f; sW[1][k] = 0.0f;
        sNX[k] = 0.0f; sNY[k] = 0.0f;
        sPX[PAD + RS + k] = 0.0f; sPY[PAD + RS + k] = 0.0f; sW[0][PAD + RS + k] = 0.0f;
        sW[1][PAD + RS + k] = 0.0f; sNX[PAD + RS + k] = 0.0f; sNY[PAD + RS + k] = 0.0f;
    }
    const float* __restrict__ Vi = d.st[in_buf][0];
    const float* __restrict__ PXi = d.st[in_buf][1];
    const float* __restrict__ PYi = d.st[in_buf][2];
    const float* __restrict__ PZi = d.st[in_buf][3];
    float* __restrict__ Vo = d.st[1 - in_buf][0];
    float* __restrict__ PXo = d.st[1 - in_buf][1];
    float* __restrict__ PYo = d.st[1 - in_buf][2];
    float* __restrict__ PZo = d.st[1 - in_buf][3];

    int gxy[CPT];
    uint32_t fxy[CPT];
    // plane s - 1: old state, its w, and the new p_z of plane s - 2
    float c1[CPT], v1[CPT], px1[CPT], py1[CPT], pz1[CPT], w1[CPT], pzn2[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int i = t + j * NT;
        const int ry = i / RX, rx = i - ry * RX;
        const int gx = ox + rx, gy = oy + ry;
        uint32_t f = 0u;
        if (i < RS && (unsigned)gx < (unsigned)d.W && (unsigned)gy < (unsigned)d.H) {
            f |= XY_IN;
            if (gx == d.W - 1) f |= CF_LASTC;
            if (gy == d.H - 1) f |= CF_LASTR;
            if (rx >= 2 && rx < 2 + BX && ry >= 2 && ry < 2 + BY) f |= XY_OUT;
        }
        fxy[j] = f;
        gxy[j] = gy * d.ld + gx;
        c1[j] = __builtin_inff(); v1[j] = 0.0f; px1[j] = 0.0f; py1[j] = 0.0f; pz1[j] = 0.0f;
        w1[j] = 0.0f; pzn2[j] = 0.0f;
    }
    // Raw loads run ahead of the planes they feed: c two planes ahead, the
    // state (v, p) of the next plane one plane ahead and only for its RD
    // voxels (the state of a frozen voxel is not used, so lines holding only
    // frozen voxels are never fetched), so that their latency overlaps the
    // three phases of the current plane.
    float lc[CPT], nc[CPT], lv[CPT], lpx[CPT], lpy[CPT], lpz[CPT];
    auto fetch_c = [&](int z, float* dst) {
        const bool zin = z >= 0 && z < d.D;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            dst[j] = __builtin_inff();
            if (zin && (fxy[j] & XY_IN)) dst[j] = d.c[z * d.lds + gxy[j]];
        }
    };
    auto fetch_state = [&](int z) {   // plane z, whose c is in lc
        const bool zin = z >= 0 && z < d.D;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            lv[j] = 0.0f; lpx[j] = 0.0f; lpy[j] = 0.0f; lpz[j] = 0.0f;
            if (zin && (fxy[j] & XY_IN) && c_active(lc[j])) {
                const int g = z * d.lds + gxy[j];
                lv[j] = Vi[g];
                lpx[j] = PXi[g];
                lpy[j] = PYi[g];
                lpz[j] = PZi[g];
            }
        }
    };
    fetch_c(z0 - 2, lc);
    fetch_state(z0 - 2);
    fetch_c(z0 - 1, nc);
    int cur = 0;
    for (int s = z0 - 2; s <= z1; ++s) {
        float c0[CPT], v0[CPT], px0[CPT], py0[CPT], pz0[CPT], w0[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const float c = lc[j];
            const bool act = c_active(c);
            c0[j] = c;
            v0[j] = act ? lv[j] : heav_from_c(c);
            px0[j] = act ? lpx[j] : 0.0f;
            py0[j] = act ? lpy[j] : 0.0f;
            pz0[j] = act ? lpz[j] : 0.0f;
        }
        if (s < z1) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) lc[j] = nc[j];
            fetch_state(s + 1);
            if (s + 2 <= z1) fetch_c(s + 2, nc);
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            if (i < RS) {
                sPX[PAD + i] = px0[j];
                sPY[PAD + i] = py0[j];
            }
        }
        __syncthreads();
        // w(s) = div p - v/theta on RD, -H(-f)/theta off RD
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            if (i < RS) {
                const float dd = div_p3(px0[j], sPX[PAD + i - 1], py0[j], sPY[PAD + i - RX],
                                        pz0[j], pz1[j]);
                w0[j] = w_of(dd, v0[j], inv_theta, c_active(c0[j]));
                sW[cur][PAD + i] = w0[j];
            }
        }
        __syncthreads();
        // dual step of plane s - 1 (from w of planes s - 1 and s)
        float pxn[CPT], pyn[CPT], pzn[CPT];
        const bool lastz = s - 1 == d.D - 1;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            pxn[j] = 0.0f; pyn[j] = 0.0f; pzn[j] = 0.0f;
            if (i < RS && s - 1 >= z0 - 1) {
                const float wc = w1[j];
                const float gx = (fxy[j] & CF_LASTC) ? 0.0f : (sW[cur ^ 1][PAD + i + 1] - wc);
                const float gy = (fxy[j] & CF_LASTR) ? 0.0f : (sW[cur ^ 1][PAD + i + RX] - wc);
                const float gz = lastz ? 0.0f : (w0[j] - wc);
                const float nn = __builtin_amdgcn_sqrtf(fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
                const float m = __builtin_amdgcn_rcpf(fmaf(tau, nn, 1.0f));
                const bool act = c_active(c1[j]);
                pxn[j] = act ? fmaf(tau, gx, px1[j]) * m : 0.0f;
                pyn[j] = act ? fmaf(tau, gy, py1[j]) * m : 0.0f;
                pzn[j] = act ? fmaf(tau, gz, pz1[j]) * m : 0.0f;
                sNX[PAD + i] = pxn[j];
                sNY[PAD + i] = pyn[j];
            }
        }
        __syncthreads();
        // u-step and v-step of plane s - 1, then its tile voxels are written
        if (s - 1 >= z0) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int i = t + j * NT;
                if (i < RS && (fxy[j] & XY_OUT) && c_active(c1[j])) {
                    float vn = v1[j];
                    const int g = (s - 1) * d.lds + gxy[j];
                    if (uv) {
                        const float dd = div_p3(pxn[j], sNX[PAD + i - 1], pyn[j],
                                                sNY[PAD + i - RX], pzn[j], pzn2[j]);
                        const float u = u_step(v1[j], dd, theta);
                        vn = v_step(u, c1[j]);
                        if (write_u) d.u[g] = u;
                    }
                    Vo[g] = vn;
                    PXo[g] = pxn[j];
                    PYo[g] = pyn[j];
                    PZo[g] = pzn[j];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            c1[j] = c0[j]; v1[j] = v0[j]; px1[j] = px0[j]; py1[j] = py0[j]; pz1[j] = pz0[j];
            w1[j] = w0[j]; pzn2[j] = pzn[j];
        }
        cur ^= 1;
    }
}

// Two time steps per pass: the second step's pipeline runs one plane behind
// the first in the same z-stream.  At step s the first level forms w^k(s) from
// the raw plane s and finishes plane s - 1 (its dual step, its u/v step when
// uv1, then w^{k+1}(s - 1)); the second level finishes plane s - 2 (its dual
// step from w^{k+1} of planes s - 2 and s - 1, its u/v step when uv2) and
// writes it.  Each level costs the x-y halo one cell low (the divergence) and
// one cell around the gradient, so the region is the tile plus 3 low and 2 high
// (checked cell by cell: the second level's u/v step is exact for region
// x, y in [3, R - 2)); in z the stream starts three planes below the chunk and
// ends one above.  Same per-voxel functions in the same order as k_stream3, so
// results are bitwise equal to two launches of it; half the HBM traffic per
// dual step.
template <int BX, int BY, int ZC, int NT>
__global__ __launch_bounds__(NT, 4) void k_stream3x2(VolDesc d, const int32_t* __restrict__ flags,
                                                  int in_buf, int uv1, int uv2, int write_u,
                                                  float theta, float inv_theta, float tau) {
    constexpr int HL = 3, HH = 2;
    constexpr int RX = BX + HL + HH, RY = BY + HL + HH, RS = RX * RY;
    constexpr int CPT = (RS + NT - 1) / NT;
    constexpr int PAD = RX + 1;
    constexpr int LS = RS + 2 * PAD;
    constexpr uint32_t XY_IN = 32u, XY_OUT = 64u;
    __shared__ float sPX[LS], sPY[LS];    // p^k of plane s
    __shared__ float sW[2][LS];           // w^k of planes s - 1 and s
    __shared__ float sNX[LS], sNY[LS];    // p^(k+1) of plane s - 1
    __shared__ float sW2[2][LS];          // w^(k+1) of planes s - 2 and s - 1
    __shared__ float sMX[LS], sMY[LS];    // p^(k+2) of plane s - 2

    const int ntx = (d.W + BX - 1) / BX, nty = (d.H + BY - 1) / BY;
    const int ntz = (d.D + ZC - 1) / ZC;
    const int n_tiles = ntx * nty * ntz;
    const int per_xcd = (n_tiles + 7) >> 3;
    const int tb = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (tb >= n_tiles || !flags[tb]) return;
    const int tz = tb / (ntx * nty), rt = tb - tz * ntx * nty;
    const int ty = rt / ntx, tx = rt - ty * ntx;
    const int ox = tx * BX - HL, oy = ty * BY - HL;
    const int z0 = tz * ZC, z1 = min(z0 + ZC, d.D);
    const int t = threadIdx.x;
    for (int k = t; k < PAD; k += NT) {
        sPX[k] = 0.0f; sPY[k] = 0.0f; sNX[k] = 0.0f; sNY[k] = 0.0f; sMX[k] = 0.0f; sMY[k] = 0.0f;
        sW[0][k] = 0.0f; sW[1][k] = 0.0f; sW2[0][k] = 0.0f; sW2[1][k] = 0.0f;
        const int e = PAD + RS + k;
        sPX[e] = 0.0f; sPY[e] = 0.0f; sNX[e] = 0.0f; sNY[e] = 0.0f; sMX[e] = 0.0f; sMY[e] = 0.0f;
        sW[0][e] = 0.0f; sW[1][e] = 0.0f; sW2[0][e] = 0.0f; sW2[1][e] = 0.0f;
    }
    const float* __restrict__ Vi = d.st[in_buf][0];
    const float* __restrict__ PXi = d.st[in_buf][1];
    const float* __restrict__ PYi = d.st[in_buf][2];
    const float* __restrict__ PZi = d.st[in_buf][3];
    float* __restrict__ Vo = d.st[1 - in_buf][0];
    float* __restrict__ PXo = d.st[1 - in_buf][1];
    float* __restrict__ PYo = d.st[1 - in_buf][2];
    float* __restrict__ PZo = d.st[1 - in_buf][3];

    int gxy[CPT];
    uint32_t fxy[CPT];
    // level 1 (plane s - 1): raw state, w^k, and p_z^(k+1) of plane s - 2
    float c1[CPT], v1[CPT], px1[CPT], py1[CPT], pz1[CPT], w1[CPT], pzn2[CPT];
    // level 2 (plane s - 2): c, v^(k+1), p^(k+1), w^(k+1); p_z^(k+2) of plane s - 3
    float c2[CPT], v2[CPT], qx2[CPT], qy2[CPT], qz2[CPT], w2b[CPT], pzm3[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int i = t + j * NT;
        const int ry = i / RX, rx = i - ry * RX;
        const int gx = ox + rx, gy = oy + ry;
        uint32_t f = 0u;
        if (i < RS && (unsigned)gx < (unsigned)d.W && (unsigned)gy < (unsigned)d.H) {
            f |= XY_IN;
            if (gx == d.W - 1) f |= CF_LASTC;
            if (gy == d.H - 1) f |= CF_LASTR;
            if (rx >= HL && rx < HL + BX && ry >= HL && ry < HL + BY) f |= XY_OUT;
        }
        fxy[j] = f;
        gxy[j] = gy * d.ld + gx;
        c1[j] = __builtin_inff(); v1[j] = 0.0f; px1[j] = 0.0f; py1[j] = 0.0f; pz1[j] = 0.0f;
        w1[j] = 0.0f; pzn2[j] = 0.0f;
        c2[j] = __builtin_inff(); v2[j] = 0.0f; qx2[j] = 0.0f; qy2[j] = 0.0f; qz2[j] = 0.0f;
        w2b[j] = 0.0f; pzm3[j] = 0.0f;
    }
    float lc[CPT], nc[CPT], lv[CPT], lpx[CPT], lpy[CPT], lpz[CPT];
    auto fetch_c = [&](int z, float* dst) {
        const bool zin = z >= 0 && z < d.D;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            dst[j] = __builtin_inff();
            if (zin && (fxy[j] & XY_IN)) dst[j] = d.c[z * d.lds + gxy[j]];
        }
    };
    auto fetch_state = [&](int z) {   // plane z, whose c is in lc
        const bool zin = z >= 0 && z < d.D;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            lv[j] = 0.0f; lpx[j] = 0.0f; lpy[j] = 0.0f; lpz[j] = 0.0f;
            if (zin && (fxy[j] & XY_IN) && c_active(lc[j])) {
                const int g = z * d.lds + gxy[j];
                lv[j] = Vi[g];
                lpx[j] = PXi[g];
                lpy[j] = PYi[g];
                lpz[j] = PZi[g];
            }
        }
    };
    const int zs = z0 - 3, ze = z1 + 1;   // raw planes streamed
    fetch_c(zs, lc);
    fetch_state(zs);
    fetch_c(zs + 1, nc);
    int cur = 0, cur2 = 0;
    for (int s = zs; s <= ze; ++s) {
        float c0[CPT], v0[CPT], px0[CPT], py0[CPT], pz0[CPT], w0[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const float c = lc[j];
            const bool act = c_active(c);
            c0[j] = c;
            v0[j] = act ? lv[j] : heav_from_c(c);
            px0[j] = act ? lpx[j] : 0.0f;
            py0[j] = act ? lpy[j] : 0.0f;
            pz0[j] = act ? lpz[j] : 0.0f;
        }
        if (s < ze) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) lc[j] = nc[j];
            fetch_state(s + 1);
            if (s + 2 <= ze) fetch_c(s + 2, nc);
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            if (i < RS) {
                sPX[PAD + i] = px0[j];
                sPY[PAD + i] = py0[j];
            }
        }
        __syncthreads();
        // level 1: w^k(s)
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            if (i < RS) {
                const float dd = div_p3(px0[j], sPX[PAD + i - 1], py0[j], sPY[PAD + i - RX],
                                        pz0[j], pz1[j]);
                w0[j] = w_of(dd, v0[j], inv_theta, c_active(c0[j]));
                sW[cur][PAD + i] = w0[j];
            }
        }
        __syncthreads();
        // level 1: dual step of plane s - 1
        float pxn[CPT], pyn[CPT], pzn[CPT];
        const bool lastz1 = s - 1 == d.D - 1;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            pxn[j] = 0.0f; pyn[j] = 0.0f; pzn[j] = 0.0f;
            if (i < RS && s - 1 >= z0 - 2) {
                const float wc = w1[j];
                const float gx = (fxy[j] & CF_LASTC) ? 0.0f : (sW[cur ^ 1][PAD + i + 1] - wc);
                const float gy = (fxy[j] & CF_LASTR) ? 0.0f : (sW[cur ^ 1][PAD + i + RX] - wc);
                const float gz = lastz1 ? 0.0f : (w0[j] - wc);
                const float nn = __builtin_amdgcn_sqrtf(fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
                const float m = __builtin_amdgcn_rcpf(fmaf(tau, nn, 1.0f));
                const bool act = c_active(c1[j]);
                pxn[j] = act ? fmaf(tau, gx, px1[j]) * m : 0.0f;
                pyn[j] = act ? fmaf(tau, gy, py1[j]) * m : 0.0f;
                pzn[j] = act ? fmaf(tau, gz, pz1[j]) * m : 0.0f;
                sNX[PAD + i] = pxn[j];
                sNY[PAD + i] = pyn[j];
            }
        }
        __syncthreads();
        // level 1: u/v step of plane s - 1, then w^(k+1)(s - 1)
        float vn1[CPT], wn[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            vn1[j] = v1[j];
            wn[j] = 0.0f;
            if (i < RS && s - 1 >= z0 - 1) {
                const float dd = div_p3(pxn[j], sNX[PAD + i - 1], pyn[j], sNY[PAD + i - RX],
                                        pzn[j], pzn2[j]);
                if (uv1) vn1[j] = v_step(u_step(v1[j], dd, theta), c1[j]);
                wn[j] = w_of(dd, vn1[j], inv_theta, c_active(c1[j]));
                sW2[cur2][PAD + i] = wn[j];
            }
        }
        __syncthreads();
        // level 2: dual step of plane s - 2
        float mxn[CPT], myn[CPT], mzn[CPT];
        const bool lastz2 = s - 2 == d.D - 1;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int i = t + j * NT;
            mxn[j] = 0.0f; myn[j] = 0.0f; mzn[j] = 0.0f;
            if (i < RS && s - 2 >= z0 - 1) {
                const float wc = w2b[j];
                const float gx = (fxy[j] & CF_LASTC) ? 0.0f : (sW2[cur2 ^ 1][PAD + i + 1] - wc);
                const float gy = (fxy[j] & CF_LASTR) ? 0.0f : (sW2[cur2 ^ 1][PAD + i + RX] - wc);
                const float gz = lastz2 ? 0.0f : (wn[j] - wc);
                const float nn = __builtin_amdgcn_sqrtf(fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
                const float m = __builtin_amdgcn_rcpf(fmaf(tau, nn, 1.0f));
                const bool act = c_active(c2[j]);
                mxn[j] = act ? fmaf(tau, gx, qx2[j]) * m : 0.0f;
                myn[j] = act ? fmaf(tau, gy, qy2[j]) * m : 0.0f;
                mzn[j] = act ? fmaf(tau, gz, qz2[j]) * m : 0.0f;
                sMX[PAD + i] = mxn[j];
                sMY[PAD + i] = myn[j];
            }
        }
        __syncthreads();
        // level 2: u/v step of plane s - 2, then its tile voxels are written
        if (s - 2 >= z0 && s - 2 < z1) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int i = t + j * NT;
                if (i < RS && (fxy[j] & XY_OUT) && c_active(c2[j])) {
                    float vn = v2[j];
                    const int g = (s - 2) * d.lds + gxy[j];
                    if (uv2) {
                        const float dd = div_p3(mxn[j], sMX[PAD + i - 1], myn[j],
                                                sMY[PAD + i - RX], mzn[j], pzm3[j]);
                        const float u = u_step(v2[j], dd, theta);
                        vn = v_step(u, c2[j]);
                        if (write_u) d.u[g] = u;
                    }
                    Vo[g] = vn;
                    PXo[g] = mxn[j];
                    PYo[g] = myn[j];
                    PZo[g] = mzn[j];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            c2[j] = c1[j]; v2[j] = vn1[j]; qx2[j] = pxn[j]; qy2[j] = pyn[j]; qz2[j] = pzn[j];
            w2b[j] = wn[j]; pzm3[j] = mzn[j];
            c1[j] = c0[j]; v1[j] = v0[j]; px1[j] = px0[j]; py1[j] = py0[j]; pz1[j] = pz0[j];
            w1[j] = w0[j]; pzn2[j] = pzn[j];
        }
        cur ^= 1;
        cur2 ^= 1;
    }
}

constexpr int kVBX = 32, kVBY = 16, kVBZ = 32, kVNT = 256;

}  // namespace

void volume_tile(int* bx, int* by, int* bz) {
    *bx = kVBX;
    *by = kVBY;
    *bz = kVBZ;
}

int launch_init3(const VolDesc& d, hipStream_t st) {
    const int64_t rows = (int64_t)d.D * d.H;
    const unsigned grid = (unsigned)std::min<int64_t>(rows, 65536);
    hipLaunchKernelGGL(k_init3, dim3(grid), dim3(256), 0, st, d);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_tile_flags3(const VolDesc& d, int64_t n_tiles, int32_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_flags3, dim3((unsigned)n_tiles), dim3(256), 0, st, d, kVBX, kVBY,
                       kVBZ, flags);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_iterate3x2(const VolDesc& d, const int32_t* flags, int64_t n_tiles, int in_buf,
                      bool uv1, bool uv2, bool write_u, float theta, float inv_theta, float tau,
                      hipStream_t st) {
    hipLaunchKernelGGL((k_stream3x2<kVBX, kVBY, kVBZ, kVNT>),
                       dim3((unsigned)((n_tiles + 7) / 8 * 8)), dim3(kVNT), 0, st, d, flags, in_buf,
                       uv1 ? 1 : 0, uv2 ? 1 : 0, write_u ? 1 : 0, theta, inv_theta, tau);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_iterate3(const VolDesc& d, const int32_t* flags, int64_t n_tiles, int in_buf, bool uv,
                    bool write_u, float theta, float inv_theta, float tau, hipStream_t st) {
    hipLaunchKernelGGL((k_stream3<kVBX, kVBY, kVBZ, kVNT>), dim3((unsigned)((n_tiles + 7) / 8 * 8)),
                       dim3(kVNT),
                       0, st, d, flags, in_buf, uv ? 1 : 0, write_u ? 1 : 0, theta, inv_theta,
                       tau);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace rdseg
