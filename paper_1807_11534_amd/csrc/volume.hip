// volume.hip -- the restricted iteration on volumes [D][H][W] (7-point
// stencil; the conclusion, Sec. 5, names 3-D problems as the extension of
// interest).  Per voxel the arithmetic is that of the images with a third
// gradient / divergence component, in the same operation order, so a volume of
// identical slices reproduces the image solve bit for bit.
//
// One launch runs one dual step on 32 x 8 x 8 blocks (plus, at the end of an
// outer iteration, the u-step and v-step).  The block loads its tile with a
// halo of two voxels on the low side and one on the high side of every axis
// into LDS (p) and registers (v, c, flags): the prologue's w is exact one voxel
// inside the region, the dual step's p on the tile plus one low layer, which
// the u-step's backward differences need.  Deeper temporal blocking would
// multiply the halo volume, so the kernel streams its 36 bytes per voxel
// (read c, v, p: 20; write v, p: 16) from HBM.  Tiles without a voxel of RD
// return at once (flags computed once per solve).
#include <algorithm>

#include "rdseg_internal.h"

namespace rdseg {

namespace {

constexpr uint32_t CF_LASTZ = 16u;

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

template <int BX, int BY, int BZ, int NT>
__global__ __launch_bounds__(NT) void k_iterate3(VolDesc d, const int32_t* __restrict__ flags,
                                                 int in_buf, int uv, int write_u, float theta,
                                                 float inv_theta, float tau) {
    constexpr int H0 = 2;   // low-side halo; high side 1
    constexpr int RX = BX + 3, RY = BY + 3, RZ = BZ + 3;
    constexpr int RS = RX * RY;             // region slice
    constexpr int RC = RS * RZ;
    constexpr int CPT = (RC + NT - 1) / NT;
    constexpr int PAD = RS + RX + 1;        // largest neighbour offset, both ends
    constexpr int LS = RC + 2 * PAD;
    __shared__ float sPX[LS], sPY[LS], sPZ[LS], sW[LS];

    const int t = blockIdx.x;
    if (!flags[t]) return;
    const int ntx = (d.W + BX - 1) / BX, nty = (d.H + BY - 1) / BY;
    const int tz = t / (ntx * nty), rt = t - tz * ntx * nty;
    const int ty = rt / ntx, tx = rt - ty * ntx;
    const int ox = tx * BX - H0, oy = ty * BY - H0, oz = tz * BZ - H0;
    const int th = threadIdx.x;
    for (int k = th; k < PAD; k += NT) {
        sPX[k] = 0.0f; sPY[k] = 0.0f; sPZ[k] = 0.0f; sW[k] = 0.0f;
        sPX[PAD + RC + k] = 0.0f; sPY[PAD + RC + k] = 0.0f;
        sPZ[PAD + RC + k] = 0.0f; sW[PAD + RC + k] = 0.0f;
    }
    const float* __restrict__ Vi = d.st[in_buf][0];
    const float* __restrict__ PXi = d.st[in_buf][1];
    const float* __restrict__ PYi = d.st[in_buf][2];
    const float* __restrict__ PZi = d.st[in_buf][3];

    float rv[CPT], rpx[CPT], rpy[CPT], rpz[CPT], rc[CPT];
    uint32_t fl[CPT];
    int gi[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int i = th + j * NT;
        rv[j] = 0.0f; rpx[j] = 0.0f; rpy[j] = 0.0f; rpz[j] = 0.0f; rc[j] = __builtin_inff();
        fl[j] = 0u; gi[j] = 0;
        if (i < RC) {
            const int rz = i / RS, rr = i - rz * RS;
            const int ry = rr / RX, rx = rr - ry * RX;
            const int gx = ox + rx, gy = oy + ry, gz = oz + rz;
            const bool inb = (unsigned)gx < (unsigned)d.W && (unsigned)gy < (unsigned)d.H &&
                             (unsigned)gz < (unsigned)d.D;
            const int g = gz * d.lds + gy * d.ld + gx;
            gi[j] = g;
            float c = __builtin_inff(), v = 0.0f, px = 0.0f, py = 0.0f, pz = 0.0f;
            if (inb) {   // issued together; state off RD is discarded below
                c = d.c[g];
                v = Vi[g];
                px = PXi[g];
                py = PYi[g];
                pz = PZi[g];
            }
            const bool act = c_active(c);
            rc[j] = c;
            rv[j] = act ? v : heav_from_c(c);
            rpx[j] = act ? px : 0.0f;
            rpy[j] = act ? py : 0.0f;
            rpz[j] = act ? pz : 0.0f;
            uint32_t f = act ? CF_ACT : 0u;
            if (gx == d.W - 1) f |= CF_LASTC;
            if (gy == d.H - 1) f |= CF_LASTR;
            if (gz == d.D - 1) f |= CF_LASTZ;
            const bool interior = rx >= H0 && rx < H0 + BX && ry >= H0 && ry < H0 + BY &&
                                  rz >= H0 && rz < H0 + BZ;
            if (interior && act) f |= CF_OUT;
            fl[j] = f;
            sPX[PAD + i] = rpx[j];
            sPY[PAD + i] = rpy[j];
            sPZ[PAD + i] = rpz[j];
        }
    }
    __syncthreads();
    // w = div p - v/theta on RD, -H(-f)/theta off RD
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int i = th + j * NT;
        if (i < RC) {
            const float dd = div_p3(rpx[j], sPX[PAD + i - 1], rpy[j], sPY[PAD + i - RX], rpz[j],
                                    sPZ[PAD + i - RS]);
            sW[PAD + i] = w_of(dd, rv[j], inv_theta, (fl[j] & CF_ACT) != 0);
        }
    }
    __syncthreads();
    // dual step
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int i = th + j * NT;
        if (i < RC) {
            const float wc = sW[PAD + i];
            const float gx = (fl[j] & CF_LASTC) ? 0.0f : (sW[PAD + i + 1] - wc);
            const float gy = (fl[j] & CF_LASTR) ? 0.0f : (sW[PAD + i + RX] - wc);
            const float gz = (fl[j] & CF_LASTZ) ? 0.0f : (sW[PAD + i + RS] - wc);
            const float nn = __builtin_amdgcn_sqrtf(fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
            const float m = __builtin_amdgcn_rcpf(fmaf(tau, nn, 1.0f));
            const bool act = (fl[j] & CF_ACT) != 0;
            rpx[j] = act ? fmaf(tau, gx, rpx[j]) * m : 0.0f;
            rpy[j] = act ? fmaf(tau, gy, rpy[j]) * m : 0.0f;
            rpz[j] = act ? fmaf(tau, gz, rpz[j]) * m : 0.0f;
            sPX[PAD + i] = rpx[j];
            sPY[PAD + i] = rpy[j];
            sPZ[PAD + i] = rpz[j];
        }
    }
    __syncthreads();
    // u-step and v-step at the end of an outer iteration; write the tile
    float* __restrict__ Vo = d.st[1 - in_buf][0];
    float* __restrict__ PXo = d.st[1 - in_buf][1];
    float* __restrict__ PYo = d.st[1 - in_buf][2];
    float* __restrict__ PZo = d.st[1 - in_buf][3];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int i = th + j * NT;
        if (i < RC && (fl[j] & CF_OUT)) {
            float vn = rv[j];
            if (uv) {
                const float dd = div_p3(rpx[j], sPX[PAD + i - 1], rpy[j], sPY[PAD + i - RX],
                                        rpz[j], sPZ[PAD + i - RS]);
                const float u = u_step(rv[j], dd, theta);
                vn = v_step(u, rc[j]);
                if (write_u) d.u[gi[j]] = u;
            }
            Vo[gi[j]] = vn;
            PXo[gi[j]] = rpx[j];
            PYo[gi[j]] = rpy[j];
            PZo[gi[j]] = rpz[j];
        }
    }
}

constexpr int kVBX = 32, kVBY = 8, kVBZ = 8, kVNT = 512;

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

int launch_iterate3(const VolDesc& d, const int32_t* flags, int64_t n_tiles, int in_buf, bool uv,
                    bool write_u, float theta, float inv_theta, float tau, hipStream_t st) {
    hipLaunchKernelGGL((k_iterate3<kVBX, kVBY, kVBZ, kVNT>), dim3((unsigned)n_tiles), dim3(kVNT),
                       0, st, d, flags, in_buf, uv ? 1 : 0, write_u ? 1 : 0, theta, inv_theta,
                       tau);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace rdseg
