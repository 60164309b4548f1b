// rdseg_device.h -- device-side data structures and per-pixel arithmetic of the
// restricted-domain dual iteration, shared by every kernel of the library so
// that all launch shapes, the batched path and the adjoint's recomputation
// produce bitwise identical FP32 states.
//
// Per pixel x of the restricted domain RD (Sec. 3), one outer iteration is
//   d   = div p          (backward differences; p = 0 beyond the first
//                         column/row, p_x = 0 on the last column and p_y = 0
//                         on the last row always hold)
//   w   = d - v/theta on RD,  -H(-f)/theta off RD
//   g   = grad w (forward differences, 0 on the last column/row)
//   p  <- (p + tau g) / (1 + tau |g|)        on RD, 0 off RD  (Sec. 3)
//   u   = v - theta div p                                      (Sec. 2.1)
//   v   = min(max(u - theta lambda f, 0), 1)                   (Sec. 2.1)
// Off RD the library stores c = -inf (Fg, f <= -delta) or +inf (Bg) in place of
// theta lambda f, so the same clamp yields v = H(-f) there.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rdseg {

// Everything a kernel needs to know about one image.  The two state buffers
// are st[0] = the caller's (v, p_x, p_y) and st[1] = the workspace's.
struct ImgDesc {
    const float* f;
    float* u;
    float* c;             // theta*lambda*f on RD, -inf on Fg, +inf on Bg
    float* st[2][3];      // [buffer][v, px, py]
    const float* u0;      // nullable start
    const float* p0x;     // nullable start (x plane)
    const float* p0y;     // nullable start (y plane)
    int32_t H, W, ld;
    int32_t tw;           // 8x8 tiles per row, ceil(W/8)
    int32_t th;           // 8x8 tile rows, ceil(H/8)
    int32_t mw;           // macro tiles per row
    int32_t mh;           // macro tile rows
    int32_t pad_;
    int64_t toff;         // first global 8x8 tile of this image
    int64_t soff;         // first global 8x64 strip of this image
    int64_t moff;         // first global macro tile of this image
    int64_t roff;         // first global row of this image
    float tl;             // (float)(theta * lambda)
    float pad2_;
    double delta;
};

// A volume [D][H][W]: voxel (z, y, x) at z * lds + y * ld + x.  The two state
// buffers are st[0] = the caller's (v, p_x, p_y, p_z), st[1] = the workspace's.
struct VolDesc {
    const float* f;
    float* u;
    float* c;
    float* st[2][4];
    const float* u0;
    const float* p0[3];
    int32_t D, H, W, ld, lds;
    float tl;             // (float)(theta * lambda)
    double delta;
};

// An image solved with the primal-dual iteration: state buffers st[b] =
// (u, ubar, p_x, p_y); c = tau*lambda*f on RD, -/+inf on Fg / Bg.
struct PdDesc {
    const float* f;
    float* c;
    float* st[2][4];
    const float* u0;
    const float* p0x;
    const float* p0y;
    int32_t H, W, ld, mw;
    float tl;             // (float)(tau * lambda)
    double delta;
};

// Cell flags kept in a register per LDS cell.
enum : uint32_t { CF_ACT = 1u, CF_LASTC = 2u, CF_LASTR = 4u, CF_OUT = 8u };

__device__ __forceinline__ float clamp01(float s) {
    return __builtin_amdgcn_fmed3f(s, 0.0f, 1.0f);
}

// Backward-difference divergence from the cell's own components and its left
// (x - e_x) and upper (y - e_y) neighbours.
__device__ __forceinline__ float div_p(float pxc, float pxl, float pyc, float pyu) {
    return (pxc - pxl) + (pyc - pyu);
}

// w = d - v/theta on RD, -v/theta off RD (v = H(-f) there).
__device__ __forceinline__ float w_of(float d, float v, float inv_theta, bool act) {
    return fmaf(-v, inv_theta, act ? d : 0.0f);
}

// Chambolle's semi-implicit dual update from w at x, x + e_x, x + e_y.
struct DualOut {
    float px, py, gx, gy, m;
};
__device__ __forceinline__ DualOut dual_update(float px, float py, float wc, float wr, float wd,
                                               uint32_t fl, float tau) {
    DualOut o;
    o.gx = (fl & CF_LASTC) ? 0.0f : (wr - wc);
    o.gy = (fl & CF_LASTR) ? 0.0f : (wd - wc);
    float nn = __builtin_amdgcn_sqrtf(fmaf(o.gx, o.gx, o.gy * o.gy));
    o.m = __builtin_amdgcn_rcpf(fmaf(tau, nn, 1.0f));
    bool act = (fl & CF_ACT) != 0;
    o.px = act ? fmaf(tau, o.gx, px) * o.m : 0.0f;
    o.py = act ? fmaf(tau, o.gy, py) * o.m : 0.0f;
    return o;
}

// u-step: u = v - theta div p.
__device__ __forceinline__ float u_step(float v, float d, float theta) {
    return fmaf(-theta, d, v);
}

// v-step: clamp(u - c) (c = theta lambda f on RD, -/+inf off RD).
__device__ __forceinline__ float v_step(float u, float c) {
    return clamp01(u - c);
}

// Fitting-term value c for one pixel: theta*lambda*f on RD, +-inf elsewhere.
__device__ __forceinline__ float c_of(float f, double delta, float tl) {
    bool act = fabs((double)f) < delta;
    float h_inf = (f < 0.0f) ? -__builtin_inff() : __builtin_inff();
    return act ? tl * f : h_inf;
}

__device__ __forceinline__ bool c_active(float c) {
    return __builtin_isfinite(c);
}

__device__ __forceinline__ float heav_from_c(float c) {
    return c < 0.0f ? 1.0f : 0.0f;
}

}  // namespace rdseg
