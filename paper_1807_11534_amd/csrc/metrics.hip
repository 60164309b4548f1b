// metrics.hip -- the evaluation measures of Sec. 4 on the device: thresholded
// labels GT = (u_ref > eps) and Omega = (u > eps), the node counts of their
// intersection and union (E1 = intersection / union, the Tanimoto
// coefficient) and E2 = sum over nodes of (u - u_ref)^2 (unit cell area).
// Labels compare the FP32 values in FP64.  Counts are exact; E2 is summed in
// FP64 in a fixed order (rows per workgroup, then a fixed tree), so repeated
// calls on the same shape return the same bits.
#include <algorithm>

#include "rdseg_internal.h"

namespace rdseg {

namespace {

constexpr int kMetricBlocks = 1024;
constexpr int kMetricThreads = 256;

__device__ void tree3(double* a, double* b, double* c) {
    const int t = threadIdx.x;
    for (int o = kMetricThreads / 2; o > 0; o >>= 1) {
        __syncthreads();
        if (t < o) {
            a[t] += a[t + o];
            b[t] += b[t + o];
            c[t] += c[t + o];
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kMetricThreads) void k_metrics_partial(
    const float* __restrict__ u, const float* __restrict__ g, int H, int W, int ld, double eps,
    double* __restrict__ part) {
    __shared__ double si[kMetricThreads], su[kMetricThreads], se[kMetricThreads];
    const int t = threadIdx.x;
    double ni = 0.0, nu = 0.0, e2 = 0.0;   // counts stay exact below 2^53
    for (int y = blockIdx.x; y < H; y += gridDim.x) {
        for (int x = t; x < W; x += kMetricThreads) {
            const int i = y * ld + x;
            const double a = (double)u[i], b = (double)g[i];
            const bool lo = a > eps, lg = b > eps;
            ni += (lo && lg) ? 1.0 : 0.0;
            nu += (lo || lg) ? 1.0 : 0.0;
            const double d = a - b;
            e2 += d * d;
        }
    }
    si[t] = ni;
    su[t] = nu;
    se[t] = e2;
    tree3(si, su, se);
    if (t == 0) {
        part[3 * blockIdx.x + 0] = si[0];
        part[3 * blockIdx.x + 1] = su[0];
        part[3 * blockIdx.x + 2] = se[0];
    }
}

__global__ __launch_bounds__(kMetricThreads) void k_metrics_final(const double* __restrict__ part,
                                                                  int n, double* __restrict__ out) {
    __shared__ double si[kMetricThreads], su[kMetricThreads], se[kMetricThreads];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = t; k < n; k += kMetricThreads) {
        a += part[3 * k + 0];
        b += part[3 * k + 1];
        c += part[3 * k + 2];
    }
    si[t] = a;
    su[t] = b;
    se[t] = c;
    tree3(si, su, se);
    if (t == 0) {
        out[0] = si[0];
        out[1] = su[0];
        out[2] = se[0];
    }
}

}  // namespace

size_t metrics_partials_bytes() { return (size_t)kMetricBlocks * 3 * sizeof(double); }

int launch_metrics(const float* u, const float* g, int H, int W, int ld, double eps,
                   double* partials, double* out, hipStream_t st) {
    const int blocks = std::min(H, kMetricBlocks);
    hipLaunchKernelGGL(k_metrics_partial, dim3(blocks), dim3(kMetricThreads), 0, st, u, g, H, W,
                       ld, eps, partials);
    RDSEG_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_metrics_final, dim3(1), dim3(kMetricThreads), 0, st,
                       (const double*)partials, blocks, out);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace rdseg
