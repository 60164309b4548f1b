// band.hip -- the band threshold q-hat from a target fraction q of nodes in
// the restricted domain (Sec. 3: q-hat grows from 0 until RD = {|f| < q-hat}
// holds a fraction q of the nodes).  q-hat is the smallest double with
// #{|f| < q-hat} >= k, k = ceil(q N): 0 for k = 0, otherwise the double just
// above a_k, the k-th smallest |f| (+inf when a_k is not finite).
//
// a_k comes from a radix select on the bits of |f|: for non-negative floats
// the 31-bit pattern (sign cleared) orders like the values, with +inf above
// every finite value and NaN above +inf, so no special casing is needed.
// Three passes over f pick bits 30..20, 19..10 and 9..0 of a_k: each pass
// histograms that digit of the keys that agree with the digits chosen so
// far (LDS histogram per workgroup, added to a global one), then one
// workgroup finds the digit whose cumulative count reaches the remaining rank.
// Counts are integers, so the result does not depend on the order of the
// atomic additions.
#include <algorithm>

#include "rdseg_internal.h"

namespace rdseg {

namespace {

constexpr int kBins = kBandHistBins;   // largest digit: 11 bits

struct PassDesc {
    int shift;   // position of the digit
    int bits;    // digit width
};
constexpr PassDesc kPasses[3] = {{20, 11}, {10, 10}, {0, 10}};

__device__ __forceinline__ uint32_t abs_key(float v) {
    return __float_as_uint(v) & 0x7fffffffu;
}

__global__ __launch_bounds__(256) void k_band_init(BandState* st, int64_t k, uint32_t* hist) {
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) hist[i] = 0u;
    if (threadIdx.x == 0) {
        st->prefix = 0u;
        st->rank = k;
    }
}

// Histogram of digit (key >> shift) & (2^bits - 1) over keys whose bits above
// shift + bits equal st->prefix (every key on the first pass).
__global__ __launch_bounds__(256) void k_band_hist(const float* __restrict__ f, int H, int W,
                                                   int ld, int shift, int bits, int first,
                                                   const BandState* __restrict__ st,
                                                   uint32_t* __restrict__ hist) {
    __shared__ uint32_t sh[kBins];
    const int nb = 1 << bits;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) sh[i] = 0u;
    __syncthreads();
    const uint32_t prefix = first ? 0u : st->prefix;
    const int hi = shift + bits;
    const uint32_t mask = (uint32_t)nb - 1u;
    for (int y = blockIdx.x; y < H; y += gridDim.x) {
        const float* row = f + (int64_t)y * ld;
        for (int x = threadIdx.x; x < W; x += blockDim.x) {
            const uint32_t key = abs_key(row[x]);
            if (first || (key >> hi) == prefix) atomicAdd(&sh[(key >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        const uint32_t c = sh[i];
        if (c) atomicAdd(&hist[i], c);
    }
}

// One workgroup of 1024 threads: the digit b with
//   sum_{j < b} hist[j] < rank <= sum_{j <= b} hist[j],
// appended to the prefix; the rank becomes relative to digit b.  Clears the
// histogram for the next pass.  After the last pass writes q-hat.
__global__ __launch_bounds__(1024) void k_band_select(BandState* __restrict__ st,
                                                      uint32_t* __restrict__ hist, int bits,
                                                      int last, double* __restrict__ out) {
    constexpr int NT = 1024;
    __shared__ int64_t part[NT];
    const int nb = 1 << bits;
    const int per = (nb + NT - 1) / NT;   // 1 or 2 bins per thread
    const int t = threadIdx.x;
    // read the state before the barriers below: the winning thread rewrites it
    const int64_t rank = st->rank;
    const uint32_t pre = st->prefix;
    int64_t own = 0;
    for (int j = 0; j < per; ++j) {
        const int b = t * per + j;
        if (b < nb) own += hist[b];
    }
    part[t] = own;
    __syncthreads();
    // inclusive scan of the per-thread sums (Hillis-Steele, fixed order)
    for (int d = 1; d < NT; d <<= 1) {
        const int64_t add = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int64_t before = part[t] - own;
    if (before < rank && rank <= part[t]) {
        for (int j = 0; j < per; ++j) {
            const int b = t * per + j;
            const int64_t c = hist[b];
            if (rank <= before + c) {
                const uint32_t prefix = (pre << bits) | (uint32_t)b;
                st->prefix = prefix;
                st->rank = rank - before;
                if (last) {
                    double q;
                    if (prefix >= 0x7f800000u) {
                        q = __builtin_inf();
                    } else {
                        const double a = (double)__uint_as_float(prefix);
                        q = __longlong_as_double(__double_as_longlong(a) + 1);
                    }
                    *out = q;
                }
                break;
            }
            before += c;
        }
    }
    __syncthreads();
    for (int j = 0; j < per; ++j) {
        const int b = t * per + j;
        if (b < nb) hist[b] = 0u;
    }
}

__global__ void k_store_double(double* out, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = v;
}

}  // namespace

int launch_band_threshold(const float* f, int H, int W, int ld, int64_t k, uint32_t* hist,
                          BandState* state, double* out, hipStream_t st) {
    if (k <= 0) {
        hipLaunchKernelGGL(k_store_double, dim3(1), dim3(64), 0, st, out, 0.0);
        return hipGetLastError() != hipSuccess;
    }
    const int64_t n = (int64_t)H * W;
    int blocks = (int)std::min<int64_t>(std::max<int64_t>(n / 8192, 1), 1024);
    blocks = std::min(blocks, H);
    hipLaunchKernelGGL(k_band_init, dim3(1), dim3(256), 0, st, state, k, hist);
    for (int p = 0; p < 3; ++p) {
        hipLaunchKernelGGL(k_band_hist, dim3(blocks), dim3(256), 0, st, f, H, W, ld,
                           kPasses[p].shift, kPasses[p].bits, p == 0 ? 1 : 0,
                           (const BandState*)state, hist);
        hipLaunchKernelGGL(k_band_select, dim3(1), dim3(1024), 0, st, state, hist,
                           kPasses[p].bits, p == 2 ? 1 : 0, out);
    }
    return hipGetLastError() != hipSuccess;
}

}  // namespace rdseg
