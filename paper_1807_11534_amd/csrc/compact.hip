// compact.hip -- stream compaction of the restricted domain RD = {|f| < delta}
// (Sec. 3: Fg / Bg / RD thresholding of the fitting term).
//
// One wave64 scans an 8-row x 64-column strip: for each of the 8 rows the
// wave's ballot of (|f| < delta) is a 64-bit row mask, and the 8 bytes of the
// 8 ballots that fall in one 8x8 tile form that tile's 64-bit mask (bit
// (y mod 8) * 8 + (x mod 8)).  Lists are built with a three-pass exclusive
// scan (block sums, one-block scan of the sums, block-local scan + scatter),
// so every list is in ascending order and identical run to run.
#include <algorithm>

#include "rdseg_internal.h"

namespace rdseg {

namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_I = 8;
constexpr int SCAN_B = SCAN_T * SCAN_I;

__device__ __forceinline__ int find_image(const int64_t* off, int n, int64_t g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int wave_incl_scan(int x) {
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ int block_excl_scan(int x, int* s_w, int& total) {
    int incl = wave_incl_scan(x);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 63) s_w[wid] = incl;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_T / 64; ++k) {
        int v = s_w[k];
        pre += (k < wid) ? v : 0;
        tot += v;
    }
    total = tot;
    __syncthreads();
    return pre + incl - x;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_partial(const int32_t* __restrict__ in,
                                                         int64_t n, int32_t* __restrict__ part) {
    __shared__ int s_w[SCAN_T / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_I;
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) s += (base + k < n) ? in[base + k] : 0;
    int tot;
    (void)block_excl_scan(s, s_w, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_top(int32_t* __restrict__ part, int64_t nb,
                                                     int32_t* __restrict__ total) {
    __shared__ int s_w[SCAN_T / 64];
    int carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_T) {
        int64_t i = b0 + threadIdx.x;
        int x = (i < nb) ? part[i] : 0;
        int tot;
        int ex = block_excl_scan(x, s_w, tot);
        if (i < nb) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_final(const int32_t* __restrict__ in, int64_t n,
                                                       const int32_t* __restrict__ part,
                                                       int32_t* __restrict__ out) {
    __shared__ int s_w[SCAN_T / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_I;
    int v[SCAN_I];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_excl_scan(s, s_w, tot) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_i32_to_i64(const int32_t* a, int64_t* b) { *b = (int64_t)*a; }

// Fixed-order sum of n int64 values (one block).
__global__ __launch_bounds__(256) void k_sum_i64(const int64_t* __restrict__ a, int n,
                                                 int64_t* __restrict__ out) {
    __shared__ int64_t s[256];
    int64_t acc = 0;
    for (int i = threadIdx.x; i < n; i += 256) acc += a[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// ---------------------------------------------------------------- tile masks
// One wave per 8-row x 64-column strip (grid-stride): 8 ballots give the 8
// tile masks.  The RD pixel count of a single image is summed per workgroup
// and added with one atomic per workgroup (thousands of waves adding to one
// counter serialise at the memory-side atomic unit); batched images keep one
// atomic per strip, on their own counters.
template <bool BATCHED>
__global__ __launch_bounds__(256) void k_tile_masks(ImgDesc d0, const ImgDesc* __restrict__ descs,
                                                    OffTables off, int n_img, int64_t n_strips,
                                                    uint64_t* __restrict__ masks,
                                                    int64_t* __restrict__ npix) {
    __shared__ unsigned long long sCnt[4];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    unsigned long long mine = 0;
    for (int64_t s = (int64_t)blockIdx.x * 4 + wv; s < n_strips; s += (int64_t)gridDim.x * 4) {
        int img = BATCHED ? find_image(off.soff, n_img, s) : 0;
        const ImgDesc& d = BATCHED ? descs[img] : d0;
        int64_t ls = s - (BATCHED ? off.soff[img] : 0);
        int sw = (d.tw + 7) >> 3;
        int ty = (int)(ls / sw);
        int sx = (int)(ls - (int64_t)ty * sw);
        int x = sx * 64 + lane;
        uint64_t b[8];
        int cnt = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            int y = ty * 8 + r;
            bool a = false;
            if (x < d.W && y < d.H) a = fabs((double)d.f[(int64_t)y * d.ld + x]) < d.delta;
            b[r] = __ballot(a);
            cnt += __popcll(b[r]);
        }
        if (lane < 8) {
            int tx = sx * 8 + lane;
            if (tx < d.tw) {
                uint64_t m = 0;
#pragma unroll
                for (int r = 0; r < 8; ++r) m |= ((b[r] >> (8 * lane)) & 0xFFull) << (8 * r);
                masks[d.toff + (int64_t)ty * d.tw + tx] = m;
            }
        }
        if (BATCHED) {
            if (lane == 0 && cnt) atomicAdd((unsigned long long*)&npix[img], (unsigned long long)cnt);
        } else {
            mine += (unsigned long long)cnt;
        }
    }
    if (!BATCHED) {
        if (lane == 0) sCnt[wv] = mine;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long tot = sCnt[0] + sCnt[1] + sCnt[2] + sCnt[3];
            if (tot) atomicAdd((unsigned long long*)npix, tot);
        }
    }
}

// Global-address-space views of the descriptor's generic pointers: global
// loads and stores are counted in order, so a load's use waits only for that
// load, where a generic (flat) access makes the compiler wait for every
// outstanding access, stores included.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// ---------------------------------------------------------------- prepare
// The initial state (u0 = H(-f) or the caller's start on RD, v0 = clamp(u0 -
// theta lambda f), p0 = 0 or the caller's; frozen pixels u = v = H(-f), p = 0)
// and the 8x8 tile masks of RD in one pass over f.  One wave per 8-row x
// 64-column strip as in k_tile_masks; each workgroup takes a contiguous run
// of 4 * `per_wave` strips, its waves every fourth one, so a batch looks up
// the image of a wave's first strip once and then walks forward (a lookup per
// strip is a chain of dependent loads that left the batched passes latency
// bound).  Writes u and the caller's state buffer (v, p_x, p_y) on every
// pixel, the workspace's state buffer only on RD pixels (no kernel reads a
// frozen pixel's state from it) and, for a single image, c (a batch's kernels
// derive c from f: one plane less to write).  With d.u == NULL only c and the
// masks are written.
template <bool BATCHED>
__global__ __launch_bounds__(256) void k_prepare(ImgDesc d0, const ImgDesc* __restrict__ descs,
                                                 OffTables off, int n_img, int64_t n_strips,
                                                 int64_t per_wave, uint64_t* __restrict__ masks,
                                                 int64_t* __restrict__ npix) {
    __shared__ unsigned long long sCnt[4];
    const int lane = threadIdx.x & 63;
    // wave-uniform (readfirstlane tells the compiler so): the strip loop, the
    // image index and its descriptor then live in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the workgroup's run of 4 * per_wave strips, its waves interleaved: the
    // four waves write adjacent strips (1 KB of each row of each plane)
    const int64_t g0 = (int64_t)blockIdx.x * 4 * per_wave;
    const int64_t s0 = g0 + wv;
    const int64_t s1 = g0 + 4 * per_wave < n_strips ? g0 + 4 * per_wave : n_strips;
    unsigned long long cnt = 0;   // RD pixels of the current image (this wave)
    // the image index is wave-uniform (readfirstlane tells the compiler so):
    // its descriptor is read with scalar loads, once per image
    int img = 0;
    int64_t img_lo = 0, img_hi = n_strips;
    ImgDesc d = d0;
    if (BATCHED && s0 < s1) {
        img = __builtin_amdgcn_readfirstlane(find_image(off.soff, n_img, s0));
        img_lo = off.soff[img];
        img_hi = off.soff[img + 1];
        d = descs[img];
    }
    for (int64_t s = s0; s < s1; s += 4) {
        if (BATCHED && s >= img_hi) {
            do {
                if (lane == 0 && cnt) atomicAdd((unsigned long long*)&npix[img], cnt);
                cnt = 0;
                ++img;
                img_lo = img_hi;
                img_hi = off.soff[img + 1];
            } while (s >= img_hi);
            img = __builtin_amdgcn_readfirstlane(img);
            d = descs[img];
        }
        const int64_t ls = s - img_lo;
        const int sw = (d.tw + 7) >> 3;
        const int ty = (int)(ls / sw);
        const int sx = (int)(ls - (int64_t)ty * sw);
        const int x = sx * 64 + lane;
        const int W = d.W, H = d.H;
        // every load of the strip is issued before its first store: a load
        // after a store waits for that store too (one counter), and a round
        // trip per row left the pass latency bound
        const auto F = as_global(d.f), U0 = as_global(d.u0);
        const auto P0X = as_global(d.p0x), P0Y = as_global(d.p0y);
        const auto C = as_global(d.c), U = as_global(d.u);
        const auto V0 = as_global(d.st[0][0]), X0 = as_global(d.st[0][1]);
        const auto Y0 = as_global(d.st[0][2]), V1 = as_global(d.st[1][0]);
        const auto X1 = as_global(d.st[1][1]), Y1 = as_global(d.st[1][2]);
        // unconditional loads (clamped into the image; the values of lanes
        // outside it are not used), so that the compiler can count them
        float fr[8], ur[8], pxr[8], pyr[8];
        const int xc = x < W ? x : W - 1;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int y = ty * 8 + r;
            const int yc = y < H ? y : H - 1;
            fr[r] = F[(int64_t)yc * d.ld + xc];
            ur[r] = 0.0f;
            pxr[r] = 0.0f;
            pyr[r] = 0.0f;
        }
        if (d.u0 || d.p0x) {   // a caller's start (single image only)
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int y = ty * 8 + r;
                const int64_t g = (int64_t)y * d.ld + x;
                const bool in = x < W && y < H;
                ur[r] = (in && d.u0) ? U0[g] : 0.0f;
                pxr[r] = (in && d.p0x) ? P0X[g] : 0.0f;
                pyr[r] = (in && d.p0y) ? P0Y[g] : 0.0f;
            }
        }
        // the whole strip's values first, then its stores (no load of this
        // strip waits behind a store of it)
        uint64_t b[8];
        float cr[8], u0r[8], v0r[8];
        uint32_t actm = 0u;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int y = ty * 8 + r;
            const bool in = x < W && y < H;
            const float fv = fr[r];
            const bool a = in && fabs((double)fv) < d.delta;
            const float c = c_of(fv, d.delta, d.tl);
            const bool act = c_active(c);
            const float h = (fv < 0.0f) ? 1.0f : 0.0f;
            cr[r] = c;
            u0r[r] = act ? (d.u0 ? ur[r] : h) : h;
            v0r[r] = v_step(u0r[r], c);
            pxr[r] = (act && x < W - 1) ? pxr[r] : 0.0f;
            pyr[r] = (act && y < H - 1) ? pyr[r] : 0.0f;
            actm |= act ? (1u << r) : 0u;
            b[r] = __ballot(a);
            cnt += (unsigned long long)__popcll(b[r]);
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int y = ty * 8 + r;
            if (x < W && y < H) {
                const int64_t g = (int64_t)y * d.ld + x;
                if (!BATCHED) C[g] = cr[r];   // a batch derives c from f where it needs it
                if (d.u) {
                    U[g] = u0r[r];
                    V0[g] = v0r[r];
                    X0[g] = pxr[r];
                    Y0[g] = pyr[r];
                    if ((actm >> r) & 1u) {
                        V1[g] = v0r[r];
                        X1[g] = pxr[r];
                        Y1[g] = pyr[r];
                    }
                }
            }
        }
        if (lane < 8) {
            const int tx = sx * 8 + lane;
            if (tx < d.tw) {
                uint64_t m = 0;
#pragma unroll
                for (int r = 0; r < 8; ++r) m |= ((b[r] >> (8 * lane)) & 0xFFull) << (8 * r);
                masks[d.toff + (int64_t)ty * d.tw + tx] = m;
            }
        }
    }
    if (BATCHED) {
        if (lane == 0 && cnt) atomicAdd((unsigned long long*)&npix[img], cnt);
    } else {
        // one atomic per workgroup on the single counter
        if (lane == 0) sCnt[wv] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long tot = sCnt[0] + sCnt[1] + sCnt[2] + sCnt[3];
            if (tot) atomicAdd((unsigned long long*)npix, tot);
        }
    }
}

__global__ void k_mask_flags(const uint64_t* __restrict__ masks, int64_t n,
                             int32_t* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = masks[i] != 0 ? 1 : 0;
}

__global__ void k_tile_scatter(const uint64_t* __restrict__ masks, int64_t n,
                               const int32_t* __restrict__ offs, int32_t* __restrict__ ids,
                               uint64_t* __restrict__ mout, int32_t* __restrict__ slot) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint64_t m = masks[t];
    if (m) {
        int o = offs[t];
        ids[o] = (int32_t)t;
        mout[o] = m;
        slot[t] = o;
    } else {
        slot[t] = -1;
    }
}

// ---------------------------------------------------------------- pixel list
__global__ __launch_bounds__(256) void k_pix_count(const float* __restrict__ f, int H, int W,
                                                   int ld, double delta, int64_t n_chunks,
                                                   int32_t* __restrict__ counts) {
    int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= n_chunks) return;
    int lane = threadIdx.x & 63;
    int64_t p = c * 64 + lane;
    bool a = false;
    if (p < (int64_t)H * W) {
        int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        a = fabs((double)f[(int64_t)y * ld + x]) < delta;
    }
    uint64_t b = __ballot(a);
    if (lane == 0) counts[c] = __popcll(b);
}

__global__ __launch_bounds__(256) void k_pix_scatter(const float* __restrict__ f, int H, int W,
                                                     int ld, double delta, int64_t n_chunks,
                                                     const int32_t* __restrict__ offs,
                                                     int32_t* __restrict__ pix) {
    int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= n_chunks) return;
    int lane = threadIdx.x & 63;
    int64_t p = c * 64 + lane;
    bool a = false;
    if (p < (int64_t)H * W) {
        int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        a = fabs((double)f[(int64_t)y * ld + x]) < delta;
    }
    uint64_t b = __ballot(a);
    if (a) {
        uint64_t below = (lane == 0) ? 0ull : (b & ((~0ull) >> (64 - lane)));
        pix[offs[c] + __popcll(below)] = (int32_t)p;
    }
}

// ---------------------------------------------------------------- work lists
// The iteration couples two RD pixels only through 4-neighbour chains of RD
// pixels (off RD, p = 0 and w = -H(-f)/theta are constants).  An 8x8 tile whose
// RD pixels have no RD 4-neighbour in another tile therefore evolves on its
// own: it is "closed" and can run every iteration on chip.  A macro tile is
// queued for the temporally blocked kernel iff it holds an open 8x8 tile
// (closed tiles inside it are computed there too); the closed tiles of the
// other macro tiles go to the closed-tile list.  One thread per macro tile.
constexpr uint64_t kCol0 = 0x0101010101010101ull;

__device__ __forceinline__ bool tile_touches_neighbour(const uint64_t* __restrict__ masks,
                                                       int64_t T, int tx, int ty, int tw, int th,
                                                       uint64_t m) {
    const uint64_t mL = tx > 0 ? masks[T - 1] : 0ull;
    const uint64_t mR = tx < tw - 1 ? masks[T + 1] : 0ull;
    const uint64_t mU = ty > 0 ? masks[T - tw] : 0ull;
    const uint64_t mD = ty < th - 1 ? masks[T + tw] : 0ull;
    uint64_t touch = (m & kCol0) & ((mL >> 7) & kCol0);   // left column vs left tile
    touch |= ((m >> 7) & kCol0) & (mR & kCol0);            // right column vs right tile
    touch |= (m & 0xFFull) & (mU >> 56);                   // top row vs upper tile
    touch |= (m >> 56) & (mD & 0xFFull);                   // bottom row vs lower tile
    return touch != 0;
}

// One wave per macro tile, one lane per 8x8 tile of it (a macro tile holds at
// most 8 x 8 of them): a tile is open when one of its RD pixels has an RD
// 4-neighbour in another tile; the macro tile is queued when it holds an open
// tile, and each closed tile of an unqueued macro tile is flagged for the
// closed-tile kernel.
template <bool BATCHED>
__global__ __launch_bounds__(256) void k_lists(ImgDesc d0, const ImgDesc* __restrict__ descs,
                                               OffTables off, int n_img, int64_t n_macro, int bx8,
                                               int by8, const uint64_t* __restrict__ masks,
                                               int use_closed, int32_t* __restrict__ mflags,
                                               int32_t* __restrict__ cflags,
                                               int32_t* __restrict__ epoch) {
    const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (m >= n_macro) return;   // uniform per wave
    const int lane = threadIdx.x & 63;
    if (epoch && lane == 0) epoch[m] = 0;   // the resident form's words start at 0
    const int img = BATCHED ? find_image(off.moff, n_img, m) : 0;
    const ImgDesc& d = BATCHED ? descs[img] : d0;
    const int64_t lm = m - (BATCHED ? off.moff[img] : 0);
    const int my = (int)(lm / d.mw), mx = (int)(lm - (int64_t)my * d.mw);
    const int tx = mx * bx8 + lane % bx8, ty = my * by8 + lane / bx8;
    const bool mine = lane < bx8 * by8 && tx < d.tw && ty < d.th;
    const int64_t T = d.toff + (int64_t)ty * d.tw + tx;
    uint64_t mk = 0;
    bool open = false;
    if (mine) {
        mk = masks[T];
        if (mk) open = !use_closed || tile_touches_neighbour(masks, T, tx, ty, d.tw, d.th, mk);
    }
    const bool any_open = __ballot(open) != 0ull;
    if (lane == 0) mflags[m] = any_open ? 1 : 0;
    if (use_closed && mine) cflags[T] = (!any_open && mk && !open) ? 1 : 0;
}

// Batched form of k_lists: each wave takes a contiguous run of macro tiles and
// covers 64 / (bx8 * by8) of them per step, one lane per 8x8 tile; a lane
// finds its image by walking forward from the image of the step's first
// macro tile (the wave looks the first one up once), instead of a lookup per
// macro tile.
__global__ __launch_bounds__(256) void k_lists_batched(const ImgDesc* __restrict__ descs,
                                                       OffTables off, int n_img, int64_t n_macro,
                                                       int64_t per_wave, int bx8, int by8,
                                                       const uint64_t* __restrict__ masks,
                                                       int use_closed,
                                                       int32_t* __restrict__ mflags,
                                                       int32_t* __restrict__ cflags) {
    const int lane = threadIdx.x & 63;
    const int tpm = bx8 * by8;   // 8x8 tiles per macro tile (<= 64)
    const int mpi = 64 / tpm;    // macro tiles per step
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + wv) * per_wave;
    const int64_t m1 = m0 + per_wave < n_macro ? m0 + per_wave : n_macro;
    if (m0 >= m1) return;   // uniform per wave
    int img = find_image(off.moff, n_img, m0);
    const int k = lane / tpm;   // macro tile of this lane within the step
    const int j = lane - k * tpm;
    for (int64_t base = m0; base < m1; base += mpi) {
        const int64_t m = base + k;
        const bool valid = k < mpi && m < m1;
        int im = img;
        if (valid)
            while (m >= off.moff[im + 1]) ++im;
        bool mine = false, open = false;
        uint64_t mk = 0;
        int64_t T = 0;
        if (valid) {
            const ImgDesc& d = descs[im];
            const int64_t lm = m - off.moff[im];
            const int my = (int)(lm / d.mw), mx = (int)(lm - (int64_t)my * d.mw);
            const int tx = mx * bx8 + j % bx8, ty = my * by8 + j / bx8;
            mine = tx < d.tw && ty < d.th;
            T = d.toff + (int64_t)ty * d.tw + tx;
            if (mine) {
                mk = masks[T];
                if (mk) open = !use_closed || tile_touches_neighbour(masks, T, tx, ty, d.tw, d.th, mk);
            }
        }
        const uint64_t bal = __ballot(open);
        const uint64_t grp = (tpm == 64) ? ~0ull : (((1ull << tpm) - 1ull) << (k * tpm));
        const bool any_open = (bal & grp) != 0ull;
        if (valid && j == 0) mflags[m] = any_open ? 1 : 0;
        if (use_closed && mine) cflags[T] = (!any_open && mk && !open) ? 1 : 0;
        // the image of the step's last macro tile starts the next step
        const int64_t mlast = (base + mpi < m1 ? base + mpi : m1) - 1;
        while (mlast >= off.moff[img + 1]) ++img;
    }
}

// Exclusive scans of up to two int32 arrays of at most SMALL_N elements, one
// 1024-thread block per array (the arrays are 16-byte aligned workspace).
constexpr int SMALL_T = 1024;
constexpr int SMALL_I = 64;
constexpr int64_t SMALL_N = (int64_t)SMALL_T * SMALL_I;

__global__ __launch_bounds__(SMALL_T) void k_scan_small2(const int32_t* __restrict__ a, int64_t na,
                                                         int32_t* __restrict__ oa,
                                                         int32_t* __restrict__ ta,
                                                         const int32_t* __restrict__ b, int64_t nb,
                                                         int32_t* __restrict__ ob,
                                                         int32_t* __restrict__ tb) {
    // Chunks of 4 * SMALL_T values: one aligned int4 per thread (coalesced),
    // a wave scan, a scan of the wave totals, and a running carry.
    __shared__ int s_w[SMALL_T / 64];
    const int32_t* in = blockIdx.x == 0 ? a : b;
    const int64_t n = blockIdx.x == 0 ? na : nb;
    int32_t* out = blockIdx.x == 0 ? oa : ob;
    int32_t* tot_out = blockIdx.x == 0 ? ta : tb;
    if (!in) return;   // uniform per block
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    int carry = 0;
    for (int64_t base = 0; base < n; base += 4 * SMALL_T) {
        const int64_t i0 = base + 4 * t;
        int4 v = make_int4(0, 0, 0, 0);
        if (i0 + 3 < n) {
            v = *reinterpret_cast<const int4*>(in + i0);
        } else if (i0 < n) {
            v.x = in[i0];
            if (i0 + 1 < n) v.y = in[i0 + 1];
            if (i0 + 2 < n) v.z = in[i0 + 2];
        }
        const int s = v.x + v.y + v.z + v.w;
        const int incl = wave_incl_scan(s);
        if (lane == 63) s_w[wid] = incl;
        __syncthreads();
        int pre = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < SMALL_T / 64; ++k) {
            const int w = s_w[k];
            pre += (k < wid) ? w : 0;
            tot += w;
        }
        int4 o;
        o.x = carry + pre + incl - s;
        o.y = o.x + v.x;
        o.z = o.y + v.y;
        o.w = o.z + v.z;
        if (i0 + 3 < n) {
            *reinterpret_cast<int4*>(out + i0) = o;
        } else if (i0 < n) {
            out[i0] = o.x;
            if (i0 + 1 < n) out[i0 + 1] = o.y;
            if (i0 + 2 < n) out[i0 + 2] = o.z;
        }
        carry += tot;
        __syncthreads();   // s_w is rewritten by the next chunk
    }
    if (t == 0) *tot_out = carry;
}

template <bool BATCHED>
__global__ void k_scatter_lists(OffTables off, int n_img, int64_t n_macro, int64_t n_tiles,
                                const int32_t* __restrict__ mflags,
                                const int32_t* __restrict__ moffs, int2* __restrict__ queue,
                                const int32_t* __restrict__ cflags,
                                const int32_t* __restrict__ coffs, int2* __restrict__ cqueue) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_macro && mflags[i]) {
        const int img = BATCHED ? find_image(off.moff, n_img, i) : 0;
        const int64_t lm = i - (BATCHED ? off.moff[img] : 0);
        queue[moffs[i]] = make_int2(img, (int)lm);
    }
    if (cqueue && i < n_tiles && cflags[i]) {
        const int img = BATCHED ? find_image(off.toff, n_img, i) : 0;
        const int64_t lt = i - (BATCHED ? off.toff[img] : 0);
        cqueue[coffs[i]] = make_int2(img, (int)lt);
    }
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int64_t scan_partials(int64_t n) { return (n + SCAN_B - 1) / SCAN_B + 1; }

int launch_scan_ints(const int32_t* counts, int64_t n, int32_t* out, int32_t* part,
                     int32_t* total, hipStream_t st) {
    int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_scan_partial, dim3((unsigned)nb), dim3(SCAN_T), 0, st, counts, n, part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, st, part, nb, total);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(SCAN_T), 0, st, counts, n, part, out);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_tile_masks(const ImgDesc* d0, const ImgDesc* descs, OffTables off, int n_img,
                      int64_t n_strips, uint64_t* masks, int64_t* npix, hipStream_t st,
                      int64_t n_clear) {
    const int64_t nz = n_clear > n_img ? n_clear : (int64_t)n_img;
    hipLaunchKernelGGL(k_fill_i64, dim3(nblk(nz, 256)), dim3(256), 0, st, npix, nz, (int64_t)0);
    if (descs)
        hipLaunchKernelGGL(k_tile_masks<true>, dim3(nblk(n_strips, 4)), dim3(256), 0, st, *d0,
                           descs, off, n_img, n_strips, masks, npix);
    else
        hipLaunchKernelGGL(k_tile_masks<false>, dim3(std::min<int64_t>(nblk(n_strips, 4), 512)),
                           dim3(256), 0, st, *d0, descs, off, n_img, n_strips, masks, npix);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_prepare(const ImgDesc* d0, const ImgDesc* descs, OffTables off, int n_img,
                   int64_t n_strips, uint64_t* masks, int64_t* npix, hipStream_t st,
                   int64_t n_clear) {
    const int64_t nz = n_clear > n_img ? n_clear : (int64_t)n_img;
    hipLaunchKernelGGL(k_fill_i64, dim3(nblk(nz, 256)), dim3(256), 0, st, npix, nz, (int64_t)0);
    // 2048 workgroups of 4 waves (8 per SIMD), or fewer for small images
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(2048, nblk(n_strips, 4)));
    const int64_t waves = grid * 4;
    const int64_t per_wave = (n_strips + waves - 1) / waves;
    if (descs)
        hipLaunchKernelGGL(k_prepare<true>, dim3((unsigned)grid), dim3(256), 0, st, *d0, descs,
                           off, n_img, n_strips, per_wave, masks, npix);
    else
        hipLaunchKernelGGL(k_prepare<false>, dim3((unsigned)grid), dim3(256), 0, st, *d0, descs,
                           off, n_img, n_strips, per_wave, masks, npix);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_sum_i64(const int64_t* a, int n, int64_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_i64, dim3(1), dim3(256), 0, st, a, n, out);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_tile_list(const uint64_t* masks, int64_t n_tiles, int32_t* flags, int32_t* offs,
                     int32_t* part, int32_t* n_listed, int32_t* tile_ids, uint64_t* tile_masks,
                     int32_t* slot_map, hipStream_t st) {
    hipLaunchKernelGGL(k_mask_flags, dim3(nblk(n_tiles, 256)), dim3(256), 0, st, masks, n_tiles,
                       flags);
    int rc = launch_scan_ints(flags, n_tiles, offs, part, n_listed, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_tile_scatter, dim3(nblk(n_tiles, 256)), dim3(256), 0, st, masks,
                       n_tiles, offs, tile_ids, tile_masks, slot_map);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_pixel_list(const float* f, int H, int W, int ld, double delta, int32_t* counts,
                      int32_t* offs, int32_t* part, int32_t* total, int32_t* pix,
                      int64_t* n_pix, hipStream_t st) {
    int64_t n_chunks = ((int64_t)H * W + 63) / 64;
    hipLaunchKernelGGL(k_pix_count, dim3(nblk(n_chunks, 4)), dim3(256), 0, st, f, H, W, ld,
                       delta, n_chunks, counts);
    int rc = launch_scan_ints(counts, n_chunks, offs, part, total, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pix_scatter, dim3(nblk(n_chunks, 4)), dim3(256), 0, st, f, H, W, ld,
                       delta, n_chunks, offs, pix);
    hipLaunchKernelGGL(k_i32_to_i64, dim3(1), dim3(1), 0, st, total, n_pix);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_macro_queue(const ImgDesc* d0, const ImgDesc* descs, OffTables off, int n_img,
                       int64_t n_macro, int bx, int by, const uint64_t* masks,
                       const QueueScratch& q, int2* queue, int32_t* n_queue, int64_t n_tiles,
                       int2* cqueue, int32_t* n_closed, hipStream_t st) {
    const bool use_closed = cqueue != nullptr;
    if (descs) {
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(2048, nblk(n_macro, 4)));
        const int64_t per_wave = (n_macro + grid * 4 - 1) / (grid * 4);
        hipLaunchKernelGGL(k_lists_batched, dim3((unsigned)grid), dim3(256), 0, st, descs, off,
                           n_img, n_macro, per_wave, bx / 8, by / 8, masks, use_closed ? 1 : 0,
                           q.mflags, q.cflags);
    } else
        hipLaunchKernelGGL(k_lists<false>, dim3(nblk(n_macro, 4)), dim3(256), 0, st, *d0, descs,
                           off, n_img, n_macro, bx / 8, by / 8, masks, use_closed ? 1 : 0,
                           q.mflags, q.cflags, q.epoch);
    if (n_macro <= SMALL_N && (!use_closed || n_tiles <= SMALL_N)) {
        hipLaunchKernelGGL(k_scan_small2, dim3(use_closed ? 2 : 1), dim3(SMALL_T), 0, st,
                           q.mflags, n_macro, q.offs, n_queue,
                           use_closed ? q.cflags : nullptr, n_tiles, q.coffs, n_closed);
    } else {
        int rc = launch_scan_ints(q.mflags, n_macro, q.offs, q.part, n_queue, st);
        if (rc) return rc;
        if (use_closed) {
            rc = launch_scan_ints(q.cflags, n_tiles, q.coffs, q.part, n_closed, st);
            if (rc) return rc;
        }
    }
    const int64_t n_all = use_closed ? std::max(n_macro, n_tiles) : n_macro;
    if (descs)
        hipLaunchKernelGGL(k_scatter_lists<true>, dim3(nblk(n_all, 256)), dim3(256), 0, st, off,
                           n_img, n_macro, n_tiles, q.mflags, q.offs, queue, q.cflags, q.coffs,
                           use_closed ? cqueue : nullptr);
    else
        hipLaunchKernelGGL(k_scatter_lists<false>, dim3(nblk(n_all, 256)), dim3(256), 0, st, off,
                           n_img, n_macro, n_tiles, q.mflags, q.offs, queue, q.cflags, q.coffs,
                           use_closed ? cqueue : nullptr);
    RDSEG_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace rdseg
