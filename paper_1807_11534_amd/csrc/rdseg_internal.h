// rdseg_internal.h -- host-side declarations shared by the library's
// translation units (kernel launchers, error helpers, configuration table).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "rdseg_device.h"

namespace rdseg {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
const char* get_error();

#define RDSEG_HIP_CHECK(expr)                                                        \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::rdseg::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));  \
            return 4; /* RDSEG_ERR_HIP */                                            \
        }                                                                            \
    } while (0)

// Offset tables of a batch (device arrays of n + 1 entries each).
struct OffTables {
    const int64_t* soff;   // 8x64 strips
    const int64_t* toff;   // 8x8 tiles
    const int64_t* moff;   // macro tiles
    const int64_t* roff;   // rows
};

// ---------------------------------------------------------------- compaction
// Exclusive prefix scan of int32 counts (n elements) into out, total into
// *total.  part: scratch of scan_partials(n) int32.  Launch order is fixed,
// so results are deterministic.
int64_t scan_partials(int64_t n);
int launch_scan_ints(const int32_t* counts, int64_t n, int32_t* out, int32_t* part,
                     int32_t* total, hipStream_t st);

// Dense 8x8 tile masks of every image (masks[toff[i] + ty * tw + tx]) and the
// number of RD pixels per image (npix[i], zeroed by this launcher together
// with the int64 slots after them up to npix[n_clear - 1]).
int launch_tile_masks(const ImgDesc* d0, const ImgDesc* descs, OffTables off, int n_img,
                      int64_t n_strips, uint64_t* masks, int64_t* npix, hipStream_t st,
                      int64_t n_clear = 0);

// Initial state and 8x8 tile masks in one pass (k_init + k_tile_masks fused;
// the workspace state buffer st[1] is written on RD pixels only).  Clears
// npix[0 .. max(n_img, n_clear)) first.
int launch_prepare(const ImgDesc* d0, const ImgDesc* descs, OffTables off, int n_img,
                   int64_t n_strips, uint64_t* masks, int64_t* npix, hipStream_t st,
                   int64_t n_clear = 0);

// Fixed-order sum of n int64 device values into *out.
int launch_sum_i64(const int64_t* a, int n, int64_t* out, hipStream_t st);

// Single-image active-set outputs from dense masks.
int launch_tile_list(const uint64_t* masks, int64_t n_tiles, int32_t* flags_scratch,
                     int32_t* offs, int32_t* part, int32_t* n_listed, int32_t* tile_ids,
                     uint64_t* tile_masks, int32_t* slot_map, hipStream_t st);
int launch_pixel_list(const float* f, int H, int W, int ld, double delta, int32_t* counts,
                      int32_t* offs, int32_t* part, int32_t* total, int32_t* pix,
                      int64_t* n_pix, hipStream_t st);

// Scratch of the queue builder: mflags, offs [n_macro]; cflags, coffs
// [n_tiles]; part [scan_partials(max(n_tiles, n_macro))].
struct QueueScratch {
    int32_t* cflags;
    int32_t* coffs;
    int32_t* mflags;
    int32_t* offs;
    int32_t* part;
    int32_t* epoch = nullptr;   // single image: one word per macro tile, zeroed on the way
};

// Work lists from dense tile masks.  Macro-tile queue (bx x by pixels,
// multiples of 8): queue[k] = (image, local macro id) for every macro tile
// holding an open 8x8 tile, ascending; *n_queue = count.  With cqueue non-NULL,
// also the closed 8x8 tiles outside queued macro tiles (cqueue[k] = (image,
// local tile id), *n_closed = count); with cqueue NULL every non-empty tile
// counts as open.
int launch_macro_queue(const ImgDesc* d0, const ImgDesc* descs, OffTables off, int n_img,
                       int64_t n_macro, int bx, int by, const uint64_t* masks,
                       const QueueScratch& q, int2* queue, int32_t* n_queue, int64_t n_tiles,
                       int2* cqueue, int32_t* n_closed, hipStream_t st);

// All iterations of the closed 8x8 tiles in one launch (one wave per tile):
// reads the initial state from buffer 0 and writes the final (v, p) there and u.
int prepare_closed(bool batched);
int launch_closed(const ImgDesc* d0, const ImgDesc* descs, bool batched, const int2* cqueue,
                  const int32_t* n_closed, int64_t max_items, int iters, float theta,
                  float inv_theta, float tau, hipStream_t st, int inner = 1);

// ---------------------------------------------------------------- band threshold
// Radix-select state: digits of the k-th smallest |f| chosen so far and the
// rank still to find among keys that share them.
struct BandState {
    uint32_t prefix;
    uint32_t pad;
    int64_t rank;
};
constexpr int kBandHistBins = 2048;
// q-hat for k = ceil(q N) into *out (device double): 0 for k = 0, else the
// double just above the k-th smallest |f| (+inf if that is not finite).
// hist: kBandHistBins uint32 of scratch.
int launch_band_threshold(const float* f, int H, int W, int ld, int64_t k, uint32_t* hist,
                          BandState* state, double* out, hipStream_t st);

// ---------------------------------------------------------------- measures
// Sec. 4 measures of u against u_ref: out[0] = #(both labels), out[1] =
// #(either label), out[2] = sum (u - u_ref)^2; partials of
// metrics_partials_bytes() bytes.
size_t metrics_partials_bytes();
int launch_metrics(const float* u, const float* g, int H, int W, int ld, double eps,
                   double* partials, double* out, hipStream_t st);

// Tile configuration of a temporally blocked kernel: bx x by macro tiles,
// `it` steps per launch (the halo depth), nt threads per workgroup.
struct TileCfg {
    int bx, by, it, nt;
};

// ---------------------------------------------------------------- primal-dual
int pd_config_count();
TileCfg pd_config_at(int i);
int pd_config_index(int bx, int by, int it);   // -1 if not compiled
int launch_pd_init(const PdDesc& d, hipStream_t st);
// nit (<= cfg.it) primal-dual iterations over the queued macro tiles, reading
// state buffer in_buf and writing 1 - in_buf.
int launch_pd_iterate(int ci, const PdDesc& d, const int2* queue, const int32_t* n_queue,
                      int64_t max_items, int in_buf, int nit, float tau, float sigma,
                      hipStream_t st);

// ---------------------------------------------------------------- volumes
void volume_tile(int* bx, int* by, int* bz);   // the volume kernel's tile
int launch_init3(const VolDesc& d, hipStream_t st);
int launch_tile_flags3(const VolDesc& d, int64_t n_tiles, int32_t* flags, hipStream_t st);
// One dual step on the flagged tiles, reading state buffer in_buf and writing
// 1 - in_buf; with uv also the u-step and v-step (u written when write_u).
int launch_iterate3(const VolDesc& d, const int32_t* flags, int64_t n_tiles, int in_buf, bool uv,
                    bool write_u, float theta, float inv_theta, float tau, hipStream_t st);
// Two consecutive dual steps in one pass (the u/v step after the first when
// uv1, after the second when uv2); reads buffer in_buf, writes 1 - in_buf.
int launch_iterate3x2(const VolDesc& d, const int32_t* flags, int64_t n_tiles, int in_buf,
                      bool uv1, bool uv2, bool write_u, float theta, float inv_theta, float tau,
                      hipStream_t st);

// ---------------------------------------------------------------- iteration
int launch_init(const ImgDesc* d0, const ImgDesc* descs, OffTables off, int n_img,
                int64_t n_rows, hipStream_t st);

int config_count();
TileCfg config_at(int i);
int config_index(int bx, int by, int it);   // -1 if not compiled

// Occupancy query for the persistent grid of configuration ci (cached).
int prepare_iterate(int ci, bool batched, bool stop = false);

// Work arrays of the small-component path (single image, indices g = y * ld
// + x of the image's [H][ld] plane): lab (union-find parent, then root; -1
// off RD), csize (pixels per root), crank (each pixel's rank in its component),
// cslot (slot of a root in its size class), lane_of (packed lane of a
// small-component pixel, -1 otherwise), wl_pix (pixel of each packed lane, -1
// for empty lanes; 2 * plane + kCompLaneExtra entries), ccount (kCompCount:
// components per size class, then [kCompFlag] set when the resident kernel
// ran the one-wave classes), npix_tile (RD pixels left to the tile path).
constexpr int kCompClasses = 9;                    // padded sizes 1, 2, 4, ..., 256
constexpr int kCompLaneExtra = kCompClasses * 64;  // a partly filled last wave per class
constexpr int kCompCount = 16;
constexpr int kCompFlag = 15;
struct CompWs {
    int32_t* lab;
    int32_t* csize;
    int32_t* crank;
    int32_t* cslot;
    int32_t* lane_of;
    int32_t* wl_pix;
    int32_t* ccount;
    int64_t* npix_tile;
};

// Small-component path of a single-image solve (components.hip): label the
// RD components of d (c already written), pack those of at most 256 pixels
// into waves or groups and freeze their pixels for the tile path (c = +inf, tile-mask
// bits cleared, w.npix_tile = the RD pixels left to it); then run every
// iteration of them.  Both do nothing on the device when more than 55 % of
// the pixels are RD (npix_tile is still written).  With a tape (inner = 1,
// ce > 0) the component kernel also writes its pixels' checkpoints (the state
// before iteration k into slot k / ce, [3][H][ld] per slot); the tile path's
// copies write only the RD pixels left to it, so the two may run side by side.
int launch_components_prepare(const ImgDesc& d, const CompWs& w, uint64_t* masks,
                              const int64_t* npix, hipStream_t st);
int launch_components(const ImgDesc& d, const CompWs& w, const int64_t* npix, int iters,
                      int inner, float theta, float inv_theta, float tau, float* tape, int ce,
                      hipStream_t st);
// The reverse sweep of the small components (all K steps of the adjoint,
// segments of ce steps recomputed from the tape checkpoints into LDS when
// (ce - 1) x 768 bytes fit a workgroup, else into seg, the (ce - 1) x
// [3][H][ld] slots of the backward): writes sacc and vbar^0 (vb_out) of their
// pixels.  Then c of those pixels back to theta lambda f.
// nwaves_hint: the packed component waves (component_waves_of the class
// counts read back), or -1 when unknown; it picks the LDS form.  group_jobs:
// the jobs of the group classes (component_group_jobs_of), -1 when unknown;
// their reverse runs first, in a launch of its own (skipped at 0).
int launch_adj_components(const ImgDesc& d, const CompWs& w, const int64_t* npix,
                          const float* tape, float* seg, int K, int ce, const float* grad_u,
                          const float* grad_v, float* vb_out, float* sacc, float theta,
                          float inv_theta, float tau, hipStream_t st, int64_t nwaves_hint,
                          int64_t group_jobs = -1);
int64_t component_waves_of(const int32_t* ccount_host);       // waves of classes 0..6
int64_t component_group_jobs_of(const int32_t* ccount_host);  // jobs of classes 7, 8
int launch_components_restore(const ImgDesc& d, const CompWs& w, const int64_t* npix,
                              hipStream_t st);

// Resident form of a whole single-image solve: whether configuration ci has a
// resident kernel whose workgroups, one per queued macro tile (at most
// max_items), all fit on the chip at once; and the launch, which runs `iters`
// outer iterations in blocks of `per` (per * inner <= cfg.it), reading buffer
// in_buf and leaving the final state where the equivalent separate launches
// would.  epoch: max_items int32 of workspace, status: one int32, zero before
// the launch (set to 1 if a bounded wait expired; u, v and p then hold NaN on
// every tile that stopped).  Returns 0 when launched,
// -1 when the resident form does not apply (nothing was enqueued), > 0 on error.
// `before` (nullable) is recorded on st right before the resident kernel.
// comp (nullable; labelled by launch_components_prepare with the full RD
// count comp_npix): the workgroups left without a tile run the small
// components' iterations and set comp->ccount[7]; a component kernel launched
// afterwards on st then returns at once (and does the work itself if no
// workgroup was left over).
bool resident_fits(int ci, int64_t max_items);
// whether configuration ci has a resident form at all
bool resident_available(int ci);
// co-resident workgroups of ci's resident form (0: none)
int resident_capacity(int ci);
// Bound of each wait of the resident kernel in ticks of the 100 MHz wall
// clock: 0 restores the default (1 s), < 0 makes every wait give up at once.
void set_resident_wait_ticks(int64_t ticks);
int64_t resident_wait_ticks();
// grid (0: one workgroup per macro tile of the image, max_items of them) is
// the number of workgroups otherwise: at least the queue length rounded up to
// a multiple of 8, and within the co-resident capacity.
int launch_resident(int ci, const ImgDesc& d, const int2* queue, const int32_t* n_queue,
                    const int32_t* mflags, int32_t* epoch, int32_t* status, int64_t max_items,
                    int in_buf, int iters, int per, int inner, float theta, float inv_theta,
                    float tau, hipStream_t st, hipEvent_t before, const CompWs* comp = nullptr,
                    const int64_t* comp_npix = nullptr, int64_t grid = 0,
                    bool epoch_cleared = false);

// Per-launch arguments of the convergence-driven solve: skip the launch when
// *skip_slot <= tol (skip_slot nullable); reduce the last iteration's change
// into *diff_slot (nullable: this launch does not end at a check).
struct StopLaunch {
    const uint32_t* skip_slot;
    uint32_t* diff_slot;
    double tol;
};

// One launch of the temporally blocked iteration kernel: `nit` outer
// iterations of `inner` dual steps each (nit * inner <= cfg.it, the halo
// depth) over the queued macro tiles, reading state buffer `in_buf` and
// writing 1 - in_buf; writes u on RD when write_u.  grid = persistent size.
int launch_iterate(int cfg_index, const ImgDesc* d0, const ImgDesc* descs, bool batched,
                   const int2* queue, const int32_t* n_queue, int64_t max_items, int in_buf,
                   int nit, bool write_u, float theta, float inv_theta, float tau,
                   hipStream_t st, const StopLaunch* stop = nullptr, int inner = 1);

// Every block of a batched solve in one cooperative launch of the persistent
// iteration kernel (grid-wide barriers between blocks of `per` iterations;
// bitwise the separate launches).  *bar is cleared first; *status is set if
// a barrier's wait expires.  Returns -1 when the form cannot be launched
// (the caller then enqueues separate launches), > 0 on a HIP error.
// The adjoint's recompute: nit (<= 8) outer iterations of the 16x16 / 8
// blocked kernel over the queued 16x16 macro tiles from state buffer in_buf
// (writing 1 - in_buf), with the state after iteration s also written to
// tape + s * tape_step (v, p_x, p_y planes tape_plane apart) on RD pixels.
int launch_recompute(const ImgDesc& d, const int2* queue, const int32_t* n_queue,
                     int64_t max_items, int in_buf, int nit, float theta, float inv_theta,
                     float tau, float* tape, int64_t tape_step, int64_t tape_plane,
                     hipStream_t st);

int prepare_iterate_persist(int cfg_index);   // occupancy query (outside graph capture)
int launch_iterate_persist(int cfg_index, const ImgDesc* d0, const ImgDesc* descs,
                           const int2* queue, const int32_t* n_queue, int iters, int per,
                           float theta, float inv_theta, float tau, int32_t* bar,
                           int32_t* status, hipStream_t st);

// After a convergence-driven solve: *iters_done = (c + 1) * check_every for
// the first check c with slots[c] <= tol (else iters), then the state of
// that check is moved into buffer 0 when it lies in buffer 1.  The check c
// ended launch (c + 1) * launches_per_check - 1 of n_launches, which wrote
// buffer 1 - (n_launches - j) % 2.
int launch_stop_finalize(const ImgDesc& d, const uint32_t* slots, int n_checks, double tol,
                         int check_every, int launches_per_check, int n_launches, int iters,
                         int32_t* iters_done, hipStream_t st);

// Copy (v, px, py) of RD pixels from a state buffer into a full-grid slot
// [3][H][ld].
int launch_state_copy(const ImgDesc& d, int buf, float* slot, hipStream_t st);

// ---------------------------------------------------------------- adjoint
struct AdjBufs {
    float* pbx[2];
    float* pby[2];
    float* vb[2];
    float* sacc;          // sum over steps of the clamp adjoint
};
// The stored state of each reverse step of one launch: s[i] holds v^{k-1-i},
// p_x at +plane and p_y at +2 plane (full-grid planes).
constexpr int kAdjMaxSteps = 8;
struct AdjSlots {
    const float* s[kAdjMaxSteps];
    int64_t plane;
};
int adj_config_count();
// index of the reverse kernel for tile x tile macro tiles and up to ns steps
// a launch, -1 if there is none
int adj_config_find(int tile, int ns);
int adj_config_steps(int ai);
int adj_config_tile(int ai);
// Reverse steps k, ..., k - ns + 1 (ns <= the kernel's step count) on the
// queued macro tiles of d's tile size: (pbar, vbar) from buffer in_buf to
// 1 - in_buf, the clamp-adjoint sum accumulated; first: k is the last
// iteration (pbar^k = 0, vbar^k = grad_v, dL/du = grad_u enters).
int launch_adj_block(int ai, const ImgDesc& d, const AdjSlots& sl, int ns, const AdjBufs& ab,
                     int in_buf, bool first, const float* grad_v, const float* grad_u,
                     const int2* queue, const int32_t* n_queue, int64_t max_items, float theta,
                     float tau, hipStream_t st);
int launch_adj_final(const ImgDesc& d, const float* sacc, const float* vb0, float* grad_f,
                     double lambda, double theta, const float* z, const float* P, double c1,
                     double c2, double* partials, int64_t n_part, double* out4,
                     hipStream_t st);
int launch_fit_forward(const float* z, const float* P, double c1, double c2, double gamma,
                       int H, int W, int ld, float* f, hipStream_t st);
int launch_fit_backward(const float* z, const float* P, const float* grad_f, double c1,
                        double c2, int H, int W, int ld, double* partials, int64_t n_part,
                        double* out3, hipStream_t st);
int64_t reduce_partials(int H);
int launch_fill(float* p, int H, int W, int ld, float v, hipStream_t st);
int launch_scatter_scalars(const double* src, double* a, double* b, double* c, double* d,
                           hipStream_t st);

int persistent_blocks(const void* kernel, int threads, size_t dyn_lds);
int cooperative_blocks(const void* kernel, int threads, size_t dyn_lds);

}  // namespace rdseg
