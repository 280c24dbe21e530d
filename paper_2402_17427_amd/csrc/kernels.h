// Host-side launchers of the rasterizer kernels.  Each enqueues on `st`
// and returns at once; shapes are validated by the C ABI layer (api.cpp)
// before any of these is called.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gs_device.h"

namespace gs {

// ---- projection (project.hip)
// nslots record slots (jobs' out0 aligned to kSlotAlign; K = SH size, the
// same for every job).  Padding slots get tiles_touched = 0.
void launch_project(const JobTab& jobs, const ViewTab& views, int K, int64_t nslots, int tw, int th, Rec* rec,
                    float* depth, ushort4* rect, uint32_t* tiles_touched, hipStream_t st);
// Chain rule per slot from g2d [9][nslots] into each job's gradient planes.
void launch_project_bwd(const JobTab& jobs, const ViewTab& views, int K, int64_t nslots,
                        const uint32_t* tiles_touched, const float* g2d, const int32_t* status, hipStream_t st);

// ---- binning (binning.hip)
// Device words to zero before a binning sort; the emission's first kernel
// clears them (saving the sort a launch).
struct ZeroList {
    uint32_t* p[3];
    int64_t n[3];
};
// Workspace for the tiles_touched scan over n Gaussians.
size_t scan_workspace_bytes(int64_t n);
// Exclusive scan of tiles_touched, then one (tile << 32 | depth bits, index)
// pair per covered tile.  Writes *pair_count and sets *status to
// GS_ERR_CAPACITY (-4) when the pairs exceed `capacity` (pairs beyond it
// are dropped).  `first` (optional, n entries) receives each Gaussian's
// first emission position.
void launch_emit_pairs(int64_t n, const uint32_t* tiles_touched, const ushort4* rect, const float* depth,
                       const JobTab& jobs, const ViewTab& views, int64_t capacity, uint64_t* keys, uint32_t* vals,
                       uint32_t* first, uint32_t* pair_count, int32_t* status, void* scan_ws, hipStream_t st,
                       const ZeroList* zero = nullptr);
// Per-tile [start, end) of sorted keys; `zeroed`: ranges already hold zeros.
void launch_tile_ranges(const uint64_t* keys, const uint32_t* pair_count, int64_t capacity, int64_t n_tiles,
                        uint32_t* ranges, hipStream_t st, bool zeroed = false);
void launch_fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t st);

// ---- radix sort (sort.hip)
size_t sort_workspace_bytes(int64_t capacity, int key_bits);
// Stable LSD sort of (key, val) on the low key_bits bits.  The sorted pairs
// end in (keys, vals); (alt_keys, alt_vals) are ping-pong buffers of the
// same capacity.  When `start_in_alt` is set the input is read from the
// alternate buffers instead (so that an odd pass count still ends in
// keys/vals).
int sort_passes(int key_bits);
void launch_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* alt_keys, uint32_t* alt_vals,
                       const uint32_t* count, int64_t capacity, int key_bits, bool start_in_alt, void* ws,
                       hipStream_t st);
// Binning sort of emitted (tile << 32 | depth bits, index) pairs: a stable
// radix sort on the tile bits, per-tile ranges, then each tile's run sorted
// stably by depth inside one workgroup -- the order of a stable sort on the
// whole key.  The emission must go to (alt_keys, alt_vals) when
// bin_sort_emit_to_alt(tile_bits), else to (keys, vals); the sorted pairs
// end in (keys, vals) and `ranges` [n_tiles][2] is written.  `ws` holds
// sort_workspace_bytes(capacity, 32 + tile_bits) bytes.
bool bin_sort_emit_to_alt(int tile_bits);
// What the emission must zero for launch_bin_sort(..., zeroed = true).
ZeroList bin_sort_zero_list(void* ws, int64_t capacity, int tile_bits, uint32_t* ranges, int64_t n_tiles);
// `tile_order` (optional, n_tiles + 1 words): [0] = n_tiles, [1..] every
// tile, the longest lists first (launch_tile_order with the empty tiles).
void launch_bin_sort(uint64_t* keys, uint32_t* vals, uint64_t* alt_keys, uint32_t* alt_vals, const uint32_t* count,
                     int64_t capacity, int tile_bits, uint32_t* ranges, int64_t n_tiles, void* ws, hipStream_t st,
                     bool zeroed = false, uint32_t* tile_order = nullptr);

// ---- direct binning (bin_direct.hip)
// For views of at most kDirectMaxTiles tiles each, the pairs are placed
// into their tile's run straight from the tile rectangles (per-block tile
// histograms, their column scan, an LDS-cursor scatter), then each run is
// sorted on (depth, index): the same keys, values, ranges, `first`, pair
// count, status and tile order as launch_emit_pairs + launch_bin_sort.
constexpr int64_t kDirectMaxTiles = 32768;
// One view of a direct binning (bin_direct_plan fills them; several views
// go to the kernels as a device table, one in the kernel arguments).
struct DView {
    int64_t s0, s1;        // the view's record slots [s0, s1), s0 a multiple of 4
    int64_t chunk;         // slots per block (a multiple of 4)
    int64_t m0;            // first word of its count-matrix rows (nb rows of n_tiles words)
    uint32_t tile_base, n_tiles;
    int ntx, nty;
    int b0, nb;            // its blocks b0 .. b0 + nb - 1 (global ids, in slot order)
    int c0;                // its first strip of 64 tiles in the column scan
};
struct DTab {
    const DView* dev;
    int n;
    DView one;
};
struct DPlan {
    int n_views = 0, nb = 0, strips = 0;
    uint32_t n_tiles = 0, max_tiles = 0;
    int64_t m_words = 0;
};
// Views 0 .. nv - 1 (slots [s0[v], s1[v]) in increasing order, tile grid
// ntx[v] x nty[v] from global tile tile_base[v]); fills out[0 .. nv - 1].
// False when a view has no tile or more than kDirectMaxTiles of them.
bool bin_direct_plan(int nv, const int64_t* s0, const int64_t* s1, const int* ntx, const int* nty,
                     const uint32_t* tile_base, DView* out, DPlan* plan);
// Device scratch of the placement (count matrix, tile and block totals);
// the placed pairs (capacity u64) are a buffer of their own.
size_t bin_direct_scratch_bytes(const DPlan& plan);
// Placement: `first` (optional, every slot of the views), ranges,
// pair_count[2], status, and the placed pairs (depth bits << 32 | slot).
void launch_bin_direct_place(const DPlan& plan, const DTab& views, const ushort4* rect, const float* depth,
                             int64_t capacity, uint32_t* first, uint32_t* ranges, uint32_t* pair_count,
                             int32_t* status, void* scratch, uint64_t* pairs, hipStream_t st);
// Per-run sort of the placed pairs into (keys, vals), and the tile order
// (optional, n_tiles + 1 words: [0] = n_tiles, [1..] every tile, the
// longest lists first).
void launch_bin_direct_sort(uint32_t n_tiles, int64_t capacity, uint64_t* keys, uint32_t* vals,
                            const uint32_t* ranges, const int32_t* status, uint32_t* tile_order,
                            uint64_t* pairs, hipStream_t st);
// One view of n Gaussians (the plain calls): workspace = scratch + pairs.
bool bin_direct_supported(int64_t n_tiles);
size_t bin_direct_ws_bytes(int64_t n, int64_t capacity, int64_t n_tiles);
void launch_bin_direct_place(int64_t n, const ushort4* rect, const float* depth, int ntx, int64_t n_tiles,
                             int64_t capacity, uint32_t* first, uint32_t* ranges, uint32_t* pair_count,
                             int32_t* status, void* ws, hipStream_t st);
void launch_bin_direct_sort(int64_t n, int64_t n_tiles, int64_t capacity, uint64_t* keys, uint32_t* vals,
                            const uint32_t* ranges, const int32_t* status, uint32_t* tile_order, void* ws,
                            hipStream_t st);

// ---- blend (render_fwd.hip / render_bwd.hip)
// What both blend passes read: records, sorted values, per-tile ranges of
// all views' tiles (global tile ids), status, the view table and the tile
// shape.  With `queue` set (one device uint32, zeroed by the launcher) and
// persistent_grid > 0 the launch is a persistent grid pulling tiles from
// `order` (a permutation of the tiles, or NULL for 0, 1, ...).
struct RenderArgs {
    const Rec* rec;
    const uint32_t* vals;
    const uint32_t* ranges;
    const int32_t* status;
    ViewTab views;
    uint32_t n_tiles;
    int tw, th;
    uint32_t* queue;
    const uint32_t* order;
    int persistent_grid;
    // Optional, render_mask_words(tw, th) words per sorted pair: the
    // forward stores each pair's cell mask of every wave of its tile, the
    // backward reads them instead of recomputing (NULL: not kept).
    uint64_t* masks;
    // One-workgroup-per-tile launches: when set, workgroup b takes tile
    // tile_order[b] and workgroups b >= *tile_order_count exit (the order
    // of launch_tile_order, so that the longest lists start first).
    const uint32_t* tile_order;
    const uint32_t* tile_order_count;
    // Persistent launches only: the forward's staged entries per batch
    // (render_fwd_batch_small() or the default) and the backward's slots
    // per chunk (render_item_cap_small() or the default); 0 = default.
    int fwd_batch, item_cap;
};

bool render_tile_supported(int tw, int th);
// Cell-mask words per sorted pair (waves of a tile's workgroup).
int render_mask_words(int tw, int th);
// image/final_T/n_contrib are the stacked planes of all views.  stats !=
// NULL runs the counting variant instead (no image written); state !=
// NULL also stores the per-entry blend state (pairs * tile pixels).
void launch_render_fwd(const RenderArgs& r, float* image, float* final_T, uint32_t* n_contrib,
                       unsigned long long* stats, float2* state, hipStream_t st);
// The counting pass with the backward's cells: adds the evaluations its walk
// performs to stats[3] (the forward's own counts go to stats[0..2]).
void launch_render_stats_bwd_cells(const RenderArgs& r, unsigned long long* stats, hipStream_t st);
// Per-pair image-space gradients of the blend.  `pairs` is the pair
// gradient buffer (pair_grad_bytes(capacity) bytes): the backward writes,
// for every (Gaussian, tile) pair of the frame, the nine sums of the
// tile's pixels (zero where the Gaussian contributes nothing) at the
// pair's emission position (first[slot] + the tile's row-major index in
// the Gaussian's rectangle), so the buffer needs no clearing; when the bin
// status is set it writes nothing and the gather yields zeros.
// state != NULL reads the stored blend state instead of recomputing it.
void launch_render_bwd(const RenderArgs& r, const float* final_T, const uint32_t* n_contrib, const float* dimg,
                       const ushort4* rect, const uint32_t* first, void* pairs, int64_t capacity,
                       const float2* state, hipStream_t st);
size_t pair_grad_bytes(int64_t capacity);
// g2d[9][nslots] = the sum of each slot's pair entries (emission order);
// zeros for culled slots and when *status != 0.
void launch_pair_gather(int64_t nslots, const uint32_t* first, const uint32_t* tiles_touched, const void* pairs,
                        int64_t capacity, const int32_t* status, float* g2d, hipStream_t st);

// Workgroups of a persistent blend launch that fit on the device at once
// (lds_knob: the fwd_batch or item_cap it will run with, 0 = default).
int render_persistent_grid(int tw, int th, bool backward, int lds_knob = 0);
int render_fwd_batch_default();
int render_fwd_batch_small();
int render_item_cap_default();
int render_item_cap_small();

// ---- batched step (batch_kernels.hip)
// L1 loss of every view against its target ([3][H][W] each; targets is a
// device array of device pointers): loss[v] = mean |I - I*| (FP64 partial
// sums added in a fixed order, the same on every run), dimg =
// sign(I - I*) / (3 W H), zero when *status != 0.  partials holds
// kL1MaxChunks doubles per view.
constexpr int kL1MaxChunks = 1024;
void launch_l1(const ViewTab& views, int n_views, int64_t max_pix, const float* const* targets, const float* image,
               float* dimg, float* loss, double* partials, const int32_t* status, hipStream_t st);
// ---- training loss (loss.hip)
// Eq. 1 / Eq. 3 loss of one [channels][height][width] image against its
// target: d_image gets the gradient (of both terms when image_l1 is NULL,
// else of the D-SSIM term, the L1 term's going to d_image_l1) and ws
// (loss_workspace_bytes()) the per-tile partial sums, which
// launch_loss_finish reduces into loss[3] = (total, L1, mean SSIM).
size_t loss_workspace_bytes(int channels, int width, int height);
void launch_loss(const float* image, const float* image_l1, const float* target, int channels, int width, int height,
                 float lambda, float* d_image, float* d_image_l1, void* ws, hipStream_t st);
// n_out = 3: loss[0..2] = (total, L1, mean SSIM); n_out = 1: the total only.
void launch_loss_finish(int channels, int width, int height, float lambda, const void* ws, float* loss,
                        hipStream_t st, int n_out = 3);
// ---- optimiser step (optim.hip)
// Adam over every raw plane of n Gaussians (stride ld; gradients with
// stride gld, grad2d [9][n]) plus the densification statistics; nothing
// changes when *status != 0.  step_size[g] = lr_g / (1 - beta1^t) for the
// groups mean, scale, quat, opacity, SH DC, SH rest.
struct AdamDev {
    float step_size[6];
    float inv_sqrt_bc2;
};
// Device-resident schedule of a sequence of steps (the batched step): the
// prepare kernel advances `step` and writes `dev`, which AdamArgs::dev
// points at.
struct AdamSched {
    int step;                 // steps taken so far
    float lr[6];
    float beta1, beta2;
    float lr_mean_final;      // <= 0: constant position rate
    int lr_mean_steps;
    AdamDev dev;
};
struct AdamArgs {
    const AdamDev* dev;  // when set, step_size and inv_sqrt_bc2 are read from it
    float *mean, *log_scale, *quat, *logit, *sh;
    float *scale_out, *opacity_out;
    const float *g_mean, *g_scale, *g_quat, *g_opacity, *g_sh, *g2d;
    float *m, *v, *accum, *count;
    const uint32_t* tiles;
    const int32_t* status;
    int64_t n, ld, gld, g2d_ld;  // g2d rows: [9][g2d_ld]
    int K;
    float step_size[6];
    float beta1, beta2, one_m_beta1, one_m_beta2, inv_sqrt_bc2, eps;
};
void launch_adam(const AdamArgs& a, hipStream_t st);
void launch_adam_prepare(AdamSched* s, hipStream_t st);
// ---- partitioning (partition.hip)
// Camera table rows: R[9], t[3], fx, fy, cx, cy, W, H, near, pad.
constexpr int kCamDoubles = 20;
// member[c][i] = 1 when point i's ground position (x, z) lies in cell c's
// closed expanded rectangle cells[c] = (x0, x1, z0, z1), else 2 when one of
// the cell's views (views[offsets[c] .. offsets[c + 1])) covers it, else 0.
// tests (optional) accumulates the projections performed.
struct SelectArgs {
    const float* points;  // [3][ld]
    int64_t n, ld;
    const double* cells;  // [n_cells][4]
    const double* cams;   // [n_views][kCamDoubles]
    const int* offsets;   // [n_cells + 1]
    const int* views;
    int n_cells;
    uint8_t* member;      // [n_cells][n]
    uint64_t* tests;
    const uint32_t* order;  // visiting order of the points (set by the launcher)
};
// Scratch of the visiting-order sort for n points.
size_t select_sort_bytes(int64_t n);
// Points are visited in the Morton order of their ground position over
// box = (x0, x1, z0, z1) (sorted in sort_ws, select_sort_bytes(n) bytes).
void launch_select_points(const SelectArgs& a, const double box[4], void* sort_ws, hipStream_t st);
// keep[i] = Gaussian i's (x, z) in [x0, x1) x [z0, z1) (closed above where asked)
void launch_merge_keep(const float* mean, int64_t n, int64_t ld, const double rect[4], int closed_x, int closed_z,
                       uint8_t* keep, hipStream_t st);
// ---- appearance model (appearance.hip)
// 3x3 convolution, zero padding 1, planar [C][H][W] maps.  Forward:
// out[o] = b[o] + sum_i w[o][i] * in[i]; transposed (the backward w.r.t. the
// input): out[i] = sum_o flip(w[o][i]) * in[o] with Cin = the forward
// layer's Cout, Cout = its Cin (CinF).  mask: the input is used only where
// mask > 0 (a ReLU's output); relu: max(0, .) on the output.
struct ConvArgs {
    const float* in;
    const float* mask;
    const float* w;
    const float* b;
    float* out;
    int Cin, Cout, H, W;
    int transposed, relu, CinF;
    // split of the input-channel reduction over conv_splits() workgroup
    // groups: raw partial sums [splits][Cout][H][W] (no bias, no ReLU),
    // added in a fixed order by a second kernel; NULL = never split
    float* part;
};
void launch_conv(const ConvArgs& a, hipStream_t st);
// input-channel splits launch_conv uses for this shape (1 = none)
int conv_splits(int Cin, int Cout, int H, int W);
// Weight and bias gradients of a forward convolution with input `in`
// [Cin][H][W] and output gradient g [Cout][H][W] (masked like ConvArgs):
// dw = [Cout][Cin][9] then [Cout] (J = Cout Cin 9 + Cout floats); partial
// holds wgrad_parts(H, W) x J floats.
struct WgradArgs {
    const float* in;
    const float* g;
    const float* mask;
    float* partial;
    int Cin, Cout, H, W;
    int64_t J;
};
int wgrad_parts(int H, int W);
void launch_wgrad(const WgradArgs& a, float* dw, hipStream_t st);
void launch_down_concat(const float* img, int H, int W, int h, int w, const float* embed, int m, float* D,
                        hipStream_t st);
void launch_down_adjoint(const float* g, int H, int W, int h, int w, float* d_img, hipStream_t st);
void launch_shuffle(const float* in, int C, int h, int w, float* out, bool inverse, hipStream_t st);
struct BilinTab {
    const int *y0, *y1, *x0, *x1;
    const float *fy, *fx;
    int *ylo, *yhi, *xlo, *xhi;   // adjoint ranges per input index (written by launch_bilinear_adj)
};
void launch_bilin_table(int n_in, int n_out, int* i0, int* i1, float* f, hipStream_t st);
void launch_bilinear(const float* in, int C, int h, int w, int H, int W, const BilinTab& t, float* out,
                     hipStream_t st);
// tmp: C H w floats of scratch
void launch_bilinear_adj(const float* g, int C, int H, int W, int h, int w, const BilinTab& t, float* tmp,
                         float* out, hipStream_t st);
void launch_mul(const float* a, const float* b, int64_t n, float* out, hipStream_t st);
void launch_mul_bwd(const float* d_adj, const float* img, const float* M, int64_t n, float* dM, float* d_img,
                    hipStream_t st);
void launch_embed_grad(const float* dD, int64_t hw, int m, float* d_embed, hipStream_t st);
// Sort keys putting the tiles with the longest lists first.
// order[0 .. *count) = the tiles with pairs, longest list first by the log2 of
// its length, then (include_empty) the empty tiles; one small launch.
void launch_tile_order(const uint32_t* ranges, uint32_t n_tiles, uint32_t* order, uint32_t* count, bool include_empty,
                       hipStream_t st);

}  // namespace gs
