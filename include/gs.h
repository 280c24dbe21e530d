/*
 * gs.h -- C ABI of the MI355X differentiable Gaussian tile rasterizer.
 *
 * The operation is the renderer R(G, C) of VastGaussian (arXiv 2402.17427),
 * section 3: a set G of 3D Gaussians (position, anisotropic covariance from
 * scale and rotation, opacity, spherical-harmonic colour) is projected to 2D
 * image-space Gaussians by EWA splatting, the 2D Gaussians are assigned to
 * screen tiles, sorted by depth within each tile and alpha-blended front to
 * back into the image I = R(G, C).  R is differentiable: given dLoss/dImage
 * the backward call returns dLoss/d(every Gaussian parameter), which is how
 * each partition cell's Gaussians are optimised (sections 3 and 4.2).
 *
 * The image-formation constants the paper leaves to 3DGS (section 5.1) are:
 *   2D dilation 0.3 px^2; affine clamp |x/z| <= 1.3 (W/2)/fx, same for y;
 *   alpha = min(0.99, o exp(power)), Gaussians with alpha < 1/255 skipped;
 *   a pixel stops before the Gaussian that would take T below 1e-4;
 *   colour = max(0, SH(view direction) + 0.5); quaternions (w, x, y, z);
 *   pixel centres at (x + 0.5, y + 0.5); depth = camera-space z of the
 *   centre, ties broken by Gaussian index.
 * A Gaussian's tile rectangle is the bounding box of the pixels where its
 * alpha can reach 1/255 (the ellipse of radius^2 = 2 ln(255 o) in its conic
 * metric), so binning never changes the image: the result is the plain
 * every-Gaussian-at-every-pixel blend in depth order, for any tile size.
 *
 * Conventions for every call:
 *  - Pointers named "device" are device memory on the current HIP device;
 *    the caller allocates and owns them (the library never frees caller
 *    memory).  Descriptor structs themselves live in host memory and are
 *    read during the call only.
 *  - Calls enqueue work on `stream` (a hipStream_t, NULL = default stream)
 *    and return without synchronising, except where stated.
 *  - Return GS_OK (0) or a negative gs_status; gs_last_error() gives a
 *    thread-local message.  Host-detectable errors (NULL pointers, negative
 *    sizes, unsupported tile sizes, SH degree > 3, ld < n, W or H <= 0) are
 *    rejected before anything is enqueued.
 *  - Device-detected pair overflow (more (Gaussian, tile) pairs than the
 *    caller's capacity) sets *status = GS_ERR_CAPACITY in device memory; the
 *    render calls then write NaN images and zero gradients instead of
 *    partial results.  Read `status` after the stream completes.
 *  - All float data is IEEE FP32 (centres of projected Gaussians are FP64).
 *    Gradients are w.r.t. the inputs as given: linear scale, opacity in
 *    (0, 1), un-normalised quaternion, raw SH coefficients.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 2

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID = -1,     /* bad argument, detected on the host */
    GS_ERR_OOM = -2,         /* allocation failed (handles only) */
    GS_ERR_HIP = -3,         /* a HIP runtime call failed */
    GS_ERR_CAPACITY = -4,    /* pair buffer too small (device status flag) */
    GS_ERR_BUSY = -5,        /* server queue full */
    GS_ERR_UNSUPPORTED = -6, /* valid but not implemented (e.g. tile size) */
    GS_ERR_TIMEOUT = -7,     /* wait timed out */
    GS_ERR_NOT_FOUND = -8    /* unknown ticket */
} gs_status;

typedef void *gs_stream; /* a hipStream_t */

int gs_abi_version(void);
const char *gs_last_error(void);

/* Gaussian set, structure of arrays, device FP32 planes with stride ld >= n
 * (element k of Gaussian i of a [P][ld] array is at [k*ld + i]):
 *   mean[3][ld]  world position          scale[3][ld] linear scale (> 0)
 *   quat[4][ld]  rotation (w, x, y, z)   opacity[ld]  in (0, 1)
 *   sh[3K][ld]   SH coefficients, plane c*K + j for colour channel c and
 *                basis j = l*l + l + m, K = (sh_degree + 1)^2, degree <= 3.
 * Non-finite parameters, centres at or behind near_z, opacity < 1/255 and
 * Gaussians whose support misses the image are culled (no pairs, zero
 * gradient). */
typedef struct {
    int64_t n, ld;
    int32_t sh_degree;
    const float *mean, *scale, *quat, *opacity, *sh;
} gs_gaussians;

/* Pinhole camera (host struct).  R: world->camera rotation, row-major;
 * t: translation (x_cam = R x_world + t).  Camera +z looks forward, +x right,
 * +y down the image.  Pixel (x, y) has centre (x + 0.5, y + 0.5).
 * bg: background colour blended with the final transmittance. */
typedef struct {
    float R[9], t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    float near_z;
    float bg[3];
} gs_camera;

/* Tuning options (host struct); pass NULL for the defaults.  Zero fields
 * take defaults.  Supported tiles: 16x16 (default), 8x8, 16x8, 32x8, 32x16,
 * 32x32.
 * The image does not depend on the tile size. */
typedef struct {
    int32_t tile_w, tile_h;
    int32_t reserved[6];
} gs_opts;

/* Projection output (caller-owned device buffers, n entries each):
 *   rec   n x 48-byte records, 16-byte aligned: { double u, v (pixel-space
 *         centre); float A, B, C (conic = inverse 2D covariance, with
 *         power = -0.5 (A dx^2 + C dy^2) - B dx dy); float opacity;
 *         float r, g, b (colour); float thr = -log2(255 opacity), the
 *         base-2 exponent above which alpha >= 1/255 }.
 *   depth n floats: camera-space z (the sort key).
 *   rect  n x 4 uint16, 8-byte aligned: tile rectangle x0, y0, x1, y1
 *         (x1, y1 exclusive).
 *   tiles_touched n uint32: (x1 - x0) (y1 - y0), 0 for culled Gaussians.
 * Records of culled Gaussians are unspecified. */
typedef struct {
    void *rec;
    float *depth;
    uint16_t *rect;
    uint32_t *tiles_touched;
} gs_proj;

/* Binning output (caller-owned device buffers):
 *   keys[pair_capacity]  sorted (tile << 32 | float32 bits of depth)
 *   vals[pair_capacity]  Gaussian index of each sorted pair
 *   first[n]             emission position of each Gaussian's first pair:
 *                        Gaussian i's pairs were emitted at positions
 *                        first[i] .. first[i] + tiles_touched[i] - 1, one
 *                        per tile of its rectangle in row-major order (the
 *                        backward keys its per-tile sums by it).  n is the
 *                        Gaussian count given to gs_bin_sort.  May be NULL
 *                        when no backward follows.
 *   ranges[n_tiles][2]   [start, end) of each tile's pairs; empty = [0, 0)
 *   pair_count[2]        written by gs_bin_sort: [0] = number of sorted
 *                        pairs P (0 on overflow), [1] = pairs the view
 *                        needs (saturated at 2^32-1), to size a retry
 *   status[1]            0, or GS_ERR_CAPACITY if the pairs needed exceed
 *                        pair_capacity (nothing is sorted then)
 *   cell_masks           optional (NULL = not kept), gs_render_mask_bytes()
 *                        bytes, 8-byte aligned: for each sorted pair, one
 *                        64-bit word per 64-lane wave of a tile's workgroup,
 *                        bit c set when the pair's Gaussian can reach cell c
 *                        of that wave (the exact alpha >= 1/255 chords of
 *                        section 3's skip rule).  gs_render_fwd writes the
 *                        words of every list entry it stages; gs_render_bwd
 *                        then reads them instead of recomputing them, so
 *                        it must get the buffer the forward of these bins
 *                        filled (or NULL).  gs_bin_sort ignores it.
 *   tile_order           optional (NULL = not kept), n_tiles + 1 uint32,
 *                        4-byte aligned: written by gs_bin_sort, [0] =
 *                        n_tiles and [1..n_tiles] every tile, those with the
 *                        longest lists first (by the floor of log2 of the
 *                        length; order within a class unspecified); both
 *                        blends then start their workgroups in that order,
 *                        so that the longest tiles do not finish last.
 *                        Results do not depend on it.
 * Tiles are numbered row-major: tile_y * ceil(W / tile_w) + tile_x. */
typedef struct {
    uint64_t *keys;
    uint32_t *vals;
    uint32_t *first;
    uint32_t *ranges;
    uint32_t *pair_count;
    int32_t *status;
    int64_t pair_capacity;
    uint64_t *cell_masks;
    uint32_t *tile_order;
} gs_bins;

/* Gradient output (caller-owned device buffers, same shapes as gs_gaussians
 * with plane stride ld; overwritten):  mean[3][ld], scale[3][ld],
 * quat[4][ld], opacity[ld], sh[3K][ld].
 * grad2d[9][n]: per-Gaussian image-space gradients (du, dv, dA, dB, dC,
 * d opacity, dr, dg, db), left holding them. */
typedef struct {
    int64_t ld;
    float *mean, *scale, *quat, *opacity, *sh;
    float *grad2d;
} gs_grads;

/* Section 3: project every Gaussian (EWA 2D covariance + dilation, conic,
 * SH colour, depth, conservative tile rectangle).  One lane per Gaussian. */
gs_status gs_project(const gs_gaussians *g, const gs_camera *cam, const gs_opts *opts,
                     gs_proj *out, gs_stream stream);

/* Workspace bytes gs_bin_sort needs for n Gaussians, a pair capacity and
 * a tile count (host query, no device work). */
gs_status gs_bin_sort_workspace(int64_t n, int64_t pair_capacity, int64_t n_tiles, size_t *bytes);

/* Section 3 (2D Gaussians binned to tiles and depth-sorted): one
 * (tile << 32 | depth bits, index) pair per covered tile, ordered by tile,
 * then depth, then Gaussian index (the order of a stable sort of the keys
 * emitted Gaussian by Gaussian, tiles row-major within each), with per-tile
 * ranges and each Gaussian's first emission position (bins.first).  Views
 * of at most 32768 tiles place every pair straight into its tile's run (per-
 * block tile histograms, a column scan, a scatter) and sort each run by
 * depth, equal depths by index; larger ones emit the pairs and radix-sort
 * them (onesweep, 8-bit digits) on the tile bits, then each run by depth.
 * `ws` is device scratch of gs_bin_sort_workspace() bytes.  No host
 * synchronisation: the pair count stays on the device.
 * pair_capacity <= 2^30 - 1. */
gs_status gs_bin_sort(const gs_proj *proj, int64_t n, const gs_camera *cam, const gs_opts *opts,
                      gs_bins *out, void *ws, size_t ws_bytes, gs_stream stream);

/* Section 3 (tiles blended front to back): one workgroup per tile.
 * image[3][H][W] (planar RGB), final_T[H][W], n_contrib[H][W] = 1-based
 * position, within the tile's list, of the last blended Gaussian (0 if
 * none).  All three are outputs (device). */
gs_status gs_render_fwd(const gs_proj *proj, const gs_bins *bins, const gs_camera *cam,
                        const gs_opts *opts, float *image, float *final_T, uint32_t *n_contrib,
                        gs_stream stream);

/* Bytes of bins->cell_masks for these bins and tiles: pair_capacity * 8 *
 * (64-lane waves per tile: 1 for 8x8, 16x8, 16x16 and 32x8 tiles, 2 for
 * 32x16, 4 for 32x32) (host query). */
gs_status gs_render_mask_bytes(const gs_bins *bins, const gs_opts *opts, size_t *bytes);

/* Bytes of the device workspace gs_render_bwd needs for these bins:
 * at most 40 bytes per pair of capacity plus 516 (host query). */
gs_status gs_render_bwd_workspace(const gs_bins *bins, size_t *bytes);

/* Section 3 (differentiable rasterizer, Gaussians optimised by gradient
 * descent): gradient of L w.r.t. every Gaussian parameter given dL/dImage
 * [3][H][W] (device) and the forward's final_T and n_contrib (device).
 * `g`, `proj` and `bins` must be the ones the forward used, and
 * bins->first must be set.  Each pixel walks its list back to front from
 * its last contributor, recovering the transmittance by division from
 * final_T; no per-contributor state is stored.  Each tile sums its pixels'
 * terms per Gaussian in a fixed order (no atomics, so the gradients are
 * bitwise repeatable) and stores the sums in `ws` (device scratch of
 * gs_render_bwd_workspace() bytes, 16-byte aligned, caller-owned, contents
 * on return unspecified) at the (Gaussian, tile) pair's emission position;
 * each Gaussian's entries are then added in emission order into
 * out->grad2d, which is overwritten.  With bins->cell_masks set, the cell
 * masks the forward kept there are read instead of recomputed.  The parameter
 * gradients are overwritten (zero for culled Gaussians, and for all
 * Gaussians when *bins->status is non-zero). */
gs_status gs_render_bwd(const gs_gaussians *g, const gs_camera *cam, const gs_opts *opts,
                        const gs_proj *proj, const gs_bins *bins, const float *final_T,
                        const uint32_t *n_contrib, const float *dL_dimage, gs_grads *out,
                        void *ws, size_t ws_bytes, gs_stream stream);

/* Stored-state variant of the blend (for comparison with the recomputing
 * backward above; same results within the gradient tolerance).
 * gs_render_state_bytes: bytes of the state buffer for these bins and
 * tiles = pair_capacity * tile_w * tile_h * 8 (host query).
 * gs_render_fwd_stored: gs_render_fwd that also writes, for every (list
 * entry, pixel) it evaluates, the entry's alpha (negated when capped at
 * 0.99, 0 when skipped) and the transmittance in front of it into `state`
 * (device, state_bytes, caller-owned).
 * gs_render_bwd_stored: gs_render_bwd reading alpha and T from `state`
 * instead of recomputing them; arguments otherwise as gs_render_bwd. */
gs_status gs_render_state_bytes(const gs_bins *bins, const gs_opts *opts, size_t *bytes);
gs_status gs_render_fwd_stored(const gs_proj *proj, const gs_bins *bins, const gs_camera *cam,
                               const gs_opts *opts, float *image, float *final_T,
                               uint32_t *n_contrib, void *state, size_t state_bytes, gs_stream stream);
gs_status gs_render_bwd_stored(const gs_gaussians *g, const gs_camera *cam, const gs_opts *opts,
                               const gs_proj *proj, const gs_bins *bins, const float *final_T,
                               const uint32_t *n_contrib, const void *state, size_t state_bytes,
                               const float *dL_dimage, gs_grads *out, void *ws, size_t ws_bytes,
                               gs_stream stream);

/* Stable LSD radix sort of (uint64 key, uint32 value) pairs on the low
 * `key_bits` bits (<= 64), the sort gs_bin_sort runs, exposed for testing
 * on arbitrary keys.  count: device pointer to the number of pairs
 * (<= capacity); keys/vals: device [capacity], sorted in place; ws: device
 * scratch of gs_sort_workspace() bytes. */
gs_status gs_sort_workspace(int64_t capacity, int32_t key_bits, size_t *bytes);
gs_status gs_sort_pairs(uint64_t *keys, uint32_t *vals, const uint32_t *count, int64_t capacity,
                        int32_t key_bits, void *ws, size_t ws_bytes, gs_stream stream);

/* ---- Training loss ---------------------------------------------------------
 * Eq. 1 (section 3): the loss of a rendered image I^r against its ground
 * truth I is (1 - lambda) L1(I^r, I) + lambda D-SSIM(I^r, I); Eq. 3
 * (section 4.2), with decoupled appearance modelling, takes the L1 term on
 * the appearance-adjusted image I^a instead and keeps D-SSIM on I^r.  D-SSIM
 * follows 3DGS (section 5.1): 1 - SSIM, SSIM averaged over every pixel and
 * channel with an 11 x 11 Gaussian window of sigma 1.5, C1 = 0.01^2,
 * C2 = 0.03^2 (dynamic range 1) and window sums that count the outside of
 * the image as zero; L1 = mean |I^a - I|, its gradient sign(I^a - I) / n
 * with sign(0) = 0; n = channels * width * height.  The prior-art weight
 * is lambda = 0.2.
 *
 * image (I^r), target (I): device [channels][height][width] FP32.
 * image_l1 (I^a): device, same shape, or NULL for Eq. 1 (then I^a = I^r).
 * loss: device float[3], overwritten with (total loss, L1, mean SSIM).
 * d_image: device, same shape, overwritten with dLoss/dI^r -- both terms
 *   for Eq. 1, the D-SSIM term only for Eq. 3.
 * d_image_l1: device, same shape, overwritten with dLoss/dI^a; required
 *   when image_l1 is set, ignored (may be NULL) otherwise.
 * ws: device scratch of gs_loss_workspace() bytes, 8-byte aligned.
 * The outputs must not overlap the inputs.  Rejected with GS_ERR_INVALID:
 * NULL buffers, channels < 1, width or height < 1, non-finite lambda, a
 * workspace that is too small or misaligned.  Deterministic: the same
 * inputs give bit-identical outputs. */
gs_status gs_loss_workspace(int32_t channels, int32_t width, int32_t height, size_t *bytes);
gs_status gs_loss(const float *image, const float *image_l1, const float *target, int32_t channels,
                  int32_t width, int32_t height, float lambda, float *loss, float *d_image,
                  float *d_image_l1, void *ws, size_t ws_bytes, gs_stream stream);

/* gs_loss without a workspace, for callers that cannot allocate device
 * memory (work recorded under stream capture, tight serving loops).  The
 * per-tile partial sums go to a fixed device array the library holds (one
 * per device, 1 MiB, kept until the process ends), so this call allocates
 * nothing and takes the same arguments as gs_loss minus the workspace.
 * Limit: channels * ceil(width / 32) * ceil(height / 32) <= 131072 (an RGB
 * image up to 7680 x 4320); a larger image is rejected with
 * GS_ERR_CAPACITY before anything is enqueued.  Calls that overlap on one
 * device share that array and race: serialise them (one stream, or events).
 * Results are bit-identical to gs_loss's.  Other errors as gs_loss. */
gs_status gs_loss_noalloc(const float *image, const float *image_l1, const float *target, int32_t channels,
                          int32_t width, int32_t height, float lambda, float *loss, float *d_image,
                          float *d_image_l1, gs_stream stream);

/* ---- Optimiser step ---------------------------------------------------------
 * Section 3: the Gaussians' properties are optimised by gradient descent on
 * the loss, interleaved with adaptive densification that is triggered by
 * each point's cumulative gradient; section 5.1 leaves the optimiser to
 * 3DGS, whose choices are these: Adam with bias correction over the raw
 * properties, one learning rate per group, every Gaussian updated every
 * step; the renderer's gradients (w.r.t. the activated scale and opacity)
 * reach the raw values through scale = exp(log_scale) and opacity =
 * 1 / (1 + exp(-logit)); for every Gaussian visible in the step's view
 * (tiles_touched > 0) the norm of its image-space centre gradient
 * |(dL/du, dL/dv)| (pixels) is added to grad_accum and visible_count is
 * incremented.  The densify/prune policy that reads them is the caller's.
 *
 * Raw properties (device, stride ld >= n, updated in place).  mean, quat and
 * sh are also the planes the rasterizer reads (gs_gaussians may point at
 * them); log_scale and logit_opacity are kept apart and their activated
 * values written to scale_out [3][ld] and opacity_out [ld], which must hold
 * exp / sigmoid of the raw values on entry (each step keeps them so). */
typedef struct {
    int64_t n, ld;
    int32_t sh_degree;
    float *mean;          /* [3][ld]  */
    float *log_scale;     /* [3][ld]  */
    float *quat;          /* [4][ld]  */
    float *logit_opacity; /* [ld]     */
    float *sh;            /* [3K][ld] */
} gs_params;

/* Optimiser state (device, stride ld of the gs_params).  m and v hold
 * 11 + 3K planes in the order mean 3, log_scale 3, quat 4, logit_opacity 1,
 * sh 3K; zero them before the first step.  grad_accum and visible_count
 * ([ld] each) may be NULL when tiles_touched is NULL. */
typedef struct {
    float *m, *v;
    float *grad_accum, *visible_count;
} gs_adam_state;

/* Hyper-parameters of one step (host struct).  step is the 1-based step
 * number t of the bias correction 1 - beta^t.  SH plane c*K + j takes
 * lr_sh_dc for j = 0 and lr_sh_rest otherwise.  3DGS uses beta1 0.9,
 * beta2 0.999, eps 1e-15, lr_scale 5e-3, lr_quat 1e-3, lr_opacity 5e-2,
 * lr_sh_dc 2.5e-3, lr_sh_rest 1.25e-4 and a position rate decayed from
 * 1.6e-4 to 1.6e-6 times the scene extent (the caller's schedule). */
typedef struct {
    float lr_mean, lr_scale, lr_quat, lr_opacity, lr_sh_dc, lr_sh_rest;
    float beta1, beta2, eps;
    int32_t step;
} gs_adam_config;

/* One Adam step of the Gaussians in p with the gradients of gs_render_bwd
 * (grads: stride grads->ld, grad2d [9][n]).  tiles_touched: device [n]
 * from the step's gs_project, or NULL to leave the statistics alone.
 * status: device flag of the step's gs_bin_sort (nothing changes when it is
 * non-zero: a step whose pairs overflowed has no valid gradient), or NULL.
 * Rejected with GS_ERR_INVALID: NULL buffers, n < 0, ld < n, grads->ld < n,
 * SH degree > 3, non-finite or out-of-range hyper-parameters (beta outside
 * [0, 1), eps < 0, step < 1).  Deterministic. */
gs_status gs_adam_step(const gs_params *p, float *scale_out, float *opacity_out, const gs_adam_state *st,
                       const gs_grads *grads, const uint32_t *tiles_touched, const int32_t *status,
                       const gs_adam_config *cfg, gs_stream stream);

/* ---- Progressive data partitioning ----------------------------------------
 * Section 4.1: the scene is split into cells by the camera positions on the
 * ground plane (world y up; ground coordinates x, z): m sections along x
 * with equal view counts, each split into n segments along z with equal
 * view counts (group sizes differ by at most one, the first groups larger;
 * boundaries midway between neighbouring camera positions; the outermost
 * ones at the bounding rectangle of all camera positions and points).  Each
 * region's rectangle is expanded by `expand` (0.2) of its side lengths about
 * its centre; views and points whose ground position lies in the (closed)
 * expanded rectangle join the cell.  Every other camera joins it when its
 * airspace-aware visibility of the cell exceeds `visibility_threshold`
 * (0.25): the fraction of its image covered by the projection of the cell's
 * box -- the axis-aligned box of the cell's points from the ground (y = 0)
 * up to the highest point -- with the part behind the near plane clipped
 * off.  Then the points covered by any view of the cell (in front of its
 * near plane, projecting inside its image; occlusion ignored) join it
 * (gs_select_points).  Section 4.3: after optimisation a cell keeps the
 * Gaussians inside its original rectangle (gs_merge_keep). */
typedef struct {
    int32_t m, n;               /* grid: m sections along x, n segments along z */
    float expand;               /* boundary expansion ratio (0.2) */
    float visibility_threshold; /* T_h (0.25) */
} gs_partition_config;

/* Host call (host buffers, FP64 geometry).  points: [n_points][3] world
 * positions (the SfM point cloud).  Outputs, cell c = i * n + j for section
 * i and segment j: bounds [m n][4] and expanded [m n][4] rectangles (x0, x1,
 * z0, z1; the original ones tile the scene, half-open above except at the
 * outermost edges); boxes [m n][6] airspace boxes (x0, y0, z0, x1, y1, z1;
 * all zero when the cell has no point); visibility [m n][n_views] (0 for
 * views selected by position); view_member [m n][n_views]: 0 = not in the
 * cell, 1 = by position, 2 = by visibility.  GS_ERR_INVALID for NULL
 * buffers, n_views < 1, a bad grid, non-finite points or cameras. */
gs_status gs_partition_views(const gs_camera *cams, int32_t n_views, const float *points, int64_t n_points,
                             const gs_partition_config *cfg, double *bounds, double *expanded, double *boxes,
                             double *visibility, uint8_t *view_member);

/* Point selection on the device.  points: device [3][ld] positions (SoA,
 * like gs_gaussians.mean); cams[n_views], expanded [n_cells][4] and
 * view_member [n_cells][n_views] are the host values of gs_partition_views.
 * point_member: device [n_cells][n_points], overwritten: 1 = in the
 * expanded rectangle, 2 = covered by a view of the cell, 0 = neither.
 * tests: device uint64 counter of the projections performed (work counter,
 * added to), or NULL.  ws: device scratch of gs_select_points_workspace()
 * bytes (n_points < 2^32); the call uploads the camera and cell tables into
 * it and synchronises `stream` once before launching.  The points are
 * visited in the Morton order of their ground position (sorted in ws), so
 * that neighbouring points, covered by the same views, share a wave. */
gs_status gs_select_points_workspace(int32_t n_views, int32_t n_cells, int64_t n_points, size_t *bytes);
gs_status gs_select_points(const float *points, int64_t n_points, int64_t ld, const gs_camera *cams,
                           int32_t n_views, const double *expanded, int32_t n_cells, const uint8_t *view_member,
                           uint8_t *point_member, uint64_t *tests, void *ws, size_t ws_bytes, gs_stream stream);

/* Section 4.3 merge mask: keep[i] = 1 when Gaussian i's (x, z) (mean, device
 * [3][ld]) lies in rect = (x0, x1, z0, z1) (host), half-open above unless
 * closed_x / closed_z (the outermost cells); keep: device [n]. */
gs_status gs_merge_keep(const float *mean, int64_t n, int64_t ld, const double *rect, int32_t closed_x,
                        int32_t closed_z, uint8_t *keep, gs_stream stream);

/* ---- Decoupled appearance modelling ----------------------------------------
 * Section 4.2 and supplement S1.1: the rendered image I^r (device [3][H][W])
 * is downsampled 32 times (ceil(H/32) x ceil(W/32) block means, border
 * blocks over the pixels they hold), an appearance embedding of length m
 * (64) is concatenated to every pixel, and a CNN maps the (3 + m)-channel
 * map to the transformation map M ([3][H][W]); the adjusted image is
 * I^a = I^r * M (pixel-wise), whose L1 loss Eq. 3 takes (gs_loss with
 * image_l1 = I^a).  The CNN: conv0 3x3 (3 + m -> 256); four blocks of pixel
 * shuffle by 2 (out[c][2y+i][2x+j] = in[4c+2i+j][y][x]), 3x3 convolution
 * halving the block input's channels (64 -> 128, 32 -> 64, 16 -> 32,
 * 8 -> 16) and ReLU; bilinear interpolation to H x W (half-pixel centres);
 * 3x3 convolution 16 -> 16, ReLU; 3x3 convolution 16 -> 3.  Every
 * convolution has a bias, zero padding 1, stride 1.
 * params: device FP32, the seven layers in that order, each its weights
 * [Cout][Cin][3][3] then its bias [Cout] (gs_appearance_param_count
 * floats).  ws: device scratch of gs_appearance_workspace() bytes, 256-byte
 * aligned; the forward keeps its activations there and the backward of the
 * same image, embedding and parameters must be given the same ws.
 * Forward: image_adj = I^a (device [3][H][W]); transform, if not NULL,
 * receives M.  Backward, for the gradient d_image_adj = dL/dI^a: d_image
 * (device [3][H][W]) is ADDED dL/dI^r through both the product and the
 * downsampling (so it can hold the D-SSIM term already); d_embedding [m]
 * and d_params (packed like params) are overwritten.  Deterministic.
 * GS_ERR_INVALID for NULL buffers, W or H < 1, m outside [0, 4096], a
 * workspace that is too small or misaligned. */
gs_status gs_appearance_param_count(int32_t embed_dim, int64_t *count);
gs_status gs_appearance_workspace(int32_t width, int32_t height, int32_t embed_dim, size_t *bytes);
gs_status gs_appearance_fwd(const float *image, int32_t width, int32_t height, const float *embedding,
                            int32_t embed_dim, const float *params, float *image_adj, float *transform, void *ws,
                            size_t ws_bytes, gs_stream stream);
gs_status gs_appearance_bwd(const float *image, int32_t width, int32_t height, const float *embedding,
                            int32_t embed_dim, const float *params, const float *d_image_adj, float *d_image,
                            float *d_embedding, float *d_params, void *ws, size_t ws_bytes, gs_stream stream);

/* ---- Batched cells (training) --------------------------------------------
 * Section 4.1: a scene is split into cells optimised independently.  A
 * gs_batch runs one training step (render, L1 image loss, backward) of
 * several cells of uneven Gaussian counts together: each stage is one
 * launch over all cells, the blends are persistent grids pulling tiles
 * longest list first, and the step is captured once as a hipGraph and
 * replayed by gs_batch_step.  With `autotune` the tile shape, the launch
 * form, the blends' LDS batch and slot capacity and the persistent grid
 * size are chosen at creation by timing each candidate on the batch.
 *
 * gs_batch_create: cells[n_cells] (device SoA planes, one SH degree for all)
 * and cams[n_cells] (host) define the cells and their training views;
 * targets[n_cells] are device [3][H][W] target images; outputs: images
 * (device, stacked: cell c's [3][H][W] image starts at the sum of 3 W H of
 * the cells before it), grads[n_cells] (device planes per cell, overwritten
 * each step) and loss (device, n_cells floats: mean |I - I*| of each cell,
 * or its Eq. 1 loss when cfg->loss_lambda > 0).  With cfg->optim the step
 * ends with the optimiser step of every cell (section 3: a complete
 * training step of every cell in one graph replay).
 * Every pointer must stay valid until gs_batch_destroy (the graph holds
 * them).  The pair capacity is sized at creation from the cells' current
 * parameters with the configured headroom; a later step that needs more
 * sets the device status to GS_ERR_CAPACITY (images NaN, gradients zero),
 * read by gs_batch_status.  Creation synchronises `stream`; it allocates
 * the batch's workspace (freed by gs_batch_destroy).
 * gs_batch_step: enqueue one step on `stream` (graph replay), no sync. */
typedef struct gs_batch gs_batch;
/* Optimiser of a batch (see gs_adam_step): params[c] are cell c's raw
 * properties, and cells[c] must read params[c].mean / quat / sh, with
 * cells[c].scale and cells[c].opacity writable (the step rewrites them
 * from the raw log-scale and logit); states[c] its moments and statistics
 * (statistics always kept).  The first gs_batch_step takes step number
 * hyper.step (>= 1), every later one the next; the position rate decays
 * log-linearly from hyper.lr_mean to lr_mean_final over lr_mean_steps
 * steps when both are > 0 (3DGS), else stays constant.  The autotune runs
 * at creation do not step the optimiser. */
typedef struct {
    const gs_params *params;
    const gs_adam_state *states;
    gs_adam_config hyper;
    float lr_mean_final;
    int32_t lr_mean_steps;
} gs_batch_optim;

typedef struct {
    int32_t tile_w, tile_h;     /* tile shape (0 = 16x16) */
    int32_t persistent;         /* 1 = persistent blend grids with a longest-first tile queue */
    int32_t use_graph;          /* 1 = capture the step as a hipGraph */
    int32_t autotune;           /* 1 = time the candidate shapes/forms at creation, keep the fastest */
    double capacity_headroom;   /* pair capacity = headroom x pairs needed at creation (<= 1: 1.25) */
    float loss_lambda;          /* Eq. 1 D-SSIM weight (gs_loss); 0 = the L1 loss alone */
    const gs_batch_optim *optim; /* NULL = no optimiser step in the batch step */
    /* Persistent blend grids only (ignored with autotune, which times its
     * own choices): */
    int32_t fwd_batch;          /* forward's staged list entries per LDS batch: 0 = 256, or 128 */
    int32_t item_cap;           /* backward's (cell, entry) slots per chunk: 0 = 512, or 256 */
    int32_t grid_pct;           /* grid = this % of the workgroups that fit at once: 0 = 100, 1..100 */
} gs_batch_config;              /* NULL = {16, 16, 1, 1, 0, 1.25, 0, NULL, 0, 0, 0} */
typedef struct {
    int32_t tile_w, tile_h, persistent, use_graph, grid_fwd, grid_bwd;
    uint32_t n_tiles;
    int64_t slots, pair_capacity;
    int32_t n_candidates;       /* autotune: candidates timed, in order */
    int32_t cand_tile_w[16], cand_tile_h[16], cand_persistent[16];
    double cand_ms[16];         /* mean step time of each candidate */
    int32_t fwd_batch, item_cap, grid_pct;   /* the chosen LDS batch, slot capacity and grid share */
    int32_t cand_fwd_batch[16], cand_item_cap[16], cand_grid_pct[16];
} gs_batch_stats;

gs_status gs_batch_create(const gs_gaussians *cells, const gs_camera *cams, const float *const *targets,
                          int32_t n_cells, float *images, gs_grads *grads, float *loss,
                          const gs_batch_config *cfg, gs_stream stream, gs_batch **out);
gs_status gs_batch_step(gs_batch *b, gs_stream stream);
/* Chosen configuration and autotune timings (host). */
gs_status gs_batch_info(const gs_batch *b, gs_batch_stats *info);
/* Device status of the last step and its pairs [P, needed]; synchronises `stream`. */
gs_status gs_batch_status(gs_batch *b, gs_stream stream, int32_t *status, uint32_t *pairs);
void gs_batch_destroy(gs_batch *b);

/* ---- Serving the merged scene ---------------------------------------------
 * Sections 4.3 and 5: the merged scene is rendered in real time from novel
 * views.  A gs_server keeps the scene resident (the caller's device planes,
 * not copied: they must outlive the server) and renders requests with
 * continuous batching: a worker thread forms a batch from the head of the
 * request queue whenever one of its pipelines (stream + workspace) is free,
 * admitting requests in arrival order while the batch's Gaussian slots,
 * pixels, tiles and estimated (Gaussian, tile) pairs fit the pipeline's share
 * of the memory budget; each batch is one projection, one joint sort and one
 * blend over all its views (mixed resolutions), and batches on different
 * pipelines overlap on the device.  Cells are culled per request on the host
 * against the view frustum.  A request's image does not depend on what it
 * was batched with.
 *
 * gs_serve_create: scene (device SoA planes), cell_aabbs (host, n_cells x 6
 * floats xmin, ymin, zmin, xmax, ymax, zmax, each bounding the alpha >= 1/255
 * support of every Gaussian of the cell, e.g. means +- 3.5 x the largest
 * scale), cell_offsets (host, n_cells + 1 ascending Gaussian indices, cell c
 * owning [cell_offsets[c], cell_offsets[c+1]), first 0 and last n).  Starts
 * the worker and completion threads and allocates the pipelines' workspace
 * (the budget split between them).  cfg NULL = defaults below.
 * gs_serve_submit: queue a render of `cam` into out_image (device [3][H][W],
 * caller-owned, untouched until the request completes); returns at once
 * with a ticket.  GS_ERR_BUSY when the queue is full, GS_ERR_INVALID when
 * the request alone can never fit a pipeline.  Thread-safe.
 * gs_serve_wait: block until the ticket's request completes (timeout_ms < 0
 * waits forever; GS_ERR_TIMEOUT otherwise) and fill its statistics (host
 * monotonic clock, ns).  Each ticket is waited for once.  The request's
 * status is returned (GS_ERR_CAPACITY if even alone its pairs overflowed).
 * gs_serve_destroy: finish queued and running requests, stop the threads,
 * free the workspace. */
typedef struct gs_server gs_server;
typedef struct {
    int64_t memory_budget;      /* device bytes for all pipelines' workspace (8 GiB) */
    int32_t pipelines;          /* batches in flight at once (2) */
    int32_t max_views;          /* requests per batch (8) */
    int32_t max_queue;          /* queued requests before GS_ERR_BUSY (1024) */
    int32_t tile_w, tile_h;     /* (16, 16) */
    int64_t max_pixels;         /* pixels of one batch, cap (4 x 3840 x 2160) */
    float widen_px;             /* frustum margin of the cell culling, pixels (64) */
    double initial_pairs_per_slot; /* admission estimate of pairs per Gaussian before any batch (3.0) */
    int32_t start_paused;       /* 1 = form no batch until gs_serve_resume (0) */
    int64_t max_pairs;          /* pair capacity per pipeline (0 = from the budget) */
} gs_serve_config;
typedef struct {
    int64_t t_arrive_ns, t_start_ns, t_done_ns;   /* submit, batch launch, completion */
    int32_t status, batch_views, attempts, cells;
    int64_t gaussians;          /* Gaussians of the cells that survived culling */
} gs_request_stats;
typedef struct {
    int64_t batches, requeues, max_batch_views, queued;
    int32_t pipelines;
    int64_t slots_cap, pairs_cap, pixels_cap;
    double pairs_per_slot;      /* current admission estimate */
} gs_serve_stats;

gs_status gs_serve_create(const gs_gaussians *scene, const float *cell_aabbs, const int64_t *cell_offsets,
                          int32_t n_cells, const gs_serve_config *cfg, gs_server **out);
gs_status gs_serve_submit(gs_server *sv, const gs_camera *cam, float *out_image, uint64_t *ticket);
gs_status gs_serve_wait(gs_server *sv, uint64_t ticket, int32_t timeout_ms, gs_request_stats *st);
gs_status gs_serve_info(gs_server *sv, gs_serve_stats *info);
/* Let a server created with start_paused form batches. */
gs_status gs_serve_resume(gs_server *sv);
void gs_serve_destroy(gs_server *sv);

/* Work counters of the blends of one view (observability; not on the
 * training path): runs the forward walk without writing an image, and the
 * same walk over the backward's cells, and stores into counters (device,
 * 4 x uint64, overwritten):
 *   [0] (pixel, list entry) evaluations the forward performs (the pixels
 *       of every cell that a list entry's support reaches),
 *   [1] evaluations with alpha >= 1/255 up to the pixel's stop,
 *   [2] blended (pixel, Gaussian) pairs,
 *   [3] evaluations over the backward's cells (2x2 pixels where the
 *       forward walks 2x1 cells: 16x16 tiles).
 * These are the units in which the blends' arithmetic work is counted. */
gs_status gs_render_stats(const gs_proj *proj, const gs_bins *bins, const gs_camera *cam,
                          const gs_opts *opts, uint64_t *counters, gs_stream stream);

/* Stage timing (observability).  gs_profile_enable(1) starts a window in
 * which every stage the library enqueues (project, scan_emit, sort,
 * tile_ranges, render_fwd, tile_order, render_bwd, pair_gather,
 * project_bwd, loss, loss_finish, adam, ...) is bracketed by HIP events on its stream;
 * gs_profile_enable(0) ends it and discards what was recorded.
 * gs_profile_select(stages) restricts the bracketing to the stages named
 * in a comma-separated list (NULL or "" = all); each event pair adds a
 * few microseconds between kernels, so a timing of the whole step brackets
 * only the stage it needs.  gs_profile_report() waits for the recorded
 * events and writes a JSON object {"stage": [total_ms, launches], ...} of
 * the window so far into buf (host, len bytes), then starts counting
 * afresh.  Process-wide; calls from several threads are serialised. */
gs_status gs_profile_enable(int on);
gs_status gs_profile_select(const char *stages);
gs_status gs_profile_report(char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* GS_H */
