// Front-to-back alpha blend of each screen tile (forward).
//
// VastGaussian (arXiv 2402.17427), section 3: the sorted 2D Gaussians of
// each tile are alpha-blended into the image in a point-based volume
// rendering manner.  Per pixel, walking the tile's list in depth order:
//   alpha = min(0.99, o exp(power)); skipped when power > 0 or
//   alpha < 1/255; the pixel stops before the Gaussian that would take T
//   below 1e-4; otherwise C += colour alpha T and T *= (1 - alpha).
// Output pixel = C + T bg.
//
// Launch: one workgroup per tile (or a persistent grid pulling tiles from
// a queue), one lane per cell of CW x CH pixels (blend_cells.h).  Batches
// of 256 list entries are staged in LDS.  For each 64 of them every lane
// computes one entry's cell mask from the exact chords of its support, a
// bit transpose gives each lane the entries that reach its cell, and each
// lane then walks its own entries of the whole batch in list order, with
// its pixels' state in registers.  Skipping the other entries never
// changes a result: they have alpha < 1/255 at every pixel of the cell.
// When the caller keeps them, every computed mask is also stored per
// sorted pair and wave, so that the backward walks the same entries
// without recomputing the chords.
// Tiles of several views are numbered consecutively; a tile finds its view
// (camera, image planes) in the view table.
#include <cstring>

#include "blend_cells.h"
#include "kernels.h"

namespace gs {

namespace {

// MODE kPlain is the forward.  kStats is the instrumented variant behind
// gs_render_stats: the same walk, counting per pixel the list entries it
// evaluates, the entries with alpha >= 1/255 before its stop, and the
// blended ones, summed into stats[0..2]; it writes no image.  kStore is the
// forward that also keeps the blend state: for every entry a pixel
// evaluates, state[(list position) * NT + pixel in tile] = (alpha, T before
// it), alpha negated when capped at 0.99 and 0 when skipped; the
// stored-state backward reads it instead of recomputing.
constexpr int kPlain = 0, kStats = 1, kStore = 2;
#ifndef GS_FWD_BATCH
#define GS_FWD_BATCH 256
#endif
constexpr int kBatch = GS_FWD_BATCH;   // staged entries per batch (one walk word per 64)
// LDS batch sizes of the persistent launch (a tuning knob of the batched
// step): kBatch, or the half of it
constexpr int kBatchSmall = kBatch / 2;
static_assert(kBatch % kWave == 0 && kBatch / kWave <= 4 && kBatchSmall % kWave == 0, "walk words");

struct FwdArgs {
    const Rec* rec;
    const uint32_t* vals;
    const uint2* ranges;
    const int32_t* status;
    ViewTab views;
    float* image;
    float* final_T;
    uint32_t* n_contrib;
    unsigned long long* stats;
    bool stats_eval_only;   // counting pass: add only the evaluations, into stats[3]
    float2* state;
    uint64_t* masks;        // per sorted pair and wave: the cell mask (NULL = not kept)
    uint32_t* queue;        // persistent launch: next queue position (zeroed before launch)
    const uint32_t* order;  // persistent launch: tiles in processing order (NULL = 0, 1, ...)
    uint32_t n_tiles;
    const uint32_t* torder;     // one workgroup per tile: workgroup b takes tile torder[b] (NULL: tile b)
    const uint32_t* torder_n;   // ... and exits when b >= *torder_n (the order holds every tile)
};

// Store a computed cell mask m of forward wave wv for list entry `pair`
// in the layout of the backward (CellsFor, Lb::WAVES words per pair).
// With 2x1 cells in the forward and 2x2 in the backward, a forward wave
// holds 64 / CPR pixel rows as cell rows of CPR bits and a backward wave
// twice as many pixel rows: backward cell row k of forward wave wv's share
// covers its cell rows 2k and 2k + 1, so the wave ORs the row pairs and
// writes them as half (wv mod 2) of the backward word of wave wv / 2.
template <class Lf, class Lb>
__device__ __forceinline__ void keep_mask(uint64_t* masks, uint32_t pair, int wv, uint64_t m) {
    if constexpr (Lf::CW == Lb::CW && Lf::CH == Lb::CH) {
        masks[(int64_t)pair * Lb::WAVES + wv] = m;
    } else {
        static_assert(Lf::TW == Lb::TW && Lf::TH == Lb::TH && Lf::CW == 2 && Lf::CH == 1 && Lb::CW == 2 &&
                          Lb::CH == 2 && Lf::WAVES == 2 * Lb::WAVES && (Lf::CPR == 8 || Lf::CPR == 16),
                      "mask layouts");
        constexpr int C = Lf::CPR;
        const uint64_t x = m | (m >> C);   // cell row 2k: rows 2k and 2k + 1
        uint32_t half;
        if constexpr (C == 8)
            half = (uint32_t)(x & 0xFFu) | (uint32_t)((x >> 8) & 0xFF00u) | (uint32_t)((x >> 16) & 0xFF0000u) |
                   (uint32_t)((x >> 24) & 0xFF000000u);
        else
            half = (uint32_t)(x & 0xFFFFu) | (uint32_t)((x >> 16) & 0xFFFF0000u);
        reinterpret_cast<uint32_t*>(masks)[2 * ((int64_t)pair * Lb::WAVES + wv / 2) + (wv & 1)] = half;
    }
}

template <int B>
struct FwdShared {
    StagedSoA<B> s;
};

// B: staged entries per batch (a multiple of 64, at most 256)
template <class L, int MODE, int B>
__device__ __forceinline__ void fwd_tile(const FwdArgs& a, uint32_t tile, FwdShared<B>& sh) {
    using LB = typename CellsFor<L::TW, L::TH>::L;   // the backward's layout (kept masks)
    constexpr int NP = L::NP;
    constexpr bool STATS = MODE == kStats;

    const View V = view_at(a.views, find_view(a.views, tile));
    const int W = V.cam.W, H = V.cam.H;
    const int local = (int)(tile - V.tile_base);
    const int tx = local % V.ntx, ty = local / V.ntx;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int cx = tid % L::CPR, cy = tid / L::CPR;
    const int x0 = tx * L::TW, y0 = ty * L::TH;
    const int wy0 = y0 + wv * L::PXROWS_W;           // the wave's first pixel row
    const int64_t npix = (int64_t)W * H;
    float* image = V.out_image ? V.out_image : a.image + V.img_base;
    float* final_T = a.final_T + V.pix_base;
    uint32_t* n_contrib = a.n_contrib + V.pix_base;

    // the lane's pixels: (px0 + i % CW, py0 + i / CW)
    const int px0 = x0 + cx * L::CW, py0 = y0 + cy * L::CH;
    bool inside[NP];
    float fxp[L::CW], fyp[L::CH];
#pragma unroll
    for (int i = 0; i < L::CW; ++i) fxp[i] = (float)(px0 + i) + 0.5f;
#pragma unroll
    for (int j = 0; j < L::CH; ++j) fyp[j] = (float)(py0 + j) + 0.5f;
#pragma unroll
    for (int p = 0; p < NP; ++p) inside[p] = (px0 + p % L::CW) < W && (py0 + p / L::CW) < H;

    if (*a.status != 0) {
        if (!STATS) {
            const float nan = __builtin_nanf("");
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if (!inside[p]) continue;
                const int64_t off = (int64_t)(py0 + p / L::CW) * W + px0 + p % L::CW;
                image[off] = nan;
                image[npix + off] = nan;
                image[2 * npix + off] = nan;
                final_T[off] = nan;
                n_contrib[off] = 0u;
            }
        }
        return;
    }

    const uint2 rg = a.ranges[tile];
    // T > 0: the pixel is blending; a pixel that has stopped (or lies
    // outside the image) keeps its transmittance negated
    float T[NP], c0[NP], c1[NP], c2[NP];
    uint32_t last[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        T[p] = inside[p] ? 1.0f : -1.0f;
        c0[p] = c1[p] = c2[p] = 0.0f;
        last[p] = 0u;
    }
    unsigned long long n_eval = 0, n_supp = 0, n_blend = 0;

    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += B) {
        bool all_done = true;
#pragma unroll
        for (int p = 0; p < NP; ++p) all_done = all_done && !(T[p] > 0.0f);
        if (__syncthreads_count(all_done) == L::NCELL) break;
        const int nb = (int)min((uint32_t)B, rg.y - b0);
        stage_batch<(B + L::NCELL - 1) / L::NCELL>(sh.s, a.rec, a.vals, b0, nb, tid, L::NCELL);
        __syncthreads();

        // the lane's walk words: entries 64 q .. 64 q + 63 of the batch that
        // reach its cell, kept in order with the empty words dropped
        uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
        int q0 = 0, q1 = 0, q2 = 0, q3 = 0, nw = 0;
#pragma unroll
        for (int q = 0; q < B / kWave; ++q) {
            if (q * kWave >= nb) break;
            const int k = q * kWave + lane;
            const uint64_t m = k < nb ? cell_mask<L>(sh.s.get(k), x0, wy0) : 0ull;
            // kept for the backward, which walks the same entries
            if (MODE != kStats && a.masks && k < nb) keep_mask<L, LB>(a.masks, b0 + (uint32_t)k, wv, m);
            uint64_t t = transpose64(m, lane);
            if (all_done) t = 0ull;
            if (t != 0ull) {
                if (nw == 0) { w0 = t; q0 = q * kWave; }
                else if (nw == 1) { w1 = t; q1 = q * kWave; }
                else if (nw == 2) { w2 = t; q2 = q * kWave; }
                else { w3 = t; q3 = q * kWave; }
                ++nw;
            }
        }

        const uint32_t pos0 = b0 - rg.x;   // list position of the batch's first entry
        // Branch-free walk: a lane with nothing left evaluates entry 0 and,
        // like a stopped pixel or an entry below the alpha threshold,
        // changes nothing.  A lane whose pixels have all stopped walks on
        // to the end of its words: testing for that at every step (and
        // dropping the lane's words) cost more than the steps it saved
        // (forward 110 -> 105 us without it).  Lanes stopped before the
        // batch have no words, and the batch loop ends once every pixel
        // of the tile has stopped.
        if (__ballot(w0 != 0ull) != 0ull) do {
            const bool has = w0 != 0ull;
            const int kk = has ? q0 + low_bit(w0) : 0;
            w0 &= w0 - 1ull;
            const Staged g = sh.s.get(kk);
            // offsets of the lane's pixel columns and rows, then each pixel's
            // base-2 exponent (a function of the pixel and the Gaussian only)
            // ca dx^2 + cb dx dy + cc dy^2 = dx (ca dx + cb dy) + cc dy^2,
            // with the dy terms formed once per pixel row
            float dxs[L::CW], rb[L::CH], rc[L::CH];
#pragma unroll
            for (int i = 0; i < L::CW; ++i) dxs[i] = (fxp[i] - g.geo.x) - g.geo.y;
#pragma unroll
            for (int j = 0; j < L::CH; ++j) {
                const float dy = (fyp[j] - g.geo.z) - g.geo.w;
                rb[j] = g.coef.y * dy;
                rc[j] = (g.coef.z * dy) * dy;
            }
            const uint32_t lastv = pos0 + (uint32_t)kk + 1u;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int i = p % L::CW, j = p / L::CW;
                const float pw = __builtin_fmaf(dxs[i], __builtin_fmaf(g.coef.x, dxs[i], rb[j]), rc[j]);
                const float G = __builtin_amdgcn_exp2f(pw);
                const float araw = g.coef.w * G;
                const float al0 = fminf(araw, kAlphaMax);
                // alpha counts when the exponent is not positive and alpha >= 1/255
                const bool above = !(pw > 0.0f) && !(al0 < kAlphaMin);
                const bool act = has && T[p] > 0.0f;
                if (MODE == kStore && act) {
                    const int pix = (py0 + j - y0) * L::TW + (px0 + i - x0);
                    const float alpha = above ? al0 : 0.0f;
                    a.state[(int64_t)(b0 + (uint32_t)kk) * L::NT + pix] =
                        make_float2(araw > kAlphaMax && above ? -alpha : alpha, T[p]);
                }
                const bool supp = act && above;
                // the weight alpha T and the next transmittance T (1 - alpha)
                // = T - alpha T from it (used only where supp)
                const float wa = al0 * T[p];
                const float Tn = T[p] - wa;
                const bool stop = supp && Tn < kTMin;
                const bool blend = supp != stop;   // stop implies supp (one compare, not two)
                if (STATS) {
                    n_eval += act ? 1u : 0u;
                    n_supp += supp ? 1u : 0u;
                    n_blend += blend ? 1u : 0u;
                }
                const float w = blend ? wa : 0.0f;
                c0[p] = __builtin_fmaf(g.col.x, w, c0[p]);
                c1[p] = __builtin_fmaf(g.col.y, w, c1[p]);
                c2[p] = __builtin_fmaf(g.col.z, w, c2[p]);
                T[p] = blend ? Tn : (stop ? -T[p] : T[p]);
                last[p] = blend ? lastv : last[p];
            }
            // a lane at the end of a word moves to its next one
            const bool adv = w0 == 0ull && nw > 1;
            w0 = adv ? w1 : w0;
            q0 = adv ? q1 : q0;
            w1 = adv ? w2 : w1;
            q1 = adv ? q2 : q1;
            w2 = adv ? w3 : w2;
            q2 = adv ? q3 : q2;
            nw = nw - (adv ? 1 : 0);
        } while (__ballot(w0 != 0ull) != 0ull);
    }
    if (STATS) {
        // one atomic per counter and wave (same-address atomics from every
        // lane serialise)
        uint32_t e32 = (uint32_t)n_eval, s32 = (uint32_t)n_supp, b32 = (uint32_t)n_blend;
        for (int d = 1; d < kWave; d <<= 1) {
            e32 += (uint32_t)__shfl_xor((int)e32, d, kWave);
            s32 += (uint32_t)__shfl_xor((int)s32, d, kWave);
            b32 += (uint32_t)__shfl_xor((int)b32, d, kWave);
        }
        if (lane == 0) {
            if (a.stats_eval_only) {   // the evaluations of another cell layout
                atomicAdd(&a.stats[3], (unsigned long long)e32);
            } else {
                atomicAdd(&a.stats[0], (unsigned long long)e32);
                atomicAdd(&a.stats[1], (unsigned long long)s32);
                atomicAdd(&a.stats[2], (unsigned long long)b32);
            }
        }
    } else {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (!inside[p]) continue;
            const int64_t off = (int64_t)(py0 + p / L::CW) * W + px0 + p % L::CW;
            const float Tf = fabsf(T[p]);
            image[off] = __builtin_fmaf(Tf, V.cam.bg[0], c0[p]);
            image[npix + off] = __builtin_fmaf(Tf, V.cam.bg[1], c1[p]);
            image[2 * npix + off] = __builtin_fmaf(Tf, V.cam.bg[2], c2[p]);
            final_T[off] = fabsf(T[p]);
            n_contrib[off] = last[p];
        }
    }
}

template <class L, int MODE>
__global__ __launch_bounds__(L::NCELL) void k_render_fwd(FwdArgs a) {
    __shared__ FwdShared<kBatch> sh;
    uint32_t tile = blockIdx.x;
    if (a.torder) {
        if (blockIdx.x >= *a.torder_n) return;
        tile = a.torder[blockIdx.x];
    }
    fwd_tile<L, MODE, kBatch>(a, tile, sh);
}

template <class L, int B>
__global__ __launch_bounds__(L::NCELL) void k_render_fwd_persistent(FwdArgs a) {
    __shared__ FwdShared<B> sh;
    __shared__ uint32_t s_next;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_next = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t q = s_next;
        if (q >= a.n_tiles) break;
        fwd_tile<L, kPlain, B>(a, a.order ? a.order[q] : q, sh);
    }
}

template <int TW, int TH>
void launch_t(const FwdArgs& a, int persistent_grid, int batch, hipStream_t st) {
    using L = typename FwdCellsFor<TW, TH>::L;
    const dim3 block(L::NCELL);
    if (a.stats)
        hipLaunchKernelGGL((k_render_fwd<L, kStats>), dim3(a.n_tiles), block, 0, st, a);
    else if (a.state)
        hipLaunchKernelGGL((k_render_fwd<L, kStore>), dim3(a.n_tiles), block, 0, st, a);
    else if (persistent_grid > 0 && batch == kBatchSmall)
        hipLaunchKernelGGL((k_render_fwd_persistent<L, kBatchSmall>), dim3(persistent_grid), block, 0, st, a);
    else if (persistent_grid > 0)
        hipLaunchKernelGGL((k_render_fwd_persistent<L, kBatch>), dim3(persistent_grid), block, 0, st, a);
    else
        hipLaunchKernelGGL((k_render_fwd<L, kPlain>), dim3(a.n_tiles), block, 0, st, a);
}

// The counting pass in the backward's cell layout (its evaluations).
template <int TW, int TH>
void launch_stats_bwd_cells_t(const FwdArgs& a, hipStream_t st) {
    using L = typename CellsFor<TW, TH>::L;
    hipLaunchKernelGGL((k_render_fwd<L, kStats>), dim3(a.n_tiles), dim3(L::NCELL), 0, st, a);
}

template <int TW, int TH>
hipError_t occupancy_t(int* per, int batch) {
    using L = typename FwdCellsFor<TW, TH>::L;
    if (batch == kBatchSmall)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_render_fwd_persistent<L, kBatchSmall>, L::NCELL, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_render_fwd_persistent<L, kBatch>, L::NCELL, 0);
}

}  // namespace

bool render_tile_supported(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 32 && th == 8) ||
           (tw == 32 && th == 16) || (tw == 32 && th == 32);
}

int render_mask_words(int tw, int th) {
    if (tw == 16 && th == 16) return CellsFor<16, 16>::L::WAVES;
    if (tw == 8 && th == 8) return CellsFor<8, 8>::L::WAVES;
    if (tw == 16 && th == 8) return CellsFor<16, 8>::L::WAVES;
    if (tw == 32 && th == 8) return CellsFor<32, 8>::L::WAVES;
    if (tw == 32 && th == 16) return CellsFor<32, 16>::L::WAVES;
    if (tw == 32 && th == 32) return CellsFor<32, 32>::L::WAVES;
    return 0;
}

void launch_render_fwd(const RenderArgs& r, float* image, float* final_T, uint32_t* n_contrib,
                       unsigned long long* stats, float2* state, hipStream_t st) {
    if (r.n_tiles == 0) return;
    FwdArgs a;
    a.rec = r.rec;
    a.vals = r.vals;
    a.ranges = reinterpret_cast<const uint2*>(r.ranges);
    a.status = r.status;
    a.views = r.views;
    a.image = image;
    a.final_T = final_T;
    a.n_contrib = n_contrib;
    a.stats = stats;
    a.stats_eval_only = false;
    a.state = state;
    a.masks = stats ? nullptr : r.masks;
    a.queue = r.queue;
    a.order = r.order;
    a.n_tiles = r.n_tiles;
    a.torder = r.tile_order;
    a.torder_n = r.tile_order_count;
    const int pg = (r.queue && !stats && !state) ? r.persistent_grid : 0;
    if (pg > 0) launch_fill_u32(r.queue, 0u, 1, st);
#define GS_FWD(x, y) launch_t<x, y>(a, pg, r.fwd_batch, st)
    if (r.tw == 16 && r.th == 16) GS_FWD(16, 16);
    else if (r.tw == 8 && r.th == 8) GS_FWD(8, 8);
    else if (r.tw == 16 && r.th == 8) GS_FWD(16, 8);
    else if (r.tw == 32 && r.th == 8) GS_FWD(32, 8);
    else if (r.tw == 32 && r.th == 16) GS_FWD(32, 16);
    else if (r.tw == 32 && r.th == 32) GS_FWD(32, 32);
#undef GS_FWD
}

void launch_render_stats_bwd_cells(const RenderArgs& r, unsigned long long* stats, hipStream_t st) {
    if (r.n_tiles == 0) return;
    FwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.rec = r.rec;
    a.vals = r.vals;
    a.ranges = reinterpret_cast<const uint2*>(r.ranges);
    a.status = r.status;
    a.views = r.views;
    a.stats = stats;
    a.stats_eval_only = true;
    a.n_tiles = r.n_tiles;
    a.torder = r.tile_order;
    a.torder_n = r.tile_order_count;
#define GS_STB(x, y) launch_stats_bwd_cells_t<x, y>(a, st)
    if (r.tw == 16 && r.th == 16) GS_STB(16, 16);
    else if (r.tw == 8 && r.th == 8) GS_STB(8, 8);
    else if (r.tw == 16 && r.th == 8) GS_STB(16, 8);
    else if (r.tw == 32 && r.th == 8) GS_STB(32, 8);
    else if (r.tw == 32 && r.th == 16) GS_STB(32, 16);
    else if (r.tw == 32 && r.th == 32) GS_STB(32, 32);
#undef GS_STB
}

int render_persistent_grid_bwd(int tw, int th, int item_cap);
int render_persistent_grid_fwd(int tw, int th, int batch);

int render_persistent_grid(int tw, int th, bool backward, int lds_knob) {
    return backward ? render_persistent_grid_bwd(tw, th, lds_knob) : render_persistent_grid_fwd(tw, th, lds_knob);
}

int render_fwd_batch_default() { return kBatch; }
int render_fwd_batch_small() { return kBatchSmall; }

int render_persistent_grid_fwd(int tw, int th, int batch) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
    if (tw == 16 && th == 16) e = occupancy_t<16, 16>(&per, batch);
    else if (tw == 8 && th == 8) e = occupancy_t<8, 8>(&per, batch);
    else if (tw == 16 && th == 8) e = occupancy_t<16, 8>(&per, batch);
    else if (tw == 32 && th == 8) e = occupancy_t<32, 8>(&per, batch);
    else if (tw == 32 && th == 16) e = occupancy_t<32, 16>(&per, batch);
    else if (tw == 32 && th == 32) e = occupancy_t<32, 32>(&per, batch);
    if (e != hipSuccess || per < 1) per = 1;
    return cus * per;
}

}  // namespace gs
