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
// Launch: one workgroup per tile, one lane per pixel.  Every wave covers an
// 8x8 block of the tile, so that a small Gaussian touches few waves.
// Batches of records are staged in LDS; for each 64 of them the wave tests
// one per lane against its block's pixel centres and walks, in list order,
// only those whose support box meets the block (a ballot mask scanned with
// scalar bit operations).  Skipping the others never changes a result: such
// a Gaussian has alpha < 1/255 at every pixel of the block.  A wave leaves
// the tile once all its pixels have stopped, the workgroup once all waves
// have.
#include "kernels.h"

namespace gs {

namespace {

// MODE kPlain is the forward.  kStats is the instrumented variant behind
// gs_render_stats: the same walk, counting per pixel the list entries it
// evaluates (after the wave culling), the entries with alpha >= 1/255
// before its stop, and the blended ones, summed into stats[0..2]; it
// writes no image.  kStore is the forward that also keeps the blend state:
// for every entry a pixel evaluates, state[(list position) * NT + lane in
// tile] = (alpha, T before it), alpha negated when capped at 0.99 and 0 when
// skipped; the stored-state backward reads it instead of recomputing.
constexpr int kPlain = 0, kStats = 1, kStore = 2;

template <int TW, int TH, int MODE>
__global__ __launch_bounds__(TW * TH) void k_render_fwd(const Rec* __restrict__ rec, const uint32_t* __restrict__ vals,
                                                        const uint2* __restrict__ ranges,
                                                        const int32_t* __restrict__ status, int W, int H, int ntx,
                                                        float bg0, float bg1, float bg2, float* __restrict__ image,
                                                        float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                                                        unsigned long long* __restrict__ stats,
                                                        float2* __restrict__ state) {
    constexpr int NT = TW * TH;
    constexpr bool STATS = MODE == kStats;
    constexpr int WX = TW / 8;
    __shared__ Staged s[NT];

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int tile = blockIdx.x;
    const int tx = tile % ntx, ty = tile / ntx;
    const int bx = (wv % WX) * 8, by = (wv / WX) * 8;
    const int lx = bx + (lane & 7), ly = by + (lane >> 3);
    const int px = tx * TW + lx, py = ty * TH + ly;
    const bool inside = px < W && py < H;
    const int64_t npix = (int64_t)W * H;
    const int64_t off = (int64_t)py * W + px;

    if (*status != 0) {
        if (!STATS && inside) {
            const float nan = __builtin_nanf("");
            image[off] = nan;
            image[npix + off] = nan;
            image[2 * npix + off] = nan;
            final_T[off] = nan;
            n_contrib[off] = 0u;
        }
        return;
    }

    const uint2 rg = ranges[tile];
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const float bx0 = (float)(tx * TW + bx) + 0.5f, bx1 = bx0 + 7.0f;
    const float by0 = (float)(ty * TH + by) + 0.5f, by1 = by0 + 7.0f;

    float T = 1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    uint32_t last = 0;
    bool done = !inside;
    unsigned long long n_eval = 0, n_supp = 0, n_blend = 0;

    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += NT) {
        if (__syncthreads_count(done) == NT) break;
        const uint32_t j = b0 + tid;
        if (j < rg.y) s[tid] = stage_rec(rec[vals[j]]);
        __syncthreads();
        const int nb = (int)min((uint32_t)NT, rg.y - b0);
        bool live = __ballot(!done) != 0ull;
        // 64 staged Gaussians at a time: each lane tests one against the
        // wave's block, the ballot lists the ones to walk, in order.
        for (int c0k = 0; live && c0k < nb; c0k += kWave) {
            const int k = c0k + lane;
            const bool ov = k < nb && box_overlaps(s[k], bx0, bx1, by0, by1);
            uint64_t mask = __ballot(ov);
            while (mask) {
                const int kk = c0k + __builtin_ctzll(mask);
                mask &= mask - 1;
                const Staged g = s[kk];
                if (!done) {
                    const Eval e = eval_pair(g, fx, fy);
                    if (MODE == kStore)
                        state[(int64_t)(b0 + (uint32_t)kk) * NT + tid] =
                            make_float2(e.capped && e.alpha > 0.0f ? -e.alpha : e.alpha, T);
                    if (STATS) ++n_eval;
                    if (e.alpha > 0.0f) {
                        const float Tn = T * (1.0f - e.alpha);
                        if (STATS) ++n_supp;
                        if (Tn < kTMin) {
                            done = true;
                        } else {
                            if (STATS) ++n_blend;
                            const float w = e.alpha * T;
                            c0 = __builtin_fmaf(g.col.x, w, c0);
                            c1 = __builtin_fmaf(g.col.y, w, c1);
                            c2 = __builtin_fmaf(g.col.z, w, c2);
                            T = Tn;
                            last = b0 - rg.x + (uint32_t)kk + 1u;
                        }
                    }
                }
                if (__ballot(!done) == 0ull) {
                    live = false;
                    break;
                }
            }
        }
    }
    if (STATS) {
        atomicAdd(&stats[0], n_eval);
        atomicAdd(&stats[1], n_supp);
        atomicAdd(&stats[2], n_blend);
    } else if (inside) {
        image[off] = __builtin_fmaf(T, bg0, c0);
        image[npix + off] = __builtin_fmaf(T, bg1, c1);
        image[2 * npix + off] = __builtin_fmaf(T, bg2, c2);
        final_T[off] = T;
        n_contrib[off] = last;
    }
}

template <int TW, int TH>
void launch_t(const Rec* rec, const uint32_t* vals, const uint32_t* ranges, const int32_t* status, const Cam& cam,
              float* image, float* final_T, uint32_t* n_contrib, unsigned long long* stats, float2* state,
              hipStream_t st) {
    const int ntx = (cam.W + TW - 1) / TW, nty = (cam.H + TH - 1) / TH;
    const dim3 grid((unsigned)(ntx * nty)), block(TW * TH);
    const uint2* rg = reinterpret_cast<const uint2*>(ranges);
    if (stats)
        hipLaunchKernelGGL((k_render_fwd<TW, TH, kStats>), grid, block, 0, st, rec, vals, rg, status, cam.W, cam.H,
                           ntx, cam.bg[0], cam.bg[1], cam.bg[2], image, final_T, n_contrib, stats, state);
    else if (state)
        hipLaunchKernelGGL((k_render_fwd<TW, TH, kStore>), grid, block, 0, st, rec, vals, rg, status, cam.W, cam.H,
                           ntx, cam.bg[0], cam.bg[1], cam.bg[2], image, final_T, n_contrib, stats, state);
    else
        hipLaunchKernelGGL((k_render_fwd<TW, TH, kPlain>), grid, block, 0, st, rec, vals, rg, status, cam.W, cam.H,
                           ntx, cam.bg[0], cam.bg[1], cam.bg[2], image, final_T, n_contrib, stats, state);
}

}  // namespace

bool render_tile_supported(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 32 && th == 8) ||
           (tw == 32 && th == 16) || (tw == 32 && th == 32);
}

void launch_render_fwd(const Rec* rec, const uint32_t* vals, const uint32_t* ranges, const int32_t* status,
                       const Cam& cam, int tw, int th, float* image, float* final_T, uint32_t* n_contrib,
                       unsigned long long* stats, float2* state, hipStream_t st) {
#define GS_FWD(a, b) launch_t<a, b>(rec, vals, ranges, status, cam, image, final_T, n_contrib, stats, state, st)
    if (tw == 16 && th == 16) GS_FWD(16, 16);
    else if (tw == 8 && th == 8) GS_FWD(8, 8);
    else if (tw == 16 && th == 8) GS_FWD(16, 8);
    else if (tw == 32 && th == 8) GS_FWD(32, 8);
    else if (tw == 32 && th == 16) GS_FWD(32, 16);
    else if (tw == 32 && th == 32) GS_FWD(32, 32);
#undef GS_FWD
}

}  // namespace gs
