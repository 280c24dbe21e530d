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
// a queue, longest list first), one lane per pixel.  Every wave covers an
// 8x8 block of the tile and each of its four 16-lane rows a 4x4 quadrant.
// Batches of records are staged in LDS; for each 64 of them every lane
// tests one against the four quadrants (an exact ellipse-rectangle test),
// and each row then walks, in list order, only the Gaussians whose support
// meets its quadrant; the rows of a wave walk different Gaussians in the
// same instructions.  Skipping the others never changes a result: such a
// Gaussian has alpha < 1/255 at every pixel of the quadrant.  A wave leaves
// the tile once all its pixels have stopped, the workgroup once all waves
// have.  Tiles of several views are numbered consecutively; a tile finds
// its view (camera, image planes) in the view table.
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
    float2* state;
    uint32_t* queue;        // persistent launch: next queue position (zeroed before launch)
    const uint32_t* order;  // persistent launch: tiles in processing order (NULL = 0, 1, ...)
    uint32_t n_tiles;
};

template <int TW, int TH, int MODE>
__device__ __forceinline__ void fwd_tile(const FwdArgs& a, uint32_t tile, Staged* s, float4* sc) {
    constexpr int NT = TW * TH;
    constexpr bool STATS = MODE == kStats;
    constexpr int WX = TW / 8;

    const View V = view_at(a.views, find_view(a.views, tile));
    const int W = V.cam.W, H = V.cam.H;
    const int local = (int)(tile - V.tile_base);
    const int tx = local % V.ntx, ty = local / V.ntx;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    // wave = 8x8 block; its 16-lane row r = the 4x4 quadrant (r & 1, r >> 1)
    const int row = lane >> 4, l16 = lane & 15;
    const int bx = (wv % WX) * 8, by = (wv / WX) * 8;
    const int lx = bx + (row & 1) * 4 + (l16 & 3), ly = by + (row >> 1) * 4 + (l16 >> 2);
    const int px = tx * TW + lx, py = ty * TH + ly;
    const bool inside = px < W && py < H;
    const int64_t npix = (int64_t)W * H;
    const int64_t off = (int64_t)py * W + px;
    float* image = V.out_image ? V.out_image : a.image + V.img_base;
    float* final_T = a.final_T + V.pix_base;
    uint32_t* n_contrib = a.n_contrib + V.pix_base;

    if (*a.status != 0) {
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

    const uint2 rg = a.ranges[tile];
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const float bx0 = (float)(tx * TW + bx) + 0.5f, by0 = (float)(ty * TH + by) + 0.5f;

    float T = 1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    uint32_t last = 0;
    bool done = !inside;
    unsigned long long n_eval = 0, n_supp = 0, n_blend = 0;

    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += NT) {
        if (__syncthreads_count(done) == NT) break;
        const uint32_t j = b0 + tid;
        if (j < rg.y) {
            const Staged st = stage_rec(a.rec[a.vals[j]]);
            s[tid] = st;
            sc[tid] = stage_cull(st);
        }
        __syncthreads();
        const int nb = (int)min((uint32_t)NT, rg.y - b0);
        // 64 staged Gaussians at a time: each lane tests one against the
        // four quadrants of the wave's block; every row then walks, in list
        // order, the Gaussians whose support meets its own quadrant (the
        // four rows of a wave walk different Gaussians in step).
        for (int c0k = 0; c0k < nb; c0k += kWave) {
            const uint64_t lv = __ballot(!done);
            if (lv == 0ull) break;
            const int k = c0k + lane;
            bool o0 = false, o1 = false, o2 = false, o3 = false;
            if (k < nb) {
                const Staged gk = staged_at(s, k);
                const float4 ck = sc[k];
                o0 = box_overlaps(gk, ck, bx0, bx0 + 3.0f, by0, by0 + 3.0f);
                o1 = box_overlaps(gk, ck, bx0 + 4.0f, bx0 + 7.0f, by0, by0 + 3.0f);
                o2 = box_overlaps(gk, ck, bx0, bx0 + 3.0f, by0 + 4.0f, by0 + 7.0f);
                o3 = box_overlaps(gk, ck, bx0 + 4.0f, bx0 + 7.0f, by0 + 4.0f, by0 + 7.0f);
            }
            const uint64_t m0 = __ballot(o0), m1 = __ballot(o1), m2 = __ballot(o2), m3 = __ballot(o3);
            uint64_t mm = row == 0 ? m0 : (row == 1 ? m1 : (row == 2 ? m2 : m3));
            if (((lv >> (16 * row)) & 0xFFFFull) == 0ull) mm = 0ull;   // this row's pixels have all stopped
            while (__ballot(mm != 0ull) != 0ull) {
                // branch-free: a row with nothing left evaluates entry
                // c0k and, like a stopped pixel or an entry below the
                // alpha threshold, changes nothing
                const bool has = mm != 0ull;
                const int kk = c0k + (has ? (int)__builtin_ctzll(mm) : 0);
                mm &= mm - 1;
                const bool act = has && !done;
                const Staged g = staged_at(s, kk);
                const Eval e = eval_pair(g, fx, fy);
                if (MODE == kStore && act)
                    a.state[(int64_t)(b0 + (uint32_t)kk) * NT + tid] =
                        make_float2(e.capped && e.alpha > 0.0f ? -e.alpha : e.alpha, T);
                const bool supp = act && e.alpha > 0.0f;
                const float Tn = T * (1.0f - e.alpha);
                const bool stop = supp && Tn < kTMin;
                const bool blend = supp && !stop;
                if (STATS) {
                    n_eval += act ? 1u : 0u;
                    n_supp += supp ? 1u : 0u;
                    n_blend += blend ? 1u : 0u;
                }
                const float w = blend ? e.alpha * T : 0.0f;
                c0 = __builtin_fmaf(g.col.x, w, c0);
                c1 = __builtin_fmaf(g.col.y, w, c1);
                c2 = __builtin_fmaf(g.col.z, w, c2);
                T = blend ? Tn : T;
                last = blend ? b0 - rg.x + (uint32_t)kk + 1u : last;
                done = done || stop;
                // a row whose pixels have all stopped leaves its walk
                // (checked only when some pixel of the wave stopped now)
                if (__ballot(stop) != 0ull) {
                    const uint64_t lv2 = __ballot(!done);
                    if (((lv2 >> (16 * row)) & 0xFFFFull) == 0ull) mm = 0ull;
                }
            }
        }
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
        if ((threadIdx.x & (kWave - 1)) == 0) {
            atomicAdd(&a.stats[0], (unsigned long long)e32);
            atomicAdd(&a.stats[1], (unsigned long long)s32);
            atomicAdd(&a.stats[2], (unsigned long long)b32);
        }
    } else if (inside) {
        image[off] = __builtin_fmaf(T, V.cam.bg[0], c0);
        image[npix + off] = __builtin_fmaf(T, V.cam.bg[1], c1);
        image[2 * npix + off] = __builtin_fmaf(T, V.cam.bg[2], c2);
        final_T[off] = T;
        n_contrib[off] = last;
    }
}

template <int TW, int TH, int MODE>
__global__ __launch_bounds__(TW * TH) void k_render_fwd(FwdArgs a) {
    __shared__ Staged s[TW * TH];
    __shared__ float4 sc[TW * TH];
    fwd_tile<TW, TH, MODE>(a, blockIdx.x, s, sc);
}

template <int TW, int TH>
__global__ __launch_bounds__(TW * TH) void k_render_fwd_persistent(FwdArgs a) {
    __shared__ Staged s[TW * TH];
    __shared__ float4 sc[TW * TH];
    __shared__ uint32_t s_next;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_next = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t q = s_next;
        if (q >= a.n_tiles) break;
        fwd_tile<TW, TH, kPlain>(a, a.order ? a.order[q] : q, s, sc);
    }
}

template <int TW, int TH>
void launch_t(const FwdArgs& a, int persistent_grid, hipStream_t st) {
    const dim3 block(TW * TH);
    if (a.stats)
        hipLaunchKernelGGL((k_render_fwd<TW, TH, kStats>), dim3(a.n_tiles), block, 0, st, a);
    else if (a.state)
        hipLaunchKernelGGL((k_render_fwd<TW, TH, kStore>), dim3(a.n_tiles), block, 0, st, a);
    else if (persistent_grid > 0)
        hipLaunchKernelGGL((k_render_fwd_persistent<TW, TH>), dim3(persistent_grid), block, 0, st, a);
    else
        hipLaunchKernelGGL((k_render_fwd<TW, TH, kPlain>), dim3(a.n_tiles), block, 0, st, a);
}

}  // namespace

bool render_tile_supported(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 32 && th == 8) ||
           (tw == 32 && th == 16) || (tw == 32 && th == 32);
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
    a.state = state;
    a.queue = r.queue;
    a.order = r.order;
    a.n_tiles = r.n_tiles;
    const int pg = (r.queue && !stats && !state) ? r.persistent_grid : 0;
    if (pg > 0) launch_fill_u32(r.queue, 0u, 1, st);
#define GS_FWD(x, y) launch_t<x, y>(a, pg, st)
    if (r.tw == 16 && r.th == 16) GS_FWD(16, 16);
    else if (r.tw == 8 && r.th == 8) GS_FWD(8, 8);
    else if (r.tw == 16 && r.th == 8) GS_FWD(16, 8);
    else if (r.tw == 32 && r.th == 8) GS_FWD(32, 8);
    else if (r.tw == 32 && r.th == 16) GS_FWD(32, 16);
    else if (r.tw == 32 && r.th == 32) GS_FWD(32, 32);
#undef GS_FWD
}

int render_persistent_grid_bwd(int tw, int th);
int render_persistent_grid_fwd(int tw, int th);

int render_persistent_grid(int tw, int th, bool backward) {
    return backward ? render_persistent_grid_bwd(tw, th) : render_persistent_grid_fwd(tw, th);
}

int render_persistent_grid_fwd(int tw, int th) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
#define GS_OCC(x, y) \
    if (tw == x && th == y) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_render_fwd_persistent<x, y>, x * y, 0)
    GS_OCC(16, 16);
    GS_OCC(8, 8);
    GS_OCC(16, 8);
    GS_OCC(32, 8);
    GS_OCC(32, 16);
    GS_OCC(32, 32);
#undef GS_OCC
    if (e != hipSuccess || per < 1) per = 1;
    return cus * per;
}

}  // namespace gs
