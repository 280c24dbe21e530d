// Backward of the tile blend: per-Gaussian image-space gradients.
//
// VastGaussian (arXiv 2402.17427), section 3: the renderer is differentiable
// and the Gaussians are optimised by gradient descent.  For a pixel with
// blended Gaussians i = 1..n (weights w_i = alpha_i T_i), colour
// C = sum_i rgb_i w_i + T_final bg, the gradients are
//   dL/drgb_i   = g w_i
//   dL/dalpha_i = g . (rgb_i T_i - S_i / (1 - alpha_i)),
//                 S_i = sum_{j > i} rgb_j w_j + T_final bg
// and, unless alpha_i was capped at 0.99, dL/do = dalpha G and
// dL/dpower = dalpha alpha, from which the conic (A, B, C) and centre (u, v)
// gradients follow.  g is dL/dpixel.
//
// No per-contributor state is stored by the forward: each pixel walks its
// tile list back to front from its last contributor, recomputes alpha with
// the same staged values and code as the forward (so it takes the same
// skip decisions), recovers T_i = T_{i+1} / (1 - alpha_i) from the stored
// final transmittance, and accumulates S_i as it goes.
//
// Walk: as in the forward, each wave covers an 8x8 block and walks only the
// staged entries whose support box meets its block (ballot mask, scanned
// from the back) and that lie before its pixels' last contributor.
// Reduction: per walked entry, a wave first checks (ballot) whether any of
// its 64 pixels contributed; only then are the nine gradient terms summed
// over each 16-lane row with DPP, added by the first lane of each row that
// has a contributing pixel into a per-tile LDS accumulator, and flushed with
// one global FP32 atomic per (Gaussian, term, tile) after the batch.
#include "kernels.h"

namespace gs {

namespace {

struct BwdArgs {
    const Rec* rec;
    const uint32_t* vals;
    const uint2* ranges;
    const int32_t* status;
    ViewTab views;
    const float* final_T;
    const uint32_t* n_contrib;
    const float* dimg;
    int64_t n;              // slots: plane stride of g2d
    float* g2d;
    const float2* state;
    uint32_t* queue;        // persistent launch: next queue position (zeroed before launch)
    const uint32_t* order;  // persistent launch: tiles in processing order (NULL = 0, 1, ...)
    uint32_t n_tiles;
};

template <int NT>
struct BwdShared {
    static constexpr int B = NT < 256 ? NT : 256;   // staged Gaussians per batch
    Staged s[B];
    uint32_t gid[B];
    float acc[B * 9];
    uint32_t max_last;
};

// STORED = true reads each entry's (alpha, T) from the state the storing
// forward wrote (alpha negated when capped) instead of recomputing them.
template <int TW, int TH, bool STORED>
__device__ __forceinline__ void bwd_tile(const BwdArgs& a, uint32_t tile, BwdShared<TW * TH>& sh) {
    constexpr int NT = TW * TH;
    constexpr int B = BwdShared<NT>::B;
    constexpr int WX = TW / 8;
    Staged* s = sh.s;
    uint32_t* s_gid = sh.gid;
    float* s_acc = sh.acc;

    if (*a.status != 0) return;

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
    const float* final_T = a.final_T + V.pix_base;
    const uint32_t* n_contrib = a.n_contrib + V.pix_base;
    const float* dimg = a.dimg + V.img_base;
    const Rec* __restrict__ rec = a.rec;
    const uint32_t* __restrict__ vals = a.vals;
    const float2* __restrict__ state = a.state;
    float* __restrict__ g2d = a.g2d;
    const int64_t n = a.n;
    const float bg0 = V.cam.bg[0], bg1 = V.cam.bg[1], bg2 = V.cam.bg[2];

    const uint2 rg = a.ranges[tile];
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const float bx0 = (float)(tx * TW + bx) + 0.5f, by0 = (float)(ty * TH + by) + 0.5f;

    uint32_t my_last = 0;
    float T = 1.0f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    if (inside) {
        my_last = n_contrib[off];
        T = final_T[off];
        g0 = dimg[off];
        g1 = dimg[npix + off];
        g2 = dimg[2 * npix + off];
    }
    // g . (T_final bg): the background's share of every suffix colour
    const float gbg = g0 * (T * bg0) + g1 * (T * bg1) + g2 * (T * bg2);
    float ga = 0.f;   // g . sum of rgb_j w_j over the blended j behind the current entry

    __syncthreads();   // the previous tile of a persistent workgroup is done with the shared state
    if (tid == 0) sh.max_last = 0u;
    __syncthreads();
    if (my_last) atomicMax(&sh.max_last, my_last);
    __syncthreads();
    // never walk past the tile's list, whatever n_contrib holds
    const uint32_t max_last = min(sh.max_last, rg.y - rg.x);

    // a row never needs entries at or beyond its pixels' last contributor
    uint32_t row_last = my_last;
    for (int d = 1; d < 16; d <<= 1) row_last = max(row_last, (uint32_t)__shfl_xor((int)row_last, d, kWave));

    for (int64_t hi = (int64_t)max_last; hi > 0; hi -= B) {
        const int64_t lo = hi - B > 0 ? hi - B : 0;
        const int nb = (int)(hi - lo);
        __syncthreads();
        if (tid < nb) {
            const uint32_t gid = vals[rg.x + lo + tid];
            s_gid[tid] = gid;
            s[tid] = stage_rec(rec[gid]);
        }
        for (int q = tid; q < B * 9; q += NT) s_acc[q] = 0.f;
        __syncthreads();

        // 64 staged entries at a time, back to front: each lane tests one
        // against the four quadrants of the wave's block; every row then
        // walks, back to front, the entries whose support meets its quadrant
        // and that lie before its pixels' last contributor (the four rows
        // of a wave walk different Gaussians in step).
        for (int c0k = ((nb - 1) / kWave) * kWave; c0k >= 0; c0k -= kWave) {
            const int k = c0k + lane;
            bool o0 = false, o1 = false, o2 = false, o3 = false;
            if (k < nb) {
                const Staged gk = s[k];
                o0 = box_overlaps(gk, bx0, bx0 + 3.0f, by0, by0 + 3.0f);
                o1 = box_overlaps(gk, bx0 + 4.0f, bx0 + 7.0f, by0, by0 + 3.0f);
                o2 = box_overlaps(gk, bx0, bx0 + 3.0f, by0 + 4.0f, by0 + 7.0f);
                o3 = box_overlaps(gk, bx0 + 4.0f, bx0 + 7.0f, by0 + 4.0f, by0 + 7.0f);
            }
            const uint64_t m0 = __ballot(o0), m1 = __ballot(o1), m2 = __ballot(o2), m3 = __ballot(o3);
            uint64_t mm = row == 0 ? m0 : (row == 1 ? m1 : (row == 2 ? m2 : m3));
            const int lim = (int)row_last - (int)(lo + c0k);
            mm = lim <= 0 ? 0ull : (lim >= kWave ? mm : (mm & ((1ull << lim) - 1ull)));
            while (__ballot(mm != 0ull) != 0ull) {
                const bool has = mm != 0ull;
                int kk = 0;
                if (has) {
                    const int j = 63 - (int)__builtin_clzll(mm);
                    mm &= ~(1ull << j);
                    kk = c0k + j;
                }
                const Staged g = s[kk];
                const uint32_t pos = (uint32_t)(lo + kk);
                const bool live = has && pos < my_last;
                // Branch-free: a pair that does not contribute gets alpha 0,
                // which leaves T and the suffix colour unchanged and makes
                // every gradient term 0.
                Eval e;
                float Ts = T;
                if (STORED) {
                    const float2 st = live ? state[(int64_t)(rg.x + pos) * NT + tid] : make_float2(0.f, 0.f);
                    e.alpha = fabsf(st.x);
                    e.capped = st.x < 0.0f;
                    e.dx = (fx - g.geo.x) - g.geo.y;
                    e.dy = (fy - g.geo.z) - g.geo.w;
                    e.G = e.alpha * __builtin_amdgcn_rcpf(g.coef.w);
                    Ts = st.y;
                } else {
                    e = eval_pair(g, fx, fy);
                }
                const bool contrib = live && e.alpha > 0.0f;
                const float a = contrib ? e.alpha : 0.0f;
                const float iom = __builtin_amdgcn_rcpf(1.0f - a);
                const float Ti = STORED ? (contrib ? Ts : T) : T * iom;
                const float w = a * Ti;
                const float grgb = g0 * g.col.x + g1 * g.col.y + g2 * g.col.z;
                // dL/dalpha = g . (rgb T_i - S_i / (1 - alpha)), S_i = suffix colour + T_final bg;
                // no gradient through a capped alpha
                const float da0 = grgb * Ti - (ga + gbg) * iom;
                const float da = (contrib && !e.capped) ? da0 : 0.0f;
                ga = __builtin_fmaf(grgb, w, ga);
                T = Ti;
                float v6 = g0 * w, v7 = g1 * w, v8 = g2 * w;
                float v5 = da * e.G;
                // moments of dL/dpower over the pixel offsets; the centre and
                // conic gradients are linear in them (formed per row below)
                const float dpow = da * a;
                const float mx = dpow * e.dx, my = dpow * e.dy;
                float v0 = mx, v1 = my, v2 = mx * e.dx, v3 = mx * e.dy, v4 = my * e.dy;
                const uint64_t cm = __ballot(contrib);
                if (cm == 0ull) continue;
                // sum each 16-lane row (DPP), then the first lane of every row
                // with a contributing pixel adds its row's sums into the
                // tile's LDS accumulator
                v0 = row_sum(v0); v1 = row_sum(v1); v2 = row_sum(v2);
                v3 = row_sum(v3); v4 = row_sum(v4); v5 = row_sum(v5);
                v6 = row_sum(v6); v7 = row_sum(v7); v8 = row_sum(v8);
                if ((lane & 15) == 0 && ((cm >> lane) & 0xFFFFull) != 0ull) {
                    // power = -(A dx^2 + C dy^2)/2 - B dx dy with dx = x - u:
                    // du = sum dpow (A dx + B dy), dA = -sum dpow dx^2 / 2, ...
                    // and A = -2 ca / log2e, B = -cb / log2e, C = -2 cc / log2e
                    const float A = -2.0f * g.coef.x * (1.0f / kLog2e), Bc = -g.coef.y * (1.0f / kLog2e),
                                C = -2.0f * g.coef.z * (1.0f / kLog2e);
                    float* acc = &s_acc[kk * 9];
                    atomicAdd(acc + 0, A * v0 + Bc * v1);
                    atomicAdd(acc + 1, Bc * v0 + C * v1);
                    atomicAdd(acc + 2, -0.5f * v2);
                    atomicAdd(acc + 3, -v3);
                    atomicAdd(acc + 4, -0.5f * v4);
                    atomicAdd(acc + 5, v5);
                    atomicAdd(acc + 6, v6);
                    atomicAdd(acc + 7, v7);
                    atomicAdd(acc + 8, v8);
                }
            }
        }
        __syncthreads();
        for (int q = tid; q < nb * 9; q += NT) {
            const float v = s_acc[q];
            if (v != 0.0f) {
                const int k = q / 9, c = q - 9 * (q / 9);
                atomicAdd(&g2d[(int64_t)c * n + s_gid[k]], v);
            }
        }
    }
}

template <int TW, int TH, bool STORED>
__global__ __launch_bounds__(TW * TH) void k_render_bwd(BwdArgs a) {
    __shared__ BwdShared<TW * TH> sh;
    bwd_tile<TW, TH, STORED>(a, blockIdx.x, sh);
}

template <int TW, int TH>
__global__ __launch_bounds__(TW * TH) void k_render_bwd_persistent(BwdArgs a) {
    __shared__ BwdShared<TW * TH> sh;
    __shared__ uint32_t s_next;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_next = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t q = s_next;
        if (q >= a.n_tiles) break;
        bwd_tile<TW, TH, false>(a, a.order ? a.order[q] : q, sh);
    }
}

template <int TW, int TH>
void launch_t(const BwdArgs& a, int persistent_grid, hipStream_t st) {
    const dim3 block(TW * TH);
    if (a.state)
        hipLaunchKernelGGL((k_render_bwd<TW, TH, true>), dim3(a.n_tiles), block, 0, st, a);
    else if (persistent_grid > 0)
        hipLaunchKernelGGL((k_render_bwd_persistent<TW, TH>), dim3(persistent_grid), block, 0, st, a);
    else
        hipLaunchKernelGGL((k_render_bwd<TW, TH, false>), dim3(a.n_tiles), block, 0, st, a);
}

}  // namespace

void launch_render_bwd(const RenderArgs& r, const float* final_T, const uint32_t* n_contrib, const float* dimg,
                       int64_t nslots, float* g2d, const float2* state, hipStream_t st) {
    if (r.n_tiles == 0) return;
    BwdArgs a;
    a.rec = r.rec;
    a.vals = r.vals;
    a.ranges = reinterpret_cast<const uint2*>(r.ranges);
    a.status = r.status;
    a.views = r.views;
    a.final_T = final_T;
    a.n_contrib = n_contrib;
    a.dimg = dimg;
    a.n = nslots;
    a.g2d = g2d;
    a.state = state;
    a.queue = r.queue;
    a.order = r.order;
    a.n_tiles = r.n_tiles;
    const int pg = (r.queue && !state) ? r.persistent_grid : 0;
    if (pg > 0) launch_fill_u32(r.queue, 0u, 1, st);
#define GS_BWD(x, y) launch_t<x, y>(a, pg, st)
    if (r.tw == 16 && r.th == 16) GS_BWD(16, 16);
    else if (r.tw == 8 && r.th == 8) GS_BWD(8, 8);
    else if (r.tw == 16 && r.th == 8) GS_BWD(16, 8);
    else if (r.tw == 32 && r.th == 8) GS_BWD(32, 8);
    else if (r.tw == 32 && r.th == 16) GS_BWD(32, 16);
    else if (r.tw == 32 && r.th == 32) GS_BWD(32, 32);
#undef GS_BWD
}

int render_persistent_grid_bwd(int tw, int th) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
#define GS_OCC(x, y) \
    if (tw == x && th == y) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_render_bwd_persistent<x, y>, x * y, 0)
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
