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
// over each 16-lane row with a transposing DPP butterfly that leaves the
// nine sums in lanes 0..8 of the row, which add them with one LDS atomic
// instruction into a per-tile accumulator.  After the batch each entry's
// sums are written, without global atomics, to its (Gaussian, tile) pair
// slot in emission order; a gather then adds each Gaussian's slots, so the
// per-Gaussian sum over tiles has a fixed order.
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
    const ushort4* rect;    // per slot: tile rectangle
    const uint32_t* first;  // per slot: emission position of its first pair
    float4* pg8;            // per pair: du, dv, dA, dB | dC, do, dr, dg
    float* pg1;             // per pair: db
    int64_t cap;            // pair capacity
    const float2* state;
    uint32_t* queue;        // persistent launch: next queue position (zeroed before launch)
    const uint32_t* order;  // persistent launch: tiles in processing order (NULL = 0, 1, ...)
    uint32_t n_tiles;
};

// One DPP exchange inside each 16-lane row: quad_perm [1,0,3,2] (partner
// lane ^ 1), quad_perm [2,3,0,1] (lane ^ 2), row_ror:4 and row_ror:8 (lane
// - 4 and lane - 8 within the row).
template <int CTRL>
__device__ __forceinline__ float xch(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kRor4 = 0x124, kRor8 = 0x128;

// Sums nine values over each 16-lane row with a transposing butterfly: in
// each of the first three exchanges a lane keeps one value of every pair and
// sends its partner the other, so the values per lane halve as the span of
// the sums doubles (27 VALU operations instead of 36 for nine plain
// butterflies, and the sums end up spread over the lanes).  On return lane
// l (0..15) of a row holds the row sum of v[l & 7] in .x and of v8 in .y.
// b0, b1, b2 are bits 0, 1, 2 of the lane index.
__device__ __forceinline__ float2 row_sum9(float v0, float v1, float v2, float v3, float v4, float v5, float v6,
                                           float v7, float v8, bool b0, bool b1, bool b2) {
    // lane ^ 1: keep v[2j + b0]
    const float r0 = (b0 ? v1 : v0) + xch<kXor1>(b0 ? v0 : v1);
    const float r1 = (b0 ? v3 : v2) + xch<kXor1>(b0 ? v2 : v3);
    const float r2 = (b0 ? v5 : v4) + xch<kXor1>(b0 ? v4 : v5);
    const float r3 = (b0 ? v7 : v6) + xch<kXor1>(b0 ? v6 : v7);
    const float r4 = v8 + xch<kXor1>(v8);
    // lane ^ 2: keep v[4k + 2 b1 + b0]
    const float s0 = (b1 ? r1 : r0) + xch<kXor2>(b1 ? r0 : r1);
    const float s1 = (b1 ? r3 : r2) + xch<kXor2>(b1 ? r2 : r3);
    const float s2 = r4 + xch<kXor2>(r4);
    // lane - 4 (opposite bit 2, same low bits): keep v[4 b2 + 2 b1 + b0]
    const float t0 = (b2 ? s1 : s0) + xch<kRor4>(b2 ? s0 : s1);
    const float t1 = s2 + xch<kRor4>(s2);
    // lane - 8: the other two quads of the row
    return make_float2(t0 + xch<kRor8>(t0), t1 + xch<kRor8>(t1));
}

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

    const bool b0 = (lane & 1) != 0, b1 = (lane & 2) != 0, b2 = (lane & 4) != 0;
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
                const Staged gk = staged_at(s, k);
                const float4 ck = stage_cull(gk);
                o0 = box_overlaps(gk, ck, bx0, bx0 + 3.0f, by0, by0 + 3.0f);
                o1 = box_overlaps(gk, ck, bx0 + 4.0f, bx0 + 7.0f, by0, by0 + 3.0f);
                o2 = box_overlaps(gk, ck, bx0, bx0 + 3.0f, by0 + 4.0f, by0 + 7.0f);
                o3 = box_overlaps(gk, ck, bx0 + 4.0f, bx0 + 7.0f, by0 + 4.0f, by0 + 7.0f);
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
                const Staged g = staged_at(s, kk);
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
                // per-lane terms; a lane without a contribution holds zeros
                const float v6 = g0 * w, v7 = g1 * w, v8 = g2 * w;
                const float v5 = (contrib && !e.capped) ? da0 * e.G : 0.0f;
                // moments of dL/dpower over the pixel offsets; the centre and
                // conic gradients are linear in them (formed at the flush)
                const float dpow = da * a;
                const float mx = dpow * e.dx, my = dpow * e.dy;
                const uint64_t cm = __ballot(contrib);
                if (cm == 0ull) continue;
                // row sums, spread over the row's lanes 0..8, added into the
                // tile's LDS accumulator of the row's entry
                const float2 r = row_sum9(mx, my, mx * e.dx, mx * e.dy, my * e.dy, v5, v6, v7, v8, b0, b1, b2);
                // LDS float atomics cost about one cycle per active lane:
                // rows without a contributing pixel add nothing
                if (l16 <= 8 && ((cm >> (lane & 48)) & 0xFFFFull) != 0ull)
                    atomicAdd(s_acc + (__umul24((uint32_t)kk, 9u) + (uint32_t)l16), l16 == 8 ? r.y : r.x);
            }
        }
        __syncthreads();
        // the accumulator holds, per entry, the sums of dpow dx, dpow dy,
        // dpow dx^2, dpow dx dy, dpow dy^2, dL/do, dL/drgb; with
        // power = -(A dx^2 + C dy^2)/2 - B dx dy and dx = x - u:
        // du = sum dpow (A dx + B dy), dv = sum dpow (B dx + C dy),
        // dA = -sum dpow dx^2 / 2, dB = -sum dpow dx dy, dC = -sum dpow dy^2 / 2,
        // where A = -2 ca / log2e, B = -cb / log2e, C = -2 cc / log2e.
        // Each entry's nine sums go, without atomics, to the entry's own
        // pair slot: one thread per entry.
        if (tid < nb) {
            const float* acc = s_acc + tid * 9;
            float m[9];
            bool any = false;
            for (int c = 0; c < 9; ++c) {
                m[c] = acc[c];
                any |= m[c] != 0.0f;
            }
            if (any) {
                const uint32_t gid = s_gid[tid];
                const ushort4 r = a.rect[gid];
                const int64_t p = (int64_t)a.first[gid] + (int64_t)(ty - (int)r.y) * ((int)r.z - (int)r.x) +
                                  (tx - (int)r.x);
                if (p >= 0 && p < a.cap) {
                    const float4 cf = s[tid].coef;
                    const float A = -2.0f * cf.x * (1.0f / kLog2e), Bc = -cf.y * (1.0f / kLog2e),
                                C = -2.0f * cf.z * (1.0f / kLog2e);
                    a.pg8[2 * p] = make_float4(A * m[0] + Bc * m[1], Bc * m[0] + C * m[1], -0.5f * m[2], -m[3]);
                    a.pg8[2 * p + 1] = make_float4(-0.5f * m[4], m[5], m[6], m[7]);
                    a.pg1[p] = m[8];
                }
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

// Clear the pair gradient buffer over the pairs of this frame.
__global__ __launch_bounds__(256) void k_pair_zero(float4* __restrict__ pg8, float* __restrict__ pg1,
                                                   const uint32_t* __restrict__ pair_count, int64_t cap) {
    const int64_t P = (int64_t)*pair_count < cap ? (int64_t)*pair_count : cap;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256) {
        pg8[2 * p] = make_float4(0.f, 0.f, 0.f, 0.f);
        pg8[2 * p + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
        pg1[p] = 0.f;
    }
}

// Per slot: the sum over its pairs (emission order, so a fixed order) of
// the per-tile image-space gradients, into g2d[9][nslots].
__global__ __launch_bounds__(256) void k_pair_gather(int64_t nslots, const uint32_t* __restrict__ first,
                                                     const uint32_t* __restrict__ tt, const float4* __restrict__ pg8,
                                                     const float* __restrict__ pg1, int64_t cap,
                                                     const int32_t* __restrict__ status, float* __restrict__ g2d) {
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= nslots) return;
    float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0;
    float s2 = 0.f;
    if (*status == 0) {
        const int64_t b = first[slot];
        int64_t e = b + (int64_t)tt[slot];
        if (e > cap) e = cap;
        for (int64_t p = b; p < e; ++p) {
            const float4 x = pg8[2 * p], y = pg8[2 * p + 1];
            s0.x += x.x; s0.y += x.y; s0.z += x.z; s0.w += x.w;
            s1.x += y.x; s1.y += y.y; s1.z += y.z; s1.w += y.w;
            s2 += pg1[p];
        }
    }
    g2d[slot] = s0.x;
    g2d[nslots + slot] = s0.y;
    g2d[2 * nslots + slot] = s0.z;
    g2d[3 * nslots + slot] = s0.w;
    g2d[4 * nslots + slot] = s1.x;
    g2d[5 * nslots + slot] = s1.y;
    g2d[6 * nslots + slot] = s1.z;
    g2d[7 * nslots + slot] = s1.w;
    g2d[8 * nslots + slot] = s2;
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

size_t pair_grad_bytes(int64_t capacity) { return (size_t)(capacity > 0 ? capacity : 0) * 36; }

void launch_pair_zero(void* pairs, const uint32_t* pair_count, int64_t capacity, hipStream_t st) {
    if (capacity <= 0) return;
    int64_t blocks = (capacity + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_pair_zero, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<float4*>(pairs),
                       reinterpret_cast<float*>(static_cast<char*>(pairs) + (size_t)capacity * 32), pair_count,
                       capacity);
}

void launch_pair_gather(int64_t nslots, const uint32_t* first, const uint32_t* tiles_touched, const void* pairs,
                        int64_t capacity, const int32_t* status, float* g2d, hipStream_t st) {
    if (nslots <= 0) return;
    const int64_t blocks = (nslots + 255) / 256;
    hipLaunchKernelGGL(k_pair_gather, dim3((unsigned)blocks), dim3(256), 0, st, nslots, first, tiles_touched,
                       static_cast<const float4*>(pairs),
                       reinterpret_cast<const float*>(static_cast<const char*>(pairs) + (size_t)capacity * 32),
                       capacity, status, g2d);
}

void launch_render_bwd(const RenderArgs& r, const float* final_T, const uint32_t* n_contrib, const float* dimg,
                       const ushort4* rect, const uint32_t* first, void* pairs, int64_t capacity,
                       const float2* state, hipStream_t st) {
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
    a.rect = rect;
    a.first = first;
    a.pg8 = static_cast<float4*>(pairs);
    a.pg1 = reinterpret_cast<float*>(static_cast<char*>(pairs) + (size_t)capacity * 32);
    a.cap = capacity;
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
