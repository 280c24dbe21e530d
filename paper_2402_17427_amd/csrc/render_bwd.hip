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
// Walk: one lane per cell of CW x CH pixels (blend_cells.h); each lane
// walks, from the back, only the list entries whose support reaches its
// cell and that lie before its pixels' last contributor (the cell masks are
// the forward's when it kept them, else recomputed the same way).  The list is
// taken in chunks of at most 64 entries from the back.  Accumulation: for
// every (cell, entry) it walks, a lane adds its pixels' nine gradient
// terms in registers and writes the sums once, with plain stores, to a slot
// of its own in LDS; the slots of one entry are contiguous (entry-major,
// then wave, then cell order), so after the chunk one thread per entry adds
// its slots in a fixed order and writes the nine sums, without global
// atomics, to the entry's (Gaussian, tile) pair slot in emission order; a
// gather then adds each Gaussian's pair slots, so the per-Gaussian sum has
// a fixed order.  A chunk ends early when its entries' slots would exceed
// the LDS capacity (Gaussians that reach many cells).
#include "blend_cells.h"
#include "kernels.h"
#include "tile_order.h"

namespace gs {

namespace {

constexpr int kChunk = 64;      // candidate entries per chunk (one walk word)
#ifndef GS_ITEM_CAP
#define GS_ITEM_CAP 512
#endif
constexpr int kItemCap = GS_ITEM_CAP;   // (cell, entry) slots per chunk (>= 64 x waves of any layout)
// slot capacities of the persistent launch (a tuning knob of the batched
// step): kItemCap, or the half of it
constexpr int kItemCapSmall = kItemCap / 2;

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
    const uint64_t* masks;  // per sorted pair and wave: the forward's cell masks (NULL = recompute)
    uint32_t* queue;        // persistent launch: next queue position (zeroed before launch)
    const uint32_t* order;  // persistent launch: tiles in processing order (NULL = 0, 1, ...)
    uint32_t n_tiles;
    const uint32_t* torder;     // one workgroup per tile: workgroup b takes tile torder[b] (NULL: tile b)
    const uint32_t* torder_n;   // ... and exits when b >= *torder_n
};

template <class L, int CAP>
struct BwdShared {
    // one entry can reach every cell of the workgroup: its slots must fit,
    // or a chunk could not take even its top candidate
    static_assert(CAP >= L::NCELL, "slot capacity below the cells of a tile");
    Staged s[kChunk];
    uint32_t gid[kChunk];
    uint64_t mask[L::WAVES][kChunk];   // per wave: the cells that walk each entry
    uint32_t base[L::WAVES][kChunk];   // items per (wave, entry), then their first slot
    uint32_t total[kChunk];            // items per entry
    float item[9][CAP];                // the nine sums of each (cell, entry)
    uint32_t max_last;
    int kmin;                          // the chunk: candidates kmin .. ncand - 1
};

// STORED = true reads each entry's (alpha, T) from the state the storing
// forward wrote (alpha negated when capped) instead of recomputing them.
template <class L, bool STORED, int CAP>
__device__ __forceinline__ void bwd_tile(const BwdArgs& a, uint32_t tile, BwdShared<L, CAP>& sh) {
    constexpr int NP = L::NP;
    if (*a.status != 0) return;

    const View V = view_at(a.views, find_view(a.views, tile));
    const int W = V.cam.W, H = V.cam.H;
    const int local = (int)(tile - V.tile_base);
    const int tx = local % V.ntx, ty = local / V.ntx;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int cx = tid % L::CPR, cy = tid / L::CPR;
    const int x0 = tx * L::TW, y0 = ty * L::TH;
    const int wy0 = y0 + wv * L::PXROWS_W;
    const int64_t npix = (int64_t)W * H;
    const float* final_T = a.final_T + V.pix_base;
    const uint32_t* n_contrib = a.n_contrib + V.pix_base;
    const float* dimg = a.dimg + V.img_base;
    const float bg0 = V.cam.bg[0], bg1 = V.cam.bg[1], bg2 = V.cam.bg[2];
    const uint2 rg = a.ranges[tile];

    const int px0 = x0 + cx * L::CW, py0 = y0 + cy * L::CH;
    float fxp[L::CW], fyp[L::CH];
#pragma unroll
    for (int i = 0; i < L::CW; ++i) fxp[i] = (float)(px0 + i) + 0.5f;
#pragma unroll
    for (int j = 0; j < L::CH; ++j) fyp[j] = (float)(py0 + j) + 0.5f;

    uint32_t my_last[NP];
    float T[NP], g0[NP], g1[NP], g2[NP], ga[NP];
    uint32_t cell_last = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int x = px0 + p % L::CW, y = py0 + p / L::CW;
        my_last[p] = 0u;
        T[p] = 1.0f;
        g0[p] = g1[p] = g2[p] = 0.0f;
        if (x < W && y < H) {
            const int64_t off = (int64_t)y * W + x;
            my_last[p] = n_contrib[off];
            T[p] = final_T[off];
            g0[p] = dimg[off];
            g1[p] = dimg[npix + off];
            g2[p] = dimg[2 * npix + off];
        }
        // g . S, S the colour behind the current entry: the background's
        // share T_final bg, then the blended rgb_j w_j as they are passed
        ga[p] = g0[p] * (T[p] * bg0) + g1[p] * (T[p] * bg1) + g2[p] * (T[p] * bg2);
        cell_last = max(cell_last, my_last[p]);
    }

    __syncthreads();   // the previous tile of a persistent workgroup is done with the shared state
    if (tid == 0) sh.max_last = 0u;
    __syncthreads();
    if (cell_last) atomicMax(&sh.max_last, cell_last);
    __syncthreads();
    // never walk past the tile's list, whatever n_contrib holds
    int hi = (int)min(sh.max_last, rg.y - rg.x);
    const int hi0 = hi;

    // The chunk's candidate values (thread tid < ncand) and this wave's
    // cell masks of them (lane < ncand): loaded here for the first chunk and
    // during the walk of the one before for each later one, so that they
    // are in flight meanwhile, like each chunk's rectangles and first pairs
    // (loaded before its walk, read by its combine).  The loads take
    // clamped indices, not conditions, so the values arrive straight in the
    // registers that read them, with no copy that would wait for them.
    // The records of the values are loaded after each walk, before the
    // combine, whose stores the next chunk's staging then need not wait for.
    uint32_t vk = 0u;
    uint64_t mk = 0ull;
    Rec rk = {};
    // Each chunk's pair-slot stores are issued after the next chunk has
    // taken its staged records and masks: loads and stores share one
    // counter here, so a wait for those loads behind the stores would
    // also wait for the stores to complete.  ds < 0: nothing pending.
    float4 d0 = make_float4(0.f, 0.f, 0.f, 0.f), d1 = d0;
    float d2 = 0.f;
    int64_t ds = -1;
    if (hi > 0) {
        const int lo0 = hi > kChunk ? hi - kChunk : 0;
        const int last = hi - lo0 - 1;
        vk = a.vals[rg.x + (uint32_t)(lo0 + min(tid, last))];
        if (a.masks) mk = a.masks[(int64_t)(rg.x + (uint32_t)(lo0 + min(lane, last))) * L::WAVES + wv];
        rk = a.rec[vk];
    }
    while (hi > 0) {
        const int lo0 = hi > kChunk ? hi - kChunk : 0;
        const int ncand = hi - lo0;
        __syncthreads();   // the previous chunk's slots and staged entries are no longer read
        if (tid < ncand) {
            sh.s[tid] = stage_rec(rk);
            sh.gid[tid] = vk;
        }
        __syncthreads();

        // entry-major cell masks of this wave, transposed into the lane's
        // walk word, cut at the cell's last contributor, and back
        const uint64_t m = lane < ncand ? (a.masks ? mk : cell_mask<L>(sh.s[lane], x0, wy0)) : 0ull;
        if (ds >= 0) {   // the previous chunk's pair slot
            a.pg8[2 * ds] = d0;
            a.pg8[2 * ds + 1] = d1;
            a.pg1[ds] = d2;
            ds = -1;
        }
        uint64_t walk = transpose64(m, lane);
        {
            const int lim = (int)cell_last - lo0;   // entries lo0 + k with k < lim
            walk = lim <= 0 ? 0ull : (lim >= kWave ? walk : (walk & ((1ull << lim) - 1ull)));
        }
        const uint64_t mw = transpose64(walk, lane);
        sh.mask[wv][lane] = mw;
        sh.base[wv][lane] = (uint32_t)__popcll(mw);
        __syncthreads();

        // one thread per candidate: its items, the chunk (the candidates from
        // the top whose items fit), and the first slot of each (wave, entry)
        if (wv == 0) {
            uint32_t tot = 0;
#pragma unroll
            for (int w = 0; w < L::WAVES; ++w) tot += sh.base[w][lane];
            // inclusive suffix sum over the candidates above (k >= lane)
            uint32_t suf = tot;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t y = (uint32_t)__shfl_down((int)suf, d, kWave);
                if (lane + d < kWave) suf += y;
            }
            const bool in = lane < ncand && suf <= (uint32_t)CAP;
            const uint64_t inm = __ballot(in);
            if (lane == 0) sh.kmin = inm ? low_bit(inm) : ncand;
            uint32_t b = suf - tot;   // slots of the entries above
#pragma unroll
            for (int w = 0; w < L::WAVES; ++w) {
                const uint32_t c = sh.base[w][lane];
                sh.base[w][lane] = b;
                b += c;
            }
            sh.total[lane] = tot;
        }
        __syncthreads();
        const int kmin = sh.kmin;
        const uint32_t pgid = sh.gid[min(tid, ncand - 1)];
        const uint2 prc = reinterpret_cast<const uint2*>(a.rect)[pgid];
        const uint32_t pfst = a.first[pgid];
        {   // the next chunk's candidates
            const int nhi = lo0 + kmin;
            const int nlo = nhi > kChunk ? nhi - kChunk : 0;
            const int nlast = max(nhi - nlo - 1, 0);
            vk = a.vals[rg.x + (uint32_t)(nlo + min(tid, nlast))];
            if (a.masks) mk = a.masks[(int64_t)(rg.x + (uint32_t)(nlo + min(lane, nlast))) * L::WAVES + wv];
        }

        // walk: entries kmin .. ncand - 1 of the lane's word, from the back.
        // The next entry's staged values and slot base are read from LDS
        // while the current entry is computed (a lane whose word is empty
        // reads entry kmin, which exists, and writes nothing).
        uint64_t wk = kmin >= kWave ? 0ull : (walk & ~((1ull << kmin) - 1ull));
        const uint64_t below = (1ull << lane) - 1ull;
        // one walked entry: its nine sums for the lane's cell, written to
        // the lane's slot
        auto entry = [&](const bool has, const int kk, const Staged& g, const uint32_t sbase, const uint64_t smask) {
            // list position of the entry; past every pixel's last
            // contributor for a lane with nothing to walk
            const uint32_t pos = has ? (uint32_t)(lo0 + kk) : 0xFFFFFFFFu;
            // the forward's exponent: dx (ca dx + cb dy) + cc dy^2, the dy
            // terms once per pixel row
            float dxs[L::CW], dys[L::CH], rb[L::CH], rc[L::CH];
#pragma unroll
            for (int i = 0; i < L::CW; ++i) dxs[i] = (fxp[i] - g.geo.x) - g.geo.y;
#pragma unroll
            for (int j = 0; j < L::CH; ++j) {
                dys[j] = (fyp[j] - g.geo.z) - g.geo.w;
                rb[j] = g.coef.y * dys[j];
                rc[j] = (g.coef.z * dys[j]) * dys[j];
            }
            // the cell's sums: dL/do, dL/drgb, and dL/dpower per pixel
            float s5 = 0.f, s6 = 0.f, s7 = 0.f, s8 = 0.f, dpow[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int i = p % L::CW, j = p / L::CW;
                float alpha, G, Ts;
                bool capped, above;
                const bool listed = pos < my_last[p];
                if (STORED) {
                    const int pix = (py0 + j - y0) * L::TW + (px0 + i - x0);
                    const float2 st = listed ? a.state[(int64_t)(rg.x + pos) * L::NT + pix] : make_float2(0.f, 0.f);
                    alpha = fabsf(st.x);
                    capped = st.x < 0.0f;
                    above = alpha > 0.0f;
                    G = alpha * __builtin_amdgcn_rcpf(g.coef.w);
                    Ts = st.y;
                } else {
                    // the forward's decision: alpha (capped at 0.99) counts
                    // when the exponent is not positive and alpha >= 1/255
                    const float pw = __builtin_fmaf(dxs[i], __builtin_fmaf(g.coef.x, dxs[i], rb[j]), rc[j]);
                    G = __builtin_amdgcn_exp2f(pw);
                    const float araw = g.coef.w * G;
                    capped = araw > kAlphaMax;
                    alpha = capped ? kAlphaMax : araw;
                    above = pw <= 0.0f && alpha >= kAlphaMin;
                    Ts = 0.0f;
                }
                // Branch-free: a pair that does not contribute gets alpha 0,
                // which leaves T and the suffix colour unchanged and makes
                // every gradient term 0.
                const bool contrib = listed && above;
                const float al = contrib ? alpha : 0.0f;
                const float iom = __builtin_amdgcn_rcpf(1.0f - al);
                const float Ti = STORED ? (contrib ? Ts : T[p]) : T[p] * iom;
                const float w = al * Ti;
                const float grgb = __builtin_fmaf(g2[p], g.col.z, __builtin_fmaf(g1[p], g.col.y, g0[p] * g.col.x));
                // dL/dalpha = g . (rgb T_i - S_i / (1 - alpha)), S_i = suffix colour + T_final bg;
                // no gradient through a capped alpha
                const float da0 = __builtin_fmaf(grgb, Ti, -(ga[p] * iom));
                const float da = (contrib && !capped) ? da0 : 0.0f;
                ga[p] = __builtin_fmaf(grgb, w, ga[p]);
                T[p] = Ti;
                s6 = __builtin_fmaf(g0[p], w, s6);
                s7 = __builtin_fmaf(g1[p], w, s7);
                s8 = __builtin_fmaf(g2[p], w, s8);
                s5 = __builtin_fmaf(da, G, s5);
                dpow[p] = da * al;
            }
            // moments of dL/dpower over the pixel offsets (the centre and
            // conic gradients are linear in them, formed at the flush):
            // s0 = sum dpow dx, s1 = sum dpow dy, s2 = sum dpow dx^2,
            // s3 = sum dpow dx dy, s4 = sum dpow dy^2, from the cell's
            // column sums (plain and dy-weighted) and row sums
            float cs[L::CW], csy[L::CW], rs[L::CH];
#pragma unroll
            for (int i = 0; i < L::CW; ++i) {
                cs[i] = dpow[i];
                csy[i] = dpow[i] * dys[0];
#pragma unroll
                for (int j = 1; j < L::CH; ++j) {
                    cs[i] += dpow[j * L::CW + i];
                    csy[i] = __builtin_fmaf(dpow[j * L::CW + i], dys[j], csy[i]);
                }
            }
#pragma unroll
            for (int j = 0; j < L::CH; ++j) {
                rs[j] = dpow[j * L::CW];
#pragma unroll
                for (int i = 1; i < L::CW; ++i) rs[j] += dpow[j * L::CW + i];
            }
            float s0 = dxs[0] * cs[0], s1 = dys[0] * rs[0];
            float s2 = s0 * dxs[0], s3 = dxs[0] * csy[0], s4 = s1 * dys[0];
#pragma unroll
            for (int i = 1; i < L::CW; ++i) {
                const float t = dxs[i] * cs[i];
                s0 += t;
                s2 = __builtin_fmaf(t, dxs[i], s2);
                s3 = __builtin_fmaf(dxs[i], csy[i], s3);
            }
#pragma unroll
            for (int j = 1; j < L::CH; ++j) {
                const float u = dys[j] * rs[j];
                s1 += u;
                s4 = __builtin_fmaf(u, dys[j], s4);
            }
            if (has) {
                const uint32_t slot = sbase + (uint32_t)__popcll(smask & below);
                sh.item[0][slot] = s0;
                sh.item[1][slot] = s1;
                sh.item[2][slot] = s2;
                sh.item[3][slot] = s3;
                sh.item[4][slot] = s4;
                sh.item[5][slot] = s5;
                sh.item[6][slot] = s6;
                sh.item[7][slot] = s7;
                sh.item[8][slot] = s8;
            }
        };
        if (__ballot(wk != 0ull) != 0ull) {
            // two entries per trip, each reading the next one's values
            // into the other register set
            int kk = wk != 0ull ? high_bit(wk) : kmin;
            Staged g = staged_at(sh.s, kk);
            uint32_t sbase = sh.base[wv][kk];
            uint64_t smask = sh.mask[wv][kk];
            for (;;) {
                bool has = wk != 0ull;
                wk &= ~(1ull << kk);
                const int kn = wk != 0ull ? high_bit(wk) : kmin;
                const Staged gn = staged_at(sh.s, kn);
                const uint32_t sbn = sh.base[wv][kn];
                const uint64_t smn = sh.mask[wv][kn];
                entry(has, kk, g, sbase, smask);
                if (__ballot(wk != 0ull) == 0ull) break;
                has = wk != 0ull;
                wk &= ~(1ull << kn);
                kk = wk != 0ull ? high_bit(wk) : kmin;
                g = staged_at(sh.s, kk);
                sbase = sh.base[wv][kk];
                smask = sh.mask[wv][kk];
                entry(has, kn, gn, sbn, smn);
                if (__ballot(wk != 0ull) == 0ull) break;
            }
        }
        rk = a.rec[vk];
        __syncthreads();

        // the accumulated sums of dpow dx, dpow dy, dpow dx^2, dpow dx dy,
        // dpow dy^2, dL/do, dL/drgb give, with
        // power = -(A dx^2 + C dy^2)/2 - B dx dy and dx = x - u:
        // du = sum dpow (A dx + B dy), dv = sum dpow (B dx + C dy),
        // dA = -sum dpow dx^2 / 2, dB = -sum dpow dx dy, dC = -sum dpow dy^2 / 2,
        // where A = -2 ca / log2e, B = -cb / log2e, C = -2 cc / log2e.
        // One thread per entry adds the entry's slots in order and writes
        // its pair slot (no atomics).
        if (tid >= kmin && tid < ncand) {
            const uint32_t b = sh.base[0][tid], n = sh.total[tid];
            float m[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) m[c] = 0.0f;
            for (uint32_t e = b; e < b + n; ++e) {
#pragma unroll
                for (int c = 0; c < 9; ++c) m[c] += sh.item[c][e];
            }
            {   // every entry's pair slot is written, zero sums included
                const int rx = (int)(prc.x & 0xFFFFu), ry = (int)(prc.x >> 16), rz = (int)(prc.y & 0xFFFFu);
                const int64_t p = (int64_t)pfst + (int64_t)(ty - ry) * (rz - rx) + (tx - rx);
                if (p >= 0 && p < a.cap) {
                    const float4 cf = sh.s[tid].coef;
                    const float A = -2.0f * cf.x * (1.0f / kLog2e), Bc = -cf.y * (1.0f / kLog2e),
                                C = -2.0f * cf.z * (1.0f / kLog2e);
                    d0 = make_float4(A * m[0] + Bc * m[1], Bc * m[0] + C * m[1], -0.5f * m[2], -m[3]);
                    d1 = make_float4(-0.5f * m[4], m[5], m[6], m[7]);
                    d2 = m[8];
                    ds = p;
                }
            }
        }
        hi = lo0 + kmin;
    }
    if (ds >= 0) {
        a.pg8[2 * ds] = d0;
        a.pg8[2 * ds + 1] = d1;
        a.pg1[ds] = d2;
    }
    // Entries behind every pixel's last contributor were never staged:
    // their pair slots get zeros here, so that every pair of the frame is
    // written by its tile's workgroup and the gather needs no cleared buffer.
    const int nlist = (int)(rg.y - rg.x);
    for (int e = hi0 + tid; e < nlist; e += L::NCELL) {
        const uint32_t gid = a.vals[rg.x + (uint32_t)e];
        const ushort4 r = a.rect[gid];
        const int64_t p = (int64_t)a.first[gid] + (int64_t)(ty - (int)r.y) * ((int)r.z - (int)r.x) + (tx - (int)r.x);
        if (p >= 0 && p < a.cap) {
            a.pg8[2 * p] = make_float4(0.f, 0.f, 0.f, 0.f);
            a.pg8[2 * p + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
            a.pg1[p] = 0.f;
        }
    }
}

template <class L, bool STORED>
__global__ __launch_bounds__(L::NCELL) void k_render_bwd(BwdArgs a) {
    __shared__ BwdShared<L, kItemCap> sh;
    uint32_t tile = blockIdx.x;
    if (a.torder) {
        if (blockIdx.x >= *a.torder_n) return;
        tile = a.torder[blockIdx.x];
    }
    bwd_tile<L, STORED, kItemCap>(a, tile, sh);
}

template <class L, int CAP>
__global__ __launch_bounds__(L::NCELL) void k_render_bwd_persistent(BwdArgs a) {
    __shared__ BwdShared<L, CAP> sh;
    __shared__ uint32_t s_next;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_next = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t q = s_next;
        if (q >= a.n_tiles) break;
        bwd_tile<L, false, CAP>(a, a.order ? a.order[q] : q, sh);
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
void launch_t(const BwdArgs& a, int persistent_grid, int cap, hipStream_t st) {
    using L = typename CellsFor<TW, TH>::L;
    const dim3 block(L::NCELL);
    if (a.state)
        hipLaunchKernelGGL((k_render_bwd<L, true>), dim3(a.n_tiles), block, 0, st, a);
    else if (persistent_grid > 0 && cap == kItemCapSmall && kItemCapSmall >= L::NCELL)
        hipLaunchKernelGGL((k_render_bwd_persistent<L, (kItemCapSmall >= L::NCELL ? kItemCapSmall : kItemCap)>),
                           dim3(persistent_grid), block, 0, st, a);
    else if (persistent_grid > 0)
        hipLaunchKernelGGL((k_render_bwd_persistent<L, kItemCap>), dim3(persistent_grid), block, 0, st, a);
    else
        hipLaunchKernelGGL((k_render_bwd<L, false>), dim3(a.n_tiles), block, 0, st, a);
}

template <int TW, int TH>
hipError_t occupancy_t(int* per, int cap) {
    using L = typename CellsFor<TW, TH>::L;
    if (cap == kItemCapSmall && kItemCapSmall >= L::NCELL)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            per, k_render_bwd_persistent<L, (kItemCapSmall >= L::NCELL ? kItemCapSmall : kItemCap)>, L::NCELL, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_render_bwd_persistent<L, kItemCap>, L::NCELL, 0);
}

}  // namespace

size_t pair_grad_bytes(int64_t capacity) { return (size_t)(capacity > 0 ? capacity : 0) * 36; }

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
    a.masks = r.masks;
    a.queue = r.queue;
    a.order = r.order;
    a.n_tiles = r.n_tiles;
    a.torder = r.tile_order;
    a.torder_n = r.tile_order_count;
    const int pg = (r.queue && !state) ? r.persistent_grid : 0;
    if (pg > 0) launch_fill_u32(r.queue, 0u, 1, st);
#define GS_BWD(x, y) launch_t<x, y>(a, pg, r.item_cap, st)
    if (r.tw == 16 && r.th == 16) GS_BWD(16, 16);
    else if (r.tw == 8 && r.th == 8) GS_BWD(8, 8);
    else if (r.tw == 16 && r.th == 8) GS_BWD(16, 8);
    else if (r.tw == 32 && r.th == 8) GS_BWD(32, 8);
    else if (r.tw == 32 && r.th == 16) GS_BWD(32, 16);
    else if (r.tw == 32 && r.th == 32) GS_BWD(32, 32);
#undef GS_BWD
}

int render_item_cap_default() { return kItemCap; }
int render_item_cap_small() { return kItemCapSmall; }

int render_persistent_grid_bwd(int tw, int th, int cap) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
    if (tw == 16 && th == 16) e = occupancy_t<16, 16>(&per, cap);
    else if (tw == 8 && th == 8) e = occupancy_t<8, 8>(&per, cap);
    else if (tw == 16 && th == 8) e = occupancy_t<16, 8>(&per, cap);
    else if (tw == 32 && th == 8) e = occupancy_t<32, 8>(&per, cap);
    else if (tw == 32 && th == 16) e = occupancy_t<32, 16>(&per, cap);
    else if (tw == 32 && th == 32) e = occupancy_t<32, 32>(&per, cap);
    if (e != hipSuccess || per < 1) per = 1;
    return cus * per;
}

}  // namespace gs
