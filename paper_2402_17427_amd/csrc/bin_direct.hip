// Binning by direct placement: every (Gaussian, tile) pair is written
// straight into its tile's run, then each run is sorted by depth.
//
// VastGaussian (arXiv 2402.17427), section 3: the projected Gaussians are
// assigned to the screen tiles their support touches, and every tile's list
// is ordered by depth before the blend.  The tile of each pair is known
// before any pair exists (the Gaussian's tile rectangle from the
// projection), so for views of at most kDirectMaxTiles tiles each no radix
// sort over the tile bits is needed.  Each view (one for the plain calls,
// several for the batched cells and the render server) is cut into blocks
// of consecutive record slots, at most 256 per view:
//   k_dcount    per block: its pairs per tile of its view (an LDS
//               histogram) -> one row of the view's count matrix
//               [blocks][tiles], and its pair total
//   k_dscan     per strip of 64 tiles of a view: exclusive scan down the
//               view's matrix columns (where each block's share of a tile's
//               run starts inside the run), the tile totals, each tile's
//               prefix within the strip and the strip's sum; one more
//               workgroup scans the block totals of all views (each block's
//               first emission position) and stores the grand total
//   k_dscatter  per block: the starts of its view's tiles (every workgroup
//               scans its view's strip sums itself; the view's first also
//               writes the view's ranges, workgroup 0 the pair count and
//               capacity status), every slot's emission position (`first`,
//               the exclusive prefix of the tile counts), and each pair
//               (depth bits << 32 | slot) written at the block's cursor in
//               the tile's run (LDS atomics, so the order inside a block's
//               share of a run is arbitrary)
//   k_dsort     one wave per run of at most 1024 pairs: stable LDS radix
//               passes over the depth bytes that vary in the run; entries
//               of equal depth are then put in index order (odd-even
//               transposition, or for long groups a second sort on (depth,
//               index), index bytes first), so the order never depends on
//               the scatter's; the sorted keys (global tile << 32 | depth
//               bits) and values are written out.  In the same launch an
//               extra first workgroup writes the blend order (longest list
//               first), and the last workgroups (one per 1025 pairs of
//               capacity, at most one per tile) sort the runs of more than
//               1024 pairs: stable passes over global memory on depth, the
//               same equal-depth fix, or the full (depth, index) sort
// The output -- keys, values, ranges, `first`, pair count, status and tile
// order -- is exactly that of the emission + stable sort of the whole key
// (global tile, then depth; equal keys in emission, i.e. slot, order).
#include <algorithm>
#include <cstring>

#include "kernels.h"
#include "tile_order.h"

namespace gs {

namespace {

constexpr int kDThreads = 1024;
constexpr int kDWaves = kDThreads / kWave;
constexpr int kDPer = 4;            // consecutive Gaussians per thread and round
constexpr int kDMaxBlocks = 256;    // blocks (count-matrix rows) per view: one per CU
constexpr int64_t kDMinChunk = 2048;  // fewest slots per block
constexpr int kDRadix = 256;
constexpr int kDSortWaves = 4;
constexpr int kDSortCap = 1024;     // longest run sorted in LDS
constexpr int kDLongThreads = 256;
constexpr int kDFixPhases = 16;     // odd-even phases for equal depths before a full re-sort

// Exclusive scan over the NT threads of a workgroup; *total = the sum.
template <int NT>
__device__ __forceinline__ uint64_t block_scan_ex(uint64_t v, uint64_t* total) {
    __shared__ uint64_t wsum[NT / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / kWave; ++k) {
        const uint64_t s = wsum[k];
        if (k < w) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// A Gaussian's tile rectangle cut to the view's grid (a no-op for the
// rectangles the projection writes for the same tile shape; it keeps the
// placement inside the runs for any input).
__device__ __forceinline__ ushort4 grid_rect(ushort4 r, int ntx, int nty) {
    r.z = (unsigned short)min((int)r.z, ntx);
    r.w = (unsigned short)min((int)r.w, nty);
    if (r.x >= r.z || r.y >= r.w) r = make_ushort4(0, 0, 0, 0);
    return r;
}

__device__ __forceinline__ uint32_t rect_area(const ushort4 r) {
    return (uint32_t)(r.z - r.x) * (uint32_t)(r.w - r.y);
}

// The block's record slots [g0, g1) within its view.
__device__ __forceinline__ void block_range(const DView& V, int lb, int64_t* g0, int64_t* g1) {
    const int64_t a = V.s0 + (int64_t)lb * V.chunk;
    *g0 = a < V.s1 ? a : V.s1;
    *g1 = a + V.chunk < V.s1 ? a + V.chunk : V.s1;
}

// The view of block b / of strip c (uniform per workgroup).  With one view
// (MULTI = false) it is the one in the kernel arguments, read with scalar
// loads; with several, the device table is searched (views in slot order).
template <bool MULTI>
__device__ __forceinline__ DView view_of_block(const DTab& t, int b) {
    if (!MULTI) return t.one;
    int lo = 0, hi = t.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.dev[mid].b0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return t.dev[lo];
}
template <bool MULTI>
__device__ __forceinline__ DView view_of_strip(const DTab& t, int c) {
    if (!MULTI) return t.one;
    int lo = 0, hi = t.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.dev[mid].c0 <= c) lo = mid;
        else hi = mid - 1;
    }
    return t.dev[lo];
}

template <bool MULTI>
__global__ __launch_bounds__(kDThreads) void k_dcount(DTab views, const ushort4* __restrict__ rect,
                                                      uint32_t* __restrict__ M, uint64_t* __restrict__ bsum) {
    extern __shared__ uint32_t s_hist[];
    const int tid = threadIdx.x;
    const DView V = view_of_block<MULTI>(views, (int)blockIdx.x);
    const int lb = (int)blockIdx.x - V.b0;
    const uint32_t n_tiles = V.n_tiles;
    const int ntx = V.ntx, nty = V.nty;
    for (uint32_t t = tid; t < n_tiles; t += kDThreads) s_hist[t] = 0u;
    __syncthreads();
    int64_t g0, g1;
    block_range(V, lb, &g0, &g1);
    uint64_t pairs = 0;
    for (int64_t base = g0; base < g1; base += (int64_t)kDThreads * kDPer) {
        // kDPer Gaussians per thread, strided by the workgroup (coalesced),
        // all loaded before any is counted
        ushort4 r[kDPer];
#pragma unroll
        for (int k = 0; k < kDPer; ++k) {
            const int64_t i = base + k * kDThreads + tid;
            r[k] = i < g1 ? rect[i] : make_ushort4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < kDPer; ++k) {
            r[k] = grid_rect(r[k], ntx, nty);
            pairs += rect_area(r[k]);
            for (int ty = r[k].y; ty < r[k].w; ++ty)
                for (int tx = r[k].x; tx < r[k].z; ++tx) atomicAdd(&s_hist[ty * ntx + tx], 1u);
        }
    }
    __syncthreads();
    uint32_t* row = M + V.m0 + (int64_t)lb * n_tiles;
    for (uint32_t t = tid; t < n_tiles; t += kDThreads) row[t] = s_hist[t];
    uint64_t tot;
    block_scan_ex<kDThreads>(pairs, &tot);
    if (tid == 0) bsum[blockIdx.x] = tot;
}

// The block that comes r-th in a tile's run.  Workgroups are dealt to the
// eight XCDs in turn (block b runs on XCD b mod 8), so the blocks are taken
// XCD by XCD: the blocks of one XCD then write one contiguous stretch of
// every run, and its L2 fills whole cache lines before it writes them back
// (in plain block order every placed pair would be a partial line of its
// own, written back to HBM alone).  r and the result count from the view's
// first block; which XCD comes first does not matter.
__device__ __forceinline__ int xcd_major_block(int r, int nb) {
    constexpr int X = 8;
    const int q = nb / X, rem = nb % X;   // XCDs x < rem hold q + 1 blocks, the others q
    int x, j;
    if (r < (q + 1) * rem) {
        x = r / (q + 1);
        j = r % (q + 1);
    } else {
        const int r2 = r - (q + 1) * rem;
        x = rem + r2 / q;
        j = r2 % q;
    }
    return x + X * j;
}

// Workgroup c < strips: tiles 64 c' .. 64 c' + 63 of its view (one per
// lane), the view's matrix rows split over the 16 waves (in XCD-major block
// order); the last workgroup scans the block totals of all views (each
// block's first emission position) and stores the grand total after them.
template <bool MULTI>
__global__ __launch_bounds__(kDThreads) void k_dscan(DTab views, int strips, int nb_all, uint32_t* __restrict__ M,
                                                     uint32_t* __restrict__ ttot, uint32_t* __restrict__ tex,
                                                     uint32_t* __restrict__ stot, uint64_t* __restrict__ bsum) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    if ((int)blockIdx.x == strips) {
        uint64_t carry = 0;
        for (int b0 = 0; b0 < nb_all; b0 += kDThreads) {
            const int b = b0 + tid;
            const uint64_t v = b < nb_all ? bsum[b] : 0u;
            uint64_t tot;
            const uint64_t ex = carry + block_scan_ex<kDThreads>(v, &tot);
            if (b < nb_all) bsum[b] = ex;
            carry += tot;
        }
        if (tid == 0) bsum[nb_all] = carry;
        return;
    }
    const DView V = view_of_strip<MULTI>(views, (int)blockIdx.x);
    const int nb = V.nb;
    const uint32_t n_tiles = V.n_tiles;
    constexpr int kRows = kDMaxBlocks / kDWaves;   // rows per wave
    __shared__ uint32_t s_part[kDWaves][kWave];
    __shared__ int s_row[kDMaxBlocks];   // the block of each place in the runs
    if (tid < nb) s_row[tid] = xcd_major_block(tid, nb);
    __syncthreads();
    const uint32_t t = ((uint32_t)blockIdx.x - (uint32_t)V.c0) * kWave + (uint32_t)lane;
    const uint32_t* Mv = M + V.m0;
    const int r0 = wv * kRows;
    uint32_t v[kRows], s = 0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int r = r0 + k;
        v[k] = (r < nb && t < n_tiles) ? Mv[(int64_t)s_row[r] * n_tiles + t] : 0u;
        s += v[k];
    }
    s_part[wv][lane] = s;
    __syncthreads();
    uint32_t run = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kDWaves; ++w) {
        const uint32_t p = s_part[w][lane];
        if (w < wv) run += p;
        tot += p;
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int r = r0 + k;
        if (r < nb && t < n_tiles) M[V.m0 + (int64_t)s_row[r] * n_tiles + t] = run;
        run += v[k];
    }
    if (wv == 0) {
        // the strip's tile totals: each tile's exclusive prefix within the
        // strip, and the strip's sum (so that a tile's start is its strip's
        // start plus this prefix)
        const uint32_t c = t < n_tiles ? tot : 0u;
        uint32_t x = c;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)x, d, kWave);
            if (lane >= d) x += y;
        }
        if (t < n_tiles) {
            ttot[V.tile_base + t] = c;
            tex[V.tile_base + t] = x - c;
        }
        if (lane == kWave - 1) stot[blockIdx.x] = x;
    }
}

// Every workgroup first forms the starts of its view's tiles itself: the
// view's first pair (the exclusive block prefix at its first block), plus
// the exclusive prefix of the view's strip sums (one workgroup scan), plus
// the tile's prefix within its strip; the grand total after the block
// totals decides the capacity.  The view's first workgroup writes the
// view's ranges, workgroup 0 the pair count and status.
template <bool MULTI>
__global__ __launch_bounds__(kDThreads) void k_dscatter(DTab views, const ushort4* __restrict__ rect,
                                                        const float* __restrict__ depth,
                                                        const uint32_t* __restrict__ M,
                                                        const uint32_t* __restrict__ ttot,
                                                        const uint32_t* __restrict__ tex,
                                                        const uint32_t* __restrict__ stot, int nb_all,
                                                        int64_t capacity, const uint64_t* __restrict__ bsum,
                                                        uint32_t* __restrict__ ranges,
                                                        uint32_t* __restrict__ pair_count,
                                                        int32_t* __restrict__ status,
                                                        uint32_t* __restrict__ first, uint64_t* __restrict__ pairs,
                                                        bool vec) {
    extern __shared__ uint32_t s_cur[];
    const int tid = threadIdx.x;
    const DView V = view_of_block<MULTI>(views, (int)blockIdx.x);
    const int lb = (int)blockIdx.x - V.b0;
    const uint32_t n_tiles = V.n_tiles;
    const int ntx = V.ntx, nty = V.nty;
    const uint64_t total = bsum[nb_all];
    const bool over = total > (uint64_t)capacity;
    // the tile starts: the view's first pair, plus its strips' exclusive
    // prefix (one workgroup scan over at most 512 strip sums), plus each
    // tile's prefix within its strip
    __shared__ uint32_t s_sp[kDirectMaxTiles / kWave];
    const int nstr = (int)((n_tiles + kWave - 1) / kWave);
    {
        const uint32_t v = tid < nstr ? stot[V.c0 + tid] : 0u;
        uint64_t tot;
        const uint64_t ex = bsum[V.b0] + block_scan_ex<kDThreads>(v, &tot);   // after the earlier views' pairs
        if (tid < nstr) s_sp[tid] = (uint32_t)ex;
    }
    __syncthreads();
    for (uint32_t t = tid; t < n_tiles; t += kDThreads) {
        const uint32_t st = s_sp[t >> 6] + tex[V.tile_base + t];
        s_cur[t] = st;
        // the view's first workgroup writes its ranges; an empty tile's
        // range is (0, 0), as a range pass over sorted keys leaves it
        if (lb == 0) {
            const uint32_t c = ttot[V.tile_base + t];
            reinterpret_cast<uint2*>(ranges)[V.tile_base + t] =
                (over || c == 0u) ? make_uint2(0u, 0u) : make_uint2(st, st + c);
        }
    }
    if (blockIdx.x == 0 && tid == 0) {
        pair_count[0] = over ? 0u : (uint32_t)total;   // pairs the later stages process
        pair_count[1] = total > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)total;   // pairs needed
        *status = over ? -4 : 0;
    }
    const bool place = !over;
    if (place) {
        const uint32_t* row = M + V.m0 + (int64_t)lb * n_tiles;
        for (uint32_t t = tid; t < n_tiles; t += kDThreads) s_cur[t] += row[t];
    }
    __syncthreads();
    int64_t g0, g1;
    block_range(V, lb, &g0, &g1);
    uint64_t carry = bsum[blockIdx.x];
    for (int64_t base = g0; base < g1; base += (int64_t)kDThreads * kDPer) {
        // kDPer consecutive Gaussians per thread, so that one scan gives
        // every emission position of the round
        // (chunk is a multiple of kDPer = 4, so i0 is, and with the three
        // arrays 16-byte aligned (`vec`) a thread's four rectangles, depths
        // and emission positions are 16-byte vectors, unless the block's
        // range ends inside them)
        const int64_t i0 = base + (int64_t)tid * kDPer;
        const bool whole = vec && i0 + kDPer <= g1;
        ushort4 r[kDPer];
        float z[kDPer];
        if (whole) {
            const uint4 r01 = *reinterpret_cast<const uint4*>(rect + i0);
            const uint4 r23 = *reinterpret_cast<const uint4*>(rect + i0 + 2);
            const uint32_t w[8] = {r01.x, r01.y, r01.z, r01.w, r23.x, r23.y, r23.z, r23.w};
#pragma unroll
            for (int k = 0; k < kDPer; ++k)
                r[k] = make_ushort4((unsigned short)(w[2 * k] & 0xFFFFu), (unsigned short)(w[2 * k] >> 16),
                                    (unsigned short)(w[2 * k + 1] & 0xFFFFu), (unsigned short)(w[2 * k + 1] >> 16));
            const float4 z4 = *reinterpret_cast<const float4*>(depth + i0);
            z[0] = z4.x; z[1] = z4.y; z[2] = z4.z; z[3] = z4.w;
        } else {
#pragma unroll
            for (int k = 0; k < kDPer; ++k) {
                r[k] = i0 + k < g1 ? rect[i0 + k] : make_ushort4(0, 0, 0, 0);
                z[k] = i0 + k < g1 ? depth[i0 + k] : 0.0f;
            }
        }
        uint32_t a[kDPer], s = 0;
#pragma unroll
        for (int k = 0; k < kDPer; ++k) {
            r[k] = grid_rect(r[k], ntx, nty);
            a[k] = rect_area(r[k]);
            s += a[k];
        }
        uint64_t tot;
        uint64_t off = carry + block_scan_ex<kDThreads>(s, &tot);
        carry += tot;
        if (first) {
            uint32_t f[kDPer];
#pragma unroll
            for (int k = 0; k < kDPer; ++k) {
                f[k] = (uint32_t)off;
                off += a[k];
            }
            if (whole) {
                *reinterpret_cast<uint4*>(first + i0) = make_uint4(f[0], f[1], f[2], f[3]);
            } else {
#pragma unroll
                for (int k = 0; k < kDPer; ++k)
                    if (i0 + k < g1) first[i0 + k] = f[k];
            }
        }
#pragma unroll
        for (int k = 0; k < kDPer; ++k) {
            const int64_t i = i0 + k;
            if (i < g1) {
                if (place && a[k]) {
                    const uint64_t hi = (uint64_t)__float_as_uint(z[k]) << 32;
                    for (int ty = r[k].y; ty < r[k].w; ++ty)
                        for (int tx = r[k].x; tx < r[k].z; ++tx) {
                            const uint32_t pos = atomicAdd(&s_cur[ty * ntx + tx], 1u);
                            pairs[pos] = hi | (uint32_t)i;
                        }
                }
            }
        }
    }
}

// One stable LDS radix pass of a wave's run s[0 .. n) on the 8 bits at
// `shift`: items ranked 64 at a time in order (match by the digit's bits
// with ballots, running digit counts), digit offsets from a scan of the
// counts, then each item stored at its place.
template <int IPL>
__device__ __forceinline__ void wave_radix_pass(uint64_t* s, uint32_t* s_cnt, uint32_t n, int nq, int shift,
                                                int lane, uint64_t lt_mask) {
    constexpr int DPL = kDRadix / kWave;   // digits per lane in the offset scan
    uint64_t it[IPL];
    uint32_t rk[IPL];
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const uint32_t idx = (uint32_t)(q * kWave + lane);
        it[q] = (q < nq && idx < n) ? s[idx] : 0ull;
    }
#pragma unroll
    for (int e = 0; e < DPL; ++e) s_cnt[e * kWave + lane] = 0u;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        if (q < nq) {
            const uint32_t idx = (uint32_t)(q * kWave + lane);
            const bool ok = idx < n;
            const uint32_t d = (uint32_t)(it[q] >> shift) & 0xFFu;
            uint64_t mt = __ballot(ok);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t vote = __ballot(bit);
                mt &= bit ? vote : ~vote;
            }
            const uint32_t below = (uint32_t)__popcll(mt & lt_mask);
            const uint32_t old = ok ? s_cnt[d] : 0u;
            rk[q] = old + below;
            __builtin_amdgcn_wave_barrier();
            if (ok && below == 0u) s_cnt[d] = old + (uint32_t)__popcll(mt);
            __builtin_amdgcn_wave_barrier();
        }
    }
    {   // digit offsets: lane l owns digits l*DPL .. l*DPL + DPL - 1
        uint32_t c[DPL], sum = 0;
#pragma unroll
        for (int e = 0; e < DPL; ++e) {
            c[e] = s_cnt[lane * DPL + e];
            sum += c[e];
        }
        uint32_t x = sum;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, kWave);
            if (lane >= d) x += y;
        }
        uint32_t run = x - sum;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int e = 0; e < DPL; ++e) {
            s_cnt[lane * DPL + e] = run;
            run += c[e];
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const uint32_t idx = (uint32_t)(q * kWave + lane);
        if (q < nq && idx < n) {
            const uint32_t d = (uint32_t)(it[q] >> shift) & 0xFFu;
            s[s_cnt[d] + rk[q]] = it[q];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v |= (uint32_t)__shfl_xor((int)v, d, kWave);
    return v;
}

// A run longer than kDSortCap, sorted by all kDLongThreads threads of a
// workgroup on (depth, index): stable 8-bit LSD passes over the depth bytes
// that vary in it, 256 items at a time in order (ballot match ranks within
// a wave, per-wave digit counts order the waves), ping-ponging between the
// placed pairs and the key output; then equal depths put in index order as
// in the short runs (or, for long groups, passes over the index bytes and
// then the depth bytes again); then the keys and values are written.
struct LongLds {
    uint32_t start[kDRadix];   // digit start in the run
    uint32_t run[kDRadix];     // items of each digit placed so far
    uint32_t wc[kDLongThreads / kWave][kDRadix];
    uint32_t w[kDRadix / kWave];
    uint32_t vary[2];
    uint32_t list[kDLongThreads];   // long runs found in a round
    uint32_t nlist;
};

__device__ __forceinline__ void sort_long_run(uint32_t tile, uint2 r, uint64_t* __restrict__ pa,
                                              uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                              LongLds& L) {
    constexpr int W = kDLongThreads / kWave;
    uint32_t* s_start = L.start;
    uint32_t* s_run = L.run;
    uint32_t (*s_wc)[kDRadix] = L.wc;
    uint32_t* s_w = L.w;
    uint32_t* s_vary = L.vary;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t n = r.y - r.x;
    __syncthreads();   // the previous run's last reads of the shared counts are done
    if (tid < 2) s_vary[tid] = 0u;
    __syncthreads();
    {
        const uint64_t x0 = pa[r.x];
        uint32_t vz = 0, vg = 0;
        for (uint32_t i = tid; i < n; i += kDLongThreads) {
            const uint64_t x = pa[r.x + i];
            vz |= (uint32_t)(x >> 32) ^ (uint32_t)(x0 >> 32);
            vg |= (uint32_t)x ^ (uint32_t)x0;
        }
        vz = wave_or(vz);
        vg = wave_or(vg);
        if (lane == 0) {
            atomicOr(&s_vary[0], vg);
            atomicOr(&s_vary[1], vz);
        }
    }
    __syncthreads();
    const uint64_t vary = ((uint64_t)s_vary[1] << 32) | s_vary[0];
    uint32_t zbytes = 0, gbytes = 0;   // bit p: byte p of the item varies in the run
    for (int p = 0; p < 4; ++p) {
        if ((vary >> (32 + 8 * p)) & 0xFFu) zbytes |= 1u << (4 + p);
        if ((vary >> (8 * p)) & 0xFFu) gbytes |= 1u << p;
    }
    bool in_a = true;
    // one stable pass over byte p, from (in_a ? pa : kout) to the other
    auto pass_over = [&](int p) {
        const int shift = 8 * p;
        const uint64_t* ki = in_a ? pa : kout;
        uint64_t* ko = in_a ? kout : pa;
        // digit counts of the run and their exclusive scan
        s_start[tid] = 0u;
        s_run[tid] = 0u;
        for (int q = 0; q < W; ++q) s_wc[q][tid] = 0u;
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kDLongThreads)
            atomicAdd(&s_start[(uint32_t)(ki[r.x + i] >> shift) & 0xFFu], 1u);
        __syncthreads();
        {
            const uint32_t v = s_start[tid];
            uint32_t x = v;
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t y = __shfl_up(x, d, kWave);
                if (lane >= d) x += y;
            }
            if (lane == kWave - 1) s_w[wv] = x;
            __syncthreads();
            uint32_t base = 0;
            for (int q = 0; q < kDRadix / kWave; ++q)
                if (q < wv) base += s_w[q];
            s_start[tid] = base + x - v;
        }
        __syncthreads();
        for (uint32_t c0 = 0; c0 < n; c0 += kDLongThreads) {
            const uint32_t i = c0 + (uint32_t)tid;
            const bool ok = i < n;
            const uint64_t key = ok ? ki[r.x + i] : 0ull;
            const uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
            uint64_t mt = __ballot(ok);
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t vote = __ballot(bit);
                mt &= bit ? vote : ~vote;
            }
            const uint32_t below = (uint32_t)__popcll(mt & lt_mask);
            if (ok && below == 0u) s_wc[wv][d] = (uint32_t)__popcll(mt);
            __syncthreads();
            if (ok) {
                uint32_t pos = s_start[d] + s_run[d] + below;
                for (int q = 0; q < W; ++q)
                    if (q < wv) pos += s_wc[q][d];
                ko[r.x + pos] = key;
            }
            __syncthreads();
            uint32_t add = 0;
            for (int q = 0; q < W; ++q) {
                add += s_wc[q][tid];
                s_wc[q][tid] = 0u;
            }
            s_run[tid] += add;
            __syncthreads();
        }
        // the next pass reads what this one wrote (same workgroup)
        __threadfence_block();
        __syncthreads();
        in_a = !in_a;
    };
    for (int p = 0; p < 8; ++p)
        if ((zbytes >> p) & 1u) pass_over(p);
    // equal depths into index order by odd-even transposition between
    // equal-depth neighbours (in place); a group too long to settle in
    // kDFixPhases phases sends the run to the full (depth, index) sort,
    // which orders it from whatever order it is in
    {
        uint64_t* X = (in_a ? pa : kout) + r.x;
        int quiet = 0;
        for (int ph = 0; ph < kDFixPhases && quiet < 2; ++ph) {
            bool sw = false;
            for (uint32_t i = 2u * (uint32_t)tid + (uint32_t)(ph & 1); i + 1 < n; i += 2u * kDLongThreads) {
                const uint64_t x = X[i], y = X[i + 1];
                if ((x >> 32) == (y >> 32) && (uint32_t)x > (uint32_t)y) {
                    X[i] = y;
                    X[i + 1] = x;
                    sw = true;
                }
            }
            __threadfence_block();
            quiet = __syncthreads_or(sw) ? 0 : quiet + 1;
        }
        if (quiet < 2)
            for (int p = 0; p < 8; ++p)
                if (((gbytes | zbytes) >> p) & 1u) pass_over(p);
    }
    const uint64_t thi = (uint64_t)tile << 32;
    const uint64_t* src = in_a ? pa : kout;
    for (uint32_t i = tid; i < n; i += kDLongThreads) {
        const uint64_t c = src[r.x + i];   // each thread reads and writes the same index
        kout[r.x + i] = thi | (c >> 32);
        vout[r.x + i] = (uint32_t)c;
    }
}

// Runs of 1 .. kDSortCap pairs, one wave each, four per workgroup.
// With `order` set, an extra first workgroup writes the blend order
// meanwhile (order[0] = the tile count, order[1..] = every tile, longest
// list first).
__global__ __launch_bounds__(kDSortWaves * kWave) void k_dsort(uint64_t* __restrict__ pin,
                                                               uint64_t* __restrict__ kout,
                                                               uint32_t* __restrict__ vout,
                                                               const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                               const int32_t* __restrict__ status,
                                                               uint32_t* __restrict__ order) {
    constexpr int IPL = kDSortCap / kWave;
    static_assert(kDLongThreads == kDSortWaves * kWave, "a long run takes a whole workgroup");
    __shared__ uint64_t s_all[kDSortWaves][kDSortCap];
    __shared__ uint32_t s_cnt_all[kDSortWaves][kDRadix];
    const int first = order ? 1 : 0;
    if (order && blockIdx.x == 0) {
        __shared__ uint32_t s_h[kDSortWaves][kTileClasses + 1];
        tile_order_block<kDSortWaves * kWave>(ranges, n_tiles, order + 1, order, 1, s_h);
        return;
    }
    if (*status != 0) return;
    const uint32_t nshort = (n_tiles + kDSortWaves - 1) / kDSortWaves;
    const uint32_t blk = (uint32_t)blockIdx.x - (uint32_t)first;
    if (blk >= nshort) {
        // long-run workgroup j of nl: the runs above kDSortCap pairs among
        // tiles j, j + nl, j + 2 nl, ..., one after another, with the
        // workgroup's LDS as their counts
        static_assert(sizeof(LongLds) <= sizeof(s_all), "long-run counts fit the run buffers");
        LongLds& L = *reinterpret_cast<LongLds*>(&s_all[0][0]);
        const uint32_t j = blk - nshort, nl = (uint32_t)gridDim.x - (uint32_t)first - nshort;
        for (uint32_t t0 = j; t0 < n_tiles; t0 += nl * kDLongThreads) {
            const uint32_t t = t0 + nl * threadIdx.x;
            bool lg = false;
            if (t < n_tiles) {
                const uint2 rr = ranges[t];
                lg = rr.y - rr.x > (uint32_t)kDSortCap;
            }
            __syncthreads();   // the previous round's list is no longer read
            if (threadIdx.x == 0) L.nlist = 0u;
            __syncthreads();
            if (lg) L.list[atomicAdd(&L.nlist, 1u)] = t;   // any order: each run is sorted on its own
            __syncthreads();
            const uint32_t cnt = L.nlist;
            for (uint32_t q = 0; q < cnt; ++q) {
                const uint32_t tile = L.list[q];
                sort_long_run(tile, ranges[tile], pin, kout, vout, L);
            }
        }
        return;
    }
    const int wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const uint32_t tile = blk * kDSortWaves + (uint32_t)wv;
    if (tile >= n_tiles) return;
    const uint2 r = ranges[tile];
    const uint32_t n = r.y - r.x;
    if (n == 0u || n > (uint32_t)kDSortCap) return;   // longer runs: the long-run workgroups
    const uint64_t thi = (uint64_t)tile << 32;
    if (n == 1u) {
        if (lane == 0) {
            const uint64_t x = pin[r.x];
            kout[r.x] = thi | (x >> 32);
            vout[r.x] = (uint32_t)x;
        }
        return;
    }
    uint64_t* s = s_all[wv];
    uint32_t* s_cnt = s_cnt_all[wv];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int nq = (int)((n + kWave - 1) / kWave);
    const uint64_t x0 = pin[r.x];
    uint32_t vz = 0, vg = 0;   // bits in which the depths / indices of the run differ
    for (uint32_t i = lane; i < n; i += kWave) {
        const uint64_t x = pin[r.x + i];
        s[i] = x;
        vz |= (uint32_t)(x >> 32) ^ (uint32_t)(x0 >> 32);
        vg |= (uint32_t)x ^ (uint32_t)x0;
    }
    vz = wave_or(vz);
    vg = wave_or(vg);
    // bytes of the item to pass over (bit p: bits 8p .. 8p + 7), lowest
    // first; a stable pass over a byte on which the whole run agrees
    // changes nothing, so only the varying ones are taken.  First the depth
    // bytes; if two entries then share a depth (their order so far is the
    // scatter's), the run is reloaded and sorted on (depth, index), index
    // bytes first.  One pass body in a loop keeps the kernel small.
    uint32_t zbytes = 0, gbytes = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        if ((vz >> (8 * p)) & 0xFFu) zbytes |= 1u << (4 + p);
        if ((vg >> (8 * p)) & 0xFFu) gbytes |= 1u << p;
    }
    uint32_t todo = zbytes;
    bool again = true;
    __builtin_amdgcn_wave_barrier();
    for (;;) {
#pragma unroll 1
        while (todo) {
            const int p = __builtin_ctz(todo);
            todo &= todo - 1u;
            wave_radix_pass<IPL>(s, s_cnt, n, nq, 8 * p, lane, lt_mask);
        }
        if (!again) break;
        again = false;
        // neighbours of equal depth into index order by odd-even
        // transposition: comparisons never cross a change of depth, so each
        // group of equal depths is sorted on its own, and two phases in a
        // row without a swap leave every neighbour pair in order; a group
        // too long to settle in kDFixPhases phases sends the run to the
        // full (depth, index) sort
        int quiet = 0;
        for (int ph = 0; ph < kDFixPhases && quiet < 2; ++ph) {
            bool sw = false;
            for (uint32_t i = 2u * (uint32_t)lane + (uint32_t)(ph & 1); i + 1 < n; i += 2u * kWave) {
                const uint64_t a = s[i], b = s[i + 1];
                if ((a >> 32) == (b >> 32) && (uint32_t)a > (uint32_t)b) {
                    s[i] = b;
                    s[i + 1] = a;
                    sw = true;
                }
            }
            __builtin_amdgcn_wave_barrier();
            quiet = __ballot(sw) != 0ull ? 0 : quiet + 1;
        }
        if (quiet >= 2) break;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < n; i += kWave) s[i] = pin[r.x + i];
        __builtin_amdgcn_wave_barrier();
        todo = gbytes | zbytes;
    }
    for (uint32_t i = lane; i < n; i += kWave) {
        const uint64_t c = s[i];
        kout[r.x + i] = thi | (c >> 32);
        vout[r.x + i] = (uint32_t)c;
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Scratch {
    uint32_t* M;      // count matrix: the views' rows
    uint32_t* ttot;   // [n_tiles]: pairs per tile
    uint32_t* tex;    // [n_tiles]: a tile's exclusive prefix within its strip of 64
    uint32_t* stot;   // [strips]: pairs per strip
    uint64_t* bsum;   // [nb + 1]: block totals, then their exclusive prefix and the grand total
};

Scratch carve_scratch(void* ws, const DPlan& plan) {
    Scratch w;
    char* p = static_cast<char*>(ws);
    w.M = reinterpret_cast<uint32_t*>(p);
    p += align256((size_t)(plan.m_words > 0 ? plan.m_words : 1) * 4);
    w.ttot = reinterpret_cast<uint32_t*>(p);
    p += align256((size_t)(plan.n_tiles > 0 ? plan.n_tiles : 1) * 4);
    w.tex = reinterpret_cast<uint32_t*>(p);
    p += align256((size_t)(plan.n_tiles > 0 ? plan.n_tiles : 1) * 4);
    w.stot = reinterpret_cast<uint32_t*>(p);
    p += align256((size_t)(plan.strips > 0 ? plan.strips : 1) * 4);
    w.bsum = reinterpret_cast<uint64_t*>(p);
    return w;
}

// The plan of one view of n Gaussians (slots 0 .. n - 1).
bool single_plan(int64_t n, int ntx, int64_t n_tiles, DView* v, DPlan* plan) {
    const int64_t s0 = 0, s1 = n;
    const int nty = ntx > 0 ? (int)((n_tiles + ntx - 1) / ntx) : 0;
    const uint32_t base = 0;
    return bin_direct_plan(1, &s0, &s1, &ntx, &nty, &base, v, plan);
}

}  // namespace

bool bin_direct_plan(int nv, const int64_t* s0, const int64_t* s1, const int* ntx, const int* nty,
                     const uint32_t* tile_base, DView* out, DPlan* plan) {
    DPlan p;
    p.n_views = nv;
    for (int v = 0; v < nv; ++v) {
        const int64_t nt = (int64_t)ntx[v] * nty[v];
        if (nt <= 0 || nt > kDirectMaxTiles) return false;
        const int64_t slots = s1[v] > s0[v] ? s1[v] - s0[v] : 0;
        int64_t nb = (slots + kDMinChunk - 1) / kDMinChunk;
        if (nb > kDMaxBlocks) nb = kDMaxBlocks;
        if (nb < 1) nb = 1;   // a view without slots still writes its ranges
        int64_t chunk = (slots + nb - 1) / nb;
        chunk = (chunk + kDPer - 1) / kDPer * kDPer;
        if (chunk < kDPer) chunk = kDPer;
        DView& d = out[v];
        d.s0 = s0[v];
        d.s1 = s0[v] + slots;
        d.chunk = chunk;
        d.m0 = p.m_words;
        d.tile_base = tile_base[v];
        d.n_tiles = (uint32_t)nt;
        d.ntx = ntx[v];
        d.nty = nty[v];
        d.b0 = p.nb;
        d.nb = (int)nb;
        d.c0 = p.strips;
        p.nb += (int)nb;
        p.strips += (int)((nt + kWave - 1) / kWave);
        p.m_words += nb * nt;
        p.n_tiles = std::max(p.n_tiles, tile_base[v] + (uint32_t)nt);
        p.max_tiles = std::max(p.max_tiles, (uint32_t)nt);
    }
    *plan = p;
    return nv > 0;
}

size_t bin_direct_scratch_bytes(const DPlan& plan) {
    return align256((size_t)(plan.m_words > 0 ? plan.m_words : 1) * 4) +
           2 * align256((size_t)(plan.n_tiles > 0 ? plan.n_tiles : 1) * 4) +
           align256((size_t)(plan.strips > 0 ? plan.strips : 1) * 4) + align256((size_t)(plan.nb + 1) * 8);
}

void launch_bin_direct_place(const DPlan& plan, const DTab& views, const ushort4* rect, const float* depth,
                             int64_t capacity, uint32_t* first, uint32_t* ranges, uint32_t* pair_count,
                             int32_t* status, void* scratch, uint64_t* pairs, hipStream_t st) {
    const Scratch w = carve_scratch(scratch, plan);
    const size_t lds = (size_t)plan.max_tiles * 4;
    const bool multi = views.dev != nullptr;
    // views start at multiples of 4 slots, so a thread's four slots are
    // 16-byte vectors when the arrays are 16-byte aligned
    const bool vec = ((reinterpret_cast<uintptr_t>(rect) | reinterpret_cast<uintptr_t>(depth) |
                       reinterpret_cast<uintptr_t>(first)) & 15u) == 0;
    if (multi) {
        hipLaunchKernelGGL(k_dcount<true>, dim3((unsigned)plan.nb), dim3(kDThreads), lds, st, views, rect, w.M,
                           w.bsum);
        hipLaunchKernelGGL(k_dscan<true>, dim3((unsigned)plan.strips + 1), dim3(kDThreads), 0, st, views,
                           plan.strips, plan.nb, w.M, w.ttot, w.tex, w.stot, w.bsum);
        hipLaunchKernelGGL(k_dscatter<true>, dim3((unsigned)plan.nb), dim3(kDThreads), lds, st, views, rect, depth,
                           w.M, w.ttot, w.tex, w.stot, plan.nb, capacity, w.bsum, ranges, pair_count, status, first,
                           pairs, vec);
    } else {
        hipLaunchKernelGGL(k_dcount<false>, dim3((unsigned)plan.nb), dim3(kDThreads), lds, st, views, rect, w.M,
                           w.bsum);
        hipLaunchKernelGGL(k_dscan<false>, dim3((unsigned)plan.strips + 1), dim3(kDThreads), 0, st, views,
                           plan.strips, plan.nb, w.M, w.ttot, w.tex, w.stot, w.bsum);
        hipLaunchKernelGGL(k_dscatter<false>, dim3((unsigned)plan.nb), dim3(kDThreads), lds, st, views, rect,
                           depth, w.M, w.ttot, w.tex, w.stot, plan.nb, capacity, w.bsum, ranges, pair_count, status,
                           first, pairs, vec);
    }
}

void launch_bin_direct_sort(uint32_t n_tiles, int64_t capacity, uint64_t* keys, uint32_t* vals,
                            const uint32_t* ranges, const int32_t* status, uint32_t* tile_order,
                            uint64_t* pairs, hipStream_t st) {
    const uint2* rg = reinterpret_cast<const uint2*>(ranges);
    if (capacity == 0) {   // nothing to sort (every range is empty); the order is still kept
        if (tile_order)
            hipLaunchKernelGGL(k_dsort, dim3(1), dim3(kDSortWaves * kWave), 0, st, pairs, keys, vals, rg, n_tiles,
                               status, tile_order);
        return;
    }
    const unsigned blocks = (unsigned)((n_tiles + kDSortWaves - 1) / kDSortWaves) + (tile_order ? 1u : 0u);
    // long-run workgroups after the others: as many as there can be long
    // runs (one per kDSortCap + 1 pairs of capacity, at most one per tile),
    // so that they run side by side
    int64_t lg = capacity / (kDSortCap + 1);
    if (lg > (int64_t)n_tiles) lg = n_tiles;
    hipLaunchKernelGGL(k_dsort, dim3(blocks + (unsigned)lg), dim3(kDSortWaves * kWave), 0, st, pairs, keys, vals,
                       rg, n_tiles, status, tile_order);
}

bool bin_direct_supported(int64_t n_tiles) { return n_tiles > 0 && n_tiles <= kDirectMaxTiles; }

size_t bin_direct_ws_bytes(int64_t n, int64_t capacity, int64_t n_tiles) {
    // the sizes depend on n and the tile count only, not on the grid's shape
    DView v;
    DPlan plan;
    if (!single_plan(n, 1, n_tiles, &v, &plan)) return 0;
    return bin_direct_scratch_bytes(plan) + align256((size_t)(capacity > 0 ? capacity : 0) * 8);
}

void launch_bin_direct_place(int64_t n, const ushort4* rect, const float* depth, int ntx, int64_t n_tiles,
                             int64_t capacity, uint32_t* first, uint32_t* ranges, uint32_t* pair_count,
                             int32_t* status, void* ws, hipStream_t st) {
    DTab t;
    std::memset(&t, 0, sizeof t);
    DPlan plan;
    if (!single_plan(n, ntx, n_tiles, &t.one, &plan)) return;
    t.n = 1;
    uint64_t* pairs = reinterpret_cast<uint64_t*>(static_cast<char*>(ws) + bin_direct_scratch_bytes(plan));
    launch_bin_direct_place(plan, t, rect, depth, capacity, first, ranges, pair_count, status, ws, pairs, st);
}

void launch_bin_direct_sort(int64_t n, int64_t n_tiles, int64_t capacity, uint64_t* keys, uint32_t* vals,
                            const uint32_t* ranges, const int32_t* status, uint32_t* tile_order, void* ws,
                            hipStream_t st) {
    DView v;
    DPlan plan;
    if (!single_plan(n, 1, n_tiles, &v, &plan)) return;
    uint64_t* pairs = reinterpret_cast<uint64_t*>(static_cast<char*>(ws) + bin_direct_scratch_bytes(plan));
    launch_bin_direct_sort((uint32_t)n_tiles, capacity, keys, vals, ranges, status, tile_order, pairs, st);
}

}  // namespace gs
