// Stable LSD radix sort of (uint64 key, uint32 value) pairs, onesweep form.
//
// VastGaussian (arXiv 2402.17427), section 3: the (Gaussian, tile) pairs are
// sorted by tile and, within a tile, by depth.  The key is
// (tile << 32) | float32 bits of the (positive) depth, so an unsigned
// integer sort gives both orders at once; the sort must be stable so that
// equal keys keep the Gaussian-index order in which they were emitted.
//
// Structure (8-bit digits, one kernel per digit pass):
//   k_sort_clear  zero the digit histograms, partition counters and
//                 look-back words of the passes to run, for the pair count
//                 on the device (in the binning sort the key emission's
//                 first kernel does this instead)
//   k_hist        one read of every key builds the histograms of all
//                 passes at once (LDS atomics, then one global atomic per
//                 non-empty bin and workgroup; few, large workgroups, since
//                 the global atomics on the same bins serialise)
//   k_onesweep    per pass: every workgroup first scans the pass's 256
//                 bins into global digit offsets, then takes the next
//                 partition of 4096 keys from an atomic counter, ranks its
//                 keys stably with wave64 ballots (match-by-digit),
//                 publishes its digit counts and resolves its global
//                 offsets by decoupled look-back over the earlier
//                 partitions (a window of eight per step, so the walk is
//                 not one dependent load per partition), sorts the
//                 partition locally in LDS and writes it out digit run by
//                 digit run (coalesced).
// The pair count stays on the device; grids are sized for the capacity
// and surplus workgroups find no partition and exit.
#include "kernels.h"
#include "tile_order.h"

namespace gs {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kIPT = 16;                        // keys per lane per partition
constexpr int kWavePart = kWave * kIPT;         // 1024
constexpr int kPart = kSortThreads * kIPT;      // 4096 keys per partition
constexpr int kRadix = 256;
constexpr int kMaxPasses = 8;
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1u;
constexpr int kMaxGrid = 2048;
constexpr int kLook = 8;                        // look-back window (partitions per step)
constexpr int kHistThreads = 1024;
constexpr int kHistGrid = 128;                  // at most: fewer flushes of the same bins

struct SortWs {
    int64_t capacity;    // pairs the buffers hold; the device count is clamped to it
    uint32_t* hist;      // [passes][256]: counts, then exclusive offsets
    uint32_t* counter;   // [passes]: next partition id
    uint32_t* look;      // [passes][max_parts][256]: look-back words
    int64_t max_parts;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SortWs carve(void* ws, int64_t capacity, int passes) {
    SortWs s;
    char* p = static_cast<char*>(ws);
    s.capacity = capacity;
    s.max_parts = (capacity + kPart - 1) / kPart;
    s.hist = reinterpret_cast<uint32_t*>(p);
    p += align256((size_t)kMaxPasses * kRadix * 4);
    s.counter = reinterpret_cast<uint32_t*>(p);
    p += align256((size_t)kMaxPasses * 4);
    s.look = reinterpret_cast<uint32_t*>(p);
    (void)passes;
    return s;
}

__device__ __forceinline__ int64_t clamp_count(const uint32_t* count, int64_t capacity) {
    const int64_t c = *count;
    return c < capacity ? c : capacity;
}

// Zero the histograms, partition counters and look-back words of passes
// p0 .. p1-1 for the pair count on the device, and zero_count words of
// `zero` (saves the caller a launch).
__global__ __launch_bounds__(256) void k_sort_clear(SortWs w, const uint32_t* __restrict__ count, int p0, int p1,
                                                    uint32_t* __restrict__ zero, int64_t zero_count) {
    const int64_t P = clamp_count(count, w.capacity);
    const int64_t parts = ((int64_t)P + kPart - 1) / kPart;
    const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
    for (int64_t j = tid; j < zero_count; j += stride) zero[j] = 0u;   // a caller's buffer (tile ranges)
    for (int64_t j = p0 * kRadix + tid; j < (int64_t)p1 * kRadix; j += stride) w.hist[j] = 0u;
    for (int64_t j = p0 + tid; j < p1; j += stride) w.counter[j] = 0u;
    for (int p = p0; p < p1; ++p)
        for (int64_t j = tid; j < parts * kRadix; j += stride) w.look[(int64_t)p * w.max_parts * kRadix + j] = 0u;
}

// Digit histograms of passes p0 .. p1-1 in one read of the keys.
__global__ __launch_bounds__(kHistThreads) void k_hist(const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ count, int p0, int p1, SortWs w) {
    __shared__ uint32_t h[kMaxPasses * kRadix];
    for (int j = threadIdx.x; j < kMaxPasses * kRadix; j += kHistThreads) h[j] = 0u;
    __syncthreads();
    const int64_t P = clamp_count(count, w.capacity);
    // eight keys per thread are loaded before any is counted, so that a
    // thread waits for memory once per eight keys (each load instruction
    // still reads consecutive keys across the workgroup)
    constexpr int kLoads = 8;
    const int64_t stride = (int64_t)gridDim.x * kHistThreads;
    for (int64_t i0 = (int64_t)blockIdx.x * kHistThreads + threadIdx.x; i0 < P; i0 += stride * kLoads) {
        uint64_t k[kLoads];
#pragma unroll
        for (int j = 0; j < kLoads; ++j) {
            const int64_t i = i0 + j * stride;
            k[j] = i < P ? keys[i] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < kLoads; ++j) {
            if (i0 + j * stride >= P) break;
            for (int p = p0; p < p1; ++p) atomicAdd(&h[p * kRadix + (uint32_t)((k[j] >> (8 * p)) & 0xFF)], 1u);
        }
    }
    __syncthreads();
    for (int j = p0 * kRadix + threadIdx.x; j < p1 * kRadix; j += kHistThreads)
        if (h[j]) atomicAdd(&w.hist[j], h[j]);
}

__device__ __forceinline__ uint64_t ballot64(bool b) { return __ballot(b); }

__global__ __launch_bounds__(kSortThreads) void k_onesweep(const uint64_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                           const uint32_t* __restrict__ count, int pass, SortWs w) {
    __shared__ uint64_t s_keys[kPart];
    __shared__ uint32_t s_vals[kPart];
    __shared__ uint32_t s_whist[kSortWaves][kRadix];  // per-wave counts, then per-wave offsets
    __shared__ uint32_t s_lofs[kRadix];               // digit start within the partition
    __shared__ uint32_t s_dbase[kRadix];              // digit start in the output
    __shared__ uint32_t s_scan[kSortWaves];
    __shared__ int64_t s_part;

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int shift = 8 * pass;
    const int64_t P = clamp_count(count, w.capacity);
    const int64_t nparts = (P + kPart - 1) / kPart;
    uint32_t* look = w.look + (int64_t)pass * w.max_parts * kRadix;
    // exclusive scan of this pass's digit counts (thread t owns digit t):
    // each workgroup forms the global digit offsets itself
    __shared__ uint32_t s_goff[kRadix];
    {
        const uint32_t v = w.hist[pass * kRadix + tid];
        uint32_t x = v;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, kWave);
            if (lane >= d) x += y;
        }
        if (lane == kWave - 1) s_scan[wv] = x;
        __syncthreads();
        uint32_t b = 0;
#pragma unroll
        for (int q = 0; q < kSortWaves; ++q)
            if (q < wv) b += s_scan[q];
        s_goff[tid] = b + x - v;
        __syncthreads();
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // When the grid covers every partition, workgroup b takes partition b
    // (workgroups are dispatched in index order, so the partitions a
    // look-back waits for are already running or done); otherwise they are
    // handed out in order by an atomic counter.
    const bool one_each = (int64_t)gridDim.x >= nparts;
    for (int round = 0;; ++round) {
        if (one_each) {
            if (round > 0) break;
            s_part = (int64_t)blockIdx.x;
        } else if (tid == 0) {
            s_part = (int64_t)atomicAdd(&w.counter[pass], 1u);
        }
        __syncthreads();
        const int64_t part = s_part;
        if (part >= nparts) break;
        const int64_t base = part * kPart;
        const int nvalid = (int)((P - base) < kPart ? (P - base) : kPart);

        for (int j = lane; j < kRadix; j += kWave) s_whist[wv][j] = 0u;

        uint64_t key[kIPT];
        uint32_t val[kIPT];
        uint32_t rank[kIPT];
        const int64_t wbase = base + (int64_t)wv * kWavePart;
#pragma unroll
        for (int k = 0; k < kIPT; ++k) {
            const int64_t idx = wbase + k * kWave + lane;
            const bool ok = idx < P;
            key[k] = ok ? kin[idx] : ~0ull;
            val[k] = ok ? vin[idx] : 0u;
        }
        __builtin_amdgcn_wave_barrier();

#pragma unroll
        for (int k = 0; k < kIPT; ++k) {
            const int64_t idx = wbase + k * kWave + lane;
            const bool ok = idx < P;
            const uint32_t d = (uint32_t)(key[k] >> shift) & 0xFFu;
            uint64_t m = ballot64(ok);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t vote = ballot64(bit);
                m &= bit ? vote : ~vote;
            }
            const uint32_t below = (uint32_t)__popcll(m & lt_mask);
            const uint32_t old = ok ? s_whist[wv][d] : 0u;
            rank[k] = old + below;
            __builtin_amdgcn_wave_barrier();
            if (ok && below == 0) s_whist[wv][d] = old + (uint32_t)__popcll(m);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();

        // thread t owns digit t: wave offsets, partition count, look-back
        {
            const int t = tid;
            uint32_t run = 0;
#pragma unroll
            for (int q = 0; q < kSortWaves; ++q) {
                const uint32_t c = s_whist[q][t];
                s_whist[q][t] = run;
                run += c;
            }
            const uint32_t total = run;
            if (part == 0) {
                store_relaxed(&look[t], kFlagInc | total);
                s_dbase[t] = s_goff[t];
            } else {
                store_relaxed(&look[part * kRadix + t], kFlagAgg | total);
                // look back over a window of kLook earlier partitions per
                // step (independent loads), nearest first: add published
                // counts until an inclusive prefix; stop at a partition
                // that has published nothing yet and read again from it
                uint32_t prefix = 0;
                int64_t j = part - 1;
                while (j >= 0) {
                    uint32_t v[kLook];
#pragma unroll
                    for (int q = 0; q < kLook; ++q)
                        v[q] = j - q >= 0 ? load_relaxed(&look[(j - q) * kRadix + t]) : kFlagInc;
                    int q = 0;
                    bool stalled = false;
#pragma unroll
                    for (; q < kLook; ++q) {
                        const uint32_t flag = v[q] & ~kValMask;
                        if (flag == 0u) {
                            stalled = true;
                            break;
                        }
                        prefix += v[q] & kValMask;
                        if (flag == kFlagInc) break;
                    }
                    if (!stalled && q < kLook) break;   // reached an inclusive prefix
                    j -= q;
                    if (stalled) __builtin_amdgcn_s_sleep(1);
                }
                store_relaxed(&look[part * kRadix + t], kFlagInc | (prefix + total));
                s_dbase[t] = s_goff[t] + prefix;
            }
            // exclusive scan of the partition's digit counts
            uint32_t x = total;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t y = __shfl_up(x, d, kWave);
                if (lane >= d) x += y;
            }
            if (lane == kWave - 1) s_scan[wv] = x;
            __syncthreads();
            uint32_t wb = 0;
#pragma unroll
            for (int q = 0; q < kSortWaves; ++q)
                if (q < wv) wb += s_scan[q];
            s_lofs[t] = wb + x - total;
        }
        __syncthreads();

#pragma unroll
        for (int k = 0; k < kIPT; ++k) {
            const int64_t idx = wbase + k * kWave + lane;
            if (idx < P) {
                const uint32_t d = (uint32_t)(key[k] >> shift) & 0xFFu;
                const uint32_t lp = s_lofs[d] + s_whist[wv][d] + rank[k];
                s_keys[lp] = key[k];
                s_vals[lp] = val[k];
            }
        }
        __syncthreads();

        for (int i = tid; i < nvalid; i += kSortThreads) {
            const uint64_t kk = s_keys[i];
            const uint32_t d = (uint32_t)(kk >> shift) & 0xFFu;
            const uint32_t gp = s_dbase[d] + (uint32_t)i - s_lofs[d];
            kout[gp] = kk;
            vout[gp] = s_vals[i];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_copy_pairs(const uint64_t* __restrict__ ks, const uint32_t* __restrict__ vs,
                                                    uint64_t* __restrict__ kd, uint32_t* __restrict__ vd,
                                                    const uint32_t* __restrict__ count, int64_t capacity) {
    const int64_t P = clamp_count(count, capacity);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < P; i += (int64_t)gridDim.x * 256) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

// ---- per-tile depth sort -------------------------------------------------
// After the stable sort on the tile bits, each tile's run is in emission
// order; sorting the run stably by the low 32 key bits (the depth) gives
// exactly the order of the stable sort on the whole key.

constexpr int kSegThreads = 256;
constexpr int kSegCap = 1024;   // longest run sorted in LDS

// Runs of 1 .. kSegCap pairs, one wave each, sorted in LDS by a stable LSD
// radix sort on the 32 depth bits: up to four 8-bit passes, skipping the
// bytes on which the whole run agrees (a stable pass over a constant digit
// leaves the order as it is).  Entries are (depth << 32 | position in the
// run), ranked in order 64 at a time with ballot matches and running digit
// counts; the values are gathered by position at the end.  One wave per
// run, four runs per workgroup: no workgroup barriers, and the loops stop
// at the run's length.  With `order` set, an extra first workgroup writes
// the tiles' blend order meanwhile (order[0] = the tile count, order[1..] =
// every tile, longest list first: tile_order_block).
constexpr int kSegWaves = 4;

__global__ __launch_bounds__(kSegWaves * kWave) void k_seg_sort_lds(const uint64_t* __restrict__ kin,
                                                                    const uint32_t* __restrict__ vin,
                                                                    uint64_t* __restrict__ kout,
                                                                    uint32_t* __restrict__ vout,
                                                                    const uint2* __restrict__ ranges,
                                                                    uint32_t n_tiles, uint32_t* __restrict__ order) {
    constexpr int IPL = kSegCap / kWave;   // entries per lane
    constexpr int DPL = kRadix / kWave;    // digits per lane in the offset scan
    __shared__ uint64_t s_all[kSegWaves][kSegCap];
    __shared__ uint32_t s_cnt_all[kSegWaves][kRadix];   // per wave: digit counts, then digit offsets
    const int first = order ? 1 : 0;
    if (order && blockIdx.x == 0) {
        __shared__ uint32_t s_h[kSegWaves][kTileClasses + 1];
        tile_order_block<kSegWaves * kWave>(ranges, n_tiles, order + 1, order, 1, s_h);
        return;
    }
    const int wv = threadIdx.x / kWave;
    const uint32_t tile = ((uint32_t)blockIdx.x - (uint32_t)first) * kSegWaves + (uint32_t)wv;
    if (tile >= n_tiles) return;
    uint64_t* s = s_all[wv];
    uint32_t* s_cnt = s_cnt_all[wv];
    const uint2 r = ranges[tile];
    const uint32_t n = r.y - r.x;
    if (n == 0u || n > (uint32_t)kSegCap) return;
    const int lane = threadIdx.x & (kWave - 1);
    if (n == 1u) {
        if (lane == 0) {
            kout[r.x] = kin[r.x];
            vout[r.x] = vin[r.x];
        }
        return;
    }
    const uint64_t tile_hi = kin[r.x] & 0xFFFFFFFF00000000ull;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t z0 = (uint32_t)kin[r.x];
    const int nq = (int)((n + kWave - 1) / kWave);
    uint32_t vary = 0;
    for (uint32_t i = lane; i < n; i += kWave) {
        const uint32_t z = (uint32_t)kin[r.x + i];
        s[i] = ((uint64_t)z << 32) | i;
        vary |= z ^ z0;
    }
    // OR over the wave
    for (int d = 1; d < kWave; d <<= 1) vary |= (uint32_t)__shfl_xor((int)vary, d, kWave);
    __builtin_amdgcn_wave_barrier();
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 32 + 8 * pass;
        if (((vary >> (8 * pass)) & 0xFFu) == 0u) continue;
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
        // digit offsets: lane l owns digits l*DPL .. l*DPL + DPL - 1
        {
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
    for (uint32_t i = lane; i < n; i += kWave) {
        const uint64_t c = s[i];
        kout[r.x + i] = tile_hi | (c >> 32);
        vout[r.x + i] = vin[r.x + (uint32_t)c];
    }
}

// Runs longer than kSegCap: one workgroup sorts the run stably by its
// 32 depth bits with four 8-bit LSD passes over global memory, 256 pairs
// at a time in order (ballot match ranks within a wave, per-wave digit
// counts order the waves), ping-ponging between the two buffers; the
// fourth pass ends in the input buffers, copied out at the end.
__global__ __launch_bounds__(kSegThreads) void k_seg_sort_long(uint64_t* __restrict__ ka, uint32_t* __restrict__ va,
                                                               uint64_t* __restrict__ kb, uint32_t* __restrict__ vb,
                                                               const uint2* __restrict__ ranges) {
    __shared__ uint32_t s_start[kRadix];   // digit start in the run
    __shared__ uint32_t s_run[kRadix];     // pairs of each digit placed so far
    __shared__ uint32_t s_wc[kSegThreads / kWave][kRadix];
    __shared__ uint32_t s_w[kRadix / kWave];
    const uint2 r = ranges[blockIdx.x];
    const uint32_t n = r.y - r.x;
    if (n <= (uint32_t)kSegCap) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int pass = 0; pass < 4; ++pass) {
        const uint64_t* ki = (pass & 1) ? kb : ka;
        const uint32_t* vi = (pass & 1) ? vb : va;
        uint64_t* ko = (pass & 1) ? ka : kb;
        uint32_t* vo = (pass & 1) ? va : vb;
        const int shift = 8 * pass;
        // digit counts of the run and their exclusive scan
        s_start[tid] = 0u;
        s_run[tid] = 0u;
        for (int q = 0; q < kSegThreads / kWave; ++q) s_wc[q][tid] = 0u;
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kSegThreads)
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
            for (int q = 0; q < kRadix / kWave; ++q)
                if (q < wv) base += s_w[q];
            s_start[tid] = base + x - v;
        }
        __syncthreads();
        for (uint32_t c0 = 0; c0 < n; c0 += kSegThreads) {
            const uint32_t i = c0 + (uint32_t)tid;
            const bool ok = i < n;
            const uint64_t key = ok ? ki[r.x + i] : 0ull;
            const uint32_t val = ok ? vi[r.x + i] : 0u;
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
                for (int q = 0; q < kSegThreads / kWave; ++q)
                    if (q < wv) pos += s_wc[q][d];
                ko[r.x + pos] = key;
                vo[r.x + pos] = val;
            }
            __syncthreads();
            uint32_t add = 0;
            for (int q = 0; q < kSegThreads / kWave; ++q) {
                add += s_wc[q][tid];
                s_wc[q][tid] = 0u;
            }
            s_run[tid] += add;
            __syncthreads();
        }
        // the next pass reads what this one wrote (same workgroup)
        __threadfence_block();
        __syncthreads();
    }
    // four passes: the run is back in (ka, va); the result goes to (kb, vb)
    for (uint32_t i = tid; i < n; i += kSegThreads) {
        kb[r.x + i] = ka[r.x + i];
        vb[r.x + i] = va[r.x + i];
    }
}

}  // namespace

int sort_passes(int key_bits) { return (key_bits + 7) / 8; }

size_t sort_workspace_bytes(int64_t capacity, int key_bits) {
    const int passes = sort_passes(key_bits);
    const int64_t parts = (capacity + kPart - 1) / kPart;
    return align256((size_t)kMaxPasses * kRadix * 4) + align256((size_t)kMaxPasses * 4) +
           align256((size_t)passes * (size_t)(parts > 0 ? parts : 1) * kRadix * 4);
}

namespace {

// Passes p0 .. p1-1 (digits 8 p .. 8 p + 7) of the stable LSD sort, reading
// the alternate buffers first when `start_in_alt`.  Returns whether the
// result sits in the alternate buffers.
// `zero` (zero_count u32 words, may be NULL) is cleared by the first kernel
// when any pass runs; the return value then has bit 1 set.
int radix_passes(uint64_t* keys, uint32_t* vals, uint64_t* alt_keys, uint32_t* alt_vals, const uint32_t* count,
                 int64_t capacity, int p0, int p1, bool start_in_alt, void* ws, hipStream_t st,
                 uint32_t* zero = nullptr, int64_t zero_count = 0, bool cleared = false) {
    if (p1 <= p0 || capacity == 0) return start_in_alt ? 1 : 0;
    SortWs w = carve(ws, capacity, p1);
    const int64_t parts = (capacity + kPart - 1) / kPart;
    if (!cleared) {
        int64_t clear_blocks = (parts * kRadix * (p1 - p0) + 255) / 256;
        if (clear_blocks > 1024) clear_blocks = 1024;
        if (clear_blocks < 1) clear_blocks = 1;
        hipLaunchKernelGGL(k_sort_clear, dim3((unsigned)clear_blocks), dim3(256), 0, st, w, count, p0, p1, zero,
                           zero ? zero_count : (int64_t)0);
    }
    const uint64_t* src = start_in_alt ? alt_keys : keys;
    // one round of eight keys per thread where the capacity is small
    int64_t hb = (capacity + kHistThreads * 8 - 1) / (kHistThreads * 8);
    if (hb > kHistGrid) hb = kHistGrid;
    if (hb < 1) hb = 1;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)hb), dim3(kHistThreads), 0, st, src, count, p0, p1, w);
    int64_t grid = parts < kMaxGrid ? parts : kMaxGrid;
    bool in_alt = start_in_alt;
    for (int p = p0; p < p1; ++p) {
        const uint64_t* ki = in_alt ? alt_keys : keys;
        const uint32_t* vi = in_alt ? alt_vals : vals;
        uint64_t* ko = in_alt ? keys : alt_keys;
        uint32_t* vo = in_alt ? vals : alt_vals;
        hipLaunchKernelGGL(k_onesweep, dim3((unsigned)grid), dim3(kSortThreads), 0, st, ki, vi, ko, vo, count, p, w);
        in_alt = !in_alt;
    }
    return (in_alt ? 1 : 0) | 2;
}

}  // namespace

void launch_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* alt_keys, uint32_t* alt_vals, const uint32_t* count,
                       int64_t capacity, int key_bits, bool start_in_alt, void* ws, hipStream_t st) {
    if (capacity == 0) return;
    const bool in_alt = (radix_passes(keys, vals, alt_keys, alt_vals, count, capacity, 0, sort_passes(key_bits),
                                      start_in_alt, ws, st) & 1) != 0;
    if (in_alt)  // result sits in the alternate buffers
        hipLaunchKernelGGL(k_copy_pairs, dim3(1024), dim3(256), 0, st, alt_keys, alt_vals, keys, vals, count,
                           capacity);
}

int bin_tile_passes(int tile_bits) { return (tile_bits + 7) / 8; }

bool bin_sort_emit_to_alt(int tile_bits) { return bin_tile_passes(tile_bits) % 2 == 0; }

ZeroList bin_sort_zero_list(void* ws, int64_t capacity, int tile_bits, uint32_t* ranges, int64_t n_tiles) {
    const int p0 = 4, p1 = 4 + bin_tile_passes(tile_bits);
    ZeroList z;
    for (int r = 0; r < 3; ++r) {
        z.p[r] = nullptr;
        z.n[r] = 0;
    }
    // the tile ranges; with pairs to sort, also the histograms and
    // partition counters (the workspace header) and the look-back words of
    // the tile passes
    if (ranges && n_tiles > 0) {
        z.p[2] = ranges;
        z.n[2] = n_tiles * 2;
    }
    if (ws && capacity > 0) {
        SortWs w = carve(ws, capacity, p1);
        z.p[0] = w.hist;
        z.n[0] = (int64_t)((reinterpret_cast<char*>(w.look) - reinterpret_cast<char*>(w.hist)) / 4);
        z.p[1] = w.look + (int64_t)p0 * w.max_parts * kRadix;
        z.n[1] = (int64_t)(p1 - p0) * w.max_parts * kRadix;
    }
    return z;
}

void launch_bin_sort(uint64_t* keys, uint32_t* vals, uint64_t* alt_keys, uint32_t* alt_vals, const uint32_t* count,
                     int64_t capacity, int tile_bits, uint32_t* ranges, int64_t n_tiles, void* ws, hipStream_t st,
                     bool zeroed, uint32_t* tile_order) {
    // tile bits: passes 4 .. 4 + ceil(tile_bits / 8) - 1, ending in the
    // alternate buffers (the emission went where bin_sort_emit_to_alt says);
    // the workspace words and ranges are zeroed by the emission when
    // `zeroed`, else by the first pass's clear
    const int r = radix_passes(keys, vals, alt_keys, alt_vals, count, capacity, 4, 4 + bin_tile_passes(tile_bits),
                               bin_sort_emit_to_alt(tile_bits), ws, st, zeroed ? nullptr : ranges, n_tiles * 2,
                               zeroed);
    launch_tile_ranges(alt_keys, count, capacity, n_tiles, ranges, st, zeroed || (r & 2) != 0);
    if (n_tiles == 0 || (capacity == 0 && !tile_order)) {
        if (tile_order) launch_fill_u32(tile_order, 0u, 1, st);
        return;
    }
    const uint2* rg = reinterpret_cast<const uint2*>(ranges);
    const unsigned blocks = (unsigned)((n_tiles + kSegWaves - 1) / kSegWaves) + (tile_order ? 1u : 0u);
    hipLaunchKernelGGL(k_seg_sort_lds, dim3(blocks), dim3(kSegWaves * kWave), 0, st, alt_keys, alt_vals, keys, vals,
                       rg, (uint32_t)n_tiles, tile_order);
    if (capacity == 0) return;
    hipLaunchKernelGGL(k_seg_sort_long, dim3((unsigned)n_tiles), dim3(kSegThreads), 0, st, alt_keys, alt_vals, keys,
                       vals, rg);
}

}  // namespace gs
