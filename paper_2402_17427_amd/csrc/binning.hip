// Tile assignment: scan of per-Gaussian tile counts, emission of one
// (tile, depth) key per covered tile, and per-tile ranges of the sorted keys.
//
// VastGaussian (arXiv 2402.17427), section 3: the projected 2D Gaussians are
// assigned to screen tiles and sorted (by tile, then by depth) before the
// blend.  A Gaussian's tiles are those its alpha >= 1/255 support touches
// (the rectangle from the projection), emitted in row-major order; the sort
// that follows is stable, so equal keys keep Gaussian-index order.
#include "kernels.h"
#include <algorithm>

namespace gs {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanTopThreads = 1024;
constexpr int kScanTopItems = 4;

// Block-wide exclusive scan of one uint32 per thread (wave64 prefix via
// shuffles, then a scan of the wave totals).  Returns the exclusive prefix;
// *total gets the block sum.
template <int NT>
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* total) {
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

__global__ __launch_bounds__(kScanThreads) void k_block_sums(const uint32_t* __restrict__ tt, int64_t n,
                                                             uint64_t* __restrict__ block_sums, ZeroList zero) {
    const int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kScanThreads;
#pragma unroll
    for (int r = 0; r < 3; ++r)
        for (int64_t j = i; j < zero.n[r]; j += stride) zero.p[r][j] = 0u;
    const int64_t nb = (n + kScanThreads - 1) / kScanThreads;
    if ((int64_t)blockIdx.x >= nb) return;   // a clearing-only workgroup
    const uint64_t v = i < n ? tt[i] : 0u;
    uint64_t tot;
    block_exclusive_scan<kScanThreads>(v, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the block sums in place, pair count and
// capacity status.
__global__ __launch_bounds__(kScanTopThreads) void k_scan_top(uint64_t* __restrict__ block_sums, int64_t nb,
                                                              int64_t capacity, uint32_t* __restrict__ pair_count,
                                                              int32_t* __restrict__ status) {
    // kScanTopItems consecutive sums per thread, so that one block-wide scan
    // covers up to kScanTopThreads * kScanTopItems of them
    uint64_t carry = 0;
    for (int64_t base = 0; base < nb; base += (int64_t)kScanTopThreads * kScanTopItems) {
        const int64_t i0 = base + (int64_t)threadIdx.x * kScanTopItems;
        uint64_t v[kScanTopItems], sum = 0;
#pragma unroll
        for (int e = 0; e < kScanTopItems; ++e) {
            v[e] = i0 + e < nb ? block_sums[i0 + e] : 0u;
            sum += v[e];
        }
        uint64_t tot;
        uint64_t run = carry + block_exclusive_scan<kScanTopThreads>(sum, &tot);
#pragma unroll
        for (int e = 0; e < kScanTopItems; ++e) {
            if (i0 + e < nb) block_sums[i0 + e] = run;
            run += v[e];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        const bool over = carry > (uint64_t)capacity;
        pair_count[0] = over ? 0u : (uint32_t)carry;   // pairs the later stages process
        pair_count[1] = carry > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)carry;   // pairs needed
        *status = over ? -4 : 0;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_emit(const uint32_t* __restrict__ tt, const ushort4* __restrict__ rect,
                                                       const float* __restrict__ depth, int64_t n, JobTab jobs,
                                                       ViewTab views, const uint64_t* __restrict__ block_prefix,
                                                       int64_t capacity, uint64_t* __restrict__ keys,
                                                       uint32_t* __restrict__ vals, uint32_t* __restrict__ first) {
    const int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    const uint32_t cnt = i < n ? tt[i] : 0u;
    uint64_t tot;
    uint64_t off = block_prefix[blockIdx.x] + block_exclusive_scan<kScanThreads>(cnt, &tot);
    // where this Gaussian's pairs start in emission order (the backward
    // writes its per-tile sums there); meaningful only when all pairs fit
    if (first && i < n) first[i] = (uint32_t)off;
    if (cnt == 0) return;
    // record slots are aligned so that a workgroup lies within one job
    const View V = view_at(views, job_at(jobs, find_job(jobs, (int64_t)blockIdx.x * kScanThreads)).view);
    const ushort4 r = rect[i];
    const uint64_t zb = (uint64_t)__float_as_uint(depth[i]);
    for (int ty = r.y; ty < r.w; ++ty)
        for (int tx = r.x; tx < r.z; ++tx) {
            if (off < (uint64_t)capacity) {
                keys[off] = ((uint64_t)(V.tile_base + (uint32_t)(ty * V.ntx + tx)) << 32) | zb;
                vals[off] = (uint32_t)i;
            }
            ++off;
        }
}

__global__ __launch_bounds__(256) void k_ranges(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ count,
                                                int64_t capacity, int64_t n_tiles, uint32_t* __restrict__ ranges) {
    const int64_t P = (int64_t)*count < capacity ? (int64_t)*count : capacity;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= P) return;
    const uint32_t t = (uint32_t)(keys[j] >> 32);
    if (t >= n_tiles) return;
    if (j == 0 || (uint32_t)(keys[j - 1] >> 32) != t) ranges[2 * (int64_t)t] = (uint32_t)j;
    if (j == (int64_t)P - 1 || (uint32_t)(keys[j + 1] >> 32) != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(j + 1);
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, size_t count) {
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < count; j += (size_t)gridDim.x * 256) p[j] = v;
}

}  // namespace

size_t scan_workspace_bytes(int64_t n) {
    const int64_t nb = (n + kScanThreads - 1) / kScanThreads;
    return (size_t)(nb > 0 ? nb : 1) * sizeof(uint64_t);
}

void launch_fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t st) {
    if (count == 0) return;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, count);
}

void launch_emit_pairs(int64_t n, const uint32_t* tt, const ushort4* rect, const float* depth, const JobTab& jobs,
                       const ViewTab& views, int64_t capacity, uint64_t* keys, uint32_t* vals, uint32_t* first,
                       uint32_t* pair_count, int32_t* status, void* scan_ws, hipStream_t st, const ZeroList* zero) {
    uint64_t* bs = static_cast<uint64_t*>(scan_ws);
    const int64_t nb = (n + kScanThreads - 1) / kScanThreads;
    ZeroList z{};
    int64_t zn = 0;
    if (zero) {
        z = *zero;
        for (int r = 0; r < 3; ++r) {
            if (!z.p[r]) z.n[r] = 0;
            zn += z.n[r];
        }
    }
    // the block-sum pass also clears what the caller listed (grid-stride),
    // with at least enough workgroups that each thread clears a few words
    int64_t grid = nb;
    const int64_t zgrid = std::min<int64_t>((zn + 4 * kScanThreads - 1) / (4 * kScanThreads), 2048);
    if (zgrid > grid) grid = zgrid;
    if (grid > 0)
        hipLaunchKernelGGL(k_block_sums, dim3((unsigned)grid), dim3(kScanThreads), 0, st, tt, n, bs, z);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTopThreads), 0, st, bs, nb, capacity, pair_count, status);
    if (nb > 0)
        hipLaunchKernelGGL(k_emit, dim3((unsigned)nb), dim3(kScanThreads), 0, st, tt, rect, depth, n, jobs, views,
                           bs, capacity, keys, vals, first);
}

void launch_tile_ranges(const uint64_t* keys, const uint32_t* pair_count, int64_t capacity, int64_t n_tiles,
                        uint32_t* ranges, hipStream_t st, bool zeroed) {
    if (!zeroed) launch_fill_u32(ranges, 0u, (size_t)n_tiles * 2, st);
    if (capacity == 0) return;
    const int64_t blocks = (capacity + 255) / 256;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, st, keys, pair_count, capacity, n_tiles,
                       ranges);
}

}  // namespace gs
