// The order in which the blend launches take their tiles: longest list
// first, so that the tiles that take longest start first and the launch
// does not end on a few of them.
#pragma once

#include "gs_device.h"

namespace gs {

// One workgroup: the tiles ordered by the log2 of their list length, longest
// first (order within a length class unspecified), then (with
// include_empty) the empty tiles; *count = the tiles written.  Every wave
// takes 64 consecutive tiles at a time and finds, with six ballots over the
// bits of the class, the lanes of its own class (match by bits, as the
// radix sort ranks its digits); the lowest of them adds the class's tiles to
// the wave's LDS counter (first pass) or moves the wave's cursor in that
// class past them, the others taking the positions by rank (second pass).
// The waves' counts meet once for the starting positions.
constexpr int kTileClasses = 33;   // 0..31: floor(log2(length)), 32: empty

__device__ __forceinline__ int tile_length_class(uint32_t n) { return n ? 31 - __builtin_clz(n) : 32; }

// Run by all NT threads of one workgroup; s_h: LDS of NT / 64 rows.
// len(t): the list length of tile t.
template <int NT, class Len>
__device__ __forceinline__ void tile_order_block_len(Len len, uint32_t n_tiles, uint32_t* __restrict__ order,
                                                     uint32_t* __restrict__ count, int include_empty,
                                                     uint32_t (*s_h)[kTileClasses + 1]) {
    constexpr int kWaves = NT / kWave;
    constexpr int kPer = 8;   // tiles per thread per block of NT x kPer, loaded together
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int i = tid; i < kWaves * (kTileClasses + 1); i += NT) (&s_h[0][0])[i] = 0u;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        // the tile of (block b0, slot k) for this thread is b0 + k * NT + tid,
        // so that a wave's 64 lanes hold 64 consecutive tiles
        for (uint32_t b0 = 0; b0 < n_tiles; b0 += NT * kPer) {
            int cl[kPer];
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const uint32_t t = b0 + (uint32_t)(k * NT + tid);
                cl[k] = t < n_tiles ? tile_length_class(len(t)) : kTileClasses;   // kTileClasses: none
            }
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const uint32_t t = b0 + (uint32_t)(k * NT + tid);
                uint64_t same = ~0ull;
#pragma unroll
                for (int bit = 0; bit < 6; ++bit) {
                    const bool on = (cl[k] >> bit) & 1;
                    const uint64_t v = __ballot(on);
                    same &= on ? v : ~v;
                }
                const uint32_t rank = (uint32_t)__popcll(same & lt);
                if (pass == 1) {
                    const uint32_t base = s_h[wv][cl[k]];
                    if (cl[k] < kTileClasses && (include_empty || cl[k] < 32)) order[base + rank] = t;
                }
                __builtin_amdgcn_wave_barrier();
                if (rank == 0u) s_h[wv][cl[k]] += (uint32_t)__popcll(same);
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (pass == 1) break;
        __syncthreads();
        // lane p of wave 0 takes the p-th class in output order (31, 30,
        // ..., 0, then the empty class 32); an exclusive scan over the lanes
        // gives the class's first position, then each wave's
        if (wv == 0) {
            const int c = lane < 32 ? 31 - lane : 32;
            uint32_t n[kWaves], tot = 0u;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                n[w] = lane < kTileClasses ? s_h[w][c] : 0u;
                tot += n[w];
            }
            uint32_t x = tot;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t y = (uint32_t)__shfl_up((int)x, d, kWave);
                if (lane >= d) x += y;
            }
            uint32_t run = x - tot;
            if (lane < kTileClasses) {
#pragma unroll
                for (int w = 0; w < kWaves; ++w) {
                    s_h[w][c] = run;
                    run += n[w];
                }
            }
            if (lane == 32) *count = include_empty ? x : x - tot;   // all tiles, or those with pairs
        }
        __syncthreads();
    }
}

// The same, with the lengths taken from per-tile [start, end) ranges.
template <int NT>
__device__ __forceinline__ void tile_order_block(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                 uint32_t* __restrict__ order, uint32_t* __restrict__ count,
                                                 int include_empty, uint32_t (*s_h)[kTileClasses + 1]) {
    tile_order_block_len<NT>([ranges](uint32_t t) { return ranges[t].y - ranges[t].x; }, n_tiles, order, count,
                             include_empty, s_h);
}

}  // namespace gs
