// Point selection of the progressive data partitioning, and the merge mask.
//
// VastGaussian (arXiv 2402.17427), section 4.1: a cell takes the points
// whose ground position lies in its expanded rectangle (position-based
// selection), and then the points covered by any of its views (coverage-
// based selection: in front of the near plane and projecting inside the
// image, occlusion ignored).  Section 4.3: after optimisation a cell keeps
// only the Gaussians inside its original rectangle.
//
// Coverage is the scalable part: points x cells x views.  One thread per
// point walks each cell's view list and stops at the first view that
// covers the point; the view index is the same for every lane of a wave,
// so the camera data come through scalar loads.  The projection test is
// FP64 (the vector FP64 rate of the chip equals its non-packed FP32 rate)
// and uses no division: 0 <= fx x/z + cx < W is tested as
// 0 <= fx x + cx z < W z with z > near > 0.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace gs {

namespace {

constexpr int kThreads = 256;

inline size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kStage = 128;  // camera rows staged in LDS at a time (20 KB)

// Morton key of a point's ground position (16 bits of x, 16 of z, over the
// box of the cells' expanded rectangles; outside points clamp to its edge):
// sorting by it puts the points of a wave close together on the ground, so
// they are covered by the same views and the wave's lanes leave the view
// scan together.
__device__ __forceinline__ uint32_t spread16(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__global__ __launch_bounds__(kThreads) void k_morton(SelectArgs a, double x0, double sx, double z0, double sz,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                     uint32_t* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i == 0) *count = (uint32_t)a.n;
    if (i >= a.n) return;
    const double qx = fmin(fmax(((double)a.points[i] - x0) * sx, 0.0), 65535.0);
    const double qz = fmin(fmax(((double)a.points[2 * a.ld + i] - z0) * sz, 0.0), 65535.0);
    keys[i] = (uint64_t)(spread16((uint32_t)qx) | (spread16((uint32_t)qz) << 1));
    vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kThreads) void k_select_points(SelectArgs a) {
    __shared__ double sv[kStage * kCamDoubles];
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool live = q < a.n;
    const int64_t i = !live ? 0 : (a.order ? (int64_t)a.order[q] : q);
    double px = 0.0, py = 0.0, pz = 0.0;
    if (live) {
        px = a.points[i];
        py = a.points[a.ld + i];
        pz = a.points[2 * a.ld + i];
    }
    uint64_t tests = 0;
    for (int c = 0; c < a.n_cells; ++c) {
        const double* r = a.cells + 4 * c;
        uint8_t mem = 0;
        if (px >= r[0] && px <= r[1] && pz >= r[2] && pz <= r[3]) mem = 1;
        bool open = live && mem == 0;
        const int v0 = a.offsets[c], v1 = a.offsets[c + 1];
        for (int base = v0; base < v1; base += kStage) {
            // the whole workgroup leaves when none of its points is open
            if (!__syncthreads_or(open)) break;
            const int cnt = min(kStage, v1 - base);
            for (int k = threadIdx.x; k < cnt * kCamDoubles; k += kThreads) {
                const int row = k / kCamDoubles;
                sv[k] = a.cams[(int64_t)kCamDoubles * a.views[base + row] + (k - row * kCamDoubles)];
            }
            __syncthreads();
            for (int k = 0; k < cnt; ++k) {
                if (__ballot(open) == 0ull) break;
                if (open) {
                    const double* w = sv + kCamDoubles * k;
                    const double x = w[0] * px + w[1] * py + w[2] * pz + w[9];
                    const double y = w[3] * px + w[4] * py + w[5] * pz + w[10];
                    const double z = w[6] * px + w[7] * py + w[8] * pz + w[11];
                    ++tests;
                    if (z > w[18]) {
                        const double u = w[12] * x + w[14] * z, v = w[13] * y + w[15] * z;
                        if (u >= 0.0 && u < w[16] * z && v >= 0.0 && v < w[17] * z) {
                            mem = 2;
                            open = false;
                        }
                    }
                }
            }
        }
        if (live) a.member[(int64_t)c * a.n + i] = mem;
    }
    if (a.tests) {
        unsigned long long t = tests;
        for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && t) atomicAdd(reinterpret_cast<unsigned long long*>(a.tests), t);
    }
}

__global__ __launch_bounds__(kThreads) void k_merge_keep(const float* __restrict__ mean, int64_t n, int64_t ld,
                                                         double x0, double x1, double z0, double z1, int closed_x,
                                                         int closed_z, uint8_t* __restrict__ keep) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double x = mean[i], z = mean[2 * ld + i];
    const bool ox = x >= x0 && (closed_x ? x <= x1 : x < x1);
    const bool oz = z >= z0 && (closed_z ? z <= z1 : z < z1);
    keep[i] = (ox && oz) ? 1 : 0;
}

}  // namespace

size_t select_sort_bytes(int64_t n) {
    return 2 * round256((size_t)n * 8) + 2 * round256((size_t)n * 4) + round256(8) + round256(sort_workspace_bytes(n, 32));
}

void launch_select_points(const SelectArgs& a_in, const double box[4], void* sort_ws, hipStream_t st) {
    if (a_in.n <= 0) return;
    SelectArgs a = a_in;
    const unsigned grid = (unsigned)((a.n + kThreads - 1) / kThreads);
    // visiting order: Morton order of the ground positions
    char* p = static_cast<char*>(sort_ws);
    uint64_t* keys = reinterpret_cast<uint64_t*>(p);
    p += round256((size_t)a.n * 8);
    uint64_t* alt_k = reinterpret_cast<uint64_t*>(p);
    p += round256((size_t)a.n * 8);
    uint32_t* vals = reinterpret_cast<uint32_t*>(p);
    p += round256((size_t)a.n * 4);
    uint32_t* alt_v = reinterpret_cast<uint32_t*>(p);
    p += round256((size_t)a.n * 4);
    uint32_t* count = reinterpret_cast<uint32_t*>(p);
    p += round256(8);
    const double wx = box[1] - box[0], wz = box[3] - box[2];
    const double sx = wx > 0.0 ? 65535.0 / wx : 0.0, sz = wz > 0.0 ? 65535.0 / wz : 0.0;
    hipLaunchKernelGGL(k_morton, dim3(grid), dim3(kThreads), 0, st, a, box[0], sx, box[2], sz, keys, vals, count);
    launch_sort_pairs(keys, vals, alt_k, alt_v, count, a.n, 32, false, p, st);
    a.order = vals;
    hipLaunchKernelGGL(k_select_points, dim3(grid), dim3(kThreads), 0, st, a);
}

void launch_merge_keep(const float* mean, int64_t n, int64_t ld, const double rect[4], int closed_x, int closed_z,
                       uint8_t* keep, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_merge_keep, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, mean, n,
                       ld, rect[0], rect[1], rect[2], rect[3], closed_x, closed_z, keep);
}

}  // namespace gs
