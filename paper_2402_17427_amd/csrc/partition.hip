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

__global__ __launch_bounds__(kThreads) void k_select_points(SelectArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool live = i < a.n;
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
        const int v1 = a.offsets[c + 1];
        for (int k = a.offsets[c]; k < v1; ++k) {
            if (__ballot(open) == 0ull) break;
            if (open) {
                const double* q = a.cams + kCamDoubles * a.views[k];
                const double x = q[0] * px + q[1] * py + q[2] * pz + q[9];
                const double y = q[3] * px + q[4] * py + q[5] * pz + q[10];
                const double z = q[6] * px + q[7] * py + q[8] * pz + q[11];
                ++tests;
                if (z > q[18]) {
                    const double u = q[12] * x + q[14] * z, v = q[13] * y + q[15] * z;
                    if (u >= 0.0 && u < q[16] * z && v >= 0.0 && v < q[17] * z) {
                        mem = 2;
                        open = false;
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

void launch_select_points(const SelectArgs& a, hipStream_t st) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_select_points, dim3((unsigned)((a.n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, a);
}

void launch_merge_keep(const float* mean, int64_t n, int64_t ld, const double rect[4], int closed_x, int closed_z,
                       uint8_t* keep, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_merge_keep, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, mean, n,
                       ld, rect[0], rect[1], rect[2], rect[3], closed_x, closed_z, keep);
}

}  // namespace gs
