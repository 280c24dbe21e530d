// Small kernels of the batched training step and of the blends: the L1
// image loss and its gradient for every view of the batch, and the
// longest-list-first tile orders the blend launches take their tiles in.
//
// VastGaussian (arXiv 2402.17427), section 3: each cell is optimised
// against its training images with an image loss; the per-pixel L1 term is
// the part of that loss this step evaluates (mean absolute error over the
// three colour planes, gradient sign(I - I*) / (3 W H), sign(0) = 0).
#include "kernels.h"
#include "tile_order.h"

namespace gs {

namespace {

constexpr int kL1Threads = 256;

// One workgroup per (view, chunk of pixels): grid.y = view.  Each
// workgroup writes its partial sum (FP64) to partials[view][chunk]; the
// finishing kernel adds them in chunk order, so the loss is the same on
// every run.
__global__ __launch_bounds__(kL1Threads) void k_l1(ViewTab views, const float* const* __restrict__ targets,
                                                   const float* __restrict__ image, float* __restrict__ dimg,
                                                   double* __restrict__ partials, const int32_t* __restrict__ status) {
    __shared__ double red[kL1Threads / kWave];
    const int v = blockIdx.y;
    const View V = view_at(views, v);
    const int64_t npix = (int64_t)V.cam.W * V.cam.H;
    const int64_t total = 3 * npix;
    const float* __restrict__ tgt = targets[v];
    const float inv = 1.0f / (float)total;
    const bool ok = *status == 0;
    double acc = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * kL1Threads + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * kL1Threads) {
        const float d = image[V.img_base + q] - tgt[q];
        acc += (double)fabsf(d);
        dimg[V.img_base + q] = ok ? (d > 0.f ? inv : (d < 0.f ? -inv : 0.f)) : 0.f;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < kL1Threads / kWave; ++k) s += red[k];
        partials[(int64_t)v * gridDim.x + blockIdx.x] = s;
    }
}

// One wave per view: loss[v] = (sum of the view's nb partials) / (3 W H).
__global__ __launch_bounds__(kWave) void k_l1_finish(ViewTab views, const double* __restrict__ partials, int nb,
                                                     float* __restrict__ loss) {
    const int v = blockIdx.x, lane = threadIdx.x;
    const View V = view_at(views, v);
    double s = 0.0;
    for (int k = lane; k < nb; k += kWave) s += partials[(int64_t)v * nb + k];
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if (lane == 0) loss[v] = (float)(s / (3.0 * (double)V.cam.W * (double)V.cam.H));
}

constexpr int kOrderThreads = 1024;

// One workgroup of 1024 threads orders the tiles (see tile_order_block).
__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                             uint32_t* __restrict__ order, uint32_t* __restrict__ count,
                                                             int include_empty) {
    __shared__ uint32_t s_h[kOrderThreads / kWave][kTileClasses + 1];
    tile_order_block<kOrderThreads>(ranges, n_tiles, order, count, include_empty, s_h);
}

}  // namespace

void launch_tile_order(const uint32_t* ranges, uint32_t n_tiles, uint32_t* order, uint32_t* count, bool include_empty,
                       hipStream_t st) {
    if (n_tiles == 0) {
        launch_fill_u32(count, 0u, 1, st);
        return;
    }
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, st, reinterpret_cast<const uint2*>(ranges),
                       n_tiles, order, count, include_empty ? 1 : 0);
}

void launch_l1(const ViewTab& views, int n_views, int64_t max_pix, const float* const* targets, const float* image,
               float* dimg, float* loss, double* partials, const int32_t* status, hipStream_t st) {
    if (n_views == 0) return;
    int64_t bx = (3 * max_pix + kL1Threads * 8 - 1) / (kL1Threads * 8);
    if (bx > kL1MaxChunks) bx = kL1MaxChunks;
    if (bx < 1) bx = 1;
    hipLaunchKernelGGL(k_l1, dim3((unsigned)bx, (unsigned)n_views), dim3(kL1Threads), 0, st, views, targets, image,
                       dimg, partials, status);
    hipLaunchKernelGGL(k_l1_finish, dim3((unsigned)n_views), dim3(kWave), 0, st, views, partials, (int)bx, loss);
}


}  // namespace gs
