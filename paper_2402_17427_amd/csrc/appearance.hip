// Kernels of the decoupled appearance model (gs_appearance_*).
//
// VastGaussian (arXiv 2402.17427), section 4.2 and supplement S1.1: the
// rendered image is downsampled 32 times, an appearance embedding is
// concatenated to every pixel, and a CNN (3x3 convolution to 256 channels;
// four blocks of pixel shuffle, 3x3 convolution halving the channels, ReLU;
// bilinear interpolation to the image size; 3x3 convolution, ReLU, 3x3
// convolution to 3 channels) produces the transformation map M; the
// adjusted image is I^r * M.
//
// Every layer works on planar FP32 maps [C][H][W].  Convolutions with more
// than four output channels are implicit GEMMs on the matrix cores
// (k_conv_mfma); the 3-channel map M uses a direct VALU kernel (k_conv).
// Both stage a pixel tile with its one-pixel halo and the weights of a few
// input channels at a time in LDS; the same kernels run the transposed
// convolutions of the backward (weights read flipped and transposed) with
// the layer's ReLU mask applied to the input as it is staged.  The
// low-resolution layers split their input channels over several workgroups
// whose partial sums a second kernel adds in a fixed order.  Weight
// gradients are per-workgroup partial sums over pixel tiles (a sliding
// 3 x 3 window in registers), reduced in a fixed order by a second kernel,
// so every result is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace gs {

namespace {

constexpr int kT = 256;
constexpr int kCI = 8;             // input channels staged per round
constexpr int kTile = 16;          // output tile width of the convolution
constexpr int kHalo = kTile + 2;   // staged tile width
constexpr int kWR = 8, kWC = 32;   // pixel tile of the weight gradient

constexpr int kXcds = 8;   // XCDs of an MI355X; workgroups are dealt to them round-robin

// Tile (x, y) of a workgroup of a 2D tile grid, in an XCD-aware order: the
// workgroups dealt to one XCD take a contiguous band of tiles (in row
// order), so horizontally adjacent tiles, which share halo columns and the
// cache lines of their output rows, go through the same L2.
__device__ __forceinline__ void xcd_tile(int* tx, int* ty) {
    const int nx = (int)gridDim.x, n = nx * (int)gridDim.y;
    const int b = (int)blockIdx.y * nx + (int)blockIdx.x;
    const int per = n / kXcds;
    const int t = b < per * kXcds ? (b % kXcds) * per + b / kXcds : b;
    *ty = t / nx;
    *tx = t - *ty * nx;
}

// Stages N floats into LDS: element k (k = tid, tid + kT, ...) is
// src[q] with (ok, q) = at(k), zero when !ok, and zero where MASK and
// mask[q] <= 0 (the ReLU mask of a backward pass).  Every load of the
// thread is issued before the first LDS write (an out-of-range element
// loads src[0] and is replaced by zero), so the loads overlap instead of
// each waiting for the previous one.
template <int N, bool MASK, typename At>
__device__ __forceinline__ void stage(float* dst, const float* __restrict__ src, const float* __restrict__ mask, At at) {
    constexpr int J = (N + kT - 1) / kT;
    float v[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int k = (int)threadIdx.x + j * kT;
        int64_t q = 0;
        const bool ok = k < N && at(k, &q);
        const int64_t qq = ok ? q : 0;
        float x = src[qq];
        if (MASK) x = mask[qq] > 0.f ? x : 0.f;
        v[j] = ok ? x : 0.f;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int k = (int)threadIdx.x + j * kT;
        if (k < N) dst[k] = v[j];
    }
}

__global__ __launch_bounds__(kT) void k_down_concat(const float* __restrict__ img, int H, int W, int h, int w,
                                                    const float* __restrict__ embed, int m, float* __restrict__ D) {
    __shared__ float red[kT / kWave][2];
    const int by = blockIdx.x / w, bx = blockIdx.x - by * w;
    const int64_t HW = (int64_t)H * W, hw = (int64_t)h * w;
    const int ny = min(32, H - 32 * by), nx = min(32, W - 32 * bx);
    for (int c = 0; c < 3; ++c) {
        float s = 0.f;
        for (int k = threadIdx.x; k < 1024; k += kT) {
            const int yy = k >> 5, xx = k & 31;
            if (yy < ny && xx < nx) s += img[c * HW + (int64_t)(32 * by + yy) * W + 32 * bx + xx];
        }
        for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave][0] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.f;
            for (int k = 0; k < kT / kWave; ++k) t += red[k][0];
            D[c * hw + blockIdx.x] = t / (float)(ny * nx);
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < m; k += kT) D[(3 + k) * hw + blockIdx.x] = embed[k];
}

// d_img[c][y][x] += g[c][y/32][x/32] / (pixels of that block)
__global__ __launch_bounds__(kT) void k_down_adjoint(const float* __restrict__ g, int H, int W, int h, int w,
                                                     float* __restrict__ d_img) {
    const int64_t HW = (int64_t)H * W;
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= 3 * HW) return;
    const int c = (int)(q / HW);
    const int64_t p = q - c * HW;
    const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
    const int by = y >> 5, bx = x >> 5;
    const int ny = min(32, H - 32 * by), nx = min(32, W - 32 * bx);
    d_img[q] += g[(int64_t)c * h * w + (int64_t)by * w + bx] / (float)(ny * nx);
}

template <int CO, int R, bool MASK>
__global__ __launch_bounds__(kT) void k_conv(ConvArgs a) {
    // input tile (16 wide, 16 R tall, one-pixel halo) and the chunk's
    // weights as [ci][tap][co], read by every lane at the same address
    constexpr int TR = kTile * R;       // output rows of the tile
    constexpr int IR = TR + 2;          // staged rows
    __shared__ float s_in[kCI * IR * kHalo];
    __shared__ float4 s_w[kCI * 9 * (CO / 4)];
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;   // rows R ty .. R ty + R - 1
    int bx, by;
    xcd_tile(&bx, &by);
    const int x0 = bx * kTile, y0 = by * TR;
    const int og = blockIdx.z * CO;
    const int64_t HW = (int64_t)a.H * a.W;
    const int px = x0 + tx, py = y0 + R * ty;
    float acc[R][CO];
#pragma unroll
    for (int k = 0; k < CO; ++k) {
        const float b = (a.b && og + k < a.Cout) ? a.b[og + k] : 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r][k] = b;
    }
    float* s_wf = reinterpret_cast<float*>(s_w);
    for (int c0 = 0; c0 < a.Cin; c0 += kCI) {
        __syncthreads();
        stage<kCI * IR * kHalo, MASK>(s_in, a.in, a.mask, [&](int k, int64_t* q) {
            const int c = k / (IR * kHalo), r = (k / kHalo) % IR, x = k % kHalo;
            const int gy = y0 - 1 + r, gx = x0 - 1 + x;
            *q = (int64_t)(c0 + c) * HW + (int64_t)gy * a.W + gx;
            return c0 + c < a.Cin && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
        });
        stage<kCI * 9 * CO, false>(s_wf, a.w, nullptr, [&](int k, int64_t* q) {
            const int c = k / (9 * CO), t = (k / CO) % 9, co = k % CO;
            const int ci = c0 + c, o = og + co;
            // forward: w[o][ci][t]; transposed: w[ci][o][8 - t] of the
            // forward layer (its output channel ci, input channel o)
            *q = a.transposed ? ((int64_t)ci * a.CinF + o) * 9 + (8 - t) : ((int64_t)o * a.Cin + ci) * 9 + t;
            return ci < a.Cin && o < a.Cout;
        });
        __syncthreads();
        const int cn = min(kCI, a.Cin - c0);
        for (int c = 0; c < cn; ++c) {
            float v[(R + 2) * 3];   // rows R ty .. R ty + R + 1 of the staged tile, columns tx .. tx + 2
#pragma unroll
            for (int t = 0; t < (R + 2) * 3; ++t) v[t] = s_in[(c * IR + R * ty + t / 3) * kHalo + tx + t % 3];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
#pragma unroll
                for (int q = 0; q < CO / 4; ++q) {
                    const float4 w4 = s_w[(c * 9 + t) * (CO / 4) + q];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float u = v[t + 3 * r];
                        acc[r][4 * q + 0] = fmaf(w4.x, u, acc[r][4 * q + 0]);
                        acc[r][4 * q + 1] = fmaf(w4.y, u, acc[r][4 * q + 1]);
                        acc[r][4 * q + 2] = fmaf(w4.z, u, acc[r][4 * q + 2]);
                        acc[r][4 * q + 3] = fmaf(w4.w, u, acc[r][4 * q + 3]);
                    }
                }
            }
        }
    }
    if (px < a.W) {
#pragma unroll
        for (int k = 0; k < CO; ++k) {
            const int o = og + k;
            if (o < a.Cout) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (py + r < a.H)
                        a.out[(int64_t)o * HW + (int64_t)(py + r) * a.W + px] =
                            a.relu ? fmaxf(acc[r][k], 0.f) : acc[r][k];
            }
        }
    }
}

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// The convolution as an implicit GEMM on the matrix cores:
// out[o][p] = sum_k W[o][k] X[k][p] with k = 8 tap + input channel (within
// a chunk of 8 channels), sixteen output channels by sixteen pixels per
// v_mfma_f32_16x16x4f32 (FP32 in, FP32 accumulate).  A workgroup computes a
// 16 x 16 pixel tile for 16 output channels; wave w owns tile rows
// 4w .. 4w + 3, one accumulator each.  Per chunk the input tile (with its
// halo) and the [k][o] weights are staged in LDS; each k-step gives every
// lane one weight (A: row o = lane % 16, k = lane / 16) and, per row, one
// input sample (B: k = lane / 16, pixel = lane % 16).  Split launches
// (splits > 1) sum input channels [s cps 8, (s + 1) cps 8) and write raw
// partial sums for k_conv_reduce.
template <bool MASK>
__global__ __launch_bounds__(kT) void k_conv_mfma(ConvArgs a, int splits, int cps) {
    constexpr int KC = kCI * 9;   // k values per chunk (72)
    __shared__ float s_in[kCI * kHalo * kHalo];
    __shared__ float s_w[16 * KC];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    int bx, by;
    xcd_tile(&bx, &by);
    const int x0 = bx * kTile, y0 = by * kTile;
    // blockIdx.z = split * (output-channel groups) + group; split s sums
    // input channels [s cps kCI, (s + 1) cps kCI)
    const int n_og = (a.Cout + 15) / 16;
    const int split = (int)blockIdx.z / n_og;
    const int og = ((int)blockIdx.z - split * n_og) * 16;
    const int cbeg = split * cps * kCI, cend = min(a.Cin, cbeg + cps * kCI);
    const int64_t HW = (int64_t)a.H * a.W;
    const int li = lane % 16, lk = lane / 16;
    mfma_f4 acc[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[g] = mfma_f4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = cbeg; c0 < cend; c0 += kCI) {
        __syncthreads();
        stage<kCI * kHalo * kHalo, MASK>(s_in, a.in, a.mask, [&](int k, int64_t* q) {
            const int c = k / (kHalo * kHalo), r = (k / kHalo) % kHalo, x = k % kHalo;
            const int gy = y0 - 1 + r, gx = x0 - 1 + x;
            *q = (int64_t)(c0 + c) * HW + (int64_t)gy * a.W + gx;
            return c0 + c < cend && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
        });
        // weights as [k][o] with k = 8 tap + channel
        stage<16 * KC, false>(s_w, a.w, nullptr, [&](int e, int64_t* q) {
            const int k = e >> 4, o = e & 15, t = k >> 3, c = k & 7;
            const int ci = c0 + c, oo = og + o;
            *q = a.transposed ? ((int64_t)ci * a.CinF + oo) * 9 + (8 - t) : ((int64_t)oo * a.Cin + ci) * 9 + t;
            return ci < cend && oo < a.Cout;
        });
        __syncthreads();
        // k-step s = 2 tap + h takes k = 4 s + lane / 16: channels 4 h ..
        // 4 h + 3 of one tap, so every operand offset is a constant from
        // the lane's base; the upper channel half is skipped when the chunk
        // has at most four channels
        const bool upper = cend - c0 > 4;
        const float* aw = s_w + lane;
        const float* bb = s_in + lk * kHalo * kHalo + 4 * wave * kHalo + li;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && !upper) continue;
                const float av = aw[64 * (2 * t + h)];
                const float* src = bb + h * 4 * kHalo * kHalo + (t / 3) * kHalo + t % 3;
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, src[g * kHalo], acc[g], 0, 0, 0);
            }
        }
    }
    // D[o = 4 (lane / 16) + r][pixel = lane % 16] of row 4 wave + g
    float bias[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = og + 4 * lk + r;
        const float bv = a.b ? a.b[o < a.Cout ? o : 0] : 0.f;
        bias[r] = (splits == 1 && o < a.Cout) ? bv : 0.f;
    }
    const int px = x0 + li;
    if (px < a.W) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int py = y0 + 4 * wave + g;
            if (py >= a.H) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = og + 4 * lk + r;
                if (o < a.Cout) {
                    const int64_t pix = (int64_t)py * a.W + px;
                    if (splits > 1) {
                        a.part[((int64_t)split * a.Cout + o) * HW + pix] = acc[g][r];
                    } else {
                        const float v = acc[g][r] + bias[r];
                        a.out[(int64_t)o * HW + pix] = a.relu ? fmaxf(v, 0.f) : v;
                    }
                }
            }
        }
    }
}

// out[o][p] = (bias[o] + sum over the splits, in order, of part[s][o][p]),
// ReLU if asked: the end of a split convolution
__global__ __launch_bounds__(kT) void k_conv_reduce(const float* __restrict__ part, int splits, int Cout, int64_t HW,
                                                    const float* __restrict__ b, int relu, float* __restrict__ out) {
    const int o = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= HW) return;
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += part[((int64_t)k * Cout + o) * HW + p];
    if (b) s += b[o];
    out[(int64_t)o * HW + p] = relu ? fmaxf(s, 0.f) : s;
}

// Per-workgroup partial sums of dW[o][i][tap] and db[o] over its pixel
// tiles (8 x 32, grid-stride).  OG = 16: thread (o, i) of a 16 x 16
// channel block.  OG = 4 (layers with at most four output channels):
// thread (column quarter, o, i) of a 4 x 16 block, each quarter of the
// tile's columns summed by its own threads and the four added in order at
// the end.
template <int OG, bool MASK>
__global__ __launch_bounds__(kT) void k_wgrad(WgradArgs a) {
    constexpr int CS = 16 / OG;          // column splits of the pixel tile
    constexpr int QW = kWC / CS;         // columns per split
    __shared__ float s_g[OG * kWR * kWC];
    __shared__ float s_in[16 * (kWR + 2) * (kWC + 2)];
    const int cs = threadIdx.x / (OG * 16);
    const int ol = (threadIdx.x / 16) % OG, il = threadIdx.x % 16;
    const int n_ig = (a.Cin + 15) / 16;
    const int o0 = (blockIdx.y / n_ig) * OG, i0 = (blockIdx.y % n_ig) * 16;
    const int64_t HW = (int64_t)a.H * a.W;
    const int tiles_x = (a.W + kWC - 1) / kWC, tiles_y = (a.H + kWR - 1) / kWR;
    const int n_tiles = tiles_x * tiles_y;
    float acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0.f;
    float bacc = 0.f;
    // the workgroups dealt to one XCD (blockIdx.x % kXcds) walk a
    // contiguous band of tiles, so neighbouring tiles' halos share an L2
    int t_beg = (int)blockIdx.x, t_end = n_tiles, t_step = (int)gridDim.x;
    if (gridDim.x % kXcds == 0) {
        const int xcd = (int)blockIdx.x % kXcds;
        t_beg = (int)((int64_t)n_tiles * xcd / kXcds) + (int)blockIdx.x / kXcds;
        t_end = (int)((int64_t)n_tiles * (xcd + 1) / kXcds);
        t_step = (int)gridDim.x / kXcds;
    }
    for (int tile = t_beg; tile < t_end; tile += t_step) {
        const int y0 = (tile / tiles_x) * kWR, x0 = (tile % tiles_x) * kWC;
        __syncthreads();
        stage<OG * kWR * kWC, MASK>(s_g, a.g, a.mask, [&](int k, int64_t* q) {
            const int o = k / (kWR * kWC), r = (k / kWC) % kWR, x = k % kWC;
            const int gy = y0 + r, gx = x0 + x;
            *q = (int64_t)(o0 + o) * HW + (int64_t)gy * a.W + gx;
            return o0 + o < a.Cout && gy < a.H && gx < a.W;
        });
        stage<16 * (kWR + 2) * (kWC + 2), false>(s_in, a.in, nullptr, [&](int k, int64_t* q) {
            const int i = k / ((kWR + 2) * (kWC + 2)), r = (k / (kWC + 2)) % (kWR + 2), x = k % (kWC + 2);
            const int gy = y0 - 1 + r, gx = x0 - 1 + x;
            *q = (int64_t)(i0 + i) * HW + (int64_t)gy * a.W + gx;
            return i0 + i < a.Cin && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
        });
        __syncthreads();
        const float* gi = s_g + ol * kWR * kWC;
        const float* xi = s_in + il * (kWR + 2) * (kWC + 2);
        const int q0 = cs * QW;
        for (int r = 0; r < kWR; ++r) {
            float w0[3], w1[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                w0[t] = xi[(r + t) * (kWC + 2) + q0];
                w1[t] = xi[(r + t) * (kWC + 2) + q0 + 1];
            }
            for (int q = q0; q < q0 + QW; ++q) {
                float w2[3];
#pragma unroll
                for (int t = 0; t < 3; ++t) w2[t] = xi[(r + t) * (kWC + 2) + q + 2];
                const float gv = gi[r * kWC + q];
                bacc += gv;
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    acc[3 * t + 0] = fmaf(gv, w0[t], acc[3 * t + 0]);
                    acc[3 * t + 1] = fmaf(gv, w1[t], acc[3 * t + 1]);
                    acc[3 * t + 2] = fmaf(gv, w2[t], acc[3 * t + 2]);
                    w0[t] = w1[t];
                    w1[t] = w2[t];
                }
            }
        }
    }
    if (CS > 1) {
        // add the column splits in order (thread (0, o, i) keeps the sum)
        float* red = s_in;
        __syncthreads();
        const int slot = (threadIdx.x % (OG * 16)) * 10;
        if (cs > 0) {
#pragma unroll
            for (int t = 0; t < 9; ++t) red[((cs - 1) * OG * 16) * 10 + slot + t] = acc[t];
            red[((cs - 1) * OG * 16) * 10 + slot + 9] = bacc;
        }
        __syncthreads();
        if (cs > 0) return;
        for (int k = 0; k < CS - 1; ++k) {
#pragma unroll
            for (int t = 0; t < 9; ++t) acc[t] += red[(k * OG * 16) * 10 + slot + t];
            bacc += red[(k * OG * 16) * 10 + slot + 9];
        }
    }
    const int o = o0 + ol, i = i0 + il;
    float* part = a.partial + (int64_t)blockIdx.x * a.J;
    if (o < a.Cout && i < a.Cin) {
#pragma unroll
        for (int t = 0; t < 9; ++t) part[((int64_t)o * a.Cin + i) * 9 + t] = acc[t];
    }
    if (o < a.Cout && i0 == 0 && il == 0) part[(int64_t)a.Cout * a.Cin * 9 + o] = bacc;
}

// out[j] = sum over the parts (in order) of partial[part][j]
__global__ __launch_bounds__(1024) void k_reduce_parts(const float* __restrict__ partial, int parts, int64_t J,
                                                       float* __restrict__ out) {
    __shared__ float red[16][64];
    const int jj = threadIdx.x % 64, pp = threadIdx.x / 64;
    const int64_t j = (int64_t)blockIdx.x * 64 + jj;
    float s = 0.f;
    if (j < J)
        for (int p = pp; p < parts; p += 16) s += partial[(int64_t)p * J + j];
    red[pp][jj] = s;
    __syncthreads();
    if (pp == 0 && j < J) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += red[k][jj];
        out[j] = t;
    }
}

// pixel shuffle by 2: out[c][2y+i][2x+j] = in[4c+2i+j][y][x] (inverse: the
// same map read the other way)
__global__ __launch_bounds__(kT) void k_shuffle(const float* __restrict__ in, int C, int h, int w,
                                                float* __restrict__ out, int inverse) {
    const int64_t n = (int64_t)4 * C * h * w;
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= n) return;
    // q indexes the shuffled map [C][2h][2w]
    const int W2 = 2 * w, H2 = 2 * h;
    const int c = (int)(q / ((int64_t)H2 * W2));
    const int64_t r = q - (int64_t)c * H2 * W2;
    const int Y = (int)(r / W2), X = (int)(r - (int64_t)Y * W2);
    const int64_t src = ((int64_t)(4 * c + 2 * (Y & 1) + (X & 1)) * h + (Y >> 1)) * w + (X >> 1);
    if (inverse) out[src] = in[q];
    else out[q] = in[src];
}

// per-axis interpolation tables (half-pixel centres), FP64 coordinates
__global__ void k_bilin_table(int n_in, int n_out, int* __restrict__ i0, int* __restrict__ i1, float* __restrict__ f) {
    const int d = blockIdx.x * kT + threadIdx.x;
    if (d >= n_out) return;
    double s = ((double)d + 0.5) * (double)n_in / (double)n_out - 0.5;
    if (s < 0.0) s = 0.0;
    int a = (int)floor(s);
    if (a > n_in - 1) a = n_in - 1;
    i0[d] = a;
    i1[d] = min(a + 1, n_in - 1);
    f[d] = (float)(s - (double)a);
}

constexpr int kRows = 8;   // rows per workgroup of the interpolation kernels

// kRows output rows (channel c, row Y) per workgroup, one column per
// thread: the column's taps are read once, the rows' loads are independent
__global__ __launch_bounds__(kT) void k_bilinear(const float* __restrict__ in, int C, int h, int w, int H, int W,
                                                 const int* __restrict__ y0, const int* __restrict__ y1,
                                                 const float* __restrict__ fy, const int* __restrict__ x0,
                                                 const int* __restrict__ x1, const float* __restrict__ fx,
                                                 float* __restrict__ out) {
    int bx, by;
    xcd_tile(&bx, &by);
    const int X = bx * kT + (int)threadIdx.x;
    if (X >= W) return;
    const int ex0 = x0[X], ex1 = x1[X];
    const float e = fx[X];
    const int rows = C * H;
    for (int r0 = by * kRows; r0 < rows; r0 += (int)gridDim.y * kRows) {
        // all loads of the kRows rows first (rows past the end repeat the
        // last one and are not stored), then the blends
        float v[kRows][4], a[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int row = min(r0 + k, rows - 1);
            const int c = row / H, Y = row - c * H;
            const float* b = in + (int64_t)c * h * w;
            const float* p0 = b + (int64_t)y0[Y] * w;
            const float* p1 = b + (int64_t)y1[Y] * w;
            a[k] = fy[Y];
            v[k][0] = p0[ex0];
            v[k][1] = p0[ex1];
            v[k][2] = p1[ex0];
            v[k][3] = p1[ex1];
        }
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            if (r0 + k >= rows) break;
            const float top = (1.f - e) * v[k][0] + e * v[k][1];
            const float bot = (1.f - e) * v[k][2] + e * v[k][3];
            out[(int64_t)(r0 + k) * W + X] = (1.f - a[k]) * top + a[k] * bot;
        }
    }
}

// Row kernels of the interpolation for images up to kRowW = 2048 wide (the
// source rows then hold at most 1024 values): a workgroup handles a
// contiguous run of rows, staging each row's sources in LDS with coalesced
// loads (every load of the thread issued before its LDS writes), and each
// thread keeps the taps of its output columns in registers for all rows.
constexpr int kRowW = 2048;
constexpr int kRowCols = kRowW / kT;   // output columns per thread (forward)
constexpr int kRowSrc = kRowW / 2 / kT;   // source values per thread and row (forward)

__global__ __launch_bounds__(kT) void k_bilinear_rows(const float* __restrict__ in, int C, int h, int w, int H,
                                                      int W, const int* __restrict__ y0, const int* __restrict__ y1,
                                                      const float* __restrict__ fy, const int* __restrict__ x0,
                                                      const int* __restrict__ x1, const float* __restrict__ fx,
                                                      float* __restrict__ out) {
    extern __shared__ float s_src[];   // the two source rows, 2 w floats
    const int tid = (int)threadIdx.x;
    int ex0[kRowCols], ex1[kRowCols];
    float e[kRowCols];
#pragma unroll
    for (int m = 0; m < kRowCols; ++m) {
        const int X = tid + m * kT;
        const bool ok = X < W;
        ex0[m] = ok ? x0[X] : 0;
        ex1[m] = ok ? x1[X] : 0;
        e[m] = ok ? fx[X] : 0.f;
    }
    const int rows = C * H;
    const int chunk = (rows + (int)gridDim.x - 1) / (int)gridDim.x;
    const int r_beg = (int)blockIdx.x * chunk, r_end = min(rows, r_beg + chunk);
    // a row's source values are loaded while the previous row is blended
    float v0[kRowSrc], v1[kRowSrc], an = 0.f;
    auto load = [&](int row) {
        const int c = row / H, Y = row - c * H;
        const float* p0 = in + ((int64_t)c * h + y0[Y]) * w;
        const float* p1 = in + ((int64_t)c * h + y1[Y]) * w;
        an = fy[Y];
#pragma unroll
        for (int j = 0; j < kRowSrc; ++j) {
            const int k = tid + j * kT;
            v0[j] = p0[k < w ? k : 0];
            v1[j] = p1[k < w ? k : 0];
        }
    };
    if (r_beg < r_end) load(r_beg);
    for (int row = r_beg; row < r_end; ++row) {
        const float a = an;
        __syncthreads();   // the previous row's blends are done with s_src
#pragma unroll
        for (int j = 0; j < kRowSrc; ++j) {
            const int k = tid + j * kT;
            if (k < w) {
                s_src[k] = v0[j];
                s_src[w + k] = v1[j];
            }
        }
        __syncthreads();
        if (row + 1 < r_end) load(row + 1);
#pragma unroll
        for (int m = 0; m < kRowCols; ++m) {
            const int X = tid + m * kT;
            if (X < W) {
                const float top = (1.f - e[m]) * s_src[ex0[m]] + e[m] * s_src[ex1[m]];
                const float bot = (1.f - e[m]) * s_src[w + ex0[m]] + e[m] * s_src[w + ex1[m]];
                out[(int64_t)row * W + X] = (1.f - a) * top + a * bot;
            }
        }
    }
}

// Outputs d reading input i along one axis are those with i0[d] <= i <=
// i1[d] (i1 is i0 or i0 + 1, both nondecreasing in d): a contiguous range,
// found by a short scan from its estimate.
__device__ __forceinline__ void axis_range(int i, int n_in, int n_out, const int* i0, const int* i1, int* lo, int* hi) {
    const float sc = (float)n_out / (float)n_in;
    int d = (int)floorf(((float)i - 0.5f) * sc - 0.5f) - 2;
    d = max(0, min(d, n_out));
    while (d > 0 && i1[d - 1] >= i) --d;
    while (d < n_out && i1[d] < i) ++d;
    int e = d;
    while (e < n_out && i0[e] <= i) ++e;
    *lo = d;
    *hi = e;
}

// per input index, the [lo, hi) range of outputs that read it
__global__ void k_bilin_ranges(int n_in, int n_out, const int* __restrict__ i0, const int* __restrict__ i1,
                               int* __restrict__ lo, int* __restrict__ hi) {
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= n_in) return;
    int a, b;
    axis_range(i, n_in, n_out, i0, i1, &a, &b);
    lo[i] = a;
    hi[i] = b;
}

// Adjoint of k_bilinear along x: tmp[c][Y][i] = sum over the outputs X
// that read input column i of their weight times g[c][Y][X] (one row per
// grid row, one input column per thread)
__device__ __forceinline__ float adj_weight(int d, int i, const int* i0, const int* i1, const float* f) {
    return (i0[d] == i ? 1.f - f[d] : 0.f) + (i1[d] == i ? f[d] : 0.f);
}

__global__ __launch_bounds__(kT) void k_bilin_adj_x(const float* __restrict__ g, int rows, int W, int w,
                                                    const int* __restrict__ i0, const int* __restrict__ i1,
                                                    const float* __restrict__ f, const int* __restrict__ rlo,
                                                    const int* __restrict__ rhi, float* __restrict__ out) {
    int bx, by;
    xcd_tile(&bx, &by);
    const int i = bx * kT + (int)threadIdx.x;
    if (i >= w) return;
    const int lo = rlo[i], hi = rhi[i];
    // upsampling by at most 2 (the only use): at most four outputs read an
    // input, five at the clamped last one; their taps are loaded once,
    // padded to six with weight-0 taps (which leave the sum unchanged);
    // longer ranges take the plain loop
    constexpr int K = 6;
    const bool fits = hi - lo <= K;
    int dk[K];
    float wk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const bool on = lo + k < hi;
        dk[k] = on ? lo + k : 0;
        wk[k] = on ? adj_weight(lo + k, i, i0, i1, f) : 0.f;
    }
    for (int r0 = by * kRows; r0 < rows; r0 += (int)gridDim.y * kRows) {
        if (fits) {
            float v[kRows][K];
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                const float* gl = g + (int64_t)min(r0 + k, rows - 1) * W;
#pragma unroll
                for (int t = 0; t < K; ++t) v[k][t] = gl[dk[t]];
            }
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                if (r0 + k >= rows) break;
                float s = 0.f;
#pragma unroll
                for (int t = 0; t < K; ++t) s = fmaf(wk[t], v[k][t], s);
                out[(int64_t)(r0 + k) * w + i] = s;
            }
        } else {
            for (int k = 0; k < kRows && r0 + k < rows; ++k) {
                const float* gl = g + (int64_t)(r0 + k) * W;
                float s = 0.f;
                for (int d = lo; d < hi; ++d) s = fmaf(adj_weight(d, i, i0, i1, f), gl[d], s);
                out[(int64_t)(r0 + k) * w + i] = s;
            }
        }
    }
}

// The x pass of the adjoint as a row kernel: the row of g (W <= kRowW) is
// staged in LDS; thread columns i = tid + m kT (i < w <= kRowW / 2) keep
// their taps in registers (at most four when upsampling by at most 2, five
// at the clamped last input; padded to six with weight-0 taps; a longer
// range falls back to the plain loop over the staged row).
__global__ __launch_bounds__(kT) void k_bilin_adj_x_rows(const float* __restrict__ g, int rows, int W, int w,
                                                         const int* __restrict__ i0, const int* __restrict__ i1,
                                                         const float* __restrict__ f, const int* __restrict__ rlo,
                                                         const int* __restrict__ rhi, float* __restrict__ out) {
    extern __shared__ float s_row[];   // W floats
    constexpr int M = kRowW / 2 / kT, K = 6, J = kRowW / kT;
    const int tid = (int)threadIdx.x;
    int dk[M][K], lo[M], hi[M];
    float wk[M][K];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = tid + m * kT;
        lo[m] = i < w ? rlo[i] : 0;
        hi[m] = i < w ? rhi[i] : 0;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const bool on = lo[m] + t < hi[m];
            dk[m][t] = on ? lo[m] + t : 0;
            wk[m][t] = on ? adj_weight(lo[m] + t, i, i0, i1, f) : 0.f;
        }
    }
    const int chunk = (rows + (int)gridDim.x - 1) / (int)gridDim.x;
    const int r_beg = (int)blockIdx.x * chunk, r_end = min(rows, r_beg + chunk);
    // a row is loaded while the previous row's sums are formed
    float v[J];
    auto load = [&](int row) {
        const float* gl = g + (int64_t)row * W;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int k = tid + j * kT;
            v[j] = gl[k < W ? k : 0];
        }
    };
    if (r_beg < r_end) load(r_beg);
    for (int row = r_beg; row < r_end; ++row) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int k = tid + j * kT;
            if (k < W) s_row[k] = v[j];
        }
        __syncthreads();
        if (row + 1 < r_end) load(row + 1);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int i = tid + m * kT;
            if (i < w) {
                float s = 0.f;
                if (hi[m] - lo[m] <= K) {
#pragma unroll
                    for (int t = 0; t < K; ++t) s = fmaf(wk[m][t], s_row[dk[m][t]], s);
                } else {
                    for (int d = lo[m]; d < hi[m]; ++d) s = fmaf(adj_weight(d, i, i0, i1, f), s_row[d], s);
                }
                out[(int64_t)row * w + i] = s;
            }
        }
    }
}

// ... and along y: out[c][i][x] = sum over the output rows Y that read
// input row i of their weight times tmp[c][Y][x] (one (c, i) per grid row,
// one column per thread)
__global__ __launch_bounds__(kT) void k_bilin_adj_y(const float* __restrict__ tmp, int C, int H, int h, int w,
                                                    const int* __restrict__ i0, const int* __restrict__ i1,
                                                    const float* __restrict__ f, const int* __restrict__ rlo,
                                                    const int* __restrict__ rhi, float* __restrict__ out) {
    int bx, by;
    xcd_tile(&bx, &by);
    const int x = bx * kT + (int)threadIdx.x;
    if (x >= w) return;
    const int rows = C * h;
    constexpr int K = 6;   // as in the x pass: at most five taps when upsampling by at most 2
    for (int r0 = by * kRows; r0 < rows; r0 += (int)gridDim.y * kRows) {
        float v[kRows][K], wt[kRows][K];
        bool fits = true;
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int row = min(r0 + k, rows - 1);
            const int c = row / h, i = row - c * h;
            const int lo = rlo[i], hi = rhi[i];
            fits = fits && hi - lo <= K;
            const float* tc = tmp + (int64_t)c * H * w + x;
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const bool on = lo + t < hi;
                const int d = on ? lo + t : 0;
                wt[k][t] = on ? adj_weight(d, i, i0, i1, f) : 0.f;
                v[k][t] = tc[(int64_t)d * w];
            }
        }
        if (fits) {
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                if (r0 + k >= rows) break;
                float s = 0.f;
#pragma unroll
                for (int t = 0; t < K; ++t) s = fmaf(wt[k][t], v[k][t], s);
                out[(int64_t)(r0 + k) * w + x] = s;
            }
        } else {
            for (int k = 0; k < kRows && r0 + k < rows; ++k) {
                const int row = r0 + k;
                const int c = row / h, i = row - c * h;
                const int lo = rlo[i], hi = rhi[i];
                const float* tc = tmp + (int64_t)c * H * w + x;
                float s = 0.f;
                for (int d = lo; d < hi; ++d) s = fmaf(adj_weight(d, i, i0, i1, f), tc[(int64_t)d * w], s);
                out[(int64_t)row * w + x] = s;
            }
        }
    }
}

__global__ __launch_bounds__(kT) void k_mul(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                            float* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q < n) out[q] = a[q] * b[q];
}

// dM = dIa * Ir; dIr += dIa * M
__global__ __launch_bounds__(kT) void k_mul_bwd(const float* __restrict__ d_adj, const float* __restrict__ img,
                                                const float* __restrict__ M, int64_t n, float* __restrict__ dM,
                                                float* __restrict__ d_img) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= n) return;
    const float g = d_adj[q];
    dM[q] = g * img[q];
    d_img[q] += g * M[q];
}

// d_embed[k] = sum over the pixels of channel 3 + k of dD
__global__ __launch_bounds__(kT) void k_embed_grad(const float* __restrict__ dD, int64_t hw, float* __restrict__ d_embed) {
    __shared__ float red[kT / kWave];
    const float* src = dD + (int64_t)(3 + blockIdx.x) * hw;
    float s = 0.f;
    for (int64_t p = threadIdx.x; p < hw; p += kT) s += src[p];
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < kT / kWave; ++k) t += red[k];
        d_embed[blockIdx.x] = t;
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

void launch_down_concat(const float* img, int H, int W, int h, int w, const float* embed, int m, float* D,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_down_concat, dim3(h * w), dim3(kT), 0, st, img, H, W, h, w, embed, m, D);
}

void launch_down_adjoint(const float* g, int H, int W, int h, int w, float* d_img, hipStream_t st) {
    hipLaunchKernelGGL(k_down_adjoint, dim3(blocks_for(3 * (int64_t)H * W)), dim3(kT), 0, st, g, H, W, h, w, d_img);
}

int conv_splits(int Cin, int Cout, int H, int W) {
    if (Cout <= 4) return 1;   // the VALU kernel
    // the low-resolution layers give too few workgroups to fill 256 CUs:
    // split their input channels until the grid has about 2048
    const int64_t wgs = (int64_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile) * ((Cout + 15) / 16);
    const int chunks = (Cin + kCI - 1) / kCI;
    if (wgs >= 1024 || chunks < 2) return 1;
    const int want = (int)std::min<int64_t>(chunks, (2048 + wgs - 1) / wgs);
    const int cps = (chunks + want - 1) / want;
    return (chunks + cps - 1) / cps;
}

void launch_conv(const ConvArgs& a, hipStream_t st) {
    if (a.Cout > 4) {
        // a dense contraction over 9 Cin: the matrix cores
        const int splits = a.part ? conv_splits(a.Cin, a.Cout, a.H, a.W) : 1;
        const int chunks = (a.Cin + kCI - 1) / kCI;
        const int cps = (chunks + splits - 1) / splits;
        const int n_og = (a.Cout + 15) / 16;
        const dim3 grid((a.W + kTile - 1) / kTile, (a.H + kTile - 1) / kTile, n_og * splits);
        if (a.mask) hipLaunchKernelGGL(k_conv_mfma<true>, grid, dim3(kT), 0, st, a, splits, cps);
        else hipLaunchKernelGGL(k_conv_mfma<false>, grid, dim3(kT), 0, st, a, splits, cps);
        if (splits > 1) {
            const int64_t HW = (int64_t)a.H * a.W;
            hipLaunchKernelGGL(k_conv_reduce, dim3(blocks_for(HW), a.Cout), dim3(kT), 0, st, a.part, splits, a.Cout,
                               HW, a.b, a.relu, a.out);
        }
        return;
    }
    // three or four output channels (the map M): most of a 16-row matrix
    // tile would be padding, so the VALU kernel, with the shape that still
    // gives every CU four workgroups
    const int r = ((int64_t)((a.W + kTile - 1) / kTile) * ((a.H + 2 * kTile - 1) / (2 * kTile)) >= 1024) ? 2 : 1;
    const unsigned gx = (a.W + kTile - 1) / kTile, gy = (a.H + kTile * r - 1) / (kTile * r);
    if (a.mask) {
        if (r == 2) hipLaunchKernelGGL((k_conv<4, 2, true>), dim3(gx, gy, 1), dim3(kT), 0, st, a);
        else hipLaunchKernelGGL((k_conv<4, 1, true>), dim3(gx, gy, 1), dim3(kT), 0, st, a);
    } else {
        if (r == 2) hipLaunchKernelGGL((k_conv<4, 2, false>), dim3(gx, gy, 1), dim3(kT), 0, st, a);
        else hipLaunchKernelGGL((k_conv<4, 1, false>), dim3(gx, gy, 1), dim3(kT), 0, st, a);
    }
}

int wgrad_parts(int H, int W) {
    const int tiles = ((W + kWC - 1) / kWC) * ((H + kWR - 1) / kWR);
    return tiles < 1024 ? tiles : 1024;
}

void launch_wgrad(const WgradArgs& a, float* dw, hipStream_t st) {
    const int parts = wgrad_parts(a.H, a.W);
    const bool m = a.mask != nullptr;
    if (a.Cout <= 4) {
        const dim3 grid(parts, (a.Cin + 15) / 16);
        if (m) hipLaunchKernelGGL((k_wgrad<4, true>), grid, dim3(kT), 0, st, a);
        else hipLaunchKernelGGL((k_wgrad<4, false>), grid, dim3(kT), 0, st, a);
    } else {
        const dim3 grid(parts, ((a.Cout + 15) / 16) * ((a.Cin + 15) / 16));
        if (m) hipLaunchKernelGGL((k_wgrad<16, true>), grid, dim3(kT), 0, st, a);
        else hipLaunchKernelGGL((k_wgrad<16, false>), grid, dim3(kT), 0, st, a);
    }
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((a.J + 63) / 64)), dim3(1024), 0, st, a.partial, parts, a.J, dw);
}

void launch_shuffle(const float* in, int C, int h, int w, float* out, bool inverse, hipStream_t st) {
    hipLaunchKernelGGL(k_shuffle, dim3(blocks_for((int64_t)4 * C * h * w)), dim3(kT), 0, st, in, C, h, w, out,
                       inverse ? 1 : 0);
}

void launch_bilin_table(int n_in, int n_out, int* i0, int* i1, float* f, hipStream_t st) {
    hipLaunchKernelGGL(k_bilin_table, dim3(blocks_for(n_out)), dim3(kT), 0, st, n_in, n_out, i0, i1, f);
}

// workgroup rows for kRows rows each (the kernels stride over the rest)
unsigned grid_rows(int64_t rows) { return (unsigned)std::min<int64_t>((rows + kRows - 1) / kRows, 65535); }

// workgroups of the row kernels: about eight per CU, each a run of rows
unsigned row_groups(int64_t rows) { return (unsigned)std::min<int64_t>(rows, 2048); }

void launch_bilinear(const float* in, int C, int h, int w, int H, int W, const BilinTab& t, float* out,
                     hipStream_t st) {
    if (W <= kRowW) {
        const int64_t rows = (int64_t)C * H;
        hipLaunchKernelGGL(k_bilinear_rows, dim3(row_groups(rows)), dim3(kT), 2 * w * sizeof(float), st, in, C, h, w,
                           H, W, t.y0, t.y1, t.fy, t.x0, t.x1, t.fx, out);
        return;
    }
    hipLaunchKernelGGL(k_bilinear, dim3(blocks_for(W), grid_rows((int64_t)C * H)), dim3(kT), 0, st, in, C, h, w, H,
                       W, t.y0, t.y1, t.fy, t.x0, t.x1, t.fx, out);
}

void launch_bilinear_adj(const float* g, int C, int H, int W, int h, int w, const BilinTab& t, float* tmp,
                         float* out, hipStream_t st) {
    // x pass: [C][H][W] -> tmp [C][H][w]; lines = C H rows
    const int64_t rows = (int64_t)C * H;
    hipLaunchKernelGGL(k_bilin_ranges, dim3(blocks_for(w)), dim3(kT), 0, st, w, W, t.x0, t.x1, t.xlo, t.xhi);
    hipLaunchKernelGGL(k_bilin_ranges, dim3(blocks_for(h)), dim3(kT), 0, st, h, H, t.y0, t.y1, t.ylo, t.yhi);
    if (W <= kRowW)
        hipLaunchKernelGGL(k_bilin_adj_x_rows, dim3(row_groups(rows)), dim3(kT), W * sizeof(float), st, g, (int)rows,
                           W, w, t.x0, t.x1, t.fx, t.xlo, t.xhi, tmp);
    else
        hipLaunchKernelGGL(k_bilin_adj_x, dim3(blocks_for(w), grid_rows(rows)), dim3(kT), 0, st, g, (int)rows, W, w,
                           t.x0, t.x1, t.fx, t.xlo, t.xhi, tmp);
    // y pass: tmp [C][H][w] -> out [C][h][w]
    hipLaunchKernelGGL(k_bilin_adj_y, dim3(blocks_for(w), grid_rows((int64_t)C * h)), dim3(kT), 0, st, tmp, C, H, h,
                       w, t.y0, t.y1, t.fy, t.ylo, t.yhi, out);
}

void launch_mul(const float* a, const float* b, int64_t n, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_mul, dim3(blocks_for(n)), dim3(kT), 0, st, a, b, n, out);
}

void launch_mul_bwd(const float* d_adj, const float* img, const float* M, int64_t n, float* dM, float* d_img,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_mul_bwd, dim3(blocks_for(n)), dim3(kT), 0, st, d_adj, img, M, n, dM, d_img);
}

void launch_embed_grad(const float* dD, int64_t hw, int m, float* d_embed, hipStream_t st) {
    hipLaunchKernelGGL(k_embed_grad, dim3(m), dim3(kT), 0, st, dD, hw, d_embed);
}

}  // namespace gs
