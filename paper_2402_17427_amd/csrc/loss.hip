// The training loss of one image and its gradient, fused in one pass.
//
// VastGaussian (arXiv 2402.17427) optimises each cell's Gaussians against
// its training images with the loss of Eq. 1 (section 3):
// (1 - lambda) L1(I^r, I) + lambda D-SSIM(I^r, I), and, with decoupled
// appearance modelling, Eq. 3 (section 4.2): the L1 term on the adjusted
// image I^a and the D-SSIM term on the rendered I^r.  D-SSIM comes from
// 3DGS: 1 - SSIM, SSIM averaged over every pixel and channel, with an
// 11 x 11 Gaussian window (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, and window
// sums that treat the outside of the image as zero.
//
// Per pixel p, with the window sums m = G*x, E = G*x^2, X = G*xy (x = I^r)
// and mu_y, E_y of the target, the SSIM map is S = a1 a2 / (b1 b2),
// a1 = 2 m mu_y + C1, a2 = 2 (X - m mu_y) + C2, b1 = m^2 + mu_y^2 + C1,
// b2 = (E - m^2) + (E_y - mu_y^2) + C2.  With g = dLoss/dS = -lambda / n,
//   dm = g 2 (mu_y (a2 - a1) - m S (b2 - b1)) / (b1 b2),
//   dE = -g S / b2,   dX = g 2 a1 / (b1 b2),
// and because the window is symmetric and zero padded, the gradient of the
// D-SSIM term at pixel q is (G*dm)(q) + 2 x(q) (G*dE)(q) + y(q) (G*dX)(q),
// the maps dm, dE, dX being zero outside the image.
//
// One workgroup computes one 32 x 32 output tile of one channel entirely
// in LDS: the input with a 10-pixel halo, the five forward window sums on
// the tile plus a 5-pixel halo (separable: a horizontal then a vertical
// 11-tap pass, three planes at a time so that three workgroups fit on a
// CU), the three SSIM partials there, their window sums on the tile (again
// two passes), and the L1 term.  Halo recompute replaces any
// intermediate HBM traffic: the kernel reads the images once (plus the
// halos, mostly from cache) and writes the gradient once.  The loss value
// is reduced from per-workgroup partial sums by a second, one-workgroup
// kernel in double precision, in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "api_internal.h"
#include "kernels.h"

namespace gs {

namespace {

constexpr int kXcds = 8;          // XCDs of an MI355X (workgroups are dealt round-robin)
constexpr int kThreads = 256;
constexpr int kT = 32;            // output tile edge
constexpr int kR = 5;             // window radius
constexpr int kTaps = 2 * kR + 1;
constexpr int kAY = kT + 4 * kR;  // input rows (52)
constexpr int kAX = 56;           // input row stride; columns loaded: 54
constexpr int kALoad = 54;
constexpr int kBY = kT + 2 * kR;  // rows of the forward sums / partials (42)
constexpr int kBX = kT + 2 * kR;  // their columns (42)
constexpr int kHX = 44;           // row stride of the horizontal sums (4 groups of 11)
constexpr int kHGroup = 11;       // columns per thread in the forward horizontal pass
constexpr int kVGroup = 7;        // rows per thread in the forward vertical pass (42 = 6 x 7)
constexpr int kQGroup = 8;        // columns per thread in the backward horizontal pass
constexpr int kDGroup = 4;        // rows per thread in the backward vertical pass

constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

constexpr int kSA = kAY * kAX;      // one input plane
constexpr int kSH = kAY * kHX;      // one horizontal-sum plane
constexpr int kSP = kBY * kHX;      // one partial plane
constexpr int kSQ = kBY * kT;       // one backward horizontal plane
constexpr int kRegX = 2 * kSA;      // inputs; later the backward horizontal sums
constexpr int kRegH = 3 * kSH;      // horizontal sums; later the partials
constexpr int kLdsFloats = kRegX + kRegH;  // 50.8 KB: three workgroups per CU
static_assert(3 * kSQ <= kRegX, "backward horizontal sums reuse the input planes");
static_assert(3 * kSP <= kRegH, "partials reuse the horizontal sums");

struct Win {
    float g[kTaps];
};

struct LossArgs {
    const float* x;    // I^r  [C][H][W]
    const float* xa;   // I^a  [C][H][W] or NULL (then x)
    const float* y;    // I    [C][H][W]
    float* dx;         // [C][H][W]
    float* dxa;        // [C][H][W] or NULL
    float2* partial;   // per workgroup (sum S, sum |xa - y|)
    int W, H;
    int tiles_x, tiles_y;
    float gs;          // dLoss/dS = -lambda / n
    float g1;          // (1 - lambda) / n
    Win win;
};

__device__ __forceinline__ float wave_sum(float v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Horizontal 11-tap sums of NM products of the input rows: thread
// (row r, group j) writes columns 11j .. 11j+10 of row r of each plane.
template <int NM, typename F>
__device__ __forceinline__ void hpass(const Win& win, const float* sx, const float* sy, float* sh, int tid, F prod) {
    if (tid >= kAY * 4) return;
    const int r = tid >> 2, c0 = (tid & 3) * kHGroup;
    float vx[kHGroup + 2 * kR], vy[kHGroup + 2 * kR];
#pragma unroll
    for (int t = 0; t < kHGroup + 2 * kR; ++t) {
        vx[t] = sx[r * kAX + c0 + t];
        vy[t] = sy[r * kAX + c0 + t];
    }
    float pr[NM][kHGroup + 2 * kR];
#pragma unroll
    for (int t = 0; t < kHGroup + 2 * kR; ++t) prod(vx[t], vy[t], pr, t);
#pragma unroll
    for (int o = 0; o < kHGroup; ++o) {
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < kTaps; ++t) s = fmaf(win.g[t], pr[m][o + t], s);
            sh[m * kSH + r * kHX + c0 + o] = s;
        }
    }
}

// Vertical 11-tap sums of NM horizontal-sum planes: thread (column vc,
// group) produces rows vr0 .. vr0+6 of the tile-plus-halo region.
template <int NM>
__device__ __forceinline__ void vpass(const Win& win, const float* sh, int vc, int vr0, float (&acc)[NM][kVGroup]) {
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        float col[kVGroup + 2 * kR];
#pragma unroll
        for (int t = 0; t < kVGroup + 2 * kR; ++t) col[t] = sh[m * kSH + (vr0 + t) * kHX + vc];
#pragma unroll
        for (int o = 0; o < kVGroup; ++o) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < kTaps; ++t) s = fmaf(win.g[t], col[o + t], s);
            acc[m][o] = s;
        }
    }
}

__global__ __launch_bounds__(kThreads, 3) void k_loss(LossArgs a) {
    __shared__ float lds[kLdsFloats];
    float* sx = lds;
    float* sy = lds + kSA;
    float* sq = lds;          // 3 planes [kBY][kT], after the inputs are consumed
    float* sh = lds + kRegX;  // 3 planes [kAY][kHX]
    float* sp = sh;           // 3 planes [kBY][kHX], after the sums are consumed
    __shared__ float red[2][kThreads / kWave];

    const int tid = threadIdx.x;
    // Workgroups are dealt round-robin to the XCDs: give each XCD a
    // contiguous band of tiles so that neighbouring tiles, which read each
    // other's halos, share an L2.
    const int nb = a.tiles_x * a.tiles_y * (int)gridDim.z;
    const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int per = nb / kXcds;
    const int lb = b < per * kXcds ? (b % kXcds) * per + b / kXcds : b;
    const int ch = lb / (a.tiles_x * a.tiles_y);
    const int rem = lb - ch * a.tiles_x * a.tiles_y;
    const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
    const int x0 = tx * kT, y0 = ty * kT;
    const int W = a.W, H = a.H;
    const int64_t plane = (int64_t)ch * W * H;
    const float* __restrict__ gx = a.x + plane;
    const float* __restrict__ gy = a.y + plane;

    // ---- input with a 10-pixel halo, zero outside the image: a wave per
    // row (lanes 0..53 load), four rows per pass
    {
        const int c = tid % kWave, px = x0 - 2 * kR + c;
        const bool col_ok = c < kALoad && px >= 0 && px < W;
        for (int r = tid / kWave; r < kAY; r += kThreads / kWave) {
            const int py = y0 - 2 * kR + r;
            float vx = 0.f, vy = 0.f;
            if (col_ok && py >= 0 && py < H) {
                const int64_t q = (int64_t)py * W + px;
                vx = gx[q];
                vy = gy[q];
            }
            if (c < kALoad) {
                sx[r * kAX + c] = vx;
                sy[r * kAX + c] = vy;
            }
        }
    }
    __syncthreads();

    // the inputs at this thread's output pixels, for the last step
    const int oc = tid % kT, or0 = (tid / kT) * kDGroup;
    float xo[kDGroup], yo[kDGroup];
#pragma unroll
    for (int o = 0; o < kDGroup; ++o) {
        const int li = (or0 + o + 2 * kR) * kAX + oc + 2 * kR;
        xo[o] = sx[li];
        yo[o] = sy[li];
    }

    // ---- forward window sums on the tile plus a 5-pixel halo: x, y, xy
    // first, then x^2, y^2 (three horizontal planes at a time)
    const bool vact = tid < kBX * (kBY / kVGroup);
    const int vc = tid % kBX, vr0 = (tid / kBX) * kVGroup;
    hpass<3>(a.win, sx, sy, sh, tid, [](float u, float v, float (&pr)[3][kHGroup + 2 * kR], int t) {
        pr[0][t] = u;
        pr[1][t] = v;
        pr[2][t] = u * v;
    });
    __syncthreads();
    float m1[3][kVGroup];
    if (vact) vpass<3>(a.win, sh, vc, vr0, m1);
    __syncthreads();
    hpass<2>(a.win, sx, sy, sh, tid, [](float u, float v, float (&pr)[2][kHGroup + 2 * kR], int t) {
        pr[0][t] = u * u;
        pr[1][t] = v * v;
    });
    __syncthreads();

    // ---- SSIM and its partials w.r.t. the window sums of x
    float pm[kVGroup], pe[kVGroup], pxy[kVGroup];
    float ssum = 0.f;
    if (vact) {
        float m2[2][kVGroup];
        vpass<2>(a.win, sh, vc, vr0, m2);
        const int px = x0 - kR + vc;
        const bool col_in = px >= 0 && px < W;
        const bool col_tile = vc >= kR && vc < kR + kT;
#pragma unroll
        for (int o = 0; o < kVGroup; ++o) {
            const int py = y0 - kR + vr0 + o;
            const float mx = m1[0][o], my = m1[1][o];
            const float vx = m2[0][o] - mx * mx, vy = m2[1][o] - my * my, cxy = m1[2][o] - mx * my;
            const float a1 = 2.f * mx * my + kC1, a2 = 2.f * cxy + kC2;
            const float b1 = mx * mx + my * my + kC1, b2 = vx + vy + kC2;
            const float inv = __builtin_amdgcn_rcpf(b1 * b2);
            const float S = a1 * a2 * inv;
            const bool in = col_in && py >= 0 && py < H;
            const int rr = vr0 + o;
            if (in && col_tile && rr >= kR && rr < kR + kT) ssum += S;
            pm[o] = in ? a.gs * 2.f * inv * (my * (a2 - a1) - mx * S * (b2 - b1)) : 0.f;
            pe[o] = in ? -a.gs * S * b1 * inv : 0.f;
            pxy[o] = in ? a.gs * 2.f * a1 * inv : 0.f;
        }
    }
    __syncthreads();  // every read of the horizontal sums is done
    if (vact) {
#pragma unroll
        for (int o = 0; o < kVGroup; ++o) {
            const int q = (vr0 + o) * kHX + vc;
            sp[q] = pm[o];
            sp[kSP + q] = pe[o];
            sp[2 * kSP + q] = pxy[o];
        }
    }
    __syncthreads();

    // ---- backward horizontal pass: rows 0..41, output columns 0..31
    if (tid < kBY * (kT / kQGroup)) {
        const int r = tid / (kT / kQGroup), c0 = (tid % (kT / kQGroup)) * kQGroup;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            float v[kQGroup + 2 * kR];
#pragma unroll
            for (int t = 0; t < kQGroup + 2 * kR; ++t) v[t] = sp[m * kSP + r * kHX + c0 + t];
#pragma unroll
            for (int o = 0; o < kQGroup; ++o) {
                float s = 0.f;
#pragma unroll
                for (int t = 0; t < kTaps; ++t) s = fmaf(a.win.g[t], v[o + t], s);
                sq[m * kSQ + r * kT + c0 + o] = s;
            }
        }
    }
    __syncthreads();

    // ---- backward vertical pass, gradient and L1 term on the tile
    float l1sum = 0.f;
    {
        float d[3][kDGroup];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            float v[kDGroup + 2 * kR];
#pragma unroll
            for (int t = 0; t < kDGroup + 2 * kR; ++t) v[t] = sq[m * kSQ + (or0 + t) * kT + oc];
#pragma unroll
            for (int o = 0; o < kDGroup; ++o) {
                float s = 0.f;
#pragma unroll
                for (int t = 0; t < kTaps; ++t) s = fmaf(a.win.g[t], v[o + t], s);
                d[m][o] = s;
            }
        }
        const int px = x0 + oc;
#pragma unroll
        for (int o = 0; o < kDGroup; ++o) {
            const int py = y0 + or0 + o;
            if (px < W && py < H) {
                const int64_t q = plane + (int64_t)py * W + px;
                const float xa = a.xa ? a.xa[q] : xo[o];
                const float df = xa - yo[o];
                l1sum += fabsf(df);
                const float d1 = df > 0.f ? a.g1 : (df < 0.f ? -a.g1 : 0.f);
                const float ds = d[0][o] + 2.f * xo[o] * d[1][o] + yo[o] * d[2][o];
                if (a.dxa) {
                    a.dx[q] = ds;
                    a.dxa[q] = d1;
                } else {
                    a.dx[q] = ds + d1;
                }
            }
        }
    }

    // ---- per-workgroup partial sums
    ssum = wave_sum(ssum);
    l1sum = wave_sum(l1sum);
    if ((tid & (kWave - 1)) == 0) {
        red[0][tid / kWave] = ssum;
        red[1][tid / kWave] = l1sum;
    }
    __syncthreads();
    if (tid == 0) {
        float s = 0.f, l = 0.f;
        for (int k = 0; k < kThreads / kWave; ++k) {
            s += red[0][k];
            l += red[1][k];
        }
        a.partial[lb] = make_float2(s, l);
    }
}

constexpr int kFinThreads = 1024;

// loss[0] = (1 - lambda) L1 + lambda (1 - SSIM), loss[1] = L1, loss[2] = SSIM
__global__ __launch_bounds__(kFinThreads) void k_loss_finish(const float2* __restrict__ partial, int64_t count,
                                                             double n, double lam, float* __restrict__ loss,
                                                             int n_out) {
    __shared__ double red[2][kFinThreads];
    double s = 0.0, l = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kFinThreads) {
        const float2 p = partial[i];
        s += (double)p.x;
        l += (double)p.y;
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = l;
    __syncthreads();
    for (int k = kFinThreads / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            red[0][threadIdx.x] += red[0][threadIdx.x + k];
            red[1][threadIdx.x] += red[1][threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ssim = red[0][0] / n, l1 = red[1][0] / n;
        loss[0] = (float)((1.0 - lam) * l1 + lam * (1.0 - ssim));
        if (n_out == 3) {
            loss[1] = (float)l1;
            loss[2] = (float)ssim;
        }
    }
}

Win make_window() {
    Win w;
    double g[kTaps], tot = 0.0;
    for (int t = 0; t < kTaps; ++t) {
        const double k = t - kR;
        g[t] = std::exp(-k * k / (2.0 * 1.5 * 1.5));
        tot += g[t];
    }
    for (int t = 0; t < kTaps; ++t) w.g[t] = (float)(g[t] / tot);
    return w;
}

}  // namespace

int64_t loss_blocks(int channels, int width, int height) {
    return (int64_t)channels * ((width + kT - 1) / kT) * ((height + kT - 1) / kT);
}

size_t loss_workspace_bytes(int channels, int width, int height) {
    return (size_t)loss_blocks(channels, width, height) * sizeof(float2);
}

void launch_loss(const float* image, const float* image_l1, const float* target, int channels, int width, int height,
                 float lambda, float* d_image, float* d_image_l1, void* ws, hipStream_t st) {
    static const Win win = make_window();
    const double n = (double)channels * width * height;
    LossArgs a;
    a.x = image;
    a.xa = image_l1;
    a.y = target;
    a.dx = d_image;
    a.dxa = image_l1 ? d_image_l1 : nullptr;
    a.partial = static_cast<float2*>(ws);
    a.W = width;
    a.H = height;
    a.gs = (float)(-(double)lambda / n);
    a.g1 = (float)((1.0 - (double)lambda) / n);
    a.win = win;
    a.tiles_x = (width + kT - 1) / kT;
    a.tiles_y = (height + kT - 1) / kT;
    const dim3 grid(a.tiles_x, a.tiles_y, channels);
    hipLaunchKernelGGL(k_loss, grid, dim3(kThreads), 0, st, a);
}

void launch_loss_finish(int channels, int width, int height, float lambda, const void* ws, float* loss,
                        hipStream_t st, int n_out) {
    const double n = (double)channels * width * height;
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(kFinThreads), 0, st, static_cast<const float2*>(ws),
                       loss_blocks(channels, width, height), n, (double)lambda, loss, n_out);
}

}  // namespace gs

// ---- the loss without a caller workspace ---------------------------------
// For callers that cannot allocate (code under stream capture, serving
// loops): the per-tile partial sums go to a fixed device array instead of
// a workspace.  Every call on a device uses that device's copy of the
// array, so calls that overlap on one device race; each call rewrites
// every partial it reads, so nothing needs clearing between calls.
namespace gs {
namespace {

constexpr size_t kLossScratchBytes = (size_t)1 << 20;   // 131072 (tile, channel) partials: 8K RGB
static __device__ __align__(256) unsigned char scratch[kLossScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];

// Device address of the current device's `scratch`, looked up once per
// device with that device current (each device holds its own copy).
gs_status scratch_of_current_device(void** out) {
    int dev = 0;
    const hipError_t ed = hipGetDevice(&dev);
    if (ed != hipSuccess) return fail(GS_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(ed));
    if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GS_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return GS_OK;
}

}  // namespace
}  // namespace gs

extern "C" gs_status gs_loss_noalloc(const float* image, const float* image_l1, const float* target,
                                     int32_t channels, int32_t width, int32_t height, float lambda, float* loss,
                                     float* d_image, float* d_image_l1, gs_stream stream) {
    using namespace gs;
    size_t need = 0;
    gs_status s;
    if ((s = gs_loss_workspace(channels, width, height, &need))) return s;
    if (!image || !target || !loss || !d_image) return fail(GS_ERR_INVALID, "buffer is NULL");
    if (image_l1 && !d_image_l1) return fail(GS_ERR_INVALID, "image_l1 given without d_image_l1");
    if (!std::isfinite(lambda)) return fail(GS_ERR_INVALID, "lambda not finite");
    if (need > kLossScratchBytes)
        return fail(GS_ERR_CAPACITY, "a %dx%dx%d image needs %zu bytes of partial sums, more than the %zu this call holds",
                    channels, height, width, need, kLossScratchBytes);
    void* ws = nullptr;
    if ((s = scratch_of_current_device(&ws))) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_loss(image, image_l1, target, channels, width, height, lambda, d_image, image_l1 ? d_image_l1 : nullptr,
                ws, st);
    launch_loss_finish(channels, width, height, lambda, ws, loss, st);
    return check_hip("gs_loss_noalloc");
}
