// Device-side definitions shared by the rasterizer kernels (gfx950).
//
// The image-formation model is the one VastGaussian (arXiv 2402.17427)
// inherits from 3D Gaussian Splatting (section 3; section 5.1 keeps the 3DGS
// settings): 2D Gaussians blended front to back with alpha = min(0.99,
// o exp(power)), contributions below 1/255 skipped and a pixel finished
// before the Gaussian that would take its transmittance below 1e-4.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace gs {

// Image-formation constants.
constexpr float kDilation = 0.3f;     // px^2 added to the projected covariance
constexpr float kFovClamp = 1.3f;     // affine-approximation clamp of x/z, y/z
constexpr double kFovClampD = 1.3;    // the same in FP64 (the projection's geometry)
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kLog2e = 1.4426950408889634f;

constexpr int kWave = 64;

// Projected Gaussian, 48 bytes, read as three 16-byte vectors.  The centre
// is kept in FP64 so that pixel offsets can be formed to a few ulp of the
// offset itself, whatever the image size.
struct alignas(16) Rec {
    double u, v;        // pixel-space centre
    float A, B, C, o;   // conic (inverse 2D covariance) and opacity
    float r, g, b;      // colour
    float thr;          // -log2(255 o): alpha >= 1/255 exactly where the
                        // base-2 exponent of the Gaussian is >= thr
};
static_assert(sizeof(Rec) == 48, "record layout");

// Camera as the kernels see it (mirrors gs_camera).
struct Cam {
    float R[9], t[3];
    float fx, fy, cx, cy;
    int W, H;
    float near_z;
    float bg[3];
    double limx, limy;   // affine-approximation clamp of x/z and y/z: 1.3 (W/2) / fx, 1.3 (H/2) / fy
};

// Gaussian SoA planes (mirrors gs_gaussians).
struct Gauss {
    int64_t n, ld;
    int deg, K;
    const float *mean, *scale, *quat, *opacity, *sh;
};

// ---- batches of views ------------------------------------------------
// The kernels render a set of views at once.  Tiles of all views are
// numbered consecutively (view v owns global tiles tile_base ..
// tile_base + ntx * nty - 1) and the images are stacked; a "job" projects
// a range of a Gaussian set into one view, into consecutive record slots
// starting at out0 (a multiple of kSlotAlign, so that a workgroup of the
// per-slot kernels never spans two jobs).  One view with one job is the
// plain single-view render.
constexpr int kSlotAlign = 256;

struct View {
    Cam cam;
    int ntx, nty;          // tiles of this view
    uint32_t tile_base;    // first global tile id of the view
    int64_t img_base;      // offset (floats) of the view's [3][H][W] image
    int64_t pix_base;      // offset of the view's [H][W] planes (final_T, n_contrib, dL/dimage is at img_base)
    float* out_image;      // when set, the forward writes this view's image here instead
};

struct Job {
    Gauss g;                        // SoA planes of the Gaussian set
    int64_t src0, count, out0;      // Gaussians src0 .. src0+count-1 -> slots out0 ..
    int view;
    float *gmean, *gscale, *gquat, *gopac, *gsh;   // gradient planes (stride gld, index src0 + k)
    int64_t gld;
};

// A table lives in device memory (dev != nullptr, n entries) or is the
// single entry carried in the kernel arguments.
struct ViewTab {
    const View* dev;
    int n;
    View one;
};
struct JobTab {
    const Job* dev;
    int n;
    Job one;
};

// Job owning record slot `slot` (jobs sorted by out0); uniform per workgroup.
__device__ __forceinline__ int find_job(const JobTab& t, int64_t slot) {
    if (!t.dev) return 0;
    int lo = 0, hi = t.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.dev[mid].out0 <= slot) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ Job job_at(const JobTab& t, int j) { return t.dev ? t.dev[j] : t.one; }

// View owning global tile `tile` (views sorted by tile_base).
__device__ __forceinline__ int find_view(const ViewTab& t, uint32_t tile) {
    if (!t.dev) return 0;
    int lo = 0, hi = t.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.dev[mid].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ View view_at(const ViewTab& t, int v) { return t.dev ? t.dev[v] : t.one; }

// One projected Gaussian staged in LDS for a tile.  The centre is held as
// an unevaluated float sum hi + lo of the FP64 centre, and a pixel offset is
// formed as (pixel centre - hi) - lo: a function of the pixel and the
// Gaussian only, so the result does not depend on the tile size or origin,
// and its error is a few ulp of the offset itself.  The conic is pre-scaled
// so that exp2(ca dx^2 + cb dx dy + cc dy^2) = exp(power).  Forward and
// backward stage the same values through stage_rec() and evaluate the
// exponent with the same expression, so both take identical decisions.
struct Staged {
    float4 geo;   // hi_u, lo_u, hi_v, lo_v
    float4 coef;  // ca, cb, cc, o
    float4 col;   // r, g, b, thr
};

__device__ __forceinline__ Staged stage_rec(const Rec& r) {
    Staged s;
    const float hu = (float)r.u, hv = (float)r.v;
    s.geo = make_float4(hu, (float)(r.u - (double)hu), hv, (float)(r.v - (double)hv));
    s.coef = make_float4(r.A * (-0.5f * kLog2e), r.B * (-kLog2e), r.C * (-0.5f * kLog2e), r.o);
    s.col = make_float4(r.r, r.g, r.b, r.thr);
    return s;
}

// The value of lane ^ s (s a power of two below 64), by the cheapest
// exchange for each distance.  Must be called by all 64 lanes of the wave.
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int s) {
    switch (s) {
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
    case 4: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);              // xor 4 in 32 lanes
    case 8: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, true);  // row_ror:8
    case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);             // xor 16 in 32 lanes
    default: return (uint32_t)__shfl_xor((int)v, 32, kWave);
    }
}

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace gs
