// Per-Gaussian projection (forward) and its chain rule (backward).
//
// VastGaussian (arXiv 2402.17427), section 3: each 3D Gaussian (position,
// anisotropic covariance from scale and rotation, opacity, SH colour) is
// projected to an image-space 2D Gaussian by EWA splatting -- the covariance
// is pushed through the Jacobian of the perspective map at the centre -- and
// gets a view-dependent colour from its SH coefficients.  The renderer is
// differentiable (section 3), so the backward pass carries image-space
// gradients back to every parameter.
//
// One lane per Gaussian; the structure-of-arrays planes are read with
// consecutive lanes on consecutive addresses.  Geometry (view transform,
// covariance, conic, centre, support rectangle) runs in FP64: it is a few
// hundred flops per Gaussian in an HBM-bound kernel, and it makes the
// centre exact enough that the per-pixel FP32 blend sees tile-local offsets
// with ~1e-6 px error even at 4K.  The SH colour runs in FP32.
#include "gs_device.h"
#include "kernels.h"

namespace gs {

namespace {

constexpr int kProjThreads = 256;
// The geometry runs in FP64 with the constants exactly as defined.
constexpr double kDilationD = 0.3;

// Real SH basis up to degree 3 (index l*l + l + m), sign pattern of 3DGS
// scenes.  Constants: 1/(2 sqrt(pi)), sqrt(3/(4 pi)), sqrt(15/pi)/2,
// sqrt(5/pi)/4, sqrt(15/pi)/4, sqrt(35/(2 pi))/4, sqrt(105/pi)/2,
// sqrt(21/(2 pi))/4, sqrt(7/pi)/4, sqrt(105/pi)/4.
constexpr float kY0 = 0.28209479177387814f;
constexpr float kY1 = 0.48860251190291992f;
constexpr float kY2a = 1.0925484305920792f;
constexpr float kY2b = 0.31539156525252005f;
constexpr float kY2c = 0.54627421529603959f;
constexpr float kY3a = 0.59004358992664352f;
constexpr float kY3b = 2.8906114426405538f;
constexpr float kY3c = 0.45704579946446572f;
constexpr float kY3d = 0.3731763325901154f;
constexpr float kY3e = 1.4453057213202769f;

__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = kY0;
    Y[1] = -kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = -kY1 * x;
    Y[4] = kY2a * x * y;
    Y[5] = -kY2a * y * z;
    Y[6] = kY2b * (2.0f * zz - xx - yy);
    Y[7] = -kY2a * x * z;
    Y[8] = kY2c * (xx - yy);
    Y[9] = -kY3a * y * (3.0f * xx - yy);
    Y[10] = kY3b * x * y * z;
    Y[11] = -kY3c * y * (4.0f * zz - xx - yy);
    Y[12] = kY3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -kY3c * x * (4.0f * zz - xx - yy);
    Y[14] = kY3e * z * (xx - yy);
    Y[15] = -kY3a * x * (xx - 3.0f * yy);
}

// Accumulate  g . dY/d(dir)  for coefficient weights w[j] (the sum over
// channels of masked dL/drgb times the coefficient): returns the gradient
// w.r.t. the (normalised) direction.
__device__ __forceinline__ void sh_dir_grad(float x, float y, float z, const float* w, int K, float* gd) {
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if (K > 1) {
        gy += -kY1 * w[1];
        gz += kY1 * w[2];
        gx += -kY1 * w[3];
    }
    if (K > 4) {
        gx += kY2a * y * w[4];            gy += kY2a * x * w[4];
        gy += -kY2a * z * w[5];           gz += -kY2a * y * w[5];
        gx += -2.f * kY2b * x * w[6];     gy += -2.f * kY2b * y * w[6];     gz += 4.f * kY2b * z * w[6];
        gx += -kY2a * z * w[7];           gz += -kY2a * x * w[7];
        gx += 2.f * kY2c * x * w[8];      gy += -2.f * kY2c * y * w[8];
    }
    if (K > 9) {
        const float xx = x * x, yy = y * y, zz = z * z;
        gx += -6.f * kY3a * x * y * w[9];
        gy += -3.f * kY3a * (xx - yy) * w[9];
        gx += kY3b * y * z * w[10];       gy += kY3b * x * z * w[10];       gz += kY3b * x * y * w[10];
        gx += 2.f * kY3c * x * y * w[11];
        gy += -kY3c * (4.f * zz - xx - 3.f * yy) * w[11];
        gz += -8.f * kY3c * y * z * w[11];
        gx += -6.f * kY3d * x * z * w[12];
        gy += -6.f * kY3d * y * z * w[12];
        gz += kY3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
        gx += -kY3c * (4.f * zz - 3.f * xx - yy) * w[13];
        gy += 2.f * kY3c * x * y * w[13];
        gz += -8.f * kY3c * x * z * w[13];
        gx += 2.f * kY3e * x * z * w[14];
        gy += -2.f * kY3e * y * z * w[14];
        gz += kY3e * (xx - yy) * w[14];
        gx += -3.f * kY3a * (xx - yy) * w[15];
        gy += 6.f * kY3a * x * y * w[15];
    }
    gd[0] = gx; gd[1] = gy; gd[2] = gz;
}

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
__device__ __forceinline__ void quat_rot(double w, double x, double y, double z, double* R) {
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Everything the forward derives from one Gaussian's geometry.
struct Geo {
    double t[3];        // camera-space centre
    double Rq[9];       // rotation of the normalised quaternion
    double qn, iqn;     // quaternion norm and its reciprocal
    double itz;         // 1 / tz
    double M[9];        // Rq diag(s)
    double S[9];        // 3D covariance M M^T
    double T[6];        // J W, 2x3
    double a, b, c;     // dilated 2D covariance
    bool clx, cly;      // affine clamp active in x / y
    double xr, yr;      // clamped x/z, y/z
};

__device__ __forceinline__ bool geometry(const Cam& cam, const double mu[3], const double s[3],
                                         const double q[4], Geo& g) {
    for (int r = 0; r < 3; ++r)
        g.t[r] = (double)cam.R[3 * r] * mu[0] + (double)cam.R[3 * r + 1] * mu[1] +
                 (double)cam.R[3 * r + 2] * mu[2] + (double)cam.t[r];
    if (!(g.t[2] > (double)cam.near_z)) return false;
    g.qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(g.qn > 0.0)) return false;
    g.iqn = 1.0 / g.qn;
    const double inv = g.iqn;
    quat_rot(q[0] * inv, q[1] * inv, q[2] * inv, q[3] * inv, g.Rq);
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) g.M[3 * r + k] = g.Rq[3 * r + k] * s[k];
    for (int r = 0; r < 3; ++r)
        for (int k = r; k < 3; ++k) {
            const double v = g.M[3 * r] * g.M[3 * k] + g.M[3 * r + 1] * g.M[3 * k + 1] + g.M[3 * r + 2] * g.M[3 * k + 2];
            g.S[3 * r + k] = v;
            g.S[3 * k + r] = v;
        }
    // one division for the Jacobian (the clamp limits come with the camera)
    g.itz = 1.0 / g.t[2];
    const double itz = g.itz, limx = cam.limx, limy = cam.limy;
    const double x0 = g.t[0] * itz, y0 = g.t[1] * itz;
    g.clx = x0 < -limx || x0 > limx;
    g.cly = y0 < -limy || y0 > limy;
    g.xr = fmin(fmax(x0, -limx), limx);
    g.yr = fmin(fmax(y0, -limy), limy);
    const double j00 = (double)cam.fx * itz, j02 = -(double)cam.fx * g.xr * itz;
    const double j11 = (double)cam.fy * itz, j12 = -(double)cam.fy * g.yr * itz;
    for (int k = 0; k < 3; ++k) {
        g.T[k] = j00 * (double)cam.R[k] + j02 * (double)cam.R[6 + k];
        g.T[3 + k] = j11 * (double)cam.R[3 + k] + j12 * (double)cam.R[6 + k];
    }
    double TS[6];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k)
            TS[3 * r + k] = g.T[3 * r] * g.S[k] + g.T[3 * r + 1] * g.S[3 + k] + g.T[3 * r + 2] * g.S[6 + k];
    g.a = TS[0] * g.T[0] + TS[1] * g.T[1] + TS[2] * g.T[2] + kDilationD;
    g.b = TS[0] * g.T[3] + TS[1] * g.T[4] + TS[2] * g.T[5];
    g.c = TS[3] * g.T[3] + TS[4] * g.T[4] + TS[5] * g.T[5] + kDilationD;
    return true;
}

// One slot of the forward projection for its job J and the job's camera.
template <int K>
__device__ __forceinline__ void project_slot(const Job& J, const Cam& cam, int64_t slot, int tw, int th,
                                             Rec* __restrict__ rec, float* __restrict__ depth,
                                             ushort4* __restrict__ rect, uint32_t* __restrict__ tt) {
    const int64_t k = slot - J.out0;
    if (k >= J.count) {   // alignment padding between jobs
        tt[slot] = 0u;
        rect[slot] = make_ushort4(0, 0, 0, 0);
        return;
    }
    const Gauss& G = J.g;
    const int64_t i = J.src0 + k;
    const int64_t ld = G.ld;
    double mu[3], s[3], q[4];
    // the finiteness tests are combined without short-circuit evaluation:
    // with && the compiler moves each later plane's load behind the test
    // of the earlier ones, one memory round trip per test
    bool fin = true;
    for (int r = 0; r < 3; ++r) {
        const float m = G.mean[r * ld + i], sc = G.scale[r * ld + i];
        fin = fin & isfinite(m) & isfinite(sc);
        mu[r] = m;
        s[r] = sc;
    }
    for (int r = 0; r < 4; ++r) {
        const float v = G.quat[r * ld + i];
        fin = fin & isfinite(v);
        q[r] = v;
    }
    const float o = G.opacity[i];
    fin = fin & isfinite(o);

    Rec out;
    out.u = 0.0; out.v = 0.0;
    out.A = out.B = out.C = 0.f;
    out.o = o;
    out.r = out.g = out.b = 0.f;
    out.thr = 0.f;
    float z = 0.f;
    ushort4 rc = make_ushort4(0, 0, 0, 0);
    uint32_t count = 0;

    Geo g;
    if (fin && geometry(cam, mu, s, q, g)) {
        const double det = g.a * g.c - g.b * g.b;
        z = (float)g.t[2];
        if (det > 0.0 && (double)o >= 1.0 / 255.0) {
            const double idet = 1.0 / det;
            out.A = (float)(g.c * idet);
            out.B = (float)(-g.b * idet);
            out.C = (float)(g.a * idet);
            out.u = (double)cam.fx * g.t[0] / g.t[2] + (double)cam.cx;
            out.v = (double)cam.fy * g.t[1] / g.t[2] + (double)cam.cy;
            // colour from the direction camera centre -> mean
            double cc[3];
            for (int r = 0; r < 3; ++r)
                cc[r] = -((double)cam.R[r] * cam.t[0] + (double)cam.R[3 + r] * cam.t[1] + (double)cam.R[6 + r] * cam.t[2]);
            double d[3] = {mu[0] - cc[0], mu[1] - cc[1], mu[2] - cc[2]};
            const double idn = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            float Y[16];
            sh_basis((float)(d[0] * idn), (float)(d[1] * idn), (float)(d[2] * idn), Y);
            // the SH coefficients are read only here, for Gaussians that
            // survive the geometry, and consumed as they arrive (a
            // non-finite coefficient culls the Gaussian like any other
            // non-finite input)
            float col[3];
            bool fin_sh = true;
            // one channel's coefficients in flight at a time (all 48 at once
            // hold 48 more registers and cost a wave per SIMD)
#pragma unroll 1
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.f;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const float cf = G.sh[(int64_t)(ch * K + j) * ld + i];
                    fin_sh = fin_sh & isfinite(cf);
                    acc += cf * Y[j];
                }
                col[ch] = fmaxf(acc + 0.5f, 0.0f);
            }
            out.r = col[0]; out.g = col[1]; out.b = col[2];
            // support: centres of pixels where alpha can reach 1/255
            const double r2 = 2.0 * log(255.0 * (double)o);
            const double ex = sqrt(r2 * g.a), ey = sqrt(r2 * g.c);
            // the blend uses thr only for its conservative cell masks (whose
            // margin is far above FP32 error), so FP32 suffices here
            out.thr = -__builtin_log2f(255.0f * o);
            double x0 = ceil(out.u - ex - 0.5), x1 = floor(out.u + ex - 0.5);
            double y0 = ceil(out.v - ey - 0.5), y1 = floor(out.v + ey - 0.5);
            x0 = fmax(x0, 0.0);
            y0 = fmax(y0, 0.0);
            x1 = fmin(x1, (double)(cam.W - 1));
            y1 = fmin(y1, (double)(cam.H - 1));
            if (!fin_sh) {   // culled: the record as for a non-finite input
                out.u = out.v = 0.0;
                out.A = out.B = out.C = 0.f;
                out.r = out.g = out.b = 0.f;
                out.thr = 0.f;
                z = 0.f;
            } else if (x0 <= x1 && y0 <= y1) {
                const int tx0 = (int)x0 / tw, tx1 = (int)x1 / tw + 1;
                const int ty0 = (int)y0 / th, ty1 = (int)y1 / th + 1;
                rc = make_ushort4((unsigned short)tx0, (unsigned short)ty0, (unsigned short)tx1, (unsigned short)ty1);
                count = (uint32_t)((tx1 - tx0) * (ty1 - ty0));
            }
        }
    }
    rec[slot] = out;
    depth[slot] = z;
    rect[slot] = rc;
    tt[slot] = count;
}

// With one job and one view (the plain calls) the job and camera are taken
// straight from the kernel arguments (scalar loads); with tables, the
// workgroup's job and view are looked up first.
template <int K>
__global__ __launch_bounds__(kProjThreads) void k_project(JobTab jobs, ViewTab views, int tw, int th, int64_t nslots,
                                                          Rec* __restrict__ rec, float* __restrict__ depth,
                                                          ushort4* __restrict__ rect, uint32_t* __restrict__ tt) {
    const int64_t slot = (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
    if (slot >= nslots) return;
    if (!jobs.dev && !views.dev) {
        project_slot<K>(jobs.one, views.one.cam, slot, tw, th, rec, depth, rect, tt);
    } else {
        const Job J = job_at(jobs, find_job(jobs, (int64_t)blockIdx.x * kProjThreads));
        project_slot<K>(J, view_at(views, J.view).cam, slot, tw, th, rec, depth, rect, tt);
    }
}

// Backward of the projection for one Gaussian.  g2d planes: du, dv, dA, dB,
// dC, d opacity, dr, dg, db (accumulated by the blend backward).
// One slot of the projection backward for its job J and the job's camera.
template <int K>
__device__ __forceinline__ void project_bwd_slot(const Job& J, const Cam& cam, int64_t slot, int64_t nslots,
                                                 const uint32_t* __restrict__ tt, const float* __restrict__ g2d,
                                                 const int32_t* __restrict__ status) {
    const int64_t k = slot - J.out0;
    if (k >= J.count) return;   // alignment padding between jobs
    const Gauss& G = J.g;
    const int64_t i = J.src0 + k, ld = G.ld, gld = J.gld, n = nslots;
    float* __restrict__ gmean = J.gmean;
    float* __restrict__ gscale = J.gscale;
    float* __restrict__ gquat = J.gquat;
    float* __restrict__ gopac = J.gopac;
    float* __restrict__ gsh = J.gsh;
    const bool live = tt[slot] != 0 && *status == 0;
    // Culled Gaussians get zero gradients.  A wave with live lanes runs
    // the whole computation on every lane and each lane stores every plane
    // once (zero where culled): storing the culled lanes' zeros in a branch
    // of their own wrote each output line in two partial pieces, which
    // reached HBM as about 1.6x the gradient bytes.
    if (__ballot(live) == 0ull) {
        for (int r = 0; r < 3; ++r) { gmean[r * gld + i] = 0.f; gscale[r * gld + i] = 0.f; }
        for (int r = 0; r < 4; ++r) gquat[r * gld + i] = 0.f;
        gopac[i] = 0.f;
        for (int j = 0; j < 3 * K; ++j) gsh[(int64_t)j * gld + i] = 0.f;
        return;
    }
    double mu[3], s[3], q[4];
    for (int r = 0; r < 3; ++r) { mu[r] = G.mean[r * ld + i]; s[r] = G.scale[r * ld + i]; }
    for (int r = 0; r < 4; ++r) q[r] = G.quat[r * ld + i];
    const double du = g2d[slot], dv = g2d[n + slot];
    const double dA = g2d[2 * n + slot], dB = g2d[3 * n + slot], dC = g2d[4 * n + slot];
    gopac[i] = live ? g2d[5 * n + slot] : 0.f;
    const float drgb[3] = {g2d[6 * n + slot], g2d[7 * n + slot], g2d[8 * n + slot]};

    Geo g = {};
    geometry(cam, mu, s, q, g);   // live implies it succeeded in the forward

    // ---- colour: rgb_c = max(0, sum_j k_cj Y_j(dir) + 0.5)
    double cc[3];
    for (int r = 0; r < 3; ++r)
        cc[r] = -((double)cam.R[r] * cam.t[0] + (double)cam.R[3 + r] * cam.t[1] + (double)cam.R[6 + r] * cam.t[2]);
    const double dd[3] = {mu[0] - cc[0], mu[1] - cc[1], mu[2] - cc[2]};
    const double dn = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]), idn = 1.0 / dn;
    const float dx = (float)(dd[0] * idn), dy = (float)(dd[1] * idn), dz = (float)(dd[2] * idn);
    float Y[16];
    sh_basis(dx, dy, dz, Y);
    float wsum[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) wsum[j] = 0.f;
    for (int ch = 0; ch < 3; ++ch) {
        float raw = 0.5f;
        float kc[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            kc[j] = G.sh[(int64_t)(ch * K + j) * ld + i];
            raw += kc[j] * Y[j];
        }
        const float gch = raw > 0.0f ? drgb[ch] : 0.0f;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            gsh[(int64_t)(ch * K + j) * gld + i] = live ? gch * Y[j] : 0.f;
            wsum[j] += gch * kc[j];
        }
    }
    float gdir[3];
    sh_dir_grad(dx, dy, dz, wsum, K, gdir);
    const double proj_d = (double)dx * gdir[0] + (double)dy * gdir[1] + (double)dz * gdir[2];
    double gmu[3] = {(gdir[0] - dx * proj_d) * idn, (gdir[1] - dy * proj_d) * idn, (gdir[2] - dz * proj_d) * idn};

    // ---- conic Q = Sigma2^{-1}: dL/dSigma2 = -Q Gq Q with Gq the gradient
    // w.r.t. Q as a full matrix (the off-diagonal B enters twice).
    const double det = g.a * g.c - g.b * g.b, idet = 1.0 / det;
    const double Q00 = g.c * idet, Q01 = -g.b * idet, Q11 = g.a * idet;
    const double G00 = dA, G01 = 0.5 * dB, G11 = dC;
    // X = Gq Q
    const double X00 = G00 * Q00 + G01 * Q01, X01 = G00 * Q01 + G01 * Q11;
    const double X10 = G01 * Q00 + G11 * Q01, X11 = G01 * Q01 + G11 * Q11;
    // D = -Q X  (symmetric)
    const double D00 = -(Q00 * X00 + Q01 * X10);
    const double D01 = -(Q00 * X01 + Q01 * X11);
    const double D11 = -(Q01 * X01 + Q11 * X11);

    // ---- Sigma2 = T Sigma T^T:  dSigma = T^T D T,  dT = 2 D T Sigma
    double DT[6];   // D T (2x3)
    for (int k = 0; k < 3; ++k) {
        DT[k] = D00 * g.T[k] + D01 * g.T[3 + k];
        DT[3 + k] = D01 * g.T[k] + D11 * g.T[3 + k];
    }
    double dS[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) dS[3 * r + k] = g.T[r] * DT[k] + g.T[3 + r] * DT[3 + k];
    double dT[6];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k)
            dT[3 * r + k] = 2.0 * (DT[3 * r] * g.S[k] + DT[3 * r + 1] * g.S[3 + k] + DT[3 * r + 2] * g.S[6 + k]);
    // T = J W: only J00, J02 (row 0) and J11, J12 (row 1) are non-zero
    const double dJ00 = dT[0] * cam.R[0] + dT[1] * cam.R[1] + dT[2] * cam.R[2];
    const double dJ02 = dT[0] * cam.R[6] + dT[1] * cam.R[7] + dT[2] * cam.R[8];
    const double dJ11 = dT[3] * cam.R[3] + dT[4] * cam.R[4] + dT[5] * cam.R[5];
    const double dJ12 = dT[3] * cam.R[6] + dT[4] * cam.R[7] + dT[5] * cam.R[8];
    const double tx = g.t[0], ty = g.t[1], tz = g.t[2];
    const double fx = cam.fx, fy = cam.fy;
    const double itz = g.itz, itz2 = itz * itz;
    double gt[3] = {0.0, 0.0, 0.0};
    // J00 = fx/tz, J11 = fy/tz
    gt[2] -= (fx * dJ00 + fy * dJ11) * itz2;
    // J02 = -fx xr / tz with xr = tx/tz (free) or a constant (clamped)
    if (!g.clx) { gt[0] -= fx * itz2 * dJ02; gt[2] += 2.0 * fx * tx * itz2 * itz * dJ02; }
    else        { gt[2] += fx * g.xr * itz2 * dJ02; }
    if (!g.cly) { gt[1] -= fy * itz2 * dJ12; gt[2] += 2.0 * fy * ty * itz2 * itz * dJ12; }
    else        { gt[2] += fy * g.yr * itz2 * dJ12; }
    // centre u = fx tx/tz + cx, v = fy ty/tz + cy
    gt[0] += fx * itz * du;
    gt[1] += fy * itz * dv;
    gt[2] -= (fx * tx * du + fy * ty * dv) * itz2;
    // t = W mu + t_v
    for (int k = 0; k < 3; ++k) gmu[k] += cam.R[k] * gt[0] + cam.R[3 + k] * gt[1] + cam.R[6 + k] * gt[2];
    for (int k = 0; k < 3; ++k) gmean[k * gld + i] = live ? (float)gmu[k] : 0.f;

    // ---- Sigma = M M^T: dM = 2 dS M;  M = Rq diag(s)
    double dM[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            dM[3 * r + k] = 2.0 * (dS[3 * r] * g.M[k] + dS[3 * r + 1] * g.M[3 + k] + dS[3 * r + 2] * g.M[6 + k]);
    double dR[9];
    for (int k = 0; k < 3; ++k) {
        gscale[k * gld + i] = live ? (float)(dM[k] * g.Rq[k] + dM[3 + k] * g.Rq[3 + k] + dM[6 + k] * g.Rq[6 + k]) : 0.f;
        for (int r = 0; r < 3; ++r) dR[3 * r + k] = dM[3 * r + k] * s[k];
    }
    // ---- Rq(qh) with qh = q/|q|
    const double inv = g.iqn;
    const double w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
    // derivative of each rotation entry w.r.t. (w, x, y, z), contracted with dR
    double gw = 2.0 * (z * (dR[3] - dR[1]) + y * (dR[2] - dR[6]) + x * (dR[7] - dR[5]));
    double gx = 2.0 * (y * (dR[1] + dR[3]) + z * (dR[2] + dR[6]) + w * (dR[7] - dR[5]) - 2.0 * x * (dR[4] + dR[8]));
    double gy = 2.0 * (x * (dR[1] + dR[3]) + w * (dR[2] - dR[6]) + z * (dR[5] + dR[7]) - 2.0 * y * (dR[0] + dR[8]));
    double gz = 2.0 * (w * (dR[3] - dR[1]) + x * (dR[2] + dR[6]) + y * (dR[5] + dR[7]) - 2.0 * z * (dR[0] + dR[4]));
    const double dot = w * gw + x * gx + y * gy + z * gz;
    gquat[0 * gld + i] = live ? (float)((gw - w * dot) * inv) : 0.f;
    gquat[1 * gld + i] = live ? (float)((gx - x * dot) * inv) : 0.f;
    gquat[2 * gld + i] = live ? (float)((gy - y * dot) * inv) : 0.f;
    gquat[3 * gld + i] = live ? (float)((gz - z * dot) * inv) : 0.f;
}

template <int K>
__global__ __launch_bounds__(kProjThreads) void k_project_bwd(JobTab jobs, ViewTab views, int64_t nslots,
                                                              const uint32_t* __restrict__ tt,
                                                              const float* __restrict__ g2d,
                                                              const int32_t* __restrict__ status) {
    const int64_t slot = (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
    if (slot >= nslots) return;
    if (!jobs.dev && !views.dev) {   // one job and one view: from the kernel arguments
        project_bwd_slot<K>(jobs.one, views.one.cam, slot, nslots, tt, g2d, status);
    } else {
        const Job J = job_at(jobs, find_job(jobs, (int64_t)blockIdx.x * kProjThreads));
        project_bwd_slot<K>(J, view_at(views, J.view).cam, slot, nslots, tt, g2d, status);
    }
}

}  // namespace

void launch_project(const JobTab& jobs, const ViewTab& views, int K, int64_t nslots, int tw, int th, Rec* rec,
                    float* depth, ushort4* rect, uint32_t* tt, hipStream_t st) {
    if (nslots == 0) return;
    const unsigned blocks = (unsigned)((nslots + kProjThreads - 1) / kProjThreads);
#define GS_PROJ(k) \
    hipLaunchKernelGGL(k_project<k>, dim3(blocks), dim3(kProjThreads), 0, st, jobs, views, tw, th, nslots, rec, depth, rect, tt)
    switch (K) {
        case 1: GS_PROJ(1); break;
        case 4: GS_PROJ(4); break;
        case 9: GS_PROJ(9); break;
        default: GS_PROJ(16); break;
    }
#undef GS_PROJ
}

void launch_project_bwd(const JobTab& jobs, const ViewTab& views, int K, int64_t nslots, const uint32_t* tt,
                        const float* g2d, const int32_t* status, hipStream_t st) {
    if (nslots == 0) return;
    const unsigned blocks = (unsigned)((nslots + kProjThreads - 1) / kProjThreads);
#define GS_PROJ_BWD(k) \
    hipLaunchKernelGGL(k_project_bwd<k>, dim3(blocks), dim3(kProjThreads), 0, st, jobs, views, nslots, tt, g2d, status)
    switch (K) {
        case 1: GS_PROJ_BWD(1); break;
        case 4: GS_PROJ_BWD(4); break;
        case 9: GS_PROJ_BWD(9); break;
        default: GS_PROJ_BWD(16); break;
    }
#undef GS_PROJ_BWD
}

}  // namespace gs
