// One optimiser step over a Gaussian set, fused in one pass over its planes.
//
// VastGaussian (arXiv 2402.17427), section 3: each cell's Gaussians are
// optimised by gradient descent on the loss, interleaved with adaptive
// densification that is triggered by each point's cumulative gradient;
// section 5.1 leaves the optimiser to 3DGS, whose choices are taken here:
// Adam with bias correction over the raw properties (position, log-scale,
// un-normalised quaternion, opacity logit, SH coefficients), one learning
// rate per group (SH degree-0 and higher-degree coefficients apart), the
// renderer's gradient carried to the raw values through scale = exp(raw)
// and opacity = sigmoid(raw), and, for every Gaussian visible in the step's
// view, the norm of its image-space centre gradient accumulated with a
// visibility count.
//
// The step is HBM-bound: per Gaussian and plane it reads the raw value, the
// gradient and both moments and writes the value and both moments (plus the
// activated scale and opacity the next forward reads).  One thread handles
// four Gaussians of one plane (coalesced plane rows, four loads of each
// stream in flight); an extra grid row updates the densification
// statistics.  Nothing is reduced, so the result is deterministic.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace gs {

namespace {

constexpr int kThreads = 256;
constexpr int kPer = 4;  // Gaussians per thread

// plane groups in the moment arrays: mean 3, log-scale 3, quat 4, logit 1, SH 3K
enum Act { kNone = 0, kExp = 1, kSigmoid = 2 };

__device__ __forceinline__ float sigmoidf(float x) { return 1.f / (1.f + expf(-x)); }

__global__ __launch_bounds__(kThreads) void k_adam(AdamArgs a) {
    if (a.status && *a.status != 0) return;
    if (a.dev) {
        // step-dependent scalars prepared on the device (graph replays)
#pragma unroll
        for (int k = 0; k < 6; ++k) a.step_size[k] = a.dev->step_size[k];
        a.inv_sqrt_bc2 = a.dev->inv_sqrt_bc2;
    }
    const int p = blockIdx.y;
    const int np = 11 + 3 * a.K;
    const int64_t i0 = (int64_t)blockIdx.x * (kThreads * kPer) + threadIdx.x;
    if (p == np) {
        // densification statistics
        if (!a.tiles) return;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = i0 + (int64_t)k * kThreads;
            if (i < a.n && a.tiles[i] > 0u) {
                const float gu = a.g2d[i], gv = a.g2d[a.g2d_ld + i];
                a.accum[i] += sqrtf(gu * gu + gv * gv);
                a.count[i] += 1.f;
            }
        }
        return;
    }
    float* raw;
    const float* grad;
    float* act_out = nullptr;
    int act = kNone;
    float ss;
    if (p < 3) {
        raw = a.mean + (int64_t)p * a.ld;
        grad = a.g_mean + (int64_t)p * a.gld;
        ss = a.step_size[0];
    } else if (p < 6) {
        raw = a.log_scale + (int64_t)(p - 3) * a.ld;
        grad = a.g_scale + (int64_t)(p - 3) * a.gld;
        act_out = a.scale_out + (int64_t)(p - 3) * a.ld;
        act = kExp;
        ss = a.step_size[1];
    } else if (p < 10) {
        raw = a.quat + (int64_t)(p - 6) * a.ld;
        grad = a.g_quat + (int64_t)(p - 6) * a.gld;
        ss = a.step_size[2];
    } else if (p == 10) {
        raw = a.logit;
        grad = a.g_opacity;
        act_out = a.opacity_out;
        act = kSigmoid;
        ss = a.step_size[3];
    } else {
        const int q = p - 11;
        raw = a.sh + (int64_t)q * a.ld;
        grad = a.g_sh + (int64_t)q * a.gld;
        ss = a.step_size[q % a.K == 0 ? 4 : 5];
    }
    float* __restrict__ m = a.m + (int64_t)p * a.ld;
    float* __restrict__ v = a.v + (int64_t)p * a.ld;
    float r[kPer], g[kPer], mm[kPer], vv[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = i0 + (int64_t)k * kThreads;
        const bool ok = i < a.n;
        r[k] = ok ? raw[i] : 0.f;
        g[k] = ok ? grad[i] : 0.f;
        mm[k] = ok ? m[i] : 0.f;
        vv[k] = ok ? v[i] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = i0 + (int64_t)k * kThreads;
        if (i >= a.n) continue;
        float gk = g[k];
        if (act == kExp) {
            gk *= expf(r[k]);
        } else if (act == kSigmoid) {
            // o (1 - o) = e / (1 + e)^2 with e = exp(-|raw|): no cancellation in 1 - o
            const float e = expf(-fabsf(r[k]));
            const float d = 1.f + e;
            gk *= e / (d * d);
        }
        const float mk = a.beta1 * mm[k] + a.one_m_beta1 * gk;
        const float vk = a.beta2 * vv[k] + a.one_m_beta2 * gk * gk;
        const float den = sqrtf(vk) * a.inv_sqrt_bc2 + a.eps;
        const float rk = r[k] - ss * (mk / den);
        raw[i] = rk;
        m[i] = mk;
        v[i] = vk;
        if (act == kExp) act_out[i] = expf(rk);
        else if (act == kSigmoid) act_out[i] = sigmoidf(rk);
    }
}

// One thread: advance the step count and derive this step's scalars
// (bias corrections in FP64; the position rate decays log-linearly from
// lr_mean to lr_mean_final over lr_mean_steps steps when those are set).
__global__ void k_adam_prepare(AdamSched* s) {
    const int t = ++s->step;
    const double b1 = s->beta1, b2 = s->beta2;
    const double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
    double lr0 = s->lr[0];
    if (s->lr_mean_final > 0.f && s->lr_mean_steps > 0) {
        const double f = fmin(1.0, (double)t / (double)s->lr_mean_steps);
        lr0 = exp(log((double)s->lr[0]) * (1.0 - f) + log((double)s->lr_mean_final) * f);
    }
    s->dev.step_size[0] = (float)(lr0 / bc1);
    for (int k = 1; k < 6; ++k) s->dev.step_size[k] = (float)((double)s->lr[k] / bc1);
    s->dev.inv_sqrt_bc2 = (float)(1.0 / sqrt(bc2));
}

}  // namespace

void launch_adam_prepare(AdamSched* s, hipStream_t st) {
    hipLaunchKernelGGL(k_adam_prepare, dim3(1), dim3(1), 0, st, s);
}

void launch_adam(const AdamArgs& a, hipStream_t st) {
    if (a.n <= 0) return;
    const int64_t bx = (a.n + kThreads * kPer - 1) / (kThreads * kPer);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)bx, 11 + 3 * a.K + 1), dim3(kThreads), 0, st, a);
}

}  // namespace gs
