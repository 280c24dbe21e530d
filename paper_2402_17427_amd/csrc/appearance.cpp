// Decoupled appearance model (gs_appearance_*): layer sequence, workspace
// layout and argument checks.  The layers are those of VastGaussian
// (arXiv 2402.17427) section 4.2 and supplement S1.1; the kernels are in
// appearance.hip.  The forward keeps every activation in the caller's
// workspace, and the backward reads them from the same workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/gs.h"
#include "api_internal.h"
#include "kernels.h"
#include "profile.h"

namespace gs {

namespace {

constexpr int kLayers = 7;

struct Layer {
    int cout, cin;
};

void layer_shapes(int m, Layer* L) {
    const Layer s[kLayers] = {{256, 3 + m}, {128, 64}, {64, 32}, {32, 16}, {16, 8}, {16, 16}, {3, 16}};
    for (int k = 0; k < kLayers; ++k) L[k] = s[k];
}

int64_t layer_params(const Layer& l) { return (int64_t)l.cout * l.cin * 9 + l.cout; }

struct Plan {
    int W, H, m, h, w;
    Layer L[kLayers];
    int64_t poff[kLayers];   // parameter offsets (weights, then bias)
    int64_t n_params;
    // workspace offsets (bytes)
    size_t D, x[5], s[5], u, f1, M, gA, gB, part, tmp, ty0, ty1, tfy, tx0, tx1, tfx, rylo, ryhi, rxlo, rxhi, bytes;
};

void make_plan(int W, int H, int m, Plan* p) {
    p->W = W;
    p->H = H;
    p->m = m;
    p->h = (H + 31) / 32;
    p->w = (W + 31) / 32;
    layer_shapes(m, p->L);
    int64_t o = 0;
    for (int k = 0; k < kLayers; ++k) {
        p->poff[k] = o;
        o += layer_params(p->L[k]);
    }
    p->n_params = o;
    const int64_t hw = (int64_t)p->h * p->w, HW = (int64_t)H * W;
    size_t off = 0;
    auto take = [&](int64_t floats) {
        const size_t at = off;
        off += align256((size_t)floats * 4);
        return at;
    };
    p->D = take((3 + m) * hw);
    int C = 256;
    int64_t area = hw;
    p->x[0] = take(C * area);
    p->s[0] = 0;
    int64_t gmax = std::max<int64_t>(16 * HW, (3 + m) * hw);
    gmax = std::max<int64_t>(gmax, C * area);
    int64_t pmax = (int64_t)wgrad_parts(p->h, p->w) * layer_params(p->L[0]);
    for (int k = 1; k <= 4; ++k) {
        area *= 4;
        p->s[k] = take((C / 4) * area);
        p->x[k] = take((C / 2) * area);
        const int sz = 1 << k;
        pmax = std::max<int64_t>(pmax, (int64_t)wgrad_parts(p->h * sz, p->w * sz) * layer_params(p->L[k]));
        gmax = std::max<int64_t>(gmax, (C / 2) * area);
        C /= 2;
    }
    p->u = take(16 * HW);
    p->f1 = take(16 * HW);
    p->M = take(3 * HW);
    pmax = std::max<int64_t>(pmax, (int64_t)wgrad_parts(H, W) * std::max(layer_params(p->L[5]), layer_params(p->L[6])));
    // split convolutions: [splits][Cout][area] partial sums, forward and
    // transposed (backward) shapes of every layer
    auto split_need = [](int cin, int cout, int hh, int ww) {
        const int sp = conv_splits(cin, cout, hh, ww);
        return sp > 1 ? (int64_t)sp * cout * hh * ww : (int64_t)0;
    };
    {
        int c = 256, hk = p->h, wk = p->w;
        pmax = std::max(pmax, split_need(3 + m, 256, hk, wk));
        pmax = std::max(pmax, split_need(256, 3 + m, hk, wk));
        for (int k = 1; k <= 4; ++k) {
            hk *= 2;
            wk *= 2;
            pmax = std::max(pmax, split_need(c / 4, c / 2, hk, wk));
            pmax = std::max(pmax, split_need(c / 2, c / 4, hk, wk));
            c /= 2;
        }
        pmax = std::max(pmax, split_need(16, 16, H, W));
        pmax = std::max(pmax, split_need(3, 16, H, W));
        pmax = std::max(pmax, split_need(16, 3, H, W));
    }
    p->gA = take(gmax);
    p->gB = take(gmax);
    p->part = take(pmax);
    p->tmp = take(16 * (int64_t)H * (p->w * 16));   // x pass of the interpolation adjoint
    p->ty0 = take(H);
    p->ty1 = take(H);
    p->tfy = take(H);
    p->tx0 = take(W);
    p->tx1 = take(W);
    p->tfx = take(W);
    p->rylo = take(p->h * 16);
    p->ryhi = take(p->h * 16);
    p->rxlo = take(p->w * 16);
    p->rxhi = take(p->w * 16);
    p->bytes = off;
}

gs_status check_shape(int W, int H, int m) {
    if (W < 1 || H < 1 || m < 0 || m > 4096) return fail(GS_ERR_INVALID, "bad shape %dx%d, embedding %d", W, H, m);
    if ((int64_t)W * H > ((int64_t)1 << 31) / 16) return fail(GS_ERR_INVALID, "image too large");
    return GS_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

BilinTab tables(const Plan& p, void* ws) {
    BilinTab t;
    t.y0 = at<int>(ws, p.ty0);
    t.y1 = at<int>(ws, p.ty1);
    t.fy = at<float>(ws, p.tfy);
    t.x0 = at<int>(ws, p.tx0);
    t.x1 = at<int>(ws, p.tx1);
    t.fx = at<float>(ws, p.tfx);
    t.ylo = at<int>(ws, p.rylo);
    t.yhi = at<int>(ws, p.ryhi);
    t.xlo = at<int>(ws, p.rxlo);
    t.xhi = at<int>(ws, p.rxhi);
    return t;
}

ConvArgs conv_args(const float* in, const float* mask, const float* w, const float* b, float* out, int cin, int cout,
                   int H, int W, bool transposed, bool relu, int cinf) {
    ConvArgs a;
    a.in = in;
    a.mask = mask;
    a.w = w;
    a.b = b;
    a.out = out;
    a.Cin = cin;
    a.Cout = cout;
    a.H = H;
    a.W = W;
    a.transposed = transposed ? 1 : 0;
    a.relu = relu ? 1 : 0;
    a.CinF = cinf;
    a.part = nullptr;
    return a;
}

void wgrad(const Plan& p, void* ws, const float* in, const float* g, const float* mask, const Layer& l, int H, int W,
           float* dw, hipStream_t st) {
    WgradArgs a;
    a.in = in;
    a.g = g;
    a.mask = mask;
    a.partial = at<float>(ws, p.part);
    a.Cin = l.cin;
    a.Cout = l.cout;
    a.H = H;
    a.W = W;
    a.J = layer_params(l);
    launch_wgrad(a, dw, st);
}

gs_status check_call(const Plan& p, void* ws, size_t ws_bytes) {
    if (!ws || ws_bytes < p.bytes) return fail(GS_ERR_INVALID, "workspace too small: %zu < %zu", ws_bytes, p.bytes);
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GS_ERR_INVALID, "workspace not 256-byte aligned");
    return GS_OK;
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" {

gs_status gs_appearance_param_count(int32_t embed_dim, int64_t* count) {
    if (!count || embed_dim < 0 || embed_dim > 4096) return fail(GS_ERR_INVALID, "bad arguments");
    Layer L[kLayers];
    layer_shapes(embed_dim, L);
    int64_t n = 0;
    for (const Layer& l : L) n += layer_params(l);
    *count = n;
    return GS_OK;
}

gs_status gs_appearance_workspace(int32_t width, int32_t height, int32_t embed_dim, size_t* bytes) {
    gs_status s;
    if (!bytes) return fail(GS_ERR_INVALID, "bytes is NULL");
    if ((s = check_shape(width, height, embed_dim))) return s;
    Plan p;
    make_plan(width, height, embed_dim, &p);
    *bytes = p.bytes;
    return GS_OK;
}

gs_status gs_appearance_fwd(const float* image, int32_t width, int32_t height, const float* embedding,
                            int32_t embed_dim, const float* params, float* image_adj, float* transform, void* ws,
                            size_t ws_bytes, gs_stream stream) {
    gs_status s;
    if ((s = check_shape(width, height, embed_dim))) return s;
    if (!image || !params || !image_adj || (embed_dim > 0 && !embedding)) return fail(GS_ERR_INVALID, "NULL buffer");
    Plan p;
    make_plan(width, height, embed_dim, &p);
    if ((s = check_call(p, ws, ws_bytes))) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int H = height, W = width, h = p.h, w = p.w;
    ProfScope ps("appearance_fwd", st);
    float* part = at<float>(ws, p.part);
    auto conv = [&](ConvArgs a) {
        a.part = part;
        launch_conv(a, st);
    };
    float* D = at<float>(ws, p.D);
    launch_down_concat(image, H, W, h, w, embedding, embed_dim, D, st);
    const Layer* L = p.L;
    float* x = at<float>(ws, p.x[0]);
    conv(conv_args(D, nullptr, params + p.poff[0], params + p.poff[0] + (int64_t)L[0].cout * L[0].cin * 9, x,
                          L[0].cin, L[0].cout, h, w, false, false, 0));
    int hk = h, wk = w, C = 256;
    for (int k = 1; k <= 4; ++k) {
        float* sk = at<float>(ws, p.s[k]);
        launch_shuffle(x, C / 4, hk, wk, sk, false, st);
        hk *= 2;
        wk *= 2;
        float* xk = at<float>(ws, p.x[k]);
        conv(conv_args(sk, nullptr, params + p.poff[k], params + p.poff[k] + (int64_t)L[k].cout * L[k].cin * 9,
                              xk, C / 4, C / 2, hk, wk, false, true, 0));
        x = xk;
        C /= 2;
    }
    const BilinTab t = tables(p, ws);
    launch_bilin_table(hk, H, const_cast<int*>(t.y0), const_cast<int*>(t.y1), const_cast<float*>(t.fy), st);
    launch_bilin_table(wk, W, const_cast<int*>(t.x0), const_cast<int*>(t.x1), const_cast<float*>(t.fx), st);
    float* u = at<float>(ws, p.u);
    launch_bilinear(x, 16, hk, wk, H, W, t, u, st);
    float* f1 = at<float>(ws, p.f1);
    conv(conv_args(u, nullptr, params + p.poff[5], params + p.poff[5] + (int64_t)L[5].cout * L[5].cin * 9, f1,
                          16, 16, H, W, false, true, 0));
    float* M = at<float>(ws, p.M);
    conv(conv_args(f1, nullptr, params + p.poff[6], params + p.poff[6] + (int64_t)L[6].cout * L[6].cin * 9, M,
                          16, 3, H, W, false, false, 0));
    const int64_t n = 3 * (int64_t)H * W;
    launch_mul(image, M, n, image_adj, st);
    if (transform && hipMemcpyAsync(transform, M, n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return check_hip("gs_appearance_fwd: transform copy");
    return check_hip("gs_appearance_fwd");
}

gs_status gs_appearance_bwd(const float* image, int32_t width, int32_t height, const float* embedding,
                            int32_t embed_dim, const float* params, const float* d_image_adj, float* d_image,
                            float* d_embedding, float* d_params, void* ws, size_t ws_bytes, gs_stream stream) {
    gs_status s;
    if ((s = check_shape(width, height, embed_dim))) return s;
    if (!image || !params || !d_image_adj || !d_image || !d_params || (embed_dim > 0 && (!embedding || !d_embedding)))
        return fail(GS_ERR_INVALID, "NULL buffer");
    Plan p;
    make_plan(width, height, embed_dim, &p);
    if ((s = check_call(p, ws, ws_bytes))) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int H = height, W = width, h = p.h, w = p.w;
    ProfScope ps("appearance_bwd", st);
    // the split convolutions' partial sums share the weight-gradient
    // partials' buffer: each weight gradient is reduced before the next
    // convolution starts on the stream
    float* part = at<float>(ws, p.part);
    auto conv = [&](ConvArgs a) {
        a.part = part;
        launch_conv(a, st);
    };
    const Layer* L = p.L;
    float* gA = at<float>(ws, p.gA);
    float* gB = at<float>(ws, p.gB);
    const float* M = at<float>(ws, p.M);
    const float* f1 = at<float>(ws, p.f1);
    const float* u = at<float>(ws, p.u);
    const int64_t n = 3 * (int64_t)H * W;
    launch_mul_bwd(d_image_adj, image, M, n, gA, d_image, st);
    // final convolutions
    wgrad(p, ws, f1, gA, nullptr, L[6], H, W, d_params + p.poff[6], st);
    conv(conv_args(gA, nullptr, params + p.poff[6], nullptr, gB, 3, 16, H, W, true, false, 16));
    wgrad(p, ws, u, gB, f1, L[5], H, W, d_params + p.poff[5], st);
    conv(conv_args(gB, f1, params + p.poff[5], nullptr, gA, 16, 16, H, W, true, false, 16));
    // interpolation
    const int h4 = h * 16, w4 = w * 16;
    launch_bilinear_adj(gA, 16, H, W, h4, w4, tables(p, ws), at<float>(ws, p.tmp), gB, st);
    // upsampling blocks, last to first
    int hk = h4, wk = w4, C = 16;   // C: the block's output channels
    for (int k = 4; k >= 1; --k) {
        const float* sk = at<float>(ws, p.s[k]);
        const float* xk = at<float>(ws, p.x[k]);
        wgrad(p, ws, sk, gB, xk, L[k], hk, wk, d_params + p.poff[k], st);
        conv(conv_args(gB, xk, params + p.poff[k], nullptr, gA, C, C / 2, hk, wk, true, false, C / 2));
        launch_shuffle(gA, C / 2, hk / 2, wk / 2, gB, true, st);
        hk /= 2;
        wk /= 2;
        C *= 2;
    }
    // first convolution
    const float* D = at<float>(ws, p.D);
    wgrad(p, ws, D, gB, nullptr, L[0], h, w, d_params + p.poff[0], st);
    conv(conv_args(gB, nullptr, params + p.poff[0], nullptr, gA, 256, 3 + embed_dim, h, w, true, false,
                          3 + embed_dim));
    if (embed_dim > 0) launch_embed_grad(gA, (int64_t)h * w, embed_dim, d_embedding, st);
    launch_down_adjoint(gA, H, W, h, w, d_image, st);
    return check_hip("gs_appearance_bwd");
}

}  // extern "C"
