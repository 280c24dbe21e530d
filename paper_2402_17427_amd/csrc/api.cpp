// C ABI of the rasterizer: argument validation, workspace carving and
// kernel dispatch.  The declarations and their contracts are in gs.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/gs.h"
#include "api_internal.h"
#include "kernels.h"
#include "profile.h"

namespace gs {

namespace {
thread_local std::string g_err;
}

const char* g_err_cstr() { return g_err.c_str(); }

gs_status fail(gs_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

gs_status check_hip(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return GS_OK;
}

gs_status to_cam(const gs_camera* c, Cam* out) {
    if (!c) return fail(GS_ERR_INVALID, "camera is NULL");
    if (c->width <= 0 || c->height <= 0) return fail(GS_ERR_INVALID, "image size %dx%d", c->width, c->height);
    if (c->width > 65535 * 8 || c->height > 65535 * 8) return fail(GS_ERR_INVALID, "image too large");
    if (!(c->fx > 0.f) || !(c->fy > 0.f) || !std::isfinite(c->fx) || !std::isfinite(c->fy))
        return fail(GS_ERR_INVALID, "focal lengths must be finite and > 0");
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(c->R[i])) return fail(GS_ERR_INVALID, "camera rotation not finite");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(c->t[i]) || !std::isfinite(c->bg[i])) return fail(GS_ERR_INVALID, "camera not finite");
    if (!std::isfinite(c->cx) || !std::isfinite(c->cy) || !std::isfinite(c->near_z))
        return fail(GS_ERR_INVALID, "camera not finite");
    std::memcpy(out->R, c->R, sizeof out->R);
    std::memcpy(out->t, c->t, sizeof out->t);
    out->fx = c->fx;
    out->fy = c->fy;
    out->cx = c->cx;
    out->cy = c->cy;
    out->W = c->width;
    out->H = c->height;
    out->near_z = c->near_z;
    std::memcpy(out->bg, c->bg, sizeof out->bg);
    out->limx = kFovClampD * (0.5 * (double)out->W) / (double)out->fx;
    out->limy = kFovClampD * (0.5 * (double)out->H) / (double)out->fy;
    return GS_OK;
}

gs_status to_gauss(const gs_gaussians* g, Gauss* out) {
    if (!g) return fail(GS_ERR_INVALID, "gaussians is NULL");
    if (g->n < 0 || g->ld < g->n) return fail(GS_ERR_INVALID, "bad n=%lld ld=%lld", (long long)g->n, (long long)g->ld);
    if (g->n > (int64_t)0xFFFFFFFF) return fail(GS_ERR_INVALID, "more than 2^32-1 Gaussians");
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(GS_ERR_INVALID, "sh_degree %d not in [0, 3]", g->sh_degree);
    if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->sh))
        return fail(GS_ERR_INVALID, "Gaussian plane pointer is NULL");
    out->n = g->n;
    out->ld = g->ld;
    out->deg = g->sh_degree;
    out->K = (g->sh_degree + 1) * (g->sh_degree + 1);
    out->mean = g->mean;
    out->scale = g->scale;
    out->quat = g->quat;
    out->opacity = g->opacity;
    out->sh = g->sh;
    return GS_OK;
}

gs_status tiles_of(const gs_opts* o, int* tw, int* th) {
    *tw = (o && o->tile_w) ? o->tile_w : 16;
    *th = (o && o->tile_h) ? o->tile_h : 16;
    if (!render_tile_supported(*tw, *th)) return fail(GS_ERR_UNSUPPORTED, "tile %dx%d not supported", *tw, *th);
    return GS_OK;
}

int tile_bits(int64_t n_tiles) {
    int b = 0;
    while (((int64_t)1 << b) < n_tiles) ++b;
    return b;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The backward's workspace: per-pair gradient slots (36 B per pair), then a
// tile order of at most one entry per pair and its count.
size_t bwd_ws_bytes(int64_t cap) {
    const size_t c = (size_t)(cap > 0 ? cap : 0);
    return align256(pair_grad_bytes(cap)) + align256((c + 1) * sizeof(uint32_t));
}

size_t bin_sort_ws_bytes(int64_t n, int64_t cap, int64_t n_tiles) {
    if (bin_direct_supported(n_tiles)) return bin_direct_ws_bytes(n, cap, n_tiles);
    const int kb = 32 + tile_bits(n_tiles);
    return align256(scan_workspace_bytes(n)) + align256((size_t)cap * 8) + align256((size_t)cap * 4) +
           align256(sort_workspace_bytes(cap, kb));
}

ViewTab single_view(const Cam& C, int tw, int th) {
    ViewTab t;
    t.dev = nullptr;
    t.n = 1;
    std::memset(&t.one, 0, sizeof t.one);
    t.one.cam = C;
    t.one.ntx = (C.W + tw - 1) / tw;
    t.one.nty = (C.H + th - 1) / th;
    t.one.tile_base = 0;
    t.one.img_base = 0;
    t.one.pix_base = 0;
    return t;
}

JobTab single_job(const Gauss& G, const gs_grads* out) {
    JobTab t;
    t.dev = nullptr;
    t.n = 1;
    std::memset(&t.one, 0, sizeof t.one);
    t.one.g = G;
    t.one.src0 = 0;
    t.one.count = G.n;
    t.one.out0 = 0;
    t.one.view = 0;
    if (out) {
        t.one.gmean = out->mean;
        t.one.gscale = out->scale;
        t.one.gquat = out->quat;
        t.one.gopac = out->opacity;
        t.one.gsh = out->sh;
        t.one.gld = out->ld;
    }
    return t;
}

RenderArgs single_render(const gs_proj* proj, const gs_bins* bins, const Cam& C, int tw, int th) {
    RenderArgs r;
    std::memset(&r, 0, sizeof r);
    r.rec = static_cast<const Rec*>(proj->rec);
    r.vals = bins->vals;
    r.ranges = bins->ranges;
    r.status = bins->status;
    r.views = single_view(C, tw, th);
    r.n_tiles = (uint32_t)(r.views.one.ntx * r.views.one.nty);
    r.tw = tw;
    r.th = th;
    r.masks = bins->cell_masks;
    if (bins->tile_order) {   // the blend order gs_bin_sort kept: [0] = count, [1..] = tiles
        r.tile_order = bins->tile_order + 1;
        r.tile_order_count = bins->tile_order;
    }
    return r;
}

gs_status check_proj(const gs_proj* p, int64_t n) {
    if (!p) return fail(GS_ERR_INVALID, "proj is NULL");
    if (n > 0 && (!p->rec || !p->depth || !p->rect || !p->tiles_touched))
        return fail(GS_ERR_INVALID, "proj buffer is NULL");
    if (reinterpret_cast<uintptr_t>(p->rec) % 16) return fail(GS_ERR_INVALID, "proj rec not 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(p->rect) % 8) return fail(GS_ERR_INVALID, "proj rect not 8-byte aligned");
    return GS_OK;
}

gs_status check_bins(const gs_bins* b) {
    if (!b) return fail(GS_ERR_INVALID, "bins is NULL");
    if (b->pair_capacity < 0 || b->pair_capacity > kMaxPairs)
        return fail(GS_ERR_INVALID, "pair_capacity %lld not in [0, 2^30-1]", (long long)b->pair_capacity);
    if (!b->ranges || !b->pair_count || !b->status) return fail(GS_ERR_INVALID, "bins buffer is NULL");
    if (b->pair_capacity > 0 && (!b->keys || !b->vals)) return fail(GS_ERR_INVALID, "bins keys/vals NULL");
    if (reinterpret_cast<uintptr_t>(b->ranges) % 8) return fail(GS_ERR_INVALID, "ranges not 8-byte aligned");
    if (reinterpret_cast<uintptr_t>(b->cell_masks) % 8)
        return fail(GS_ERR_INVALID, "cell_masks not 8-byte aligned");
    if (reinterpret_cast<uintptr_t>(b->tile_order) % 4) return fail(GS_ERR_INVALID, "tile_order not 4-byte aligned");
    return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" {

int gs_abi_version(void) { return GS_ABI_VERSION; }

const char* gs_last_error(void) { return g_err_cstr(); }

gs_status gs_project(const gs_gaussians* g, const gs_camera* cam, const gs_opts* opts, gs_proj* out,
                     gs_stream stream) {
    Gauss G;
    Cam C;
    int tw, th;
    gs_status s;
    if ((s = to_gauss(g, &G)) || (s = to_cam(cam, &C)) || (s = tiles_of(opts, &tw, &th))) return s;
    if ((s = check_proj(out, G.n))) return s;
    const int ntx = (C.W + tw - 1) / tw, nty = (C.H + th - 1) / th;
    if (ntx > 65535 || nty > 65535) return fail(GS_ERR_INVALID, "too many tiles");
    {
        ProfScope ps("project", static_cast<hipStream_t>(stream));
        launch_project(single_job(G, nullptr), single_view(C, tw, th), G.K, G.n, tw, th, static_cast<Rec*>(out->rec),
                       out->depth, reinterpret_cast<ushort4*>(out->rect), out->tiles_touched,
                       static_cast<hipStream_t>(stream));
    }
    return check_hip("gs_project");
}

gs_status gs_bin_sort_workspace(int64_t n, int64_t pair_capacity, int64_t n_tiles, size_t* bytes) {
    if (!bytes) return fail(GS_ERR_INVALID, "bytes is NULL");
    if (n < 0 || pair_capacity < 0 || pair_capacity > kMaxPairs || n_tiles <= 0)
        return fail(GS_ERR_INVALID, "bad sizes");
    *bytes = bin_sort_ws_bytes(n, pair_capacity, n_tiles);
    return GS_OK;
}

gs_status gs_bin_sort(const gs_proj* proj, int64_t n, const gs_camera* cam, const gs_opts* opts, gs_bins* out,
                      void* ws, size_t ws_bytes, gs_stream stream) {
    Cam C;
    int tw, th;
    gs_status s;
    if (n < 0 || n > (int64_t)0xFFFFFFFF) return fail(GS_ERR_INVALID, "bad n");
    if ((s = to_cam(cam, &C)) || (s = tiles_of(opts, &tw, &th)) || (s = check_proj(proj, n)) ||
        (s = check_bins(out)))
        return s;
    const int ntx = (C.W + tw - 1) / tw, nty = (C.H + th - 1) / th;
    const int64_t n_tiles = (int64_t)ntx * nty;
    const int64_t cap = out->pair_capacity;
    const size_t need = bin_sort_ws_bytes(n, cap, n_tiles);
    if (!ws || ws_bytes < need) return fail(GS_ERR_INVALID, "workspace too small: %zu < %zu", ws_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (bin_direct_supported(n_tiles)) {   // pairs placed into their tile runs, then each run sorted
        {
            ProfScope ps("scan_emit", st);
            launch_bin_direct_place(n, reinterpret_cast<const ushort4*>(proj->rect), proj->depth,
                                    (C.W + tw - 1) / tw, n_tiles, cap, out->first, out->ranges, out->pair_count,
                                    out->status, ws, st);
        }
        {
            ProfScope ps("sort", st);
            launch_bin_direct_sort(n, n_tiles, cap, out->keys, out->vals, out->ranges, out->status, out->tile_order,
                                   ws, st);
        }
        return check_hip("gs_bin_sort");
    }
    char* p = static_cast<char*>(ws);
    void* scan_ws = p;
    p += align256(scan_workspace_bytes(n));
    uint64_t* alt_k = reinterpret_cast<uint64_t*>(p);
    p += align256((size_t)cap * 8);
    uint32_t* alt_v = reinterpret_cast<uint32_t*>(p);
    p += align256((size_t)cap * 4);
    void* sort_ws = p;
    const int tb = tile_bits(n_tiles);
    const bool to_alt = bin_sort_emit_to_alt(tb);
    {
        ProfScope ps("scan_emit", st);
        Gauss G0;
        std::memset(&G0, 0, sizeof G0);
        G0.n = n;
        const ZeroList z = bin_sort_zero_list(sort_ws, cap, tb, out->ranges, n_tiles);
        launch_emit_pairs(n, proj->tiles_touched, reinterpret_cast<const ushort4*>(proj->rect), proj->depth,
                          single_job(G0, nullptr), single_view(C, tw, th), cap, to_alt ? alt_k : out->keys,
                          to_alt ? alt_v : out->vals, out->first, out->pair_count, out->status, scan_ws, st, &z);
    }
    {
        ProfScope ps("sort", st);
        launch_bin_sort(out->keys, out->vals, alt_k, alt_v, out->pair_count, cap, tb, out->ranges, n_tiles, sort_ws,
                        st, true, out->tile_order);
    }
    return check_hip("gs_bin_sort");
}

gs_status gs_render_fwd(const gs_proj* proj, const gs_bins* bins, const gs_camera* cam, const gs_opts* opts,
                        float* image, float* final_T, uint32_t* n_contrib, gs_stream stream) {
    Cam C;
    int tw, th;
    gs_status s;
    if ((s = to_cam(cam, &C)) || (s = tiles_of(opts, &tw, &th)) || (s = check_bins(bins))) return s;
    if (!proj || !proj->rec) return fail(GS_ERR_INVALID, "proj is NULL");
    if (!image || !final_T || !n_contrib) return fail(GS_ERR_INVALID, "output buffer is NULL");
    {
        ProfScope ps("render_fwd", static_cast<hipStream_t>(stream));
        launch_render_fwd(single_render(proj, bins, C, tw, th), image, final_T, n_contrib, nullptr, nullptr,
                          static_cast<hipStream_t>(stream));
    }
    return check_hip("gs_render_fwd");
}

gs_status gs_render_state_bytes(const gs_bins* bins, const gs_opts* opts, size_t* bytes) {
    int tw, th;
    gs_status s;
    if ((s = tiles_of(opts, &tw, &th)) || (s = check_bins(bins))) return s;
    if (!bytes) return fail(GS_ERR_INVALID, "bytes is NULL");
    *bytes = (size_t)bins->pair_capacity * (size_t)(tw * th) * sizeof(float) * 2;
    return GS_OK;
}

gs_status gs_render_mask_bytes(const gs_bins* bins, const gs_opts* opts, size_t* bytes) {
    int tw, th;
    gs_status s;
    if ((s = tiles_of(opts, &tw, &th)) || (s = check_bins(bins))) return s;
    if (!bytes) return fail(GS_ERR_INVALID, "bytes is NULL");
    *bytes = (size_t)bins->pair_capacity * (size_t)render_mask_words(tw, th) * sizeof(uint64_t);
    return GS_OK;
}

gs_status gs_render_fwd_stored(const gs_proj* proj, const gs_bins* bins, const gs_camera* cam, const gs_opts* opts,
                               float* image, float* final_T, uint32_t* n_contrib, void* state,
                               size_t state_bytes, gs_stream stream) {
    Cam C;
    int tw, th;
    gs_status s;
    size_t need = 0;
    if ((s = to_cam(cam, &C)) || (s = tiles_of(opts, &tw, &th)) || (s = check_bins(bins)) ||
        (s = gs_render_state_bytes(bins, opts, &need)))
        return s;
    if (!proj || !proj->rec) return fail(GS_ERR_INVALID, "proj is NULL");
    if (!image || !final_T || !n_contrib) return fail(GS_ERR_INVALID, "output buffer is NULL");
    if (!state || state_bytes < need) return fail(GS_ERR_INVALID, "state buffer too small: %zu < %zu", state_bytes, need);
    {
        ProfScope ps("render_fwd_stored", static_cast<hipStream_t>(stream));
        launch_render_fwd(single_render(proj, bins, C, tw, th), image, final_T, n_contrib, nullptr,
                          static_cast<float2*>(state), static_cast<hipStream_t>(stream));
    }
    return check_hip("gs_render_fwd_stored");
}

gs_status gs_render_stats(const gs_proj* proj, const gs_bins* bins, const gs_camera* cam, const gs_opts* opts,
                          uint64_t* counters, gs_stream stream) {
    Cam C;
    int tw, th;
    gs_status s;
    if ((s = to_cam(cam, &C)) || (s = tiles_of(opts, &tw, &th)) || (s = check_bins(bins))) return s;
    if (!proj || !proj->rec) return fail(GS_ERR_INVALID, "proj is NULL");
    if (!counters) return fail(GS_ERR_INVALID, "counters is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_fill_u32(reinterpret_cast<uint32_t*>(counters), 0u, 8, st);
    const RenderArgs r = single_render(proj, bins, C, tw, th);
    launch_render_fwd(r, nullptr, nullptr, nullptr, reinterpret_cast<unsigned long long*>(counters), nullptr, st);
    launch_render_stats_bwd_cells(r, reinterpret_cast<unsigned long long*>(counters), st);
    return check_hip("gs_render_stats");
}

namespace {

gs_status render_bwd_impl(const gs_gaussians* g, const gs_camera* cam, const gs_opts* opts, const gs_proj* proj,
                          const gs_bins* bins, const float* final_T, const uint32_t* n_contrib,
                          const float* dL_dimage, gs_grads* out, const void* state, size_t state_bytes, void* ws,
                          size_t ws_bytes, gs_stream stream) {
    Gauss G;
    Cam C;
    int tw, th;
    gs_status s;
    if ((s = to_gauss(g, &G)) || (s = to_cam(cam, &C)) || (s = tiles_of(opts, &tw, &th)) ||
        (s = check_proj(proj, G.n)) || (s = check_bins(bins)))
        return s;
    if (!final_T || !n_contrib || !dL_dimage || !out) return fail(GS_ERR_INVALID, "buffer is NULL");
    if (out->ld < G.n) return fail(GS_ERR_INVALID, "gradient ld < n");
    if (G.n > 0 && (!out->mean || !out->scale || !out->quat || !out->opacity || !out->sh || !out->grad2d))
        return fail(GS_ERR_INVALID, "gradient buffer is NULL");
    if (state) {
        size_t need = 0;
        if ((s = gs_render_state_bytes(bins, opts, &need))) return s;
        if (state_bytes < need) return fail(GS_ERR_INVALID, "state buffer too small: %zu < %zu", state_bytes, need);
    }
    if (G.n > 0 && !bins->first) return fail(GS_ERR_INVALID, "bins first is NULL");
    const size_t need_ws = bwd_ws_bytes(bins->pair_capacity);
    if (!ws || ws_bytes < need_ws) return fail(GS_ERR_INVALID, "workspace too small: %zu < %zu", ws_bytes, need_ws);
    if (reinterpret_cast<uintptr_t>(ws) % 16) return fail(GS_ERR_INVALID, "workspace not 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t cap = bins->pair_capacity;
    // workspace: the per-pair gradient slots, then the tiles with pairs in
    // longest-list-first order (at most one per pair) and their count
    uint32_t* order = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + align256(pair_grad_bytes(cap)));
    uint32_t* order_n = order + (cap > 0 ? cap : 0);
    RenderArgs r = single_render(proj, bins, C, tw, th);
    if (!bins->tile_order) {   // else the order gs_bin_sort kept
        ProfScope ps("tile_order", st);
        launch_tile_order(bins->ranges, r.n_tiles, order, order_n, false, st);
        r.tile_order = order;
        r.tile_order_count = order_n;
    }
    {
        ProfScope ps(state ? "render_bwd_stored" : "render_bwd", st);
        launch_render_bwd(r, final_T, n_contrib, dL_dimage, reinterpret_cast<const ushort4*>(proj->rect),
                          bins->first, ws, cap, static_cast<const float2*>(state), st);
    }
    {
        ProfScope ps("pair_gather", st);
        launch_pair_gather(G.n, bins->first, proj->tiles_touched, ws, cap, bins->status, out->grad2d, st);
    }
    {
        ProfScope ps("project_bwd", st);
        launch_project_bwd(single_job(G, out), single_view(C, tw, th), G.K, G.n, proj->tiles_touched, out->grad2d,
                           bins->status, st);
    }
    return check_hip("gs_render_bwd");
}

}  // namespace

gs_status gs_render_bwd_workspace(const gs_bins* bins, size_t* bytes) {
    gs_status s;
    if ((s = check_bins(bins))) return s;
    if (!bytes) return fail(GS_ERR_INVALID, "bytes is NULL");
    *bytes = bwd_ws_bytes(bins->pair_capacity);
    return GS_OK;
}

gs_status gs_render_bwd(const gs_gaussians* g, const gs_camera* cam, const gs_opts* opts, const gs_proj* proj,
                        const gs_bins* bins, const float* final_T, const uint32_t* n_contrib,
                        const float* dL_dimage, gs_grads* out, void* ws, size_t ws_bytes, gs_stream stream) {
    return render_bwd_impl(g, cam, opts, proj, bins, final_T, n_contrib, dL_dimage, out, nullptr, 0, ws, ws_bytes,
                           stream);
}

gs_status gs_render_bwd_stored(const gs_gaussians* g, const gs_camera* cam, const gs_opts* opts,
                               const gs_proj* proj, const gs_bins* bins, const float* final_T,
                               const uint32_t* n_contrib, const void* state, size_t state_bytes,
                               const float* dL_dimage, gs_grads* out, void* ws, size_t ws_bytes,
                               gs_stream stream) {
    if (!state) return fail(GS_ERR_INVALID, "state is NULL");
    return render_bwd_impl(g, cam, opts, proj, bins, final_T, n_contrib, dL_dimage, out, state, state_bytes, ws,
                           ws_bytes, stream);
}

gs_status gs_loss_workspace(int32_t channels, int32_t width, int32_t height, size_t* bytes) {
    if (!bytes) return fail(GS_ERR_INVALID, "bytes is NULL");
    if (channels < 1 || width < 1 || height < 1)
        return fail(GS_ERR_INVALID, "image shape %dx%dx%d", channels, height, width);
    if ((height + 31) / 32 > 65535 || channels > 65535 ||
        (int64_t)channels * ((width + 31) / 32) * ((height + 31) / 32) > INT32_MAX)
        return fail(GS_ERR_INVALID, "image too large");
    *bytes = loss_workspace_bytes(channels, width, height);
    return GS_OK;
}

gs_status gs_loss(const float* image, const float* image_l1, const float* target, int32_t channels, int32_t width,
                  int32_t height, float lambda, float* loss, float* d_image, float* d_image_l1, void* ws,
                  size_t ws_bytes, gs_stream stream) {
    size_t need = 0;
    gs_status s;
    if ((s = gs_loss_workspace(channels, width, height, &need))) return s;
    if (!image || !target || !loss || !d_image) return fail(GS_ERR_INVALID, "buffer is NULL");
    if (image_l1 && !d_image_l1) return fail(GS_ERR_INVALID, "image_l1 given without d_image_l1");
    if (!std::isfinite(lambda)) return fail(GS_ERR_INVALID, "lambda not finite");
    if (!ws || ws_bytes < need) return fail(GS_ERR_INVALID, "workspace too small: %zu < %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % 8) return fail(GS_ERR_INVALID, "workspace not 8-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    {
        ProfScope ps("loss", st);
        launch_loss(image, image_l1, target, channels, width, height, lambda, d_image,
                    image_l1 ? d_image_l1 : nullptr, ws, st);
    }
    {
        ProfScope ps("loss_finish", st);
        launch_loss_finish(channels, width, height, lambda, ws, loss, st);
    }
    return check_hip("gs_loss");
}

gs_status gs_adam_step(const gs_params* p, float* scale_out, float* opacity_out, const gs_adam_state* st,
                       const gs_grads* grads, const uint32_t* tiles_touched, const int32_t* status,
                       const gs_adam_config* cfg, gs_stream stream) {
    if (!p || !st || !grads || !cfg) return fail(GS_ERR_INVALID, "NULL argument");
    if (p->n < 0 || p->ld < p->n) return fail(GS_ERR_INVALID, "bad sizes n=%lld ld=%lld", (long long)p->n,
                                              (long long)p->ld);
    if (p->sh_degree < 0 || p->sh_degree > 3) return fail(GS_ERR_INVALID, "sh_degree %d", p->sh_degree);
    if (grads->ld < p->n) return fail(GS_ERR_INVALID, "gradient ld < n");
    if (p->n > 0) {
        if (!p->mean || !p->log_scale || !p->quat || !p->logit_opacity || !p->sh || !scale_out || !opacity_out)
            return fail(GS_ERR_INVALID, "parameter buffer is NULL");
        if (!st->m || !st->v) return fail(GS_ERR_INVALID, "moment buffer is NULL");
        if (!grads->mean || !grads->scale || !grads->quat || !grads->opacity || !grads->sh)
            return fail(GS_ERR_INVALID, "gradient buffer is NULL");
        if (tiles_touched && (!grads->grad2d || !st->grad_accum || !st->visible_count))
            return fail(GS_ERR_INVALID, "statistics buffer is NULL");
    }
    const float lrs[6] = {cfg->lr_mean, cfg->lr_scale, cfg->lr_quat, cfg->lr_opacity, cfg->lr_sh_dc, cfg->lr_sh_rest};
    for (float lr : lrs)
        if (!std::isfinite(lr)) return fail(GS_ERR_INVALID, "learning rate not finite");
    if (!(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) ||
        !(cfg->eps >= 0.f) || !std::isfinite(cfg->eps) || cfg->step < 1)
        return fail(GS_ERR_INVALID, "bad Adam hyper-parameters");
    AdamArgs a;
    a.dev = nullptr;
    a.mean = p->mean;
    a.log_scale = p->log_scale;
    a.quat = p->quat;
    a.logit = p->logit_opacity;
    a.sh = p->sh;
    a.scale_out = scale_out;
    a.opacity_out = opacity_out;
    a.g_mean = grads->mean;
    a.g_scale = grads->scale;
    a.g_quat = grads->quat;
    a.g_opacity = grads->opacity;
    a.g_sh = grads->sh;
    a.g2d = grads->grad2d;
    a.m = st->m;
    a.v = st->v;
    a.accum = st->grad_accum;
    a.count = st->visible_count;
    a.tiles = tiles_touched;
    a.status = status;
    a.n = p->n;
    a.ld = p->ld;
    a.gld = grads->ld;
    a.g2d_ld = p->n;
    a.K = (p->sh_degree + 1) * (p->sh_degree + 1);
    const double b1 = cfg->beta1, b2 = cfg->beta2;
    const double bc1 = 1.0 - std::pow(b1, (double)cfg->step), bc2 = 1.0 - std::pow(b2, (double)cfg->step);
    for (int k = 0; k < 6; ++k) a.step_size[k] = (float)((double)lrs[k] / bc1);
    a.beta1 = cfg->beta1;
    a.beta2 = cfg->beta2;
    a.one_m_beta1 = (float)(1.0 - b1);
    a.one_m_beta2 = (float)(1.0 - b2);
    a.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
    a.eps = cfg->eps;
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        ProfScope ps("adam", s);
        launch_adam(a, s);
    }
    return check_hip("gs_adam_step");
}

gs_status gs_sort_workspace(int64_t capacity, int32_t key_bits, size_t* bytes) {
    if (!bytes || capacity < 0 || capacity > kMaxPairs || key_bits < 0 || key_bits > 64)
        return fail(GS_ERR_INVALID, "bad arguments");
    *bytes = align256((size_t)capacity * 8) + align256((size_t)capacity * 4) +
             align256(sort_workspace_bytes(capacity, key_bits));
    return GS_OK;
}

gs_status gs_sort_pairs(uint64_t* keys, uint32_t* vals, const uint32_t* count, int64_t capacity, int32_t key_bits,
                        void* ws, size_t ws_bytes, gs_stream stream) {
    size_t need = 0;
    gs_status s;
    if ((s = gs_sort_workspace(capacity, key_bits, &need))) return s;
    if (!count || (capacity > 0 && (!keys || !vals))) return fail(GS_ERR_INVALID, "NULL buffer");
    if (!ws || ws_bytes < need) return fail(GS_ERR_INVALID, "workspace too small: %zu < %zu", ws_bytes, need);
    char* p = static_cast<char*>(ws);
    uint64_t* alt_k = reinterpret_cast<uint64_t*>(p);
    p += align256((size_t)capacity * 8);
    uint32_t* alt_v = reinterpret_cast<uint32_t*>(p);
    p += align256((size_t)capacity * 4);
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_sort_pairs(keys, vals, alt_k, alt_v, count, capacity, key_bits, false, p, st);
    return check_hip("gs_sort_pairs");
}

}  // extern "C"
