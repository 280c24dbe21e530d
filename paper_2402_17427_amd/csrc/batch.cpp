// Batched training step over several partition cells (gs_batch_*).
//
// VastGaussian (arXiv 2402.17427), section 4.1: the scene is split into
// cells that are optimised independently.  Here several cells of uneven
// Gaussian counts take one training step each together: every stage runs as
// one launch over all cells (one projection over the concatenated Gaussian
// slots, one joint sort whose keys carry each view's tile range, one blend
// forward and one backward over all views' tiles, pulled from a
// longest-list-first queue by a persistent grid), the whole step is captured
// once as a hipGraph and replayed, and the tile shape and launch form are
// chosen by timing the candidates on the batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gs.h"
#include "api_internal.h"
#include "kernels.h"

namespace gs {

namespace {

// An autotune candidate: tile shape, launch form and, for persistent grids,
// the LDS knobs (small = half the default forward batch and backward slot
// capacity) and the grid's share of the workgroups that fit at once.
struct Cand {
    int tw, th, persistent, small_lds, grid_pct;
};

const Cand kCands[] = {{16, 16, 1, 0, 100}, {16, 16, 0, 0, 100}, {32, 16, 1, 0, 100}, {32, 16, 0, 0, 100},
                       {16, 8, 1, 0, 100},  {32, 8, 1, 0, 100},  {16, 16, 1, 1, 100}, {32, 16, 1, 1, 100},
                       {16, 16, 1, 0, 75},  {32, 16, 1, 0, 75}};
static_assert(sizeof(kCands) / sizeof(kCands[0]) <= 16, "gs_batch_stats holds 16 candidates");

template <typename T>
gs_status dmalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ERR_OOM, "device allocation of %zu bytes failed", count * sizeof(T));
    }
    return GS_OK;
}

// The optimiser of a batch must update the planes the cells are rendered
// from, with the moments and statistics of each cell.
gs_status check_batch_optim(const gs_batch_optim* o, const gs_gaussians* cells, const gs_grads* grads, int n) {
    if (!o->params || !o->states) return fail(GS_ERR_INVALID, "optim params or states is NULL");
    const gs_adam_config& y = o->hyper;
    const float lrs[6] = {y.lr_mean, y.lr_scale, y.lr_quat, y.lr_opacity, y.lr_sh_dc, y.lr_sh_rest};
    for (float lr : lrs)
        if (!std::isfinite(lr)) return fail(GS_ERR_INVALID, "learning rate not finite");
    if (!(y.beta1 >= 0.f && y.beta1 < 1.f) || !(y.beta2 >= 0.f && y.beta2 < 1.f) || !(y.eps >= 0.f) ||
        !std::isfinite(y.eps) || y.step < 1 || !std::isfinite(o->lr_mean_final))
        return fail(GS_ERR_INVALID, "bad Adam hyper-parameters");
    for (int c = 0; c < n; ++c) {
        const gs_params& P = o->params[c];
        const gs_adam_state& S = o->states[c];
        if (P.n != cells[c].n || P.ld != cells[c].ld || P.sh_degree != cells[c].sh_degree)
            return fail(GS_ERR_INVALID, "optim params of cell %d do not match the cell", c);
        if (P.n > 0 && (P.mean != cells[c].mean || P.quat != cells[c].quat || P.sh != cells[c].sh))
            return fail(GS_ERR_INVALID, "cell %d must be rendered from its optimised planes", c);
        if (P.n > 0 && (!P.log_scale || !P.logit_opacity || !S.m || !S.v || !S.grad_accum || !S.visible_count))
            return fail(GS_ERR_INVALID, "optimiser buffers of cell %d", c);
        if (grads[c].ld < P.n) return fail(GS_ERR_INVALID, "gradient ld of cell %d", c);
    }
    return GS_OK;
}

}  // namespace

}  // namespace gs

using namespace gs;

struct gs_batch {
    int n = 0;
    int K = 1;
    std::vector<Gauss> cells;
    std::vector<Cam> cams;
    std::vector<int64_t> out0;
    int64_t nslots = 0;
    int64_t img_floats = 0, pix_count = 0, max_pix = 0;
    double headroom = 1.25;

    // chosen configuration
    int tw = 16, th = 16, persistent = 1, use_graph = 1;
    int grid_fwd = 0, grid_bwd = 0;
    int fwd_batch = 0, item_cap = 0, grid_pct = 100;   // persistent grids: LDS knobs (0 = default), grid share
    uint32_t n_tiles = 0;
    int64_t capacity = 0;
    std::vector<double> tune_ms;   // per candidate (autotune), -1 when skipped

    // tables
    View* d_views = nullptr;
    Job* d_jobs = nullptr;
    const float** d_targets = nullptr;
    std::vector<View> h_views;
    std::vector<Job> h_jobs;

    // per-slot buffers
    Rec* rec = nullptr;
    float* depth = nullptr;
    ushort4* rect = nullptr;
    uint32_t* tt = nullptr;
    float* g2d = nullptr;
    uint32_t* first = nullptr;   // emission position of each slot's first pair
    void* scan_ws = nullptr;
    // pair buffers (capacity) and per-tile buffers (max over candidates)
    uint64_t *keys = nullptr, *alt_k = nullptr;
    uint32_t *vals = nullptr, *alt_v = nullptr;
    void* pair_grad = nullptr;   // per-pair image-space gradients of the backward
    uint64_t* masks = nullptr;   // per-pair cell masks the forward keeps for the backward
    int mask_words = 1;          // mask words per pair (most over the candidate tile shapes)
    void* sort_ws = nullptr;
    size_t sort_ws_bytes = 0;
    uint32_t* ranges = nullptr;
    uint32_t* pair_count = nullptr;
    int32_t* status = nullptr;
    uint32_t* queue = nullptr;
    uint32_t* torder = nullptr;   // the blend order the sort keeps: [0] = n_tiles, [1..] every tile
    uint32_t max_tiles = 0;
    // direct binning (every view of the tile shape at most kDirectMaxTiles
    // tiles): the plan of the current shape and its device table; the
    // placed pairs go to alt_k
    bool direct = false;
    DPlan dplan;
    std::vector<DView> h_dviews;
    DView* d_dviews = nullptr;
    void* dscratch = nullptr;
    size_t dscratch_bytes = 0;
    // per-pixel buffers
    float* final_T = nullptr;
    uint32_t* n_contrib = nullptr;
    float* dimg = nullptr;
    // caller outputs
    float* images = nullptr;
    float* loss = nullptr;
    double* l1_part = nullptr;    // per view: the L1 loss's partial sums
    // Eq. 1 loss (lambda > 0) per view, and the optimiser step of every cell
    float lambda = 0.f;
    std::vector<const float*> h_targets;
    void* loss_ws = nullptr;
    std::vector<size_t> loss_ws_off;
    AdamSched* sched = nullptr;   // device schedule advanced inside the step
    std::vector<AdamArgs> adam;   // one launch per cell (empty: no optimiser)
    bool optim_on = false;        // off during sizing and autotune

    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~gs_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        void* ptrs[] = {d_views, d_jobs, d_targets, rec, depth, rect, tt, g2d, first, scan_ws, keys, alt_k, vals,
                        alt_v, pair_grad, masks, sort_ws, ranges, pair_count, status, queue, torder, d_dviews,
                        dscratch,
                        final_T, n_contrib, dimg, loss_ws, sched, l1_part};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
    }

    uint32_t tiles_for(int w, int h) const {
        uint32_t t = 0;
        for (const Cam& c : cams) t += (uint32_t)(((c.W + w - 1) / w) * ((c.H + h - 1) / h));
        return t;
    }

    // LDS knobs and grid share of an autotune candidate.
    void set_knobs(const Cand& c) {
        fwd_batch = c.small_lds ? render_fwd_batch_small() : 0;
        item_cap = c.small_lds ? render_item_cap_small() : 0;
        grid_pct = c.grid_pct;
    }

    // The direct-binning plan of the views for a tile shape (false: some
    // view has too many tiles, so the emission path bins them).
    bool plan_direct(int w, int h, std::vector<DView>* dv, DPlan* plan) const {
        std::vector<int64_t> s0(n), s1(n);
        std::vector<int> ntx(n), nty(n);
        std::vector<uint32_t> base(n);
        uint32_t b = 0;
        for (int c = 0; c < n; ++c) {
            s0[c] = h_jobs[c].out0;
            s1[c] = h_jobs[c].out0 + h_jobs[c].count;
            ntx[c] = (cams[c].W + w - 1) / w;
            nty[c] = (cams[c].H + h - 1) / h;
            base[c] = b;
            b += (uint32_t)(ntx[c] * nty[c]);
        }
        dv->assign(n, DView{});
        return bin_direct_plan(n, s0.data(), s1.data(), ntx.data(), nty.data(), base.data(), dv->data(), plan);
    }

    // View table for a tile shape (host copy + upload).
    gs_status set_tiles(int w, int h, hipStream_t st) {
        tw = w;
        th = h;
        uint32_t base = 0;
        for (int c = 0; c < n; ++c) {
            View& v = h_views[c];
            v.ntx = (cams[c].W + w - 1) / w;
            v.nty = (cams[c].H + h - 1) / h;
            v.tile_base = base;
            base += (uint32_t)(v.ntx * v.nty);
        }
        n_tiles = base;
        direct = d_dviews && plan_direct(w, h, &h_dviews, &dplan) && bin_direct_scratch_bytes(dplan) <= dscratch_bytes;
        if (hipMemcpyAsync(d_views, h_views.data(), sizeof(View) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
            (direct && hipMemcpyAsync(d_dviews, h_dviews.data(), sizeof(DView) * n, hipMemcpyHostToDevice, st) !=
                           hipSuccess) ||
            hipStreamSynchronize(st) != hipSuccess)
            return check_hip("gs_batch: view table upload");
        grid_fwd = std::max(1, render_persistent_grid(w, h, false, fwd_batch) * grid_pct / 100);
        grid_bwd = std::max(1, render_persistent_grid(w, h, true, item_cap) * grid_pct / 100);
        return GS_OK;
    }

    ViewTab vt() const {
        ViewTab t;
        std::memset(&t, 0, sizeof t);
        t.dev = d_views;
        t.n = n;
        return t;
    }
    JobTab jt() const {
        JobTab t;
        std::memset(&t, 0, sizeof t);
        t.dev = d_jobs;
        t.n = n;
        return t;
    }

    void enqueue_project_bin(hipStream_t st) {
        launch_project(jt(), vt(), K, nslots, tw, th, rec, depth, rect, tt, st);
        if (direct) {
            DTab t;
            std::memset(&t, 0, sizeof t);
            t.dev = d_dviews;
            t.n = n;
            launch_bin_direct_place(dplan, t, rect, depth, capacity, first, ranges, pair_count, status, dscratch,
                                    alt_k, st);
            return;
        }
        const bool to_alt = bin_sort_emit_to_alt(tile_bits(n_tiles));
        const ZeroList z = bin_sort_zero_list(sort_ws, capacity, tile_bits(n_tiles), ranges, n_tiles);
        launch_emit_pairs(nslots, tt, rect, depth, jt(), vt(), capacity, to_alt ? alt_k : keys, to_alt ? alt_v : vals,
                          first, pair_count, status, scan_ws, st, &z);
    }

    // One training step of every cell: project, bin, sort, ranges, blend,
    // L1 loss gradient, blend backward, projection backward.
    void enqueue_step(hipStream_t st) {
        enqueue_project_bin(st);
        if (direct)
            launch_bin_direct_sort(n_tiles, capacity, keys, vals, ranges, status, torder, alt_k, st);
        else
            launch_bin_sort(keys, vals, alt_k, alt_v, pair_count, capacity, tile_bits(n_tiles), ranges, n_tiles,
                            sort_ws, st, true, torder);
        RenderArgs r;
        std::memset(&r, 0, sizeof r);
        r.rec = rec;
        r.vals = vals;
        r.ranges = ranges;
        r.status = status;
        r.views = vt();
        r.n_tiles = n_tiles;
        r.tw = tw;
        r.th = th;
        r.masks = masks;
        r.fwd_batch = fwd_batch;
        r.item_cap = item_cap;
        // both launch forms take the tiles longest list first, in the order
        // the sort kept
        r.tile_order = torder + 1;
        r.tile_order_count = torder;
        if (persistent) {
            r.queue = queue;
            r.order = torder + 1;
            r.persistent_grid = grid_fwd;
        }
        launch_render_fwd(r, images, final_T, n_contrib, nullptr, nullptr, st);
        if (lambda > 0.f) {
            for (int c = 0; c < n; ++c) {
                const View& v = h_views[c];
                void* ws = static_cast<char*>(loss_ws) + loss_ws_off[c];
                launch_loss(images + v.img_base, nullptr, h_targets[c], 3, cams[c].W, cams[c].H, lambda,
                            dimg + v.img_base, nullptr, ws, st);
                launch_loss_finish(3, cams[c].W, cams[c].H, lambda, ws, loss + c, st, 1);
            }
        } else {
            launch_l1(vt(), n, max_pix, d_targets, images, dimg, loss, l1_part, status, st);
        }
        if (persistent) r.persistent_grid = grid_bwd;
        launch_render_bwd(r, final_T, n_contrib, dimg, rect, first, pair_grad, capacity, nullptr, st);
        launch_pair_gather(nslots, first, tt, pair_grad, capacity, status, g2d, st);
        launch_project_bwd(jt(), vt(), K, nslots, tt, g2d, status, st);
        if (optim_on && !adam.empty()) {
            launch_adam_prepare(sched, st);
            for (const AdamArgs& a : adam) launch_adam(a, st);
        }
    }

    // Pairs the current tile shape needs (one projection + emission, synchronous).
    gs_status pairs_needed(hipStream_t st, uint32_t* need) {
        const int64_t cap = capacity;
        capacity = 0;   // count only
        enqueue_project_bin(st);
        capacity = cap;
        uint32_t pc[2] = {0, 0};
        if (hipMemcpyAsync(pc, pair_count, sizeof pc, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return check_hip("gs_batch: sizing pass");
        *need = pc[1];
        return GS_OK;
    }

    gs_status alloc_pairs(int64_t cap) {
        if (cap > kMaxPairs) return fail(GS_ERR_CAPACITY, "batch needs %lld pairs (> 2^30-1)", (long long)cap);
        for (void* p : {(void*)keys, (void*)alt_k, (void*)vals, (void*)alt_v, pair_grad, (void*)masks, sort_ws})
            if (p) (void)hipFree(p);
        keys = alt_k = nullptr;
        vals = alt_v = nullptr;
        pair_grad = sort_ws = nullptr;
        masks = nullptr;
        gs_status s;
        sort_ws_bytes = sort_workspace_bytes(cap, 64);
        if ((s = dmalloc(&keys, cap)) || (s = dmalloc(&alt_k, cap)) || (s = dmalloc(&vals, cap)) ||
            (s = dmalloc(&alt_v, cap)) || (s = dmalloc(reinterpret_cast<char**>(&sort_ws), sort_ws_bytes)) ||
            (s = dmalloc(reinterpret_cast<char**>(&pair_grad), pair_grad_bytes(cap))) ||
            (s = dmalloc(&masks, cap * mask_words)))
            return s;
        capacity = cap;
        return GS_OK;
    }

    gs_status capture(hipStream_t st) {
        if (exec) {
            (void)hipGraphExecDestroy(exec);
            exec = nullptr;
        }
        if (graph) {
            (void)hipGraphDestroy(graph);
            graph = nullptr;
        }
        if (!use_graph) return GS_OK;
        if (hipStreamSynchronize(st) != hipSuccess) return check_hip("gs_batch: capture");
        if (hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return check_hip("gs_batch: begin capture");
        enqueue_step(cap_stream);
        if (hipStreamEndCapture(cap_stream, &graph) != hipSuccess) return check_hip("gs_batch: end capture");
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
            return check_hip("gs_batch: instantiate");
        return GS_OK;
    }

    gs_status run(hipStream_t st) {
        if (use_graph && exec) {
            if (hipGraphLaunch(exec, st) != hipSuccess) return check_hip("gs_batch_step: graph launch");
            return GS_OK;
        }
        enqueue_step(st);
        return check_hip("gs_batch_step");
    }

    // Mean step time of the current configuration over `iters` launches.
    gs_status time_steps(hipStream_t st, int warm, int iters, double* ms) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return check_hip("gs_batch: events");
        gs_status s = GS_OK;
        for (int i = 0; i < warm && !s; ++i) s = run(st);
        if (!s && hipEventRecord(a, st) != hipSuccess) s = check_hip("gs_batch: event");
        for (int i = 0; i < iters && !s; ++i) s = run(st);
        float f = 0.f;
        if (!s && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                   hipEventElapsedTime(&f, a, b) != hipSuccess))
            s = check_hip("gs_batch: timing");
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        *ms = f / (iters > 0 ? iters : 1);
        return s;
    }

    gs_status device_status(hipStream_t st, int32_t* out) {
        if (hipMemcpyAsync(out, status, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return check_hip("gs_batch: status");
        return GS_OK;
    }
};

extern "C" {

gs_status gs_batch_create(const gs_gaussians* cells, const gs_camera* cams, const float* const* targets,
                          int32_t n_cells, float* images, gs_grads* grads, float* loss,
                          const gs_batch_config* cfg, gs_stream stream, gs_batch** out) {
    if (!out) return fail(GS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n_cells <= 0 || !cells || !cams || !targets || !images || !grads || !loss)
        return fail(GS_ERR_INVALID, "NULL argument or n_cells <= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    gs_batch* b = new gs_batch();
    b->n = n_cells;
    gs_status s = GS_OK;
    for (int c = 0; c < n_cells && !s; ++c) {
        Gauss G;
        Cam C;
        if ((s = to_gauss(&cells[c], &G)) || (s = to_cam(&cams[c], &C))) break;
        if (c == 0) b->K = G.K;
        else if (G.K != b->K) s = fail(GS_ERR_INVALID, "cells must share one SH degree");
        if (!targets[c]) s = fail(GS_ERR_INVALID, "target %d is NULL", c);
        if (grads[c].ld < G.n || (G.n > 0 && (!grads[c].mean || !grads[c].scale || !grads[c].quat ||
                                              !grads[c].opacity || !grads[c].sh)))
            s = fail(GS_ERR_INVALID, "gradient buffers of cell %d", c);
        b->cells.push_back(G);
        b->cams.push_back(C);
    }
    int tw0 = cfg && cfg->tile_w ? cfg->tile_w : 16, th0 = cfg && cfg->tile_h ? cfg->tile_h : 16;
    const int autotune = cfg ? cfg->autotune : 0;
    b->persistent = cfg ? (cfg->persistent != 0) : 1;
    b->use_graph = cfg ? (cfg->use_graph != 0) : 1;
    b->headroom = cfg && cfg->capacity_headroom > 1.0 ? cfg->capacity_headroom : 1.25;
    b->lambda = cfg ? cfg->loss_lambda : 0.f;
    if (cfg && cfg->fwd_batch) {
        if (cfg->fwd_batch == render_fwd_batch_small()) b->fwd_batch = cfg->fwd_batch;
        else if (cfg->fwd_batch != render_fwd_batch_default())
            s = fail(GS_ERR_INVALID, "fwd_batch %d: 0, %d or %d", cfg->fwd_batch, render_fwd_batch_default(),
                     render_fwd_batch_small());
    }
    if (cfg && cfg->item_cap) {
        if (cfg->item_cap == render_item_cap_small()) b->item_cap = cfg->item_cap;
        else if (cfg->item_cap != render_item_cap_default())
            s = fail(GS_ERR_INVALID, "item_cap %d: 0, %d or %d", cfg->item_cap, render_item_cap_default(),
                     render_item_cap_small());
    }
    if (cfg && cfg->grid_pct) {
        if (cfg->grid_pct < 1 || cfg->grid_pct > 100) s = fail(GS_ERR_INVALID, "grid_pct %d not in 1..100", cfg->grid_pct);
        else b->grid_pct = cfg->grid_pct;
    }
    if (!s && (!std::isfinite(b->lambda) || b->lambda < 0.f)) s = fail(GS_ERR_INVALID, "loss_lambda must be >= 0");
    const gs_batch_optim* opt = cfg ? cfg->optim : nullptr;
    if (!s && opt) s = check_batch_optim(opt, cells, grads, n_cells);
    if (!s && !render_tile_supported(tw0, th0)) s = fail(GS_ERR_UNSUPPORTED, "tile %dx%d not supported", tw0, th0);
    if (s) {
        delete b;
        return s;
    }
    // slots, images, tables
    int64_t slot = 0, img = 0, pix = 0;
    b->h_views.resize(n_cells);
    b->h_jobs.resize(n_cells);
    for (int c = 0; c < n_cells; ++c) {
        const Gauss& G = b->cells[c];
        const Cam& C = b->cams[c];
        b->out0.push_back(slot);
        Job& j = b->h_jobs[c];
        std::memset(&j, 0, sizeof j);
        j.g = G;
        j.src0 = 0;
        j.count = G.n;
        j.out0 = slot;
        j.view = c;
        j.gmean = grads[c].mean;
        j.gscale = grads[c].scale;
        j.gquat = grads[c].quat;
        j.gopac = grads[c].opacity;
        j.gsh = grads[c].sh;
        j.gld = grads[c].ld;
        slot += (G.n + kSlotAlign - 1) / kSlotAlign * kSlotAlign;
        View& v = b->h_views[c];
        std::memset(&v, 0, sizeof v);
        v.cam = C;
        v.img_base = img;
        v.pix_base = pix;
        img += 3 * (int64_t)C.W * C.H;
        pix += (int64_t)C.W * C.H;
        b->max_pix = std::max<int64_t>(b->max_pix, (int64_t)C.W * C.H);
    }
    if (slot > (int64_t)0xFFFFFFFF) s = fail(GS_ERR_INVALID, "more than 2^32-1 Gaussian slots");
    b->nslots = slot;
    b->img_floats = img;
    b->pix_count = pix;
    b->images = images;
    b->loss = loss;
    // tile buffers sized for the candidate with the most tiles
    uint32_t max_tiles = b->tiles_for(tw0, th0);
    if (autotune)
        for (const Cand& c : kCands) max_tiles = std::max(max_tiles, b->tiles_for(c.tw, c.th));
    b->max_tiles = max_tiles;
    if (!s) {
        if ((s = dmalloc(&b->d_views, n_cells)) || (s = dmalloc(&b->d_jobs, n_cells)) ||
            (s = dmalloc(&b->d_targets, n_cells)) || (s = dmalloc(&b->rec, slot)) || (s = dmalloc(&b->depth, slot)) ||
            (s = dmalloc(&b->rect, slot)) || (s = dmalloc(&b->tt, slot)) || (s = dmalloc(&b->g2d, slot * 9)) || (s = dmalloc(&b->first, slot)) ||
            (s = dmalloc(reinterpret_cast<char**>(&b->scan_ws), scan_workspace_bytes(slot))) ||
            (s = dmalloc(&b->ranges, (size_t)max_tiles * 2)) || (s = dmalloc(&b->pair_count, 2)) ||
            (s = dmalloc(&b->status, 1)) || (s = dmalloc(&b->queue, 1)) || (s = dmalloc(&b->torder, (size_t)max_tiles + 1)) ||
            (s = dmalloc(&b->final_T, pix)) ||
            (s = dmalloc(&b->n_contrib, pix)) || (s = dmalloc(&b->dimg, img)) ||
            (s = dmalloc(&b->l1_part, (size_t)n_cells * kL1MaxChunks)))
            ;
    }
    if (!s) {   // direct-binning scratch for the largest plan over the tile shapes tried
        std::vector<DView> dv;
        DPlan plan;
        size_t need = 0;
        if (b->plan_direct(tw0, th0, &dv, &plan)) need = bin_direct_scratch_bytes(plan);
        if (autotune)
            for (const Cand& c : kCands)
                if (b->plan_direct(c.tw, c.th, &dv, &plan)) need = std::max(need, bin_direct_scratch_bytes(plan));
        if (need > 0 && (s = dmalloc(&b->d_dviews, n_cells)) == GS_OK &&
            (s = dmalloc(reinterpret_cast<char**>(&b->dscratch), need)) == GS_OK)
            b->dscratch_bytes = need;
    }
    if (!s) {
        b->h_targets.assign(targets, targets + n_cells);
        size_t off = 0;
        for (int c = 0; c < n_cells; ++c) {
            b->loss_ws_off.push_back(off);
            off += (loss_workspace_bytes(3, b->cams[c].W, b->cams[c].H) + 255) / 256 * 256;
        }
        if (b->lambda > 0.f) s = dmalloc(reinterpret_cast<char**>(&b->loss_ws), off);
    }
    if (!s && opt) {
        AdamSched h;
        std::memset(&h, 0, sizeof h);
        h.step = opt->hyper.step - 1;
        const gs_adam_config& y = opt->hyper;
        const float lrs[6] = {y.lr_mean, y.lr_scale, y.lr_quat, y.lr_opacity, y.lr_sh_dc, y.lr_sh_rest};
        for (int k = 0; k < 6; ++k) h.lr[k] = lrs[k];
        h.beta1 = y.beta1;
        h.beta2 = y.beta2;
        h.lr_mean_final = opt->lr_mean_final;
        h.lr_mean_steps = opt->lr_mean_steps;
        if ((s = dmalloc(&b->sched, 1)) == GS_OK &&
            (hipMemcpyAsync(b->sched, &h, sizeof h, hipMemcpyHostToDevice, st) != hipSuccess ||
             hipStreamSynchronize(st) != hipSuccess))
            s = check_hip("gs_batch: optimiser schedule upload");
        for (int c = 0; c < n_cells && !s; ++c) {
            const gs_params& P = opt->params[c];
            const gs_adam_state& S = opt->states[c];
            AdamArgs a;
            std::memset(&a, 0, sizeof a);
            a.dev = &b->sched->dev;
            a.mean = P.mean;
            a.log_scale = P.log_scale;
            a.quat = P.quat;
            a.logit = P.logit_opacity;
            a.sh = P.sh;
            a.scale_out = const_cast<float*>(cells[c].scale);
            a.opacity_out = const_cast<float*>(cells[c].opacity);
            a.g_mean = grads[c].mean;
            a.g_scale = grads[c].scale;
            a.g_quat = grads[c].quat;
            a.g_opacity = grads[c].opacity;
            a.g_sh = grads[c].sh;
            a.g2d = b->g2d + b->out0[c];
            a.g2d_ld = b->nslots;
            a.m = S.m;
            a.v = S.v;
            a.accum = S.grad_accum;
            a.count = S.visible_count;
            a.tiles = b->tt + b->out0[c];
            a.status = b->status;
            a.n = P.n;
            a.ld = P.ld;
            a.gld = grads[c].ld;
            a.K = b->K;
            a.beta1 = y.beta1;
            a.beta2 = y.beta2;
            a.one_m_beta1 = (float)(1.0 - (double)y.beta1);
            a.one_m_beta2 = (float)(1.0 - (double)y.beta2);
            a.eps = y.eps;
            if (P.n > 0) b->adam.push_back(a);
        }
    }
    if (!s && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
        s = check_hip("gs_batch: stream");
    if (!s) {
        std::vector<const float*> tg(targets, targets + n_cells);
        if (hipMemcpyAsync(b->d_jobs, b->h_jobs.data(), sizeof(Job) * n_cells, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(b->d_targets, tg.data(), sizeof(float*) * n_cells, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(b->status, "\0\0\0\0", 4, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            s = check_hip("gs_batch: table upload");
    }
    // capacity: the most pairs any candidate tile shape needs, with headroom
    std::vector<Cand> cands;
    if (autotune) cands.assign(std::begin(kCands), std::end(kCands));
    else cands.push_back({tw0, th0, b->persistent, 0, b->grid_pct});
    uint32_t need = 0;
    for (const Cand& c : cands) {
        if (s) break;
        uint32_t p = 0;
        if ((s = b->set_tiles(c.tw, c.th, st)) || (s = b->pairs_needed(st, &p))) break;
        need = std::max(need, p);
        b->mask_words = std::max(b->mask_words, render_mask_words(c.tw, c.th));
    }
    if (!s) s = b->alloc_pairs((int64_t)std::ceil(need * b->headroom) + 4096);
    // autotune: time every candidate (eager launches), keep the fastest
    if (!s && autotune) {
        double best = 1e30;
        Cand pick = cands[0];
        const int saved_graph = b->use_graph;
        b->use_graph = 0;
        for (const Cand& c : cands) {
            double ms = -1;
            b->persistent = c.persistent;
            b->set_knobs(c);
            if ((s = b->set_tiles(c.tw, c.th, st)) || (s = b->time_steps(st, 2, 5, &ms))) break;
            int32_t dst = 0;
            if ((s = b->device_status(st, &dst))) break;
            if (dst != 0) ms = -1;   // did not fit (cannot happen with the sized capacity)
            b->tune_ms.push_back(ms);
            if (ms > 0 && ms < best) {
                best = ms;
                pick = c;
            }
        }
        b->use_graph = saved_graph;
        b->persistent = pick.persistent;
        b->set_knobs(pick);
        if (!s) s = b->set_tiles(pick.tw, pick.th, st);
    } else if (!s) {
        s = b->set_tiles(tw0, th0, st);
    }
    b->optim_on = true;
    if (!s) s = b->capture(st);
    if (s) {
        delete b;
        return s;
    }
    *out = b;
    return GS_OK;
}

gs_status gs_batch_step(gs_batch* b, gs_stream stream) {
    if (!b) return fail(GS_ERR_INVALID, "batch is NULL");
    return b->run(static_cast<hipStream_t>(stream));
}

gs_status gs_batch_info(const gs_batch* b, gs_batch_stats* info) {
    if (!b || !info) return fail(GS_ERR_INVALID, "NULL argument");
    std::memset(info, 0, sizeof *info);
    info->tile_w = b->tw;
    info->tile_h = b->th;
    info->persistent = b->persistent;
    info->use_graph = b->use_graph && b->exec != nullptr;
    info->grid_fwd = b->grid_fwd;
    info->grid_bwd = b->grid_bwd;
    info->fwd_batch = b->fwd_batch ? b->fwd_batch : render_fwd_batch_default();
    info->item_cap = b->item_cap ? b->item_cap : render_item_cap_default();
    info->grid_pct = b->grid_pct;
    info->n_tiles = b->n_tiles;
    info->slots = b->nslots;
    info->pair_capacity = b->capacity;
    info->n_candidates = (int32_t)b->tune_ms.size();
    for (size_t i = 0; i < b->tune_ms.size() && i < 16; ++i) {
        info->cand_tile_w[i] = kCands[i].tw;
        info->cand_tile_h[i] = kCands[i].th;
        info->cand_persistent[i] = kCands[i].persistent;
        info->cand_fwd_batch[i] = kCands[i].small_lds ? render_fwd_batch_small() : render_fwd_batch_default();
        info->cand_item_cap[i] = kCands[i].small_lds ? render_item_cap_small() : render_item_cap_default();
        info->cand_grid_pct[i] = kCands[i].grid_pct;
        info->cand_ms[i] = b->tune_ms[i];
    }
    return GS_OK;
}

gs_status gs_batch_status(gs_batch* b, gs_stream stream, int32_t* status, uint32_t* pairs) {
    if (!b || !status) return fail(GS_ERR_INVALID, "NULL argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint32_t pc[2] = {0, 0};
    if (hipMemcpyAsync(status, b->status, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(pc, b->pair_count, sizeof pc, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return check_hip("gs_batch_status");
    if (pairs) {
        pairs[0] = pc[0];
        pairs[1] = pc[1];
    }
    return GS_OK;
}

void gs_batch_destroy(gs_batch* b) { delete b; }

}  // extern "C"
