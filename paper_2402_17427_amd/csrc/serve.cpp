// Render server over a merged scene resident in HBM (gs_serve_*).
//
// VastGaussian (arXiv 2402.17427), sections 4.3 and 5: the optimised cells
// are merged into one scene that is rendered in real time from novel
// views.  The server keeps that scene in device memory and renders
// requests of mixed resolutions with continuous batching:
//   * submit() culls the scene's cells against the request's view frustum
//     on the host (cell AABBs widened by the Gaussians' support), queues the
//     request and returns a ticket;
//   * a worker thread forms a batch from the head of the queue whenever a
//     pipeline (stream + workspace) is free, admitting requests in arrival
//     order while the batch's Gaussian slots, pixels, tiles and estimated
//     (Gaussian, tile) pairs fit the pipeline's share of the memory budget;
//     the batch is one projection, one joint sort (each view owns a range
//     of tile ids) and one blend launch over all its views' tiles, writing
//     each image straight into the caller's buffer;
//   * requests arriving while batches run are admitted into the next batch
//     on another pipeline, so batches overlap on the device;
//   * a completion thread waits for each batch, requeues its requests at
//     the head of the queue if the pairs overflowed (the pair estimate is
//     then raised), and otherwise stamps their completion times.
// A request's image does not depend on what it was batched with: its
// tiles, their sorted lists and every per-pixel operation are the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/gs.h"
#include "api_internal.h"
#include "kernels.h"

namespace gs {

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int64_t align_slots(int64_t n) { return (n + kSlotAlign - 1) / kSlotAlign * kSlotAlign; }

struct Req {
    uint64_t ticket = 0;
    Cam cam;
    float* out = nullptr;
    std::vector<int> cells;
    int64_t slots = 0, pix = 0;
    uint32_t tiles = 0;
    int64_t t_arrive = 0, t_start = 0, t_done = 0;
    int32_t status = GS_OK;
    int32_t batch_views = 0;
    int32_t attempts = 0;
    bool done = false;
};

struct Pipe {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    // capacities
    int64_t slots_cap = 0, pairs_cap = 0, pix_cap = 0;
    uint32_t tiles_cap = 0;
    int views_cap = 0, jobs_cap = 0;
    // device
    Rec* rec = nullptr;
    float* depth = nullptr;
    ushort4* rect = nullptr;
    uint32_t* tt = nullptr;
    void* scan_ws = nullptr;
    uint64_t *keys = nullptr, *alt_k = nullptr;
    uint32_t *vals = nullptr, *alt_v = nullptr;
    void* sort_ws = nullptr;
    uint32_t* ranges = nullptr;
    uint32_t* torder = nullptr;   // the blend order the sort keeps: [0] = tile count, [1..] the tiles
    uint32_t* pair_count = nullptr;
    int32_t* status = nullptr;
    float* final_T = nullptr;
    uint32_t* n_contrib = nullptr;
    View* d_views = nullptr;
    Job* d_jobs = nullptr;
    DView* d_dviews = nullptr;   // direct binning: the batch's plan
    void* dscratch = nullptr;
    size_t dscratch_bytes = 0;
    // pinned host
    View* h_views = nullptr;
    Job* h_jobs = nullptr;
    DView* h_dviews = nullptr;
    int32_t* h_status = nullptr;   // status, pairs processed, pairs needed
    // batch in flight
    std::vector<uint64_t> tickets;
    int64_t slots_used = 0;
};

template <typename T>
bool dalloc(T** p, size_t count) {
    *p = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(p), (count ? count : 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

// Conservative frustum test of an axis-aligned box (world) for a camera:
// false only when every point of the box lies behind the near plane or
// outside one side plane of the (widened) view frustum.
bool box_visible(const Cam& c, const float* box, float widen) {
    double cz[8], cx[8], cy[8];
    for (int k = 0; k < 8; ++k) {
        const double p[3] = {box[(k & 1) ? 3 : 0], box[(k & 2) ? 4 : 1], box[(k & 4) ? 5 : 2]};
        cx[k] = c.R[0] * p[0] + c.R[1] * p[1] + c.R[2] * p[2] + c.t[0];
        cy[k] = c.R[3] * p[0] + c.R[4] * p[1] + c.R[5] * p[2] + c.t[1];
        cz[k] = c.R[6] * p[0] + c.R[7] * p[1] + c.R[8] * p[2] + c.t[2];
    }
    const double m = widen;   // pixels of margin on every side of the image
    const double xl = -(c.cx + m) / c.fx, xr = (c.W - c.cx + m) / c.fx;
    const double yt = -(c.cy + m) / c.fy, yb = (c.H - c.cy + m) / c.fy;
    bool all_near = true, all_l = true, all_r = true, all_t = true, all_b = true;
    for (int k = 0; k < 8; ++k) {
        all_near &= cz[k] <= c.near_z;
        all_l &= cx[k] < xl * cz[k];
        all_r &= cx[k] > xr * cz[k];
        all_t &= cy[k] < yt * cz[k];
        all_b &= cy[k] > yb * cz[k];
    }
    return !(all_near || all_l || all_r || all_t || all_b);
}

}  // namespace

}  // namespace gs

using namespace gs;

struct gs_server {
    Gauss scene;
    std::vector<float> boxes;        // [n_cells][6], widened by the support radius
    std::vector<int64_t> cell_off;   // [n_cells + 1]
    int n_cells = 0;
    int tw = 16, th = 16;
    int max_queue = 1024;
    float widen_px = 64.f;
    std::vector<Pipe> pipes;

    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_inflight;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<int> inflight;        // pipelines in launch order
    uint64_t next_ticket = 1;
    bool stop = false;
    bool paused = false;
    bool worker_done = false;
    double pairs_per_slot = 3.0;     // admission estimate, raised on overflow
    int64_t batches = 0, requeues = 0, max_batch_views = 0;
    std::thread worker, completer;
    std::atomic<int> fatal{0};

    int64_t est_pairs(const Req& r) const { return (int64_t)std::ceil(pairs_per_slot * (double)r.slots) + 1024; }

    bool fits_alone(const Req& r, const Pipe& p) const {
        return align_slots(r.slots) + 256 * (int64_t)r.cells.size() <= p.slots_cap && r.pix <= p.pix_cap &&
               r.tiles <= p.tiles_cap && (int)r.cells.size() <= p.jobs_cap;
    }

    void worker_loop() {
        for (;;) {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                if (stop && queue.empty() && all_idle()) return true;
                if (queue.empty() || (paused && !stop)) return false;
                for (const Pipe& p : pipes)
                    if (!p.busy) return true;
                return false;
            });
            if (stop && queue.empty() && all_idle()) break;
            int pi = 0;
            while (pipes[pi].busy) ++pi;
            Pipe& p = pipes[pi];
            // admit from the head of the queue while the batch fits
            std::vector<uint64_t> batch;
            int64_t slots = 0, pix = 0, pairs = 0;
            uint32_t tiles = 0;
            int jobs = 0;
            while (!queue.empty() && (int)batch.size() < p.views_cap) {
                Req& r = reqs[queue.front()];
                const int64_t rs = (int64_t)r.cells.size() * kSlotAlign + r.slots;
                const int64_t rp = est_pairs(r);
                const bool first = batch.empty();
                if (!first && (slots + rs > p.slots_cap || pix + r.pix > p.pix_cap || tiles + r.tiles > p.tiles_cap ||
                               pairs + rp > p.pairs_cap || jobs + (int)r.cells.size() > p.jobs_cap))
                    break;
                slots += rs;
                pix += r.pix;
                tiles += r.tiles;
                pairs += rp;
                jobs += (int)r.cells.size();
                batch.push_back(r.ticket);
                queue.pop_front();
            }
            const int64_t t0 = now_ns();
            std::vector<Req*> rs;
            for (uint64_t t : batch) {
                Req& r = reqs[t];
                r.t_start = t0;
                r.batch_views = (int32_t)batch.size();
                ++r.attempts;
                rs.push_back(&r);
            }
            p.busy = true;
            p.tickets = batch;
            ++batches;
            max_batch_views = std::max<int64_t>(max_batch_views, (int64_t)batch.size());
            lk.unlock();
            launch(p, rs);
            lk.lock();
            inflight.push_back(pi);
            cv_inflight.notify_one();
        }
        std::lock_guard<std::mutex> lk(mu);
        worker_done = true;
        cv_inflight.notify_all();
    }

    // Enqueue one batch on pipeline p (called without the lock; the
    // requests are not touched by other threads while in flight).
    void launch(Pipe& p, const std::vector<Req*>& rs) {
        int nv = 0, nj = 0;
        int64_t slot = 0, pix = 0;
        uint32_t tile = 0;
        for (Req* r : rs) {
            View& v = p.h_views[nv];
            std::memset(&v, 0, sizeof v);
            v.cam = r->cam;
            v.ntx = (r->cam.W + tw - 1) / tw;
            v.nty = (r->cam.H + th - 1) / th;
            v.tile_base = tile;
            v.pix_base = pix;
            v.img_base = 0;
            v.out_image = r->out;
            tile += (uint32_t)(v.ntx * v.nty);
            pix += (int64_t)r->cam.W * r->cam.H;
            for (int c : r->cells) {
                Job& j = p.h_jobs[nj++];
                std::memset(&j, 0, sizeof j);
                j.g = scene;
                j.src0 = cell_off[c];
                j.count = cell_off[c + 1] - cell_off[c];
                j.out0 = slot;
                j.view = nv;
                slot += align_slots(j.count);
            }
            ++nv;
        }
        hipStream_t st = p.st;
        ViewTab vt;
        JobTab jt;
        std::memset(&vt, 0, sizeof vt);
        std::memset(&jt, 0, sizeof jt);
        vt.dev = p.d_views;
        vt.n = nv;
        jt.dev = p.d_jobs;
        jt.n = nj;
        (void)hipMemcpyAsync(p.d_views, p.h_views, sizeof(View) * nv, hipMemcpyHostToDevice, st);
        if (nj) (void)hipMemcpyAsync(p.d_jobs, p.h_jobs, sizeof(Job) * nj, hipMemcpyHostToDevice, st);
        if (nj == 0) {   // nothing visible: every view is its background
            slot = 0;
        }
        const int64_t cap = p.pairs_cap;
        launch_project(jt, vt, scene.K, slot, tw, th, p.rec, p.depth, p.rect, p.tt, st);
        // direct binning when every view fits it: the views' slot ranges
        // (their jobs are consecutive) and tile grids
        bool direct = nv > 0;
        DPlan plan;
        if (direct) {
            std::vector<int64_t> s0(nv), s1(nv);
            std::vector<int> ntx(nv), nty(nv);
            std::vector<uint32_t> base(nv);
            int jv = 0;
            for (int v = 0; v < nv; ++v) {
                const int j0 = jv;
                while (jv < nj && p.h_jobs[jv].view == v) ++jv;
                s0[v] = j0 < jv ? p.h_jobs[j0].out0 : (jv < nj ? p.h_jobs[jv].out0 : slot);
                s1[v] = j0 < jv ? p.h_jobs[jv - 1].out0 + p.h_jobs[jv - 1].count : s0[v];
                ntx[v] = p.h_views[v].ntx;
                nty[v] = p.h_views[v].nty;
                base[v] = p.h_views[v].tile_base;
            }
            direct = bin_direct_plan(nv, s0.data(), s1.data(), ntx.data(), nty.data(), base.data(), p.h_dviews,
                                     &plan) &&
                     bin_direct_scratch_bytes(plan) <= p.dscratch_bytes;
        }
        if (direct) {
            (void)hipMemcpyAsync(p.d_dviews, p.h_dviews, sizeof(DView) * nv, hipMemcpyHostToDevice, st);
            DTab dt;
            std::memset(&dt, 0, sizeof dt);
            dt.dev = p.d_dviews;
            dt.n = nv;
            launch_bin_direct_place(plan, dt, p.rect, p.depth, cap, nullptr, p.ranges, p.pair_count, p.status,
                                    p.dscratch, p.alt_k, st);
            launch_bin_direct_sort(tile, cap, p.keys, p.vals, p.ranges, p.status, p.torder, p.alt_k, st);
        } else {
            const int tb = tile_bits(std::max<uint32_t>(tile, 1));
            const bool to_alt = bin_sort_emit_to_alt(tb);
            const ZeroList z = bin_sort_zero_list(p.sort_ws, cap, tb, p.ranges, tile);
            launch_emit_pairs(slot, p.tt, p.rect, p.depth, jt, vt, cap, to_alt ? p.alt_k : p.keys,
                              to_alt ? p.alt_v : p.vals, nullptr, p.pair_count, p.status, p.scan_ws, st, &z);
            launch_bin_sort(p.keys, p.vals, p.alt_k, p.alt_v, p.pair_count, cap, tb, p.ranges, tile, p.sort_ws, st,
                            true, p.torder);
        }
        RenderArgs r;
        std::memset(&r, 0, sizeof r);
        r.rec = p.rec;
        r.vals = p.vals;
        r.ranges = p.ranges;
        r.status = p.status;
        r.views = vt;
        r.n_tiles = tile;
        r.tw = tw;
        r.th = th;
        r.tile_order = p.torder + 1;   // longest lists first
        r.tile_order_count = p.torder;
        launch_render_fwd(r, nullptr, p.final_T, p.n_contrib, nullptr, nullptr, st);
        (void)hipMemcpyAsync(p.h_status, p.status, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        (void)hipMemcpyAsync(p.h_status + 1, p.pair_count, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
        p.slots_used = slot;
        if (hipEventRecord(p.ev, st) != hipSuccess) fatal = 1;
        if (hipGetLastError() != hipSuccess) fatal = 1;
    }

    void completer_loop() {
        for (;;) {
            std::unique_lock<std::mutex> lk(mu);
            cv_inflight.wait(lk, [&] { return !inflight.empty() || worker_done; });
            if (inflight.empty()) break;
            const int pi = inflight.front();
            inflight.pop_front();
            Pipe& p = pipes[pi];
            lk.unlock();
            const bool ok = hipEventSynchronize(p.ev) == hipSuccess;
            const int64_t t1 = now_ns();
            lk.lock();
            const int32_t st = ok ? p.h_status[0] : GS_ERR_HIP;
            const uint32_t needed = (uint32_t)p.h_status[2];
            if (st == GS_ERR_CAPACITY && p.tickets.size() > 1) {
                // pairs overflowed: raise the estimate, retry at the head of the queue
                const double ratio = (double)needed / (double)std::max<int64_t>(p.slots_used, 1);
                pairs_per_slot = std::max(pairs_per_slot, 1.25 * ratio);
                for (auto it = p.tickets.rbegin(); it != p.tickets.rend(); ++it) queue.push_front(*it);
                ++requeues;
            } else {
                if (st == GS_OK && p.slots_used > 0) {
                    const double ratio = (double)needed / (double)p.slots_used;
                    pairs_per_slot = std::max(0.9 * pairs_per_slot + 0.1 * 1.25 * ratio, 1.25 * ratio);
                }
                for (uint64_t t : p.tickets) {
                    Req& r = reqs[t];
                    r.status = st;
                    r.t_done = t1;
                    r.done = true;
                }
            }
            p.tickets.clear();
            p.busy = false;
            cv_work.notify_all();
            cv_done.notify_all();
        }
    }

    bool all_idle() const {
        for (const Pipe& p : pipes)
            if (p.busy) return false;
        return true;
    }

    ~gs_server() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
        cv_inflight.notify_all();
        if (worker.joinable()) worker.join();
        {
            std::lock_guard<std::mutex> lk(mu);
            cv_inflight.notify_all();
        }
        if (completer.joinable()) completer.join();
        for (Pipe& p : pipes) {
            if (p.st) (void)hipStreamSynchronize(p.st);
            void* ptrs[] = {p.rec, p.depth, p.rect, p.tt, p.scan_ws, p.keys, p.alt_k, p.vals, p.alt_v, p.sort_ws,
                            p.ranges, p.torder, p.pair_count, p.status, p.final_T, p.n_contrib, p.d_views, p.d_jobs,
                            p.d_dviews, p.dscratch};
            for (void* q : ptrs)
                if (q) (void)hipFree(q);
            if (p.h_views) (void)hipHostFree(p.h_views);
            if (p.h_jobs) (void)hipHostFree(p.h_jobs);
            if (p.h_status) (void)hipHostFree(p.h_status);
            if (p.h_dviews) (void)hipHostFree(p.h_dviews);
            if (p.ev) (void)hipEventDestroy(p.ev);
            if (p.st) (void)hipStreamDestroy(p.st);
        }
    }
};

extern "C" {

gs_status gs_serve_create(const gs_gaussians* scene, const float* cell_aabbs, const int64_t* cell_offsets,
                          int32_t n_cells, const gs_serve_config* cfg, gs_server** out) {
    if (!out) return fail(GS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    Gauss G;
    gs_status s;
    if ((s = to_gauss(scene, &G))) return s;
    if (n_cells <= 0 || !cell_aabbs || !cell_offsets) return fail(GS_ERR_INVALID, "cells missing");
    if (cell_offsets[0] != 0 || cell_offsets[n_cells] != G.n) return fail(GS_ERR_INVALID, "cell offsets must span [0, n]");
    for (int c = 0; c < n_cells; ++c)
        if (cell_offsets[c + 1] < cell_offsets[c]) return fail(GS_ERR_INVALID, "cell offsets not ascending");
    gs_serve_config d;
    std::memset(&d, 0, sizeof d);
    d.memory_budget = (int64_t)8 << 30;
    d.pipelines = 2;
    d.max_views = 8;
    d.max_queue = 1024;
    d.tile_w = d.tile_h = 16;
    d.max_pixels = (int64_t)4 * 3840 * 2160;
    d.widen_px = 64.f;
    d.initial_pairs_per_slot = 3.0;
    const gs_serve_config c = cfg ? *cfg : d;
    const int pipes = c.pipelines > 0 ? c.pipelines : d.pipelines;
    const int tw = c.tile_w ? c.tile_w : 16, th = c.tile_h ? c.tile_h : 16;
    if (!render_tile_supported(tw, th)) return fail(GS_ERR_UNSUPPORTED, "tile %dx%d not supported", tw, th);
    if (c.memory_budget <= 0 || c.max_views <= 0 || c.max_pixels <= 0) return fail(GS_ERR_INVALID, "bad config");

    gs_server* sv = new gs_server();
    sv->scene = G;
    sv->n_cells = n_cells;
    sv->tw = tw;
    sv->th = th;
    sv->max_queue = c.max_queue > 0 ? c.max_queue : 1024;
    sv->widen_px = c.widen_px > 0 ? c.widen_px : 64.f;
    sv->pairs_per_slot = c.initial_pairs_per_slot > 0 ? c.initial_pairs_per_slot : 3.0;
    sv->paused = c.start_paused != 0;
    sv->cell_off.assign(cell_offsets, cell_offsets + n_cells + 1);
    sv->boxes.assign(cell_aabbs, cell_aabbs + 6 * (size_t)n_cells);

    // capacities per pipeline from the budget: bytes per slot, pair, pixel, tile
    const double per_slot = sizeof(Rec) + 4 + 8 + 4 + 8.0 / 256;
    const double per_pair = 2 * (8 + 4) + 16.0;   // keys/vals + alternates + sort look-back share
    const double per_pix = 8;
    const int64_t share = c.memory_budget / pipes;
    const int64_t pix_cap = std::min<int64_t>(c.max_pixels, (int64_t)(0.15 * share / per_pix));
    const int64_t slots_cap = (int64_t)(0.40 * share / per_slot);
    const int64_t pairs_cap =
        c.max_pairs > 0 ? std::min<int64_t>(kMaxPairs, c.max_pairs)
                        : std::min<int64_t>(kMaxPairs, (int64_t)(0.45 * share / per_pair));
    const uint32_t tiles_cap = (uint32_t)std::min<int64_t>(pix_cap / (tw * th) + 64 * c.max_views, 1 << 24);
    bool ok = true;
    sv->pipes.resize(pipes);
    for (Pipe& p : sv->pipes) {
        p.slots_cap = slots_cap / kSlotAlign * kSlotAlign;
        p.pairs_cap = pairs_cap;
        p.pix_cap = pix_cap;
        p.tiles_cap = tiles_cap;
        p.views_cap = c.max_views;
        p.jobs_cap = c.max_views * n_cells;
        ok = ok && hipStreamCreateWithFlags(&p.st, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&p.ev, hipEventDisableTiming) == hipSuccess && dalloc(&p.rec, p.slots_cap) &&
             dalloc(&p.depth, p.slots_cap) && dalloc(&p.rect, p.slots_cap) && dalloc(&p.tt, p.slots_cap) &&
             dalloc(reinterpret_cast<char**>(&p.scan_ws), scan_workspace_bytes(p.slots_cap)) &&
             dalloc(&p.keys, p.pairs_cap) && dalloc(&p.alt_k, p.pairs_cap) && dalloc(&p.vals, p.pairs_cap) &&
             dalloc(&p.alt_v, p.pairs_cap) &&
             dalloc(reinterpret_cast<char**>(&p.sort_ws), sort_workspace_bytes(p.pairs_cap, 64)) &&
             dalloc(&p.ranges, (size_t)p.tiles_cap * 2) && dalloc(&p.torder, (size_t)p.tiles_cap + 1) && dalloc(&p.pair_count, 2) && dalloc(&p.status, 1) &&
             dalloc(&p.final_T, p.pix_cap) && dalloc(&p.n_contrib, p.pix_cap) && dalloc(&p.d_views, p.views_cap) &&
             dalloc(&p.d_jobs, p.jobs_cap) &&
             hipHostMalloc(reinterpret_cast<void**>(&p.h_views), sizeof(View) * p.views_cap, 0) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&p.h_jobs), sizeof(Job) * p.jobs_cap, 0) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&p.h_status), 4 * sizeof(int32_t), 0) == hipSuccess;
        // direct binning: at most 256 count-matrix rows per view, each of
        // the view's tiles, so the matrix holds at most 256 x tiles_cap words
        if (ok) {
            p.dscratch_bytes = ((size_t)256 * p.tiles_cap * 4 + 255) / 256 * 256 +
                               ((size_t)p.tiles_cap * 4 + 255) / 256 * 256 +
                               ((size_t)(256 * p.views_cap + 1) * 8 + 255) / 256 * 256;
            ok = dalloc(&p.d_dviews, p.views_cap) &&
                 dalloc(reinterpret_cast<char**>(&p.dscratch), p.dscratch_bytes) &&
                 hipHostMalloc(reinterpret_cast<void**>(&p.h_dviews), sizeof(DView) * p.views_cap, 0) == hipSuccess;
        }
        if (!ok) break;
    }
    if (!ok) {
        (void)hipGetLastError();
        delete sv;
        return fail(GS_ERR_OOM, "server workspace allocation failed");
    }
    sv->worker = std::thread([sv] { sv->worker_loop(); });
    sv->completer = std::thread([sv] { sv->completer_loop(); });
    *out = sv;
    return GS_OK;
}

gs_status gs_serve_submit(gs_server* sv, const gs_camera* cam, float* out_image, uint64_t* ticket) {
    if (!sv || !cam || !out_image || !ticket) return fail(GS_ERR_INVALID, "NULL argument");
    Req r;
    gs_status s;
    if ((s = to_cam(cam, &r.cam))) return s;
    r.out = out_image;
    r.pix = (int64_t)r.cam.W * r.cam.H;
    r.tiles = (uint32_t)(((r.cam.W + sv->tw - 1) / sv->tw) * ((r.cam.H + sv->th - 1) / sv->th));
    for (int c = 0; c < sv->n_cells; ++c)
        if (sv->cell_off[c + 1] > sv->cell_off[c] && box_visible(r.cam, &sv->boxes[6 * c], sv->widen_px)) {
            r.cells.push_back(c);
            r.slots += sv->cell_off[c + 1] - sv->cell_off[c];
        }
    if (!sv->fits_alone(r, sv->pipes[0]))
        return fail(GS_ERR_INVALID, "request exceeds the server's memory budget (%lld slots, %lld pixels)",
                    (long long)r.slots, (long long)r.pix);
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return fail(GS_ERR_INVALID, "server is stopping");
    if ((int)sv->queue.size() >= sv->max_queue) return fail(GS_ERR_BUSY, "queue full (%d requests)", sv->max_queue);
    r.ticket = sv->next_ticket++;
    r.t_arrive = now_ns();
    *ticket = r.ticket;
    sv->queue.push_back(r.ticket);
    sv->reqs.emplace(r.ticket, std::move(r));
    sv->cv_work.notify_one();
    return GS_OK;
}

gs_status gs_serve_wait(gs_server* sv, uint64_t ticket, int32_t timeout_ms, gs_request_stats* st) {
    if (!sv) return fail(GS_ERR_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return fail(GS_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    auto pred = [&] { return sv->reqs[ticket].done; };
    if (timeout_ms < 0) sv->cv_done.wait(lk, pred);
    else if (!sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
        return fail(GS_ERR_TIMEOUT, "ticket %llu not done", (unsigned long long)ticket);
    Req& r = sv->reqs[ticket];
    if (st) {
        st->t_arrive_ns = r.t_arrive;
        st->t_start_ns = r.t_start;
        st->t_done_ns = r.t_done;
        st->status = r.status;
        st->batch_views = r.batch_views;
        st->attempts = r.attempts;
        st->cells = (int32_t)r.cells.size();
        st->gaussians = r.slots;
    }
    const int32_t status = r.status;
    sv->reqs.erase(ticket);
    if (status != GS_OK) return fail((gs_status)status, "request failed");
    return GS_OK;
}

gs_status gs_serve_info(gs_server* sv, gs_serve_stats* info) {
    if (!sv || !info) return fail(GS_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    std::memset(info, 0, sizeof *info);
    info->batches = sv->batches;
    info->requeues = sv->requeues;
    info->max_batch_views = sv->max_batch_views;
    info->queued = (int64_t)sv->queue.size();
    info->pipelines = (int32_t)sv->pipes.size();
    info->slots_cap = sv->pipes[0].slots_cap;
    info->pairs_cap = sv->pipes[0].pairs_cap;
    info->pixels_cap = sv->pipes[0].pix_cap;
    info->pairs_per_slot = sv->pairs_per_slot;
    return GS_OK;
}

gs_status gs_serve_resume(gs_server* sv) {
    if (!sv) return fail(GS_ERR_INVALID, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->paused = false;
    }
    sv->cv_work.notify_all();
    return GS_OK;
}

void gs_serve_destroy(gs_server* sv) { delete sv; }

}  // extern "C"
