// Progressive data partitioning of a scene into cells (gs_partition_views),
// host side.
//
// VastGaussian (arXiv 2402.17427), section 4.1: the camera centres are
// projected on the ground plane (world y is up, the ground coordinates are
// x and z) and split into m sections along x with equal view counts, each
// section into n segments along z with equal view counts; each region's
// rectangle, expanded by a ratio (20 %) of its sides, selects the views and
// points whose ground position lies in it; then every other camera whose
// airspace-aware visibility of the cell exceeds a threshold (25 %) joins
// the cell.  The visibility is the fraction of the image covered by the
// projection of the cell's airspace box: the axis-aligned box of the
// cell's points, from the ground up to their highest point.
//
// Conventions where the paper leaves a choice (the same in the test
// oracle): group sizes differ by at most one, the first groups taking the
// extra view; boundaries lie midway between neighbouring camera positions;
// the outermost boundaries are the bounding rectangle of all camera
// positions and points; the expansion keeps each rectangle's centre; the
// box's part behind the near plane is clipped off before it is projected;
// the projected outline is the convex hull of the clipped box's vertices,
// cut to the image rectangle.  All arithmetic is FP64; the work is
// O(views x cells + points x cells), small next to the coverage test of
// the points (partition.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/gs.h"
#include "api_internal.h"
#include "kernels.h"
#include "profile.h"

namespace gs {

namespace {

struct V2 {
    double x, y;
};
struct V3 {
    double x, y, z;
};

struct PinCam {
    double R[9], t[3], fx, fy, cx, cy, W, H, near_z;
    V3 to_cam(const V3& p) const {
        return {R[0] * p.x + R[1] * p.y + R[2] * p.z + t[0], R[3] * p.x + R[4] * p.y + R[5] * p.z + t[1],
                R[6] * p.x + R[7] * p.y + R[8] * p.z + t[2]};
    }
    V3 centre() const {  // -R^T t
        return {-(R[0] * t[0] + R[3] * t[1] + R[6] * t[2]), -(R[1] * t[0] + R[4] * t[1] + R[7] * t[2]),
                -(R[2] * t[0] + R[5] * t[1] + R[8] * t[2])};
    }
};

PinCam pin(const gs_camera& c) {
    PinCam p;
    for (int k = 0; k < 9; ++k) p.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) p.t[k] = c.t[k];
    p.fx = c.fx;
    p.fy = c.fy;
    p.cx = c.cx;
    p.cy = c.cy;
    p.W = c.width;
    p.H = c.height;
    p.near_z = c.near_z;
    return p;
}

// sizes of `count` items split into `parts` groups, the first count % parts
// groups one larger
std::vector<int> group_sizes(int count, int parts) {
    std::vector<int> s(parts, count / parts);
    for (int k = 0; k < count % parts; ++k) ++s[k];
    return s;
}

// group edges over sorted values: lo, midpoints between groups, hi
std::vector<double> group_edges(const std::vector<double>& sorted, const std::vector<int>& sizes, double lo,
                                double hi) {
    std::vector<double> e{lo};
    int k = 0;
    for (size_t g = 0; g + 1 < sizes.size(); ++g) {
        k += sizes[g];
        if (k <= 0 || k >= (int)sorted.size()) e.push_back(e.back());
        else e.push_back(0.5 * (sorted[k - 1] + sorted[k]));
    }
    e.push_back(hi);
    return e;
}

double cross(const V2& o, const V2& a, const V2& b) { return (a.x - o.x) * (b.y - o.y) - (a.y - o.y) * (b.x - o.x); }

// convex hull, counter-clockwise (monotone chain)
std::vector<V2> hull(std::vector<V2> p) {
    std::sort(p.begin(), p.end(), [](const V2& a, const V2& b) { return a.x < b.x || (a.x == b.x && a.y < b.y); });
    p.erase(std::unique(p.begin(), p.end(), [](const V2& a, const V2& b) { return a.x == b.x && a.y == b.y; }),
            p.end());
    if (p.size() < 3) return p;
    std::vector<V2> h(2 * p.size());
    size_t k = 0;
    for (size_t i = 0; i < p.size(); ++i) {
        while (k >= 2 && cross(h[k - 2], h[k - 1], p[i]) <= 0) --k;
        h[k++] = p[i];
    }
    for (size_t i = p.size() - 1, t = k + 1; i-- > 0;) {
        while (k >= t && cross(h[k - 2], h[k - 1], p[i]) <= 0) --k;
        h[k++] = p[i];
    }
    h.resize(k - 1);
    return h;
}

// keep the part of a polygon on one side of x = v (axis 0) or y = v (axis 1)
std::vector<V2> clip(const std::vector<V2>& poly, int axis, double v, bool keep_greater) {
    std::vector<V2> out;
    const size_t n = poly.size();
    for (size_t k = 0; k < n; ++k) {
        const V2 &a = poly[k], &b = poly[(k + 1) % n];
        const double ca = axis ? a.y : a.x, cb = axis ? b.y : b.x;
        const bool ia = keep_greater ? ca >= v : ca <= v;
        const bool ib = keep_greater ? cb >= v : cb <= v;
        if (ia) out.push_back(a);
        if (ia != ib) {
            const double s = (v - ca) / (cb - ca);
            out.push_back({a.x + s * (b.x - a.x), a.y + s * (b.y - a.y)});
        }
    }
    return out;
}

double area(const std::vector<V2>& p) {
    if (p.size() < 3) return 0.0;
    double s = 0.0;
    for (size_t k = 0; k < p.size(); ++k) {
        const V2 &a = p[k], &b = p[(k + 1) % p.size()];
        s += a.x * b.y - b.x * a.y;
    }
    return std::fabs(s) * 0.5;
}

// fraction of the image covered by the box [lo, hi] beyond the near plane
double box_visibility(const PinCam& c, const double lo[3], const double hi[3]) {
    V3 cw[8];
    for (int k = 0; k < 8; ++k) {
        const V3 p{(k & 4) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 1) ? hi[2] : lo[2]};
        cw[k] = c.to_cam(p);
    }
    std::vector<V3> verts;
    for (int k = 0; k < 8; ++k)
        if (cw[k].z > c.near_z) verts.push_back(cw[k]);
    for (int a = 0; a < 8; ++a)
        for (int bit = 1; bit < 8; bit <<= 1) {
            const int b = a | bit;
            if (b == a) continue;  // each edge once: a has the bit clear
            const double za = cw[a].z - c.near_z, zb = cw[b].z - c.near_z;
            if ((za > 0) != (zb > 0)) {
                const double s = za / (za - zb);
                verts.push_back({cw[a].x + s * (cw[b].x - cw[a].x), cw[a].y + s * (cw[b].y - cw[a].y),
                                 cw[a].z + s * (cw[b].z - cw[a].z)});
            }
        }
    if (verts.size() < 3) return 0.0;
    std::vector<V2> uv;
    for (const V3& v : verts) uv.push_back({c.fx * v.x / v.z + c.cx, c.fy * v.y / v.z + c.cy});
    std::vector<V2> poly = hull(uv);
    const double lim[4] = {0.0, c.W, 0.0, c.H};
    for (int e = 0; e < 4; ++e) {
        if (poly.size() < 3) return 0.0;
        poly = clip(poly, e / 2, lim[e], e % 2 == 0);
    }
    return area(poly) / (c.W * c.H);
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" {

gs_status gs_partition_views(const gs_camera* cams, int32_t n_views, const float* points, int64_t n_points,
                             const gs_partition_config* cfg, double* bounds, double* expanded, double* boxes,
                             double* visibility, uint8_t* view_member) {
    if (!cams || !cfg || !bounds || !expanded || !boxes || !visibility || !view_member)
        return fail(GS_ERR_INVALID, "NULL argument");
    if (n_views < 1 || n_points < 0 || (n_points > 0 && !points)) return fail(GS_ERR_INVALID, "bad sizes");
    if (cfg->m < 1 || cfg->n < 1 || (int64_t)cfg->m * cfg->n > 65535) return fail(GS_ERR_INVALID, "bad grid");
    if (!(cfg->expand >= 0.f) || !std::isfinite(cfg->expand) || !std::isfinite(cfg->visibility_threshold))
        return fail(GS_ERR_INVALID, "bad expansion or threshold");
    std::vector<PinCam> pc;
    for (int i = 0; i < n_views; ++i) {
        Cam tmp;
        gs_status s;
        if ((s = to_cam(&cams[i], &tmp))) return s;
        pc.push_back(pin(cams[i]));
    }
    for (int64_t k = 0; k < 3 * n_points; ++k)
        if (!std::isfinite(points[k])) return fail(GS_ERR_INVALID, "point %lld not finite", (long long)(k / 3));
    const int m = cfg->m, n = cfg->n, ncell = m * n;
    // 1. region division on the camera centres' ground positions
    std::vector<V3> cen;
    double X0 = INFINITY, X1 = -INFINITY, Z0 = INFINITY, Z1 = -INFINITY;
    for (const PinCam& c : pc) {
        cen.push_back(c.centre());
        X0 = std::min(X0, cen.back().x);
        X1 = std::max(X1, cen.back().x);
        Z0 = std::min(Z0, cen.back().z);
        Z1 = std::max(Z1, cen.back().z);
    }
    for (int64_t k = 0; k < n_points; ++k) {
        X0 = std::min(X0, (double)points[3 * k]);
        X1 = std::max(X1, (double)points[3 * k]);
        Z0 = std::min(Z0, (double)points[3 * k + 2]);
        Z1 = std::max(Z1, (double)points[3 * k + 2]);
    }
    std::vector<int> order(n_views);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cen[a].x < cen[b].x; });
    std::vector<double> xs;
    for (int i : order) xs.push_back(cen[i].x);
    const std::vector<int> xsz = group_sizes(n_views, m);
    const std::vector<double> xe = group_edges(xs, xsz, X0, X1);
    int k0 = 0;
    for (int i = 0; i < m; ++i) {
        std::vector<double> zs;
        for (int k = k0; k < k0 + xsz[i]; ++k) zs.push_back(cen[order[k]].z);
        k0 += xsz[i];
        std::stable_sort(zs.begin(), zs.end());
        const std::vector<int> zsz = group_sizes((int)zs.size(), n);
        const std::vector<double> ze = group_edges(zs, zsz, Z0, Z1);
        for (int j = 0; j < n; ++j) {
            double* b = bounds + 4 * (i * n + j);
            b[0] = xe[i];
            b[1] = xe[i + 1];
            b[2] = ze[j];
            b[3] = ze[j + 1];
        }
    }
    // 2-3. expansion, position-based selection, airspace box, visibility:
    // cells are independent (each writes only its own rows), so they run on
    // host threads; the per-cell computation, and so the result, is the
    // same for any thread count
    const double r = cfg->expand;
    auto one_cell = [&](int c) {
        const double* b = bounds + 4 * c;
        double* e = expanded + 4 * c;
        const double hx = 0.5 * r * (b[1] - b[0]), hz = 0.5 * r * (b[3] - b[2]);
        e[0] = b[0] - hx;
        e[1] = b[1] + hx;
        e[2] = b[2] - hz;
        e[3] = b[3] + hz;
        uint8_t* vm = view_member + (int64_t)c * n_views;
        double* vis = visibility + (int64_t)c * n_views;
        for (int i = 0; i < n_views; ++i) {
            vm[i] = (cen[i].x >= e[0] && cen[i].x <= e[1] && cen[i].z >= e[2] && cen[i].z <= e[3]) ? 1 : 0;
            vis[i] = 0.0;
        }
        double lo[3] = {INFINITY, 0.0, INFINITY}, hi[3] = {-INFINITY, 0.0, -INFINITY};
        bool any = false;
        for (int64_t k = 0; k < n_points; ++k) {
            const double x = points[3 * k], y = points[3 * k + 1], z = points[3 * k + 2];
            if (x >= e[0] && x <= e[1] && z >= e[2] && z <= e[3]) {
                any = true;
                lo[0] = std::min(lo[0], x);
                hi[0] = std::max(hi[0], x);
                lo[2] = std::min(lo[2], z);
                hi[2] = std::max(hi[2], z);
                hi[1] = std::max(hi[1], y);
            }
        }
        double* bx = boxes + 6 * c;
        if (!any) {
            std::memset(bx, 0, 6 * sizeof(double));
            return;
        }
        bx[0] = lo[0];
        bx[1] = 0.0;
        bx[2] = lo[2];
        bx[3] = hi[0];
        bx[4] = hi[1];
        bx[5] = hi[2];
        for (int i = 0; i < n_views; ++i) {
            if (vm[i]) continue;
            vis[i] = box_visibility(pc[i], lo, hi);
            if (vis[i] > cfg->visibility_threshold) vm[i] = 2;
        }
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int workers = (int)std::min<unsigned>(hw, (unsigned)ncell);
    if (workers <= 1) {
        for (int c = 0; c < ncell; ++c) one_cell(c);
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < workers; ++t)
            pool.emplace_back([&, t] {
                for (int c = t; c < ncell; c += workers) one_cell(c);
            });
        for (std::thread& th : pool) th.join();
    }
    return GS_OK;
}

namespace {
size_t table_bytes(int32_t n_views, int32_t n_cells) {
    return align256((size_t)n_views * kCamDoubles * 8) + align256((size_t)n_cells * 4 * 8) +
           align256((size_t)(n_cells + 1) * 4) + align256((size_t)n_cells * n_views * 4);
}
}  // namespace

gs_status gs_select_points_workspace(int32_t n_views, int32_t n_cells, int64_t n_points, size_t* bytes) {
    if (!bytes || n_views < 1 || n_cells < 1 || n_cells > 65535 || n_points < 0 || n_points > 0xFFFFFFFFll)
        return fail(GS_ERR_INVALID, "bad arguments");
    *bytes = table_bytes(n_views, n_cells) + select_sort_bytes(n_points);
    return GS_OK;
}

gs_status gs_select_points(const float* points, int64_t n_points, int64_t ld, const gs_camera* cams,
                           int32_t n_views, const double* expanded, int32_t n_cells, const uint8_t* view_member,
                           uint8_t* point_member, uint64_t* tests, void* ws, size_t ws_bytes, gs_stream stream) {
    size_t need = 0;
    gs_status s;
    if ((s = gs_select_points_workspace(n_views, n_cells, n_points, &need))) return s;
    const size_t tbytes = table_bytes(n_views, n_cells);
    if (!cams || !expanded || !view_member) return fail(GS_ERR_INVALID, "NULL host table");
    if (n_points < 0 || ld < n_points) return fail(GS_ERR_INVALID, "bad sizes");
    if (n_points > 0 && (!points || !point_member)) return fail(GS_ERR_INVALID, "NULL device buffer");
    if (!ws || ws_bytes < need) return fail(GS_ERR_INVALID, "workspace too small: %zu < %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % 8) return fail(GS_ERR_INVALID, "workspace not 8-byte aligned");
    // host tables, laid out as in the workspace
    std::vector<char> host(tbytes, 0);
    double* tc = reinterpret_cast<double*>(host.data());
    for (int i = 0; i < n_views; ++i) {
        Cam tmp;
        if ((s = to_cam(&cams[i], &tmp))) return s;
        const PinCam p = pin(cams[i]);
        double* q = tc + (size_t)kCamDoubles * i;
        for (int k = 0; k < 9; ++k) q[k] = p.R[k];
        for (int k = 0; k < 3; ++k) q[9 + k] = p.t[k];
        q[12] = p.fx;
        q[13] = p.fy;
        q[14] = p.cx;
        q[15] = p.cy;
        q[16] = p.W;
        q[17] = p.H;
        q[18] = p.near_z;
        if (!(p.near_z > 0.0)) return fail(GS_ERR_INVALID, "camera %d: near_z must be > 0", i);
    }
    size_t off = align256((size_t)n_views * kCamDoubles * 8);
    double* cells = reinterpret_cast<double*>(host.data() + off);
    for (int c = 0; c < 4 * n_cells; ++c) {
        if (!std::isfinite(expanded[c])) return fail(GS_ERR_INVALID, "expanded rectangle not finite");
        cells[c] = expanded[c];
    }
    const size_t off_cells = off;
    off += align256((size_t)n_cells * 4 * 8);
    int* offsets = reinterpret_cast<int*>(host.data() + off);
    const size_t off_offsets = off;
    off += align256((size_t)(n_cells + 1) * 4);
    int* views = reinterpret_cast<int*>(host.data() + off);
    const size_t off_views = off;
    int nv = 0;
    for (int c = 0; c < n_cells; ++c) {
        offsets[c] = nv;
        for (int i = 0; i < n_views; ++i)
            if (view_member[(int64_t)c * n_views + i]) views[nv++] = i;
    }
    offsets[n_cells] = nv;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(ws, host.data(), tbytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return check_hip("gs_select_points: table upload");
    SelectArgs a;
    a.points = points;
    a.n = n_points;
    a.ld = ld;
    char* w = static_cast<char*>(ws);
    a.cams = reinterpret_cast<const double*>(w);
    a.cells = reinterpret_cast<const double*>(w + off_cells);
    a.offsets = reinterpret_cast<const int*>(w + off_offsets);
    a.views = reinterpret_cast<const int*>(w + off_views);
    a.n_cells = n_cells;
    a.member = point_member;
    a.tests = tests;
    a.order = nullptr;
    // Morton box: the union of the expanded rectangles
    double box[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int c = 0; c < n_cells; ++c) {
        box[0] = std::min(box[0], expanded[4 * c]);
        box[1] = std::max(box[1], expanded[4 * c + 1]);
        box[2] = std::min(box[2], expanded[4 * c + 2]);
        box[3] = std::max(box[3], expanded[4 * c + 3]);
    }
    {
        ProfScope ps("select_points", st);
        launch_select_points(a, box, w + tbytes, st);
    }
    return check_hip("gs_select_points");
}

gs_status gs_merge_keep(const float* mean, int64_t n, int64_t ld, const double* rect, int32_t closed_x,
                        int32_t closed_z, uint8_t* keep, gs_stream stream) {
    if (!rect || n < 0 || ld < n || (n > 0 && (!mean || !keep))) return fail(GS_ERR_INVALID, "bad arguments");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(rect[k])) return fail(GS_ERR_INVALID, "rectangle not finite");
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_merge_keep(mean, n, ld, rect, closed_x, closed_z, keep, st);
    return check_hip("gs_merge_keep");
}

}  // extern "C"
