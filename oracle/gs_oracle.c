/*
 * FP64 reference renderer for 3D Gaussian splatting -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header or constant table with
 * the GPU path.
 *
 * What it computes (VastGaussian, arXiv 2402.17427, section 3 "Preliminaries"):
 * a scene is a set of 3D Gaussians, each with a position, an anisotropic
 * covariance (scale and rotation), an opacity and spherical-harmonic colour
 * coefficients.  For a camera C the rendered image is R(G, C): every Gaussian
 * is projected to a 2D image-space Gaussian by EWA splatting (the local affine
 * approximation of the perspective map), and the 2D Gaussians are composited
 * front to back by volume-rendering alpha blending.  The tiles and the sort the
 * paper mentions are an acceleration of that blend; this file evaluates the
 * plain definition: every Gaussian at every pixel, in global depth order.
 * Section 3 also states that R is differentiable and G is optimised by
 * gradients, so the analytic gradient of the image w.r.t. every Gaussian
 * parameter is given as well.  The paper leaves the image-formation constants
 * to the 3DGS method it builds on (section 5.1 keeps every setting it does not
 * list at its 3DGS value); the readings taken here are:
 *   * 2D dilation of 0.3 px^2 added to the projected covariance
 *   * affine-approximation clamp of |x/z| to 1.3 * (W/2)/fx (same for y)
 *   * alpha = min(0.99, o * exp(power)); Gaussians with alpha < 1/255 skipped
 *   * blending stops before the Gaussian that would drop T below 1e-4
 *   * colour = max(0, SH(dir) + 0.5), dir from the camera centre to the mean
 *   * quaternion order (w, x, y, z); pixel centres at (px + 0.5, py + 0.5)
 *   * global per-Gaussian depth = camera-space z of the centre; ties broken
 *     by the float32 bit pattern of that depth and then by Gaussian index
 * The binning functions at the end re-derive, from this file's own FP64
 * projection, the per-tile sorted lists and ranges a tiled renderer must
 * produce when each Gaussian's tile rectangle is the bounding box of the
 * pixels where its alpha can reach 1/255.
 *
 * Everything is double precision; the caller passes float32 inputs widened
 * to double so that finite differences can perturb them freely.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_DILATION 0.3
#define ORC_FOV_CLAMP 1.3
#define ORC_ALPHA_MAX 0.99
#define ORC_ALPHA_MIN (1.0 / 255.0)
#define ORC_T_MIN 1e-4

/* camera as 22 doubles: R[9] (world->camera, row-major), t[3], fx, fy, cx,
 * cy, width, height, near, bg[3] */
typedef struct {
    double R[9], t[3], fx, fy, cx, cy;
    int W, H;
    double near_z, bg[3];
} cam_t;

static cam_t read_cam(const double *c) {
    cam_t k;
    for (int i = 0; i < 9; ++i) k.R[i] = c[i];
    for (int i = 0; i < 3; ++i) k.t[i] = c[9 + i];
    k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
    k.W = (int)c[16]; k.H = (int)c[17];
    k.near_z = c[18];
    for (int i = 0; i < 3; ++i) k.bg[i] = c[19 + i];
    return k;
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics up to degree 3 (section 3: SH coefficients for  */
/* view-dependent colour).  Index j = l*l + l + m.  Constants are written    */
/* from their closed forms; the sign pattern is the one 3DGS scenes use.    */

int orc_sh_basis(const double *d, double *Y) {
    const double x = d[0], y = d[1], z = d[2];
    const double pi = M_PI;
    const double c0 = 0.5 * sqrt(1.0 / pi);
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi);
    const double c2b = 0.25 * sqrt(5.0 / pi);
    const double c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi));
    const double c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi));
    const double c3d = 0.25 * sqrt(7.0 / pi);
    const double c3e = 0.25 * sqrt(105.0 / pi);
    Y[0] = c0;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0 * z * z - x * x - y * y);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (x * x - y * y);
    Y[9] = -c3a * y * (3.0 * x * x - y * y);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0 * z * z - x * x - y * y);
    Y[12] = c3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    Y[13] = -c3c * x * (4.0 * z * z - x * x - y * y);
    Y[14] = c3e * z * (x * x - y * y);
    Y[15] = -c3a * x * (x * x - 3.0 * y * y);
    return 16;
}

/* dY[j][k] = dY_j / d d_k (derivative w.r.t. the un-normalised polynomial
 * arguments x, y, z). */
int orc_sh_basis_grad(const double *d, double *dY) {
    const double x = d[0], y = d[1], z = d[2];
    const double pi = M_PI;
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi);
    const double c2b = 0.25 * sqrt(5.0 / pi);
    const double c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi));
    const double c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi));
    const double c3d = 0.25 * sqrt(7.0 / pi);
    const double c3e = 0.25 * sqrt(105.0 / pi);
    memset(dY, 0, sizeof(double) * 48);
#define G(j, a, b, c) do { dY[3 * (j)] = (a); dY[3 * (j) + 1] = (b); dY[3 * (j) + 2] = (c); } while (0)
    G(1, 0, -c1, 0);
    G(2, 0, 0, c1);
    G(3, -c1, 0, 0);
    G(4, c2a * y, c2a * x, 0);
    G(5, 0, -c2a * z, -c2a * y);
    G(6, -2.0 * c2b * x, -2.0 * c2b * y, 4.0 * c2b * z);
    G(7, -c2a * z, 0, -c2a * x);
    G(8, 2.0 * c2c * x, -2.0 * c2c * y, 0);
    G(9, -c3a * 6.0 * x * y, -c3a * (3.0 * x * x - 3.0 * y * y), 0);
    G(10, c3b * y * z, c3b * x * z, c3b * x * y);
    G(11, c3c * 2.0 * x * y, -c3c * (4.0 * z * z - x * x - 3.0 * y * y), -c3c * 8.0 * y * z);
    G(12, -c3d * 6.0 * x * z, -c3d * 6.0 * y * z, c3d * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y));
    G(13, -c3c * (4.0 * z * z - 3.0 * x * x - y * y), c3c * 2.0 * x * y, -c3c * 8.0 * x * z);
    G(14, c3e * 2.0 * x * z, -c3e * 2.0 * y * z, c3e * (x * x - y * y));
    G(15, -c3a * (3.0 * x * x - 3.0 * y * y), c3a * 6.0 * x * y, 0);
#undef G
    return 48;
}

/* ------------------------------------------------------------------------ */
/* Projection (section 3: each 3D Gaussian is projected to the image as a   */
/* 2D Gaussian; EWA splatting).                                             */

typedef struct {
    int valid;
    double t[3];            /* camera-space centre */
    double u, v;            /* pixel-space centre */
    double a, b, c;         /* 2D covariance incl. dilation: [[a, b], [b, c]] */
    double A, B, C;         /* conic = inverse of the 2D covariance */
    double rgb[3], raw[3];  /* clamped and un-clamped colour */
    double o;
    double ex, ey;          /* half-extents of the alpha >= 1/255 ellipse */
    double lnthr;           /* power below which alpha < 1/255: -ln(255 o) */
    int px0, py0, px1, py1; /* inclusive pixel bounds, clamped to the image */
} proj_t;

static void quat_to_rot(const double *q, double *Rq) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z);     Rq[2] = 2 * (x * z + w * y);
    Rq[3] = 2 * (x * y + w * z);     Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
    Rq[6] = 2 * (x * z - w * y);     Rq[7] = 2 * (y * z + w * x);     Rq[8] = 1 - 2 * (x * x + y * y);
}

typedef struct {
    int64_t n, ld;
    int deg, K;
    const double *mean, *scale, *quat, *opac, *sh;
} gauss_t;

static double P(const double *plane, int64_t ld, int k, int64_t i) { return plane[(int64_t)k * ld + i]; }

static void camera_centre(const cam_t *k, double *cc) {
    for (int r = 0; r < 3; ++r)
        cc[r] = -(k->R[r] * k->t[0] + k->R[3 + r] * k->t[1] + k->R[6 + r] * k->t[2]);
}

static void project_one(const gauss_t *g, const cam_t *k, int64_t i, proj_t *p) {
    memset(p, 0, sizeof(*p));
    double mu[3], s[3], q[4];
    int finite = 1;
    for (int r = 0; r < 3; ++r) { mu[r] = P(g->mean, g->ld, r, i); s[r] = P(g->scale, g->ld, r, i); }
    for (int r = 0; r < 4; ++r) q[r] = P(g->quat, g->ld, r, i);
    double o = g->opac[i];
    for (int r = 0; r < 3; ++r) finite &= isfinite(mu[r]) && isfinite(s[r]);
    for (int r = 0; r < 4; ++r) finite &= isfinite(q[r]);
    finite &= isfinite(o);
    for (int j = 0; j < 3 * g->K; ++j) finite &= isfinite(P(g->sh, g->ld, j, i));
    if (!finite) return;
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(qn > 0)) return;

    /* view transform */
    for (int r = 0; r < 3; ++r)
        p->t[r] = k->R[3 * r] * mu[0] + k->R[3 * r + 1] * mu[1] + k->R[3 * r + 2] * mu[2] + k->t[r];
    const double tx = p->t[0], ty = p->t[1], tz = p->t[2];
    if (!(tz > k->near_z)) return;

    /* 3D covariance Sigma = M M^T with M = R(q) diag(s) */
    double qh[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
    double Rq[9], M[9], S[9];
    quat_to_rot(qh, Rq);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * s[c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            S[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];

    /* Jacobian of the perspective map at the (clamped) centre */
    const double limx = ORC_FOV_CLAMP * (0.5 * k->W) / k->fx;
    const double limy = ORC_FOV_CLAMP * (0.5 * k->H) / k->fy;
    double xr = tx / tz, yr = ty / tz;
    xr = xr < -limx ? -limx : (xr > limx ? limx : xr);
    yr = yr < -limy ? -limy : (yr > limy ? limy : yr);
    const double J[6] = {k->fx / tz, 0.0, -k->fx * xr / tz, 0.0, k->fy / tz, -k->fy * yr / tz};
    double T[6]; /* T = J W (2x3), W = camera rotation */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            T[3 * r + c] = J[3 * r] * k->R[c] + J[3 * r + 1] * k->R[3 + c] + J[3 * r + 2] * k->R[6 + c];
    double TS[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            TS[3 * r + c] = T[3 * r] * S[c] + T[3 * r + 1] * S[3 + c] + T[3 * r + 2] * S[6 + c];
    p->a = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2] + ORC_DILATION;
    p->b = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
    p->c = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5] + ORC_DILATION;
    const double det = p->a * p->c - p->b * p->b;
    if (!(det > 0)) return;
    p->A = p->c / det;
    p->B = -p->b / det;
    p->C = p->a / det;
    p->u = k->fx * tx / tz + k->cx;
    p->v = k->fy * ty / tz + k->cy;

    /* colour */
    double cc[3], d[3], Y[16];
    camera_centre(k, cc);
    for (int r = 0; r < 3; ++r) d[r] = mu[r] - cc[r];
    const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int r = 0; r < 3; ++r) d[r] /= dn;
    orc_sh_basis(d, Y);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int j = 0; j < g->K; ++j) acc += P(g->sh, g->ld, ch * g->K + j, i) * Y[j];
        p->raw[ch] = acc + 0.5;
        p->rgb[ch] = p->raw[ch] > 0.0 ? p->raw[ch] : 0.0;
    }
    p->o = o;

    /* support: pixels whose centre can see alpha >= 1/255 */
    if (!(o >= ORC_ALPHA_MIN)) return;
    const double r2 = 2.0 * log(255.0 * o);
    p->lnthr = -0.5 * r2;
    p->ex = sqrt(r2 * p->a);
    p->ey = sqrt(r2 * p->c);
    double x0 = ceil(p->u - p->ex - 0.5), x1 = floor(p->u + p->ex - 0.5);
    double y0 = ceil(p->v - p->ey - 0.5), y1 = floor(p->v + p->ey - 0.5);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > k->W - 1) x1 = k->W - 1;
    if (y1 > k->H - 1) y1 = k->H - 1;
    if (x0 > x1 || y0 > y1) return;
    p->px0 = (int)x0; p->px1 = (int)x1; p->py0 = (int)y0; p->py1 = (int)y1;
    p->valid = 1;
}

static gauss_t make_gauss(int64_t n, int64_t ld, int deg, const double *mean, const double *scale,
                          const double *quat, const double *opac, const double *sh) {
    gauss_t g = {n, ld, deg, (deg + 1) * (deg + 1), mean, scale, quat, opac, sh};
    return g;
}

/* Projection of every Gaussian.  Outputs (each may be NULL):
 *   valid[n] (int32), uv[n][2], conic[n][3] (A,B,C), cov[n][3] (a,b,c),
 *   rgb[n][3], depth[n] (camera z), ext[n][2], pxrect[n][4] (x0,y0,x1,y1). */
int orc_project(int64_t n, int64_t ld, int deg, const double *mean, const double *scale,
                const double *quat, const double *opac, const double *sh, const double *camv,
                int32_t *valid, double *uv, double *conic, double *cov, double *rgb, double *depth,
                double *ext, int32_t *pxrect) {
    if (deg < 0 || deg > 3 || n < 0 || ld < n) return -1;
    const cam_t k = read_cam(camv);
    const gauss_t g = make_gauss(n, ld, deg, mean, scale, quat, opac, sh);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        proj_t p;
        project_one(&g, &k, i, &p);
        if (valid) valid[i] = p.valid;
        if (uv) { uv[2 * i] = p.u; uv[2 * i + 1] = p.v; }
        if (conic) { conic[3 * i] = p.A; conic[3 * i + 1] = p.B; conic[3 * i + 2] = p.C; }
        if (cov) { cov[3 * i] = p.a; cov[3 * i + 1] = p.b; cov[3 * i + 2] = p.c; }
        if (rgb) for (int c = 0; c < 3; ++c) rgb[3 * i + c] = p.rgb[c];
        if (depth) depth[i] = p.t[2];
        if (ext) { ext[2 * i] = p.ex; ext[2 * i + 1] = p.ey; }
        if (pxrect) { pxrect[4 * i] = p.px0; pxrect[4 * i + 1] = p.py0; pxrect[4 * i + 2] = p.px1; pxrect[4 * i + 3] = p.py1; }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Depth order: ascending float32 bit pattern of the camera-space depth,    */
/* ties by Gaussian index.                                                  */

typedef struct { uint32_t zbits; int64_t idx; } zkey_t;

static uint32_t f32_bits(double z) {
    float f = (float)z;
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

static int cmp_zkey(const void *a, const void *b) {
    const zkey_t *x = (const zkey_t *)a, *y = (const zkey_t *)b;
    if (x->zbits != y->zbits) return x->zbits < y->zbits ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

/* ------------------------------------------------------------------------ */
/* Blend (section 3: alpha blending, point-based volume rendering).         */

typedef struct {
    double eps_alpha, eps_T, eps_power;
} flagcfg_t;

typedef struct {
    int64_t gid;
    double alpha, T, G, dx, dy;
    int capped;
} contrib_t;

/* Composite one pixel front to back.  Returns the number of blended
 * Gaussians; fills `list` (capacity cap, may be NULL) with them in order.
 * flags: bit0 = a discontinuous image decision lies near its threshold,
 *        bit1 = an alpha lies near the 0.99 cap (only the gradient changes). */
static int64_t blend_pixel(const proj_t *pr, const int64_t *order, int64_t nv, double x, double y,
                           const flagcfg_t *fc, double *T_out, double *C_out, int64_t *last_out,
                           int *flags, contrib_t *list, int64_t cap) {
    double T = 1.0, C[3] = {0, 0, 0};
    int64_t last = -1, nb = 0;
    int fl = 0;
    for (int64_t k = 0; k < nv; ++k) {
        const proj_t *p = &pr[order[k]];
        const double dx = x - p->u, dy = y - p->v;
        const double quad = 0.5 * (p->A * dx * dx + p->C * dy * dy);
        const double cross = p->B * dx * dy;
        const double power = -quad - cross;
        /* alpha < 1/255 certainly (far from the threshold): skip without exp */
        if (power < p->lnthr - 1e-3) continue;
        if (fabs(power) < fc->eps_power * (quad + fabs(cross))) fl |= 1;
        if (power > 0.0) continue;
        const double G = exp(power);
        const double araw = p->o * G;
        if (fabs(araw - ORC_ALPHA_MIN) <= fc->eps_alpha * ORC_ALPHA_MIN) fl |= 1;
        if (fabs(araw - ORC_ALPHA_MAX) <= fc->eps_alpha * ORC_ALPHA_MAX) fl |= 2;
        const int capped = araw > ORC_ALPHA_MAX;
        const double alpha = capped ? ORC_ALPHA_MAX : araw;
        if (alpha < ORC_ALPHA_MIN) continue;
        const double Tn = T * (1.0 - alpha);
        if (fabs(Tn - ORC_T_MIN) <= fc->eps_T * ORC_T_MIN) fl |= 1;
        if (Tn < ORC_T_MIN) break;
        for (int c = 0; c < 3; ++c) C[c] += p->rgb[c] * alpha * T;
        if (list && nb < cap) {
            contrib_t *e = &list[nb];
            e->gid = order[k]; e->alpha = alpha; e->T = T; e->G = G; e->dx = dx; e->dy = dy; e->capped = capped;
        }
        ++nb;
        T = Tn;
        last = order[k];
    }
    *T_out = T;
    for (int c = 0; c < 3; ++c) C_out[c] = C[c];
    *last_out = last;
    *flags = fl;
    return nb;
}

typedef struct {
    proj_t *pr;
    int64_t *order;
    int64_t nv;
} scene_t;

static int build_scene(const gauss_t *g, const cam_t *k, scene_t *sc) {
    sc->pr = (proj_t *)malloc(sizeof(proj_t) * (size_t)(g->n > 0 ? g->n : 1));
    zkey_t *zk = (zkey_t *)malloc(sizeof(zkey_t) * (size_t)(g->n > 0 ? g->n : 1));
    sc->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->n > 0 ? g->n : 1));
    if (!sc->pr || !zk || !sc->order) { free(sc->pr); free(zk); free(sc->order); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; ++i) project_one(g, k, i, &sc->pr[i]);
    int64_t nv = 0;
    for (int64_t i = 0; i < g->n; ++i)
        if (sc->pr[i].valid) { zk[nv].zbits = f32_bits(sc->pr[i].t[2]); zk[nv].idx = i; ++nv; }
    qsort(zk, (size_t)nv, sizeof(zkey_t), cmp_zkey);
    for (int64_t i = 0; i < nv; ++i) sc->order[i] = zk[i].idx;
    sc->nv = nv;
    free(zk);
    return 0;
}

static void free_scene(scene_t *sc) { free(sc->pr); free(sc->order); }

/* Forward render at a list of pixels (npix >= 0; pix = NULL means the full
 * frame in row-major order).  Outputs per listed pixel:
 *   img[npix][3], final_T[npix], last_id[npix] (Gaussian index of the last
 *   blended Gaussian, -1 if none), nblend[npix], flags[npix].
 * eps: {eps_alpha, eps_T, eps_power} relative windows for the flags. */
int orc_render(int64_t n, int64_t ld, int deg, const double *mean, const double *scale,
               const double *quat, const double *opac, const double *sh, const double *camv,
               int64_t npix, const int32_t *pix_x, const int32_t *pix_y, const double *eps,
               double *img, double *final_T, int64_t *last_id, int64_t *nblend, int32_t *flags) {
    if (deg < 0 || deg > 3 || n < 0 || ld < n) return -1;
    const cam_t k = read_cam(camv);
    const gauss_t g = make_gauss(n, ld, deg, mean, scale, quat, opac, sh);
    scene_t sc;
    if (build_scene(&g, &k, &sc)) return -2;
    const flagcfg_t fc = {eps[0], eps[1], eps[2]};
    const int64_t np = pix_x ? npix : (int64_t)k.W * k.H;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < np; ++q) {
        const int px = pix_x ? pix_x[q] : (int)(q % k.W);
        const int py = pix_x ? pix_y[q] : (int)(q / k.W);
        double T, C[3];
        int64_t last;
        int fl;
        int64_t nb = blend_pixel(sc.pr, sc.order, sc.nv, px + 0.5, py + 0.5, &fc, &T, C, &last, &fl, NULL, 0);
        for (int c = 0; c < 3; ++c) img[3 * q + c] = C[c] + T * k.bg[c];
        if (final_T) final_T[q] = T;
        if (last_id) last_id[q] = last;
        if (nblend) nblend[q] = nb;
        if (flags) flags[q] = fl;
    }
    free_scene(&sc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Backward: gradient of L = sum_p dL/dI_p . I_p w.r.t. the Gaussian        */
/* parameters (section 3: differentiable rasterizer, gradient-based          */
/* optimisation of G).                                                      */

/* 2D stage: per pixel, walk the blended list back to front with the suffix
 * colour S_i = sum_{j after i} rgb_j w_j + T_final bg.  Accumulates into
 * g2[n][9] = (du, dv, dA, dB, dC, do, dr, dg, db). */
static void backward_2d(const scene_t *sc, const cam_t *k, const double *dimg, int64_t npix,
                        const int32_t *pix_x, const int32_t *pix_y, const flagcfg_t *fc, int64_t n,
                        double *g2, int32_t *flags_out) {
    const int64_t np = pix_x ? npix : (int64_t)k->W * k->H;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nthr * (size_t)n * 9 + 1, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *my = acc + (size_t)tid * (size_t)n * 9;
        int64_t cap = 256;
        contrib_t *list = (contrib_t *)malloc(sizeof(contrib_t) * (size_t)cap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < np; ++q) {
            const int px = pix_x ? pix_x[q] : (int)(q % k->W);
            const int py = pix_x ? pix_y[q] : (int)(q / k->W);
            const int64_t off = (int64_t)py * k->W + px;
            const int64_t npx = (int64_t)k->W * k->H;
            const double gp[3] = {dimg[off], dimg[npx + off], dimg[2 * npx + off]};
            if (gp[0] == 0.0 && gp[1] == 0.0 && gp[2] == 0.0) { if (flags_out) flags_out[q] = 0; continue; }
            double T, C[3];
            int64_t last;
            int fl;
            int64_t nb = blend_pixel(sc->pr, sc->order, sc->nv, px + 0.5, py + 0.5, fc, &T, C, &last, &fl, list, cap);
            while (nb > cap) {
                cap = 2 * nb;
                list = (contrib_t *)realloc(list, sizeof(contrib_t) * (size_t)cap);
                nb = blend_pixel(sc->pr, sc->order, sc->nv, px + 0.5, py + 0.5, fc, &T, C, &last, &fl, list, cap);
            }
            if (flags_out) flags_out[q] = fl;
            double S[3] = {T * k->bg[0], T * k->bg[1], T * k->bg[2]};
            for (int64_t e = nb - 1; e >= 0; --e) {
                const contrib_t *c = &list[e];
                const proj_t *p = &sc->pr[c->gid];
                double *out = my + 9 * c->gid;
                const double w = c->alpha * c->T;
                double dalpha = 0.0;
                for (int ch = 0; ch < 3; ++ch) {
                    out[6 + ch] += gp[ch] * w;
                    dalpha += gp[ch] * (p->rgb[ch] * c->T - S[ch] / (1.0 - c->alpha));
                }
                for (int ch = 0; ch < 3; ++ch) S[ch] += p->rgb[ch] * w;
#ifdef ORC_PLANT_CAPPED_DOPACITY
                /* a planted slip for the tests: keep dL/do = dalpha G under
                 * the cap (the correct gradient is zero there) */
                if (c->capped) { out[5] += dalpha * c->G; continue; }
#endif
                /* alpha capped at 0.99 does not depend on o or power */
                if (c->capped) continue;
                out[5] += dalpha * c->G;
                const double dpow = dalpha * c->alpha;
                out[2] += -0.5 * c->dx * c->dx * dpow;
                out[3] += -c->dx * c->dy * dpow;
                out[4] += -0.5 * c->dy * c->dy * dpow;
                out[0] += (p->A * c->dx + p->B * c->dy) * dpow;
                out[1] += (p->B * c->dx + p->C * c->dy) * dpow;
            }
        }
        free(list);
    }
    for (int t = 0; t < nthr; ++t)
        for (int64_t j = 0; j < n * 9; ++j) g2[j] += acc[(size_t)t * (size_t)n * 9 + (size_t)j];
    free(acc);
}

/* 3D stage for one Gaussian: chain rule from the 2D gradients back to the
 * mean, scale, quaternion, opacity and SH coefficients. */
static void backward_3d_one(const gauss_t *g, const cam_t *k, int64_t i, const proj_t *p, const double *g2,
                            double *gmean, double *gscale, double *gquat, double *gopac, double *gsh,
                            int64_t gld) {
    double mu[3], s[3], q[4];
    for (int r = 0; r < 3; ++r) { mu[r] = P(g->mean, g->ld, r, i); s[r] = P(g->scale, g->ld, r, i); }
    for (int r = 0; r < 4; ++r) q[r] = P(g->quat, g->ld, r, i);
    const double du = g2[0], dv = g2[1], dA = g2[2], dB = g2[3], dC = g2[4], dop = g2[5];
    const double drgb[3] = {g2[6], g2[7], g2[8]};
    gopac[i] = dop;

    /* colour: rgb = max(0, sum_j k_j Y_j(dir) + 0.5) */
    double cc[3], d[3], Y[16], dY[48];
    camera_centre(k, cc);
    for (int r = 0; r < 3; ++r) d[r] = mu[r] - cc[r];
    const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double dh[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
    orc_sh_basis(dh, Y);
    orc_sh_basis_grad(dh, dY);
    double ddh[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
        const double gr = p->raw[ch] > 0.0 ? drgb[ch] : 0.0;
        for (int j = 0; j < g->K; ++j) {
            gsh[(int64_t)(ch * g->K + j) * gld + i] = gr * Y[j];
            const double kj = P(g->sh, g->ld, ch * g->K + j, i);
            for (int r = 0; r < 3; ++r) ddh[r] += gr * kj * dY[3 * j + r];
        }
    }
    /* dir = d / |d|: d(dir) -> d(d) = (I - dir dir^T) d(dir) / |d| */
    const double dd = dh[0] * ddh[0] + dh[1] * ddh[1] + dh[2] * ddh[2];
    double dmu[3];
    for (int r = 0; r < 3; ++r) dmu[r] = (ddh[r] - dh[r] * dd) / dn;

    /* conic (A, B, C) = (c, -b, a) / (a c - b^2) */
    const double a = p->a, b = p->b, c = p->c;
    const double det = a * c - b * b, det2 = det * det;
    const double da = dA * (-c * c / det2) + dB * (b * c / det2) + dC * (1.0 / det - a * c / det2);
    const double db = dA * (2.0 * b * c / det2) + dB * (-1.0 / det - 2.0 * b * b / det2) + dC * (2.0 * a * b / det2);
    const double dc = dA * (1.0 / det - a * c / det2) + dB * (a * b / det2) + dC * (-a * a / det2);
    /* note dA/dc etc. written from A = c/det: dA/da = -c^2/det^2,
     * dA/db = 2bc/det^2, dA/dc = 1/det - ac/det^2 (= -b^2/det^2). */

    /* recompute the forward intermediates */
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double qh[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
    double Rq[9], M[9], S[9];
    quat_to_rot(qh, Rq);
    for (int r = 0; r < 3; ++r)
        for (int cc2 = 0; cc2 < 3; ++cc2) M[3 * r + cc2] = Rq[3 * r + cc2] * s[cc2];
    for (int r = 0; r < 3; ++r)
        for (int cc2 = 0; cc2 < 3; ++cc2)
            S[3 * r + cc2] = M[3 * r] * M[3 * cc2] + M[3 * r + 1] * M[3 * cc2 + 1] + M[3 * r + 2] * M[3 * cc2 + 2];
    const double tx = p->t[0], ty = p->t[1], tz = p->t[2];
    const double limx = ORC_FOV_CLAMP * (0.5 * k->W) / k->fx;
    const double limy = ORC_FOV_CLAMP * (0.5 * k->H) / k->fy;
    const double xr0 = tx / tz, yr0 = ty / tz;
    const int clx = xr0 < -limx || xr0 > limx, cly = yr0 < -limy || yr0 > limy;
    const double xr = xr0 < -limx ? -limx : (xr0 > limx ? limx : xr0);
    const double yr = yr0 < -limy ? -limy : (yr0 > limy ? limy : yr0);
    const double J[6] = {k->fx / tz, 0.0, -k->fx * xr / tz, 0.0, k->fy / tz, -k->fy * yr / tz};
    double T[6];
    for (int r = 0; r < 2; ++r)
        for (int cc2 = 0; cc2 < 3; ++cc2)
            T[3 * r + cc2] = J[3 * r] * k->R[cc2] + J[3 * r + 1] * k->R[3 + cc2] + J[3 * r + 2] * k->R[6 + cc2];

    /* Sigma2 = T Sigma T^T (+ dilation).  G = dL/dSigma2 as a symmetric
     * matrix: the off-diagonal parameter b appears twice, so G01 = db / 2. */
    const double G2[4] = {da, 0.5 * db, 0.5 * db, dc};
    /* dL/dSigma = T^T G T (3x3) */
    double dS[9];
    for (int r = 0; r < 3; ++r)
        for (int cc2 = 0; cc2 < 3; ++cc2) {
            double acc = 0.0;
            for (int x = 0; x < 2; ++x)
                for (int y = 0; y < 2; ++y) acc += T[3 * x + r] * G2[2 * x + y] * T[3 * y + cc2];
            dS[3 * r + cc2] = acc;
        }
    /* dL/dT = 2 G T Sigma (2x3) */
    double dT[6];
    for (int r = 0; r < 2; ++r)
        for (int cc2 = 0; cc2 < 3; ++cc2) {
            double acc = 0.0;
            for (int x = 0; x < 2; ++x)
                for (int y = 0; y < 3; ++y) acc += G2[2 * r + x] * T[3 * x + y] * S[3 * y + cc2];
            dT[3 * r + cc2] = 2.0 * acc;
        }
    /* T = J W  =>  dJ = dT W^T */
    double dJ[6];
    for (int r = 0; r < 2; ++r)
        for (int cc2 = 0; cc2 < 3; ++cc2)
            dJ[3 * r + cc2] = dT[3 * r] * k->R[3 * cc2] + dT[3 * r + 1] * k->R[3 * cc2 + 1] + dT[3 * r + 2] * k->R[3 * cc2 + 2];
    /* J entries as functions of t:
     *   J00 = fx/tz, J11 = fy/tz
     *   J02 = -fx*tx/tz^2 (unclamped)  or  -fx*lim/tz (clamped, lim = +-limx)
     *   J12 likewise with y */
    double dt[3] = {0, 0, 0};
    const double tz2 = tz * tz, tz3 = tz2 * tz;
    dt[2] += -k->fx / tz2 * dJ[0] - k->fy / tz2 * dJ[4];
    if (!clx) { dt[0] += -k->fx / tz2 * dJ[2]; dt[2] += 2.0 * k->fx * tx / tz3 * dJ[2]; }
    else      { dt[2] += k->fx * xr / tz2 * dJ[2]; }
    if (!cly) { dt[1] += -k->fy / tz2 * dJ[5]; dt[2] += 2.0 * k->fy * ty / tz3 * dJ[5]; }
    else      { dt[2] += k->fy * yr / tz2 * dJ[5]; }
    /* centre u = fx tx/tz + cx, v = fy ty/tz + cy */
    dt[0] += k->fx / tz * du;
    dt[1] += k->fy / tz * dv;
    dt[2] += -k->fx * tx / tz2 * du - k->fy * ty / tz2 * dv;
    /* t = W mu + t_v */
    for (int r = 0; r < 3; ++r)
        dmu[r] += k->R[r] * dt[0] + k->R[3 + r] * dt[1] + k->R[6 + r] * dt[2];
    for (int r = 0; r < 3; ++r) gmean[(int64_t)r * gld + i] = dmu[r];

    /* Sigma = M M^T  =>  dM = (dS + dS^T) M = 2 dS M (dS symmetric) */
    double dM[9];
    for (int r = 0; r < 3; ++r)
        for (int cc2 = 0; cc2 < 3; ++cc2)
            dM[3 * r + cc2] = 2.0 * (dS[3 * r] * M[cc2] + dS[3 * r + 1] * M[3 + cc2] + dS[3 * r + 2] * M[6 + cc2]);
    /* M = Rq diag(s) */
    double dRq[9];
    for (int cc2 = 0; cc2 < 3; ++cc2) {
        double acc = 0.0;
        for (int r = 0; r < 3; ++r) { acc += dM[3 * r + cc2] * Rq[3 * r + cc2]; dRq[3 * r + cc2] = dM[3 * r + cc2] * s[cc2]; }
        gscale[(int64_t)cc2 * gld + i] = acc;
    }
    /* Rq(qh): derivative of each entry w.r.t. (w, x, y, z) */
    const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    double dqh[4];
    dqh[0] = 2 * (-z * dRq[1] + y * dRq[2] + z * dRq[3] - x * dRq[5] - y * dRq[6] + x * dRq[7]);
    dqh[1] = 2 * (y * dRq[1] + z * dRq[2] + y * dRq[3] - 2 * x * dRq[4] - w * dRq[5] + z * dRq[6] + w * dRq[7] - 2 * x * dRq[8]);
    dqh[2] = 2 * (-2 * y * dRq[0] + x * dRq[1] + w * dRq[2] + x * dRq[3] + z * dRq[5] - w * dRq[6] + z * dRq[7] - 2 * y * dRq[8]);
    dqh[3] = 2 * (-2 * z * dRq[0] - w * dRq[1] + x * dRq[2] + w * dRq[3] - 2 * z * dRq[4] + y * dRq[5] + x * dRq[6] + y * dRq[7]);
    /* qh = q / |q| */
    const double dot = qh[0] * dqh[0] + qh[1] * dqh[1] + qh[2] * dqh[2] + qh[3] * dqh[3];
    for (int r = 0; r < 4; ++r) gquat[(int64_t)r * gld + i] = (dqh[r] - qh[r] * dot) / qn;
}

/* Full backward.  dimg is dL/dI as [3][H][W].  If pix_x is given only the
 * listed pixels contribute (dimg is still indexed by pixel position).
 * Outputs gradients in the input layout with plane stride n:
 *   gmean[3][n], gscale[3][n], gquat[4][n], gopac[n], gsh[3K][n];
 * g2d[n][9] receives the 2D-stage gradients (may be NULL);
 * pflags[npix] the per-pixel flags (may be NULL);
 * touch[n] (may be NULL): 1 if the Gaussian's alpha reaches
 * (1/255)(1 - eps_alpha) at a flagged pixel (its gradient is ambiguous). */
int orc_backward(int64_t n, int64_t ld, int deg, const double *mean, const double *scale,
                 const double *quat, const double *opac, const double *sh, const double *camv,
                 const double *dimg, int64_t npix, const int32_t *pix_x, const int32_t *pix_y,
                 const double *eps, double *gmean, double *gscale, double *gquat, double *gopac,
                 double *gsh, double *g2d, int32_t *pflags, int32_t *touch) {
    if (deg < 0 || deg > 3 || n < 0 || ld < n) return -1;
    const cam_t k = read_cam(camv);
    const gauss_t g = make_gauss(n, ld, deg, mean, scale, quat, opac, sh);
    scene_t sc;
    if (build_scene(&g, &k, &sc)) return -2;
    const flagcfg_t fc = {eps[0], eps[1], eps[2]};
    const int64_t np = pix_x ? npix : (int64_t)k.W * k.H;
    double *g2 = (double *)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
    int32_t *fl = (int32_t *)calloc((size_t)(np > 0 ? np : 1), sizeof(int32_t));
    backward_2d(&sc, &k, dimg, npix, pix_x, pix_y, &fc, n, g2, fl);
    const int K = g.K;
    for (int64_t i = 0; i < n; ++i) {
        if (!sc.pr[i].valid) {
            for (int r = 0; r < 3; ++r) { gmean[r * n + i] = 0; gscale[r * n + i] = 0; }
            for (int r = 0; r < 4; ++r) gquat[r * n + i] = 0;
            gopac[i] = 0;
            for (int j = 0; j < 3 * K; ++j) gsh[(int64_t)j * n + i] = 0;
            continue;
        }
        backward_3d_one(&g, &k, i, &sc.pr[i], g2 + 9 * i, gmean, gscale, gquat, gopac, gsh, n);
    }
    if (g2d) memcpy(g2d, g2, sizeof(double) * (size_t)n * 9);
    if (pflags) memcpy(pflags, fl, sizeof(int32_t) * (size_t)np);
    if (touch) {
        memset(touch, 0, sizeof(int32_t) * (size_t)n);
        for (int64_t q = 0; q < np; ++q) {
            if (!fl[q]) continue;
            const int px = pix_x ? pix_x[q] : (int)(q % k.W);
            const int py = pix_x ? pix_y[q] : (int)(q / k.W);
            const double x = px + 0.5, y = py + 0.5;
            for (int64_t e = 0; e < sc.nv; ++e) {
                const proj_t *p = &sc.pr[sc.order[e]];
                const double dx = x - p->u, dy = y - p->v;
                const double power = -0.5 * (p->A * dx * dx + p->C * dy * dy) - p->B * dx * dy;
                if (p->o * exp(power) >= ORC_ALPHA_MIN * (1.0 - fc.eps_alpha)) touch[sc.order[e]] = 1;
            }
        }
    }
    free(g2);
    free(fl);
    free_scene(&sc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Binning (section 3: projected Gaussians are assigned to tiles and        */
/* sorted).  From this file's FP64 projection: every valid Gaussian emits   */
/* one (tile << 32 | float32 bits of depth, index) pair per tile its pixel  */
/* rectangle touches, tiles in row-major order; the pairs are ordered by    */
/* (key, Gaussian index) and each tile gets the [start, end) range of its   */
/* pairs (empty tiles get [0, 0)).                                          */

typedef struct { uint64_t key; uint32_t val; } pair_t;

static int cmp_pair(const void *a, const void *b) {
    const pair_t *x = (const pair_t *)a, *y = (const pair_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->val < y->val ? -1 : (x->val > y->val ? 1 : 0);
}

/* Pass keys/vals = NULL to query the pair count only.  tiles_touched[n],
 * trect[n][4] (tile x0, y0, x1, y1 exclusive) and zbits[n] may be NULL.
 * ranges[n_tiles][2].  amb[n] (may be NULL) flags Gaussians whose FP64
 * extent lies within `eps_px` pixels of a boundary that changes their
 * tile rectangle, or whose depth lies within a relative 1e-12 of a float32
 * rounding boundary. */
int64_t orc_bin(int64_t n, int64_t ld, int deg, const double *mean, const double *scale,
                const double *quat, const double *opac, const double *sh, const double *camv,
                int tile_w, int tile_h, double eps_px, uint64_t *keys, uint32_t *vals, int64_t cap,
                uint32_t *ranges, uint32_t *tiles_touched, int32_t *trect, uint32_t *zbits, int32_t *amb) {
    if (deg < 0 || deg > 3 || n < 0 || ld < n || tile_w <= 0 || tile_h <= 0) return -1;
    const cam_t k = read_cam(camv);
    const gauss_t g = make_gauss(n, ld, deg, mean, scale, quat, opac, sh);
    const int tx = (k.W + tile_w - 1) / tile_w, ty = (k.H + tile_h - 1) / tile_h;
    proj_t *pr = (proj_t *)malloc(sizeof(proj_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) project_one(&g, &k, i, &pr[i]);
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        const proj_t *p = &pr[i];
        int x0 = 0, y0 = 0, x1 = 0, y1 = 0;
        if (p->valid) { x0 = p->px0 / tile_w; x1 = p->px1 / tile_w + 1; y0 = p->py0 / tile_h; y1 = p->py1 / tile_h + 1; }
        const uint32_t cnt = (uint32_t)((x1 - x0) * (y1 - y0));
        if (tiles_touched) tiles_touched[i] = cnt;
        if (trect) { trect[4 * i] = x0; trect[4 * i + 1] = y0; trect[4 * i + 2] = x1; trect[4 * i + 3] = y1; }
        if (zbits) zbits[i] = p->valid ? f32_bits(p->t[2]) : 0u;
        if (amb) {
            int a = 0;
            /* pixel-rectangle edges: a flip of ceil/floor changes the tile
             * rectangle only across a tile or image boundary; flag every edge
             * within eps_px of an integer near such a boundary */
            if (p->ex > 0 || p->ey > 0) {
                const double e[4] = {p->u - p->ex - 0.5, p->u + p->ex - 0.5, p->v - p->ey - 0.5, p->v + p->ey - 0.5};
                const int tsz[4] = {tile_w, tile_w, tile_h, tile_h};
                const int lim[4] = {k.W, k.W, k.H, k.H};
                for (int j = 0; j < 4; ++j) {
                    const double r = floor(e[j] + 0.5);
                    if (fabs(e[j] - r) <= eps_px) {
                        const long ri = (long)r;
                        if (ri <= 0 || ri >= lim[j] - 1 || ri % tsz[j] == 0 || (ri + 1) % tsz[j] == 0) a = 1;
                    }
                }
            }
            /* cull thresholds */
            if (fabs(p->o - ORC_ALPHA_MIN) <= 1e-6 * ORC_ALPHA_MIN) a = 1;
            if (fabs(p->t[2] - k.near_z) <= 1e-6 * fabs(k.near_z)) a = 1;
            /* depth near a float32 rounding midpoint */
            if (p->valid) {
                const float f = (float)p->t[2];
                const double lo = (double)nextafterf(f, -INFINITY), hi = (double)nextafterf(f, INFINITY);
                const double m1 = 0.5 * ((double)f + lo), m2 = 0.5 * ((double)f + hi);
                if (fabs(p->t[2] - m1) <= 1e-12 * p->t[2] || fabs(p->t[2] - m2) <= 1e-12 * p->t[2]) a = 1;
            }
            amb[i] = a;
        }
        total += cnt;
    }
    if (!keys) { free(pr); return total; }
    if (total > cap) { free(pr); return -3; }
    pair_t *pp = (pair_t *)malloc(sizeof(pair_t) * (size_t)(total > 0 ? total : 1));
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        const proj_t *p = &pr[i];
        if (!p->valid) continue;
        const uint64_t zb = f32_bits(p->t[2]);
        for (int yy = p->py0 / tile_h; yy <= p->py1 / tile_h; ++yy)
            for (int xx = p->px0 / tile_w; xx <= p->px1 / tile_w; ++xx) {
                pp[w].key = ((uint64_t)(yy * tx + xx) << 32) | zb;
                pp[w].val = (uint32_t)i;
                ++w;
            }
    }
    qsort(pp, (size_t)total, sizeof(pair_t), cmp_pair);
    for (int64_t t = 0; t < (int64_t)tx * ty; ++t) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t j = 0; j < total; ++j) {
        keys[j] = pp[j].key;
        vals[j] = pp[j].val;
        const uint32_t t = (uint32_t)(pp[j].key >> 32);
        if (j == 0 || (uint32_t)(pp[j - 1].key >> 32) != t) ranges[2 * t] = (uint32_t)j;
        if (j == total - 1 || (uint32_t)(pp[j + 1].key >> 32) != t) ranges[2 * t + 1] = (uint32_t)(j + 1);
    }
    free(pp);
    free(pr);
    return total;
}

/* Tiled re-evaluation of the forward image from orc_bin's lists: each pixel
 * walks only its tile's list.  Equal to orc_render's all-pairs image when
 * the tile rectangles are conservative. */
int orc_render_tiled(int64_t n, int64_t ld, int deg, const double *mean, const double *scale,
                     const double *quat, const double *opac, const double *sh, const double *camv,
                     int tile_w, int tile_h, const uint32_t *vals, const uint32_t *ranges, double *img,
                     double *final_T) {
    if (deg < 0 || deg > 3 || n < 0 || ld < n) return -1;
    const cam_t k = read_cam(camv);
    const gauss_t g = make_gauss(n, ld, deg, mean, scale, quat, opac, sh);
    proj_t *pr = (proj_t *)malloc(sizeof(proj_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) project_one(&g, &k, i, &pr[i]);
    const int tx = (k.W + tile_w - 1) / tile_w;
    const flagcfg_t fc = {0, 0, 0};
#pragma omp parallel for schedule(dynamic, 4)
    for (int py = 0; py < k.H; ++py) {
        int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        for (int px = 0; px < k.W; ++px) {
            const int t = (py / tile_h) * tx + px / tile_w;
            const uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
            for (uint32_t j = s; j < e; ++j) ord[j - s] = vals[j];
            double T, C[3];
            int64_t last;
            int fl;
            blend_pixel(pr, ord, (int64_t)(e - s), px + 0.5, py + 0.5, &fc, &T, C, &last, &fl, NULL, 0);
            const int64_t q = (int64_t)py * k.W + px;
            for (int c = 0; c < 3; ++c) img[3 * q + c] = C[c] + T * k.bg[c];
            if (final_T) final_T[q] = T;
        }
        free(ord);
    }
    free(pr);
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel regions (timing with one thread). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
