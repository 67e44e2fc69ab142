/*
 * FP64 CPU oracle for the Gaussian-splatting rasterizer of RT-GuIDE
 * (arXiv 2409.18122).  TEST INFRASTRUCTURE ONLY: nothing on the product path
 * may link or call this file; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.
 *
 * What it computes, each piece written from its definition:
 *   - projection of a Gaussian (Sec. III, Gaussian Splatting paragraph:
 *     mu_2D = K R^T (mu - T) / d, d = e3^T R^T (mu - T)); the paper's
 *     isotropic radius r_2D = f r / d is generalised to the EWA covariance
 *     Sigma_2D = J R^T Sigma R J^T of the cited 3DGS work, which equals
 *     (f r / d)^2 I on the optical axis for an isotropic Gaussian;
 *   - depth ordering "in increasing order of depth relative to the camera"
 *     (Sec. III), ties by Gaussian index;
 *   - alpha compositing C(p) = sum_i c_i f_i(p) prod_{j<i} (1 - f_j(p)) and
 *     the depth image with c_i replaced by d_i (Sec. III), plus the accumulated
 *     alpha and the same sum with c_i replaced by the per-Gaussian uncertainty;
 *   - the L1 part of the mapping loss (Sec. III eq. (4)) with colour weight 1
 *     and depth weight w_d, mean over pixels;
 *   - the view score: sum over pixels of the composited uncertainty, the
 *     rendered form of the trace proxy of Sec. IV-A eq. (7);
 *   - the exact reverse-mode adjoint of all of the above (the gradient used to
 *     refine the map, Sec. IV-A "refined through backpropagation").
 *
 * Readings where the paper is silent (all are parameters, see rtgo_settings):
 *   a Gaussian with alpha < alpha_min at a pixel is skipped there; compositing
 *   stops before the Gaussian that would take transmittance below T_min;
 *   alpha is clamped to alpha_max; Gaussians with depth <= z_near, opacity <
 *   alpha_min, a non-positive 2D covariance determinant, a zero quaternion,
 *   non-finite geometry or an empty pixel box are culled; pixel centres are at
 *   integer coordinates; the depth image is not normalised; there is no
 *   background term.
 *
 * All arithmetic is IEEE binary64.  The file is compiled without floating
 * point contraction so that the camera depth, whose binary32 rounding is the
 * sort key, is evaluated exactly as the formula is written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Inputs                                                                   */
/* ------------------------------------------------------------------------ */

/* camera array layout: w, h, fx, fy, cx, cy, R[9] (camera->world,
 * row-major), T[3] (camera centre in world) -> 18 doubles */
typedef struct {
    int w, h;
    double fx, fy, cx, cy;
    double R[9];
    double T[3];
} ocam;

/* settings array layout: T_min, alpha_min, alpha_max, z_near, eps2d, isotropic */
typedef struct {
    double T_min, alpha_min, alpha_max, z_near, eps2d;
    int iso; /* the paper's 8-parameter isotropic Gaussians (Sec. III) */
} oset;

/* Gaussians: planar arrays of N entries each */
typedef struct {
    int64_t n;
    const double *means;      /* 3 x N */
    const double *log_scales; /* 3 x N */
    const double *quats;      /* 4 x N: w, x, y, z (any norm) */
    const double *opacity;    /* N */
    const double *colors;     /* 3 x N */
    const double *uncert;     /* N */
} ogauss;

static void read_cam(const double *a, ocam *c)
{
    c->w = (int)a[0];
    c->h = (int)a[1];
    c->fx = a[2];
    c->fy = a[3];
    c->cx = a[4];
    c->cy = a[5];
    for (int i = 0; i < 9; i++) c->R[i] = a[6 + i];
    for (int i = 0; i < 3; i++) c->T[i] = a[15 + i];
}

static void read_set(const double *a, oset *s)
{
    s->T_min = a[0];
    s->alpha_min = a[1];
    s->alpha_max = a[2];
    s->z_near = a[3];
    s->eps2d = a[4];
    s->iso = a[5] != 0.0;
}

/* ------------------------------------------------------------------------ */
/* Projection (Sec. III, Gaussian Splatting paragraph)                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int valid;
    double qn[4];   /* normalised quaternion */
    double qnorm;   /* norm of the raw quaternion */
    double Rq[9];   /* rotation of the Gaussian, row-major */
    double s[3];    /* scales exp(log_scale) */
    double Sw[9];   /* world covariance Rq diag(s^2) Rq^T */
    double t[3];    /* camera-frame mean R^T (mu - T) */
    double Sc[9];   /* camera-frame covariance R^T Sw R */
    double J[6];    /* 2x3 Jacobian of the perspective map at t */
    double cov[3];  /* Sigma_2D: xx, xy, yy */
    double con[3];  /* Sigma_2D^{-1}: xx, xy, yy */
    double mx, my;  /* projected mean */
    double depth;   /* t_z */
    uint32_t dbits; /* bits of the binary32 rounding of depth */
    double hx, hy;  /* half extents of the alpha >= alpha_min region */
    int u0, u1, v0, v1; /* inclusive pixel box, clipped to the image */
} oproj;

/* Isotropic Gaussians read one log-radius per Gaussian (the first n
 * log-scale values) and no quaternion. */
static int finite_geometry(const ogauss *g, int64_t i, int iso)
{
    int64_t n = g->n;
    for (int k = 0; k < 3; k++)
        if (!isfinite(g->means[k * n + i])) return 0;
    if (iso)
        return isfinite(g->log_scales[i]) && isfinite(g->opacity[i]);
    for (int k = 0; k < 3; k++)
        if (!isfinite(g->log_scales[k * n + i])) return 0;
    for (int k = 0; k < 4; k++)
        if (!isfinite(g->quats[k * n + i])) return 0;
    return isfinite(g->opacity[i]);
}

static uint32_t f32_bits(double d)
{
    float f = (float)d;
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

/* Projected mean, inverse covariance and the pixel box of {alpha >= alpha_min}
 * (d^T Q d <= 2 ln(o / alpha_min), exact half extents sqrt(rho^2 Sigma_aa)),
 * from p->t and p->cov; sets p->valid. */
static void finish_projection(const ocam *c, const oset *st, double o, oproj *p)
{
    double cxx = p->cov[0], cxy = p->cov[1], cyy = p->cov[2];
    double det = cxx * cyy - cxy * cxy;
    if (!(det > 0.0) || !isfinite(det)) return;
    p->con[0] = cyy / det;
    p->con[1] = -cxy / det;
    p->con[2] = cxx / det;
    double tx = p->t[0], ty = p->t[1], tz = p->t[2];
    p->mx = c->fx * tx / tz + c->cx;
    p->my = c->fy * ty / tz + c->cy;
    double rho2 = 2.0 * log(o / st->alpha_min);
    p->hx = sqrt(rho2 * cxx);
    p->hy = sqrt(rho2 * cyy);
    double ulo = ceil(p->mx - p->hx), uhi = floor(p->mx + p->hx);
    double vlo = ceil(p->my - p->hy), vhi = floor(p->my + p->hy);
    if (!(ulo <= uhi) || !(vlo <= vhi)) return;
    if (ulo < 0.0) ulo = 0.0;
    if (vlo < 0.0) vlo = 0.0;
    if (uhi > (double)(c->w - 1)) uhi = (double)(c->w - 1);
    if (vhi > (double)(c->h - 1)) vhi = (double)(c->h - 1);
    if (ulo > uhi || vlo > vhi) return;
    p->u0 = (int)ulo; p->u1 = (int)uhi;
    p->v0 = (int)vlo; p->v1 = (int)vhi;
    p->valid = 1;
}

/* camera-frame mean t = R^T (mu - T); depth d = t_z written in a fixed order.
 * Returns 0 if the Gaussian is at or before the near plane. */
static int camera_mean(const ogauss *g, int64_t i, const ocam *c, const oset *st, oproj *p)
{
    int64_t n = g->n;
    double dx = g->means[0 * n + i] - c->T[0];
    double dy = g->means[1 * n + i] - c->T[1];
    double dz = g->means[2 * n + i] - c->T[2];
    const double *R = c->R;
    p->t[0] = (dx * R[0] + dy * R[3]) + dz * R[6];
    p->t[1] = (dx * R[1] + dy * R[4]) + dz * R[7];
    p->t[2] = (dx * R[2] + dy * R[5]) + dz * R[8];
    p->depth = p->t[2];
    if (!(p->depth > st->z_near)) return 0;
    p->dbits = f32_bits(p->depth);
    return 1;
}

/* The paper's isotropic splat (Sec. III): radius r = exp(log-radius),
 * projected radius r_2D = f r / d per image axis, so
 * Sigma_2D = diag((fx r / d)^2, (fy r / d)^2) (+ eps2d). */
static void project_isotropic(const ogauss *g, int64_t i, const ocam *c, const oset *st, oproj *p)
{
    double r = exp(g->log_scales[i]);
    p->s[0] = p->s[1] = p->s[2] = r;
    if (!camera_mean(g, i, c, st, p)) return;
    double rx = c->fx * r / p->t[2], ry = c->fy * r / p->t[2];
    p->cov[0] = rx * rx + st->eps2d;
    p->cov[1] = 0.0;
    p->cov[2] = ry * ry + st->eps2d;
    finish_projection(c, st, g->opacity[i], p);
}

static void project_one(const ogauss *g, int64_t i, const ocam *c, const oset *st, oproj *p)
{
    int64_t n = g->n;
    memset(p, 0, sizeof(*p));
    p->valid = 0;
    if (!finite_geometry(g, i, st->iso)) return;
    double o = g->opacity[i];
    if (o < st->alpha_min) return;
    if (st->iso) {
        project_isotropic(g, i, c, st, p);
        return;
    }

    /* quaternion -> rotation (w, x, y, z), normalised first */
    double qw = g->quats[0 * n + i], qx = g->quats[1 * n + i];
    double qy = g->quats[2 * n + i], qz = g->quats[3 * n + i];
    double qnorm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    if (!(qnorm > 0.0)) return;
    double w = qw / qnorm, x = qx / qnorm, y = qy / qnorm, z = qz / qnorm;
    p->qnorm = qnorm;
    p->qn[0] = w; p->qn[1] = x; p->qn[2] = y; p->qn[3] = z;
    double *Rq = p->Rq;
    Rq[0] = 1.0 - 2.0 * (y * y + z * z);
    Rq[1] = 2.0 * (x * y - w * z);
    Rq[2] = 2.0 * (x * z + w * y);
    Rq[3] = 2.0 * (x * y + w * z);
    Rq[4] = 1.0 - 2.0 * (x * x + z * z);
    Rq[5] = 2.0 * (y * z - w * x);
    Rq[6] = 2.0 * (x * z - w * y);
    Rq[7] = 2.0 * (y * z + w * x);
    Rq[8] = 1.0 - 2.0 * (x * x + y * y);

    for (int k = 0; k < 3; k++) p->s[k] = exp(g->log_scales[k * n + i]);
    /* Sw = Rq diag(s^2) Rq^T */
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += Rq[a * 3 + k] * p->s[k] * p->s[k] * Rq[b * 3 + k];
            p->Sw[a * 3 + b] = acc;
        }

    if (!camera_mean(g, i, c, st, p)) return;
    const double *R = c->R;

    /* Sc = R^T Sw R */
    double tmp[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += p->Sw[a * 3 + k] * R[k * 3 + b];
            tmp[a * 3 + b] = acc;
        }
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += R[k * 3 + a] * tmp[k * 3 + b];
            p->Sc[a * 3 + b] = acc;
        }

    /* perspective Jacobian and 2D covariance */
    double tx = p->t[0], ty = p->t[1], tz = p->t[2];
    double *J = p->J;
    J[0] = c->fx / tz; J[1] = 0.0; J[2] = -c->fx * tx / (tz * tz);
    J[3] = 0.0; J[4] = c->fy / tz; J[5] = -c->fy * ty / (tz * tz);
    double JS[6];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += J[a * 3 + k] * p->Sc[k * 3 + b];
            JS[a * 3 + b] = acc;
        }
    double cxx = 0.0, cxy = 0.0, cyy = 0.0;
    for (int k = 0; k < 3; k++) {
        cxx += JS[0 * 3 + k] * J[0 * 3 + k];
        cxy += JS[0 * 3 + k] * J[1 * 3 + k];
        cyy += JS[1 * 3 + k] * J[1 * 3 + k];
    }
    cxx += st->eps2d;
    cyy += st->eps2d;
    p->cov[0] = cxx; p->cov[1] = cxy; p->cov[2] = cyy;
    finish_projection(c, st, o, p);
}

/* Depth order: ascending binary32 depth bits, ties by Gaussian index. */
typedef struct {
    uint32_t dbits;
    int64_t idx;
} okey;

static int okey_cmp(const void *a, const void *b)
{
    const okey *x = (const okey *)a, *y = (const okey *)b;
    if (x->dbits != y->dbits) return x->dbits < y->dbits ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

typedef struct {
    ogauss g;
    ocam c;
    oset s;
    oproj *P;       /* N projections */
    int64_t *order; /* visible Gaussians in depth order */
    int64_t nvis;
    double ev_a, ev_t; /* relative widths of the near-threshold event bands */
} oview;

static int view_setup(oview *V, const ogauss *g, const double *cam, const double *set)
{
    V->g = *g;
    read_cam(cam, &V->c);
    read_set(set, &V->s);
    V->P = (oproj *)malloc(sizeof(oproj) * (size_t)(g->n > 0 ? g->n : 1));
    if (!V->P) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; i++) project_one(g, i, &V->c, &V->s, &V->P[i]);
    int64_t nv = 0;
    for (int64_t i = 0; i < g->n; i++) nv += V->P[i].valid;
    okey *keys = (okey *)malloc(sizeof(okey) * (size_t)(nv > 0 ? nv : 1));
    V->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv > 0 ? nv : 1));
    if (!keys || !V->order) return -1;
    nv = 0;
    for (int64_t i = 0; i < g->n; i++)
        if (V->P[i].valid) {
            keys[nv].dbits = V->P[i].dbits;
            keys[nv].idx = i;
            nv++;
        }
    qsort(keys, (size_t)nv, sizeof(okey), okey_cmp);
    for (int64_t k = 0; k < nv; k++) V->order[k] = keys[k].idx;
    free(keys);
    V->nvis = nv;
    return 0;
}

static void view_free(oview *V)
{
    free(V->P);
    free(V->order);
}

/* Per-tile candidate lists: the depth-ordered visible Gaussians whose pixel
 * box meets the tile.  Only an index; every pixel still evaluates its own
 * predicate on each candidate, so the result equals the all-Gaussian loop. */
typedef struct {
    int tw, th, ntx, nty;
    int64_t *start; /* ntx*nty + 1 */
    int64_t *items;
} otiles;

static int tiles_build(const oview *V, int tw, int th, otiles *T)
{
    T->tw = tw;
    T->th = th;
    T->ntx = (V->c.w + tw - 1) / tw;
    T->nty = (V->c.h + th - 1) / th;
    int64_t nt = (int64_t)T->ntx * T->nty;
    T->start = (int64_t *)calloc((size_t)(nt + 1), sizeof(int64_t));
    if (!T->start) return -1;
    for (int64_t k = 0; k < V->nvis; k++) {
        const oproj *p = &V->P[V->order[k]];
        for (int ty = p->v0 / th; ty <= p->v1 / th; ty++)
            for (int tx = p->u0 / tw; tx <= p->u1 / tw; tx++) T->start[(int64_t)ty * T->ntx + tx + 1]++;
    }
    for (int64_t t = 0; t < nt; t++) T->start[t + 1] += T->start[t];
    T->items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T->start[nt] > 0 ? T->start[nt] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt > 0 ? nt : 1));
    if (!T->items || !fill) return -1;
    for (int64_t t = 0; t < nt; t++) fill[t] = T->start[t];
    for (int64_t k = 0; k < V->nvis; k++) {
        int64_t i = V->order[k];
        const oproj *p = &V->P[i];
        for (int ty = p->v0 / th; ty <= p->v1 / th; ty++)
            for (int tx = p->u0 / tw; tx <= p->u1 / tw; tx++) T->items[fill[(int64_t)ty * T->ntx + tx]++] = i;
    }
    free(fill);
    return 0;
}

static void tiles_free(otiles *T)
{
    free(T->start);
    free(T->items);
}

/* ------------------------------------------------------------------------ */
/* Compositing of one pixel (Sec. III)                                      */
/* ------------------------------------------------------------------------ */

#define OEV_CAP 8

typedef struct {
    int pos;  /* position in the candidate list */
    int kind; /* 0: the alpha_min skip test, 1: the T_min stop test */
} oevent;

typedef struct {
    double out[6]; /* r, g, b, depth, alpha, uncertainty */
    double ub;     /* sum of u over the contributing Gaussians (binary-J trace) */
    double T;      /* final transmittance */
    int ncontrib;  /* Gaussians that contributed */
    int nevents;   /* near-threshold decisions (may exceed OEV_CAP) */
    oevent ev[OEV_CAP];
} opix;

static int forced(const oevent *f, int nf, int pos, int kind)
{
    for (int k = 0; k < nf; k++)
        if (f[k].pos == pos && f[k].kind == kind) return 1;
    return 0;
}

static void alpha_at(const oview *V, int64_t i, double u, double v,
                     double *alpha, double *G, int *clamped, double *ddx, double *ddy)
{
    const oproj *p = &V->P[i];
    double dx = u - p->mx, dy = v - p->my;
    double power = p->con[0] * dx * dx + 2.0 * p->con[1] * dx * dy + p->con[2] * dy * dy;
    double Gv = exp(-0.5 * power);
    double a = V->g.opacity[i] * Gv;
    *clamped = 0;
    if (a > V->s.alpha_max) {
        a = V->s.alpha_max;
        *clamped = 1;
    }
    *alpha = a;
    *G = Gv;
    *ddx = dx;
    *ddy = dy;
}

/* Composites the candidates list[0..n) at pixel (u, v) front to back.  The
 * decisions named in `force` are taken the other way. */
static void composite(const oview *V, const int64_t *list, int64_t n, int u, int v,
                      const oevent *force, int nforce, opix *r)
{
    const double *col = V->g.colors, *unc = V->g.uncert;
    int64_t N = V->g.n;
    double T = 1.0, C0 = 0.0, C1 = 0.0, C2 = 0.0, D = 0.0, U = 0.0, UB = 0.0;
    int nc = 0, ne = 0;
    for (int64_t k = 0; k < n; k++) {
        int64_t i = list[k];
        double a, G, ddx, ddy;
        int cl;
        alpha_at(V, i, (double)u, (double)v, &a, &G, &cl, &ddx, &ddy);
        int skip = a < V->s.alpha_min;
        if (fabs(a - V->s.alpha_min) <= V->ev_a * V->s.alpha_min) {
            if (ne < OEV_CAP) { r->ev[ne].pos = (int)k; r->ev[ne].kind = 0; }
            ne++;
        }
        if (nforce && forced(force, nforce, (int)k, 0)) skip = !skip;
        if (skip) continue;
        double Tn = T * (1.0 - a);
        int stop = Tn < V->s.T_min;
        if (fabs(Tn - V->s.T_min) <= V->ev_t * V->s.T_min) {
            if (ne < OEV_CAP) { r->ev[ne].pos = (int)k; r->ev[ne].kind = 1; }
            ne++;
        }
        if (nforce && forced(force, nforce, (int)k, 1)) stop = !stop;
        if (stop) break;
        double w = a * T;
        C0 += col[0 * N + i] * w;
        C1 += col[1 * N + i] * w;
        C2 += col[2 * N + i] * w;
        D += V->P[i].depth * w;
        U += unc[i] * w;
        UB += unc[i];
        T = Tn;
        nc++;
    }
    r->out[0] = C0; r->out[1] = C1; r->out[2] = C2;
    r->out[3] = D; r->out[4] = 1.0 - T; r->out[5] = U;
    r->ub = UB;
    r->T = T;
    r->ncontrib = nc;
    r->nevents = ne;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                    */
/* ------------------------------------------------------------------------ */

static void gauss_from(ogauss *g, int64_t n, const double *means, const double *ls,
                       const double *q, const double *o, const double *c, const double *u)
{
    g->n = n;
    g->means = means;
    g->log_scales = ls;
    g->quats = q;
    g->opacity = o;
    g->colors = c;
    g->uncert = u;
}

void rtgo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int rtgo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Per-Gaussian projection for one camera.
 * outputs (N each unless noted): valid (int32), mean2d (2N: x then y planes),
 * cov2d (3N), conic (3N), depth (N), depth_bits (uint32), half-extent (2N),
 * box (4N int32: u0, u1, v0, v1 planes). */
int rtgo_project(int64_t n, const double *means, const double *ls, const double *q,
                 const double *o, const double *cam, const double *set,
                 int32_t *valid, double *mean2d, double *cov2d, double *conic,
                 double *depth, uint32_t *dbits, double *half, int32_t *box)
{
    ogauss g;
    gauss_from(&g, n, means, ls, q, o, NULL, NULL);
    ocam c;
    oset s;
    read_cam(cam, &c);
    read_set(set, &s);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        oproj p;
        project_one(&g, i, &c, &s, &p);
        valid[i] = p.valid;
        mean2d[i] = p.mx; mean2d[n + i] = p.my;
        cov2d[i] = p.cov[0]; cov2d[n + i] = p.cov[1]; cov2d[2 * n + i] = p.cov[2];
        conic[i] = p.con[0]; conic[n + i] = p.con[1]; conic[2 * n + i] = p.con[2];
        depth[i] = p.depth;
        dbits[i] = p.dbits;
        half[i] = p.hx; half[n + i] = p.hy;
        box[i] = p.u0; box[n + i] = p.u1; box[2 * n + i] = p.v0; box[3 * n + i] = p.v1;
    }
    return 0;
}

/* Renders one camera.
 *   mode 0: every pixel walks every visible Gaussian (the definition);
 *   mode 1: every pixel walks the candidates of its tw x th tile.
 *   roi = {x0, y0, x1, y1}: only pixels with x0 <= u < x1, y0 <= v < y1 are
 *   written (others are left untouched).
 * Image outputs are planar: rgb (3 x H x W), depth, alpha, unc, T_final
 * (H x W each), ncontrib and nevents (int32, H x W).
 * For pixels with 1..2 near-threshold events, all 2^k decision combinations
 * are written to alt_val (alt_cap x 4 x 6; combination 0 is the primary
 * result, unused slots repeat it), with the pixel index in alt_pix.  Returns
 * the number of such pixels (may exceed alt_cap, then the surplus is
 * dropped), or -1 on allocation failure. */
int64_t rtgo_render(int64_t n, const double *means, const double *ls, const double *q,
                    const double *o, const double *colors, const double *unc,
                    const double *cam, const double *set, int mode, int tw, int th,
                    const int32_t *roi, double ev_a, double ev_t,
                    double *rgb, double *depth, double *alpha, double *uimg, double *Tfin,
                    int32_t *ncontrib, int32_t *nevents,
                    int64_t alt_cap, int64_t *alt_pix, double *alt_val)
{
    ogauss g;
    gauss_from(&g, n, means, ls, q, o, colors, unc);
    oview V;
    if (view_setup(&V, &g, cam, set)) return -1;
    V.ev_a = ev_a;
    V.ev_t = ev_t;
    otiles T;
    memset(&T, 0, sizeof(T));
    if (mode == 1 && tiles_build(&V, tw, th, &T)) return -1;
    int W = V.c.w, H = V.c.h;
    int x0 = roi ? roi[0] : 0, y0 = roi ? roi[1] : 0;
    int x1 = roi ? roi[2] : W, y1 = roi ? roi[3] : H;
    int64_t P = (int64_t)W * H;
    int64_t nalt = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t pix = 0; pix < P; pix++) {
        int u = (int)(pix % W), v = (int)(pix / W);
        if (u < x0 || u >= x1 || v < y0 || v >= y1) continue;
        const int64_t *list;
        int64_t len;
        if (mode == 1) {
            int64_t t = (int64_t)(v / th) * T.ntx + u / tw;
            list = T.items + T.start[t];
            len = T.start[t + 1] - T.start[t];
        } else {
            list = V.order;
            len = V.nvis;
        }
        opix r;
        composite(&V, list, len, u, v, NULL, 0, &r);
        for (int ch = 0; ch < 3; ch++) rgb[ch * P + pix] = r.out[ch];
        depth[pix] = r.out[3];
        alpha[pix] = r.out[4];
        uimg[pix] = r.out[5];
        Tfin[pix] = r.T;
        ncontrib[pix] = r.ncontrib;
        nevents[pix] = r.nevents;
        if (r.nevents >= 1 && r.nevents <= 2) {
            int64_t slot;
#pragma omp atomic capture
            slot = nalt++;
            if (slot < alt_cap) {
                alt_pix[slot] = pix;
                double *dst = alt_val + slot * 24;
                int ncomb = 1 << r.nevents;
                for (int cmb = 0; cmb < 4; cmb++) {
                    opix a;
                    if (cmb == 0 || cmb >= ncomb) {
                        a = r;
                    } else {
                        oevent f[2];
                        int nf = 0;
                        for (int e = 0; e < r.nevents; e++)
                            if (cmb & (1 << e)) f[nf++] = r.ev[e];
                        composite(&V, list, len, u, v, f, nf, &a);
                    }
                    for (int ch = 0; ch < 6; ch++) dst[cmb * 6 + ch] = a.out[ch];
                }
            }
        }
    }
    if (mode == 1) tiles_free(&T);
    view_free(&V);
    return nalt;
}

/* Number of visible Gaussians and of (tile, Gaussian) pairs for one camera. */
/* Whether Gaussian i's support meets tile (tx, ty): some pixel centre of the
 * tile, inside its pixel box, where alpha >= alpha_min (the skip test of the
 * compositing loop).  Pixels of other tiles never composite Gaussian i. */
static int support_meets_tile(const oview *V, int64_t i, int tx, int ty, int tw, int th)
{
    const oproj *p = &V->P[i];
    int ulo = tx * tw > p->u0 ? tx * tw : p->u0, uhi = tx * tw + tw - 1 < p->u1 ? tx * tw + tw - 1 : p->u1;
    int vlo = ty * th > p->v0 ? ty * th : p->v0, vhi = ty * th + th - 1 < p->v1 ? ty * th + th - 1 : p->v1;
    for (int v = vlo; v <= vhi; v++)
        for (int u = ulo; u <= uhi; u++) {
            double a, G, dx, dy;
            int cl;
            alpha_at(V, i, (double)u, (double)v, &a, &G, &cl, &dx, &dy);
            if (a >= V->s.alpha_min) return 1;
        }
    return 0;
}

/* Tiles Gaussian i is binned to: every tile its pixel box meets, or with
 * support != 0 only those its support meets. */
static int64_t tiles_of(const oview *V, int64_t i, int tw, int th, int support, int ntx, int64_t tile_base,
                        uint64_t *keys, uint32_t *vals, int64_t k)
{
    const oproj *p = &V->P[i];
    for (int ty = p->v0 / th; ty <= p->v1 / th; ty++)
        for (int tx = p->u0 / tw; tx <= p->u1 / tw; tx++) {
            if (support && !support_meets_tile(V, i, tx, ty, tw, th)) continue;
            if (keys) {
                keys[k] = ((uint64_t)(tile_base + (int64_t)ty * ntx + tx) << 32) | p->dbits;
                vals[k] = (uint32_t)i;
            }
            k++;
        }
    return k;
}

int rtgo_count(int64_t n, const double *means, const double *ls, const double *q,
               const double *o, const double *cam, const double *set, int tw, int th, int support,
               int64_t *nvis, int64_t *npairs)
{
    ogauss g;
    gauss_from(&g, n, means, ls, q, o, NULL, NULL);
    oview V;
    if (view_setup(&V, &g, cam, set)) return -1;
    int ntx = (V.c.w + tw - 1) / tw;
    int64_t k = 0;
    for (int64_t j = 0; j < V.nvis; j++) k = tiles_of(&V, V.order[j], tw, th, support, ntx, 0, NULL, NULL, k);
    *nvis = V.nvis;
    *npairs = k;
    view_free(&V);
    return 0;
}

/* Sorted binning of one camera: for every visible Gaussian i and every tile
 * (tx, ty) it is binned to (tiles_of), the pair key
 * ((tile_base + ty*ntx + tx) << 32 | depth_bits) with value i, listed in
 * ascending (key, i) order: a stable sort by tile of the depth-ordered pairs.
 * The caller sizes keys/vals from rtgo_count with the same `support`. */
int rtgo_keys(int64_t n, const double *means, const double *ls, const double *q,
              const double *o, const double *cam, const double *set, int tw, int th, int support,
              int64_t tile_base, uint64_t *keys, uint32_t *vals)
{
    ogauss g;
    gauss_from(&g, n, means, ls, q, o, NULL, NULL);
    oview V;
    if (view_setup(&V, &g, cam, set)) return -1;
    int ntx = (V.c.w + tw - 1) / tw;
    int nty = (V.c.h + th - 1) / th;
    int64_t nt = (int64_t)ntx * nty;
    int64_t total = 0;
    for (int64_t j = 0; j < V.nvis; j++) total = tiles_of(&V, V.order[j], tw, th, support, ntx, 0, NULL, NULL, total);
    uint64_t *dk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(total > 0 ? total : 1));
    uint32_t *dv = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(total > 0 ? total : 1));
    int64_t *start = (int64_t *)calloc((size_t)(nt + 1), sizeof(int64_t));
    if (!dk || !dv || !start) return -1;
    /* pairs in depth order, then a counting sort by tile (stable) */
    int64_t k = 0;
    for (int64_t j = 0; j < V.nvis; j++) k = tiles_of(&V, V.order[j], tw, th, support, ntx, 0, dk, dv, k);
    for (int64_t m = 0; m < total; m++) start[(dk[m] >> 32) + 1]++;
    for (int64_t t = 0; t < nt; t++) start[t + 1] += start[t];
    for (int64_t m = 0; m < total; m++) {
        int64_t t = (int64_t)(dk[m] >> 32);
        int64_t at = start[t]++;
        keys[at] = ((uint64_t)(tile_base + t) << 32) | (dk[m] & 0xffffffffu);
        vals[at] = dv[m];
    }
    free(dk);
    free(dv);
    free(start);
    view_free(&V);
    return 0;
}

/* L1 mapping loss of Sec. III eq. (4) without the SSIM term, colour weight 1,
 * depth weight wd:  L = (1/P) sum_p [sum_ch |c - c*| + wd |d - d*|], and its
 * gradient with sign(0) = 0.  Inputs/outputs planar (rgb 3 x P). */
double rtgo_loss(int64_t P, const double *rgb, const double *dep, const double *trgb,
                 const double *tdep, double wd, double *grgb, double *gdep)
{
    double L = 0.0;
    for (int64_t p = 0; p < P; p++) {
        for (int ch = 0; ch < 3; ch++) {
            double e = rgb[ch * P + p] - trgb[ch * P + p];
            L += fabs(e);
            grgb[ch * P + p] = (e > 0.0 ? 1.0 : (e < 0.0 ? -1.0 : 0.0)) / (double)P;
        }
        double e = dep[p] - tdep[p];
        L += wd * fabs(e);
        gdep[p] = wd * (e > 0.0 ? 1.0 : (e < 0.0 ? -1.0 : 0.0)) / (double)P;
    }
    return L / (double)P;
}

/* SSIM term of the mapping loss of Sec. III eq. (4).  The paper names SSIM
 * without defining it; this is the structural similarity index of Wang et
 * al. (2004) in the form the 3DGS mappers it builds on use: per colour
 * channel, local statistics under an 11 x 11 Gaussian window (sigma 1.5,
 * weights w(a, b) = g(a) g(b) with g normalised to sum 1 over -5..5), pixels
 * outside the image read as 0, C1 = 0.01^2, C2 = 0.03^2 (data range 1):
 *   mx = sum w x,  sx = sum w x^2 - mx^2,  sxy = sum w x y - mx my,
 *   S  = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sx + sy + C2)),
 * and SSIM = the mean of S over the three channels and all pixels. */
#define SSIM_R 5
#define SSIM_C1 (0.01 * 0.01)
#define SSIM_C2 (0.03 * 0.03)

static void ssim_window(double g[2 * SSIM_R + 1])
{
    double sum = 0.0;
    for (int k = -SSIM_R; k <= SSIM_R; k++) {
        g[k + SSIM_R] = exp(-(double)(k * k) / (2.0 * 1.5 * 1.5));
        sum += g[k + SSIM_R];
    }
    for (int k = 0; k <= 2 * SSIM_R; k++)
        g[k] /= sum;
}

/* Mapping loss of Sec. III eq. (4) for one W x H view (planar rgb 3 x P):
 *   L = (1/P) sum_p ( wd |D - D*| + l1 sum_ch |C - C*| ) + l2 (1 - SSIM(C, C*)),
 * with its gradient with respect to the rendered C and D (the target gets
 * none; sign(0) = 0).  The SSIM gradient is the exact reverse mode of the
 * definition above: pixel p's S depends on x(q) for q in its window through
 *   dS(p)/dx(q) = w(q - p) [dS/dmx + 2 (x(q) - mx) dS/dsx + (y(q) - my) dS/dsxy](p),
 * gathered per q.  smap (3 x P) receives S when not NULL. */
double rtgo_loss_ssim(int W, int H, const double *rgb, const double *dep, const double *trgb,
                      const double *tdep, double wd, double l1, double l2, double *grgb, double *gdep,
                      double *smap)
{
    const int64_t P = (int64_t)W * H;
    double g[2 * SSIM_R + 1];
    ssim_window(g);
    double L = 0.0;
    for (int64_t p = 0; p < P; p++) {
        double row = 0.0;
        for (int ch = 0; ch < 3; ch++) {
            double e = rgb[ch * P + p] - trgb[ch * P + p];
            row += fabs(e);
            grgb[ch * P + p] = l1 * (e > 0.0 ? 1.0 : (e < 0.0 ? -1.0 : 0.0)) / (double)P;
        }
        double e = dep[p] - tdep[p];
        L += wd * fabs(e) + l1 * row;
        gdep[p] = wd * (e > 0.0 ? 1.0 : (e < 0.0 ? -1.0 : 0.0)) / (double)P;
    }
    L /= (double)P;
    /* per pixel: mx, my, dS/dmx, dS/dsx, dS/dsxy */
    double *st = (double *)malloc(sizeof(double) * 5 * (size_t)P);
    if (!st)
        return NAN;
    double ssum = 0.0;
    for (int ch = 0; ch < 3; ch++) {
        const double *x = rgb + ch * P, *y = trgb + ch * P;
        double csum = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : csum)
        for (int v = 0; v < H; v++) {
            for (int u = 0; u < W; u++) {
                double mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
                for (int b = -SSIM_R; b <= SSIM_R; b++) {
                    int vv = v + b;
                    if (vv < 0 || vv >= H)
                        continue;
                    for (int a = -SSIM_R; a <= SSIM_R; a++) {
                        int uu = u + a;
                        if (uu < 0 || uu >= W)
                            continue;
                        double w = g[a + SSIM_R] * g[b + SSIM_R];
                        double xv = x[(int64_t)vv * W + uu], yv = y[(int64_t)vv * W + uu];
                        mx += w * xv;
                        my += w * yv;
                        exx += w * (xv * xv);
                        eyy += w * (yv * yv);
                        exy += w * (xv * yv);
                    }
                }
                double sx = exx - mx * mx, sy = eyy - my * my, sxy = exy - mx * my;
                double n1 = 2.0 * mx * my + SSIM_C1, n2 = 2.0 * sxy + SSIM_C2;
                double d1 = mx * mx + my * my + SSIM_C1, d2 = sx + sy + SSIM_C2;
                double S = (n1 * n2) / (d1 * d2);
                int64_t p = (int64_t)v * W + u;
                if (smap)
                    smap[ch * P + p] = S;
                csum += S;
                st[5 * p + 0] = mx;
                st[5 * p + 1] = my;
                st[5 * p + 2] = (2.0 * my * n2 - S * 2.0 * mx * d2) / (d1 * d2); /* dS/dmx */
                st[5 * p + 3] = -S / d2;                                        /* dS/dsx */
                st[5 * p + 4] = 2.0 * n1 / (d1 * d2);                           /* dS/dsxy */
            }
        }
        ssum += csum;
        const double k = -l2 / (3.0 * (double)P);
#pragma omp parallel for schedule(static)
        for (int v = 0; v < H; v++) {
            for (int u = 0; u < W; u++) {
                int64_t q = (int64_t)v * W + u;
                double acc = 0.0;
                for (int b = -SSIM_R; b <= SSIM_R; b++) {
                    int vv = v + b;
                    if (vv < 0 || vv >= H)
                        continue;
                    for (int a = -SSIM_R; a <= SSIM_R; a++) {
                        int uu = u + a;
                        if (uu < 0 || uu >= W)
                            continue;
                        const double *sp = st + 5 * ((int64_t)vv * W + uu);
                        double w = g[a + SSIM_R] * g[b + SSIM_R];
                        acc += w * (sp[2] + 2.0 * (x[q] - sp[0]) * sp[3] + (y[q] - sp[1]) * sp[4]);
                    }
                }
                grgb[ch * P + q] += k * acc;
            }
        }
    }
    free(st);
    return L + l2 * (1.0 - ssum / (3.0 * (double)P));
}

/* Sum over pixels of the composited uncertainty for each of nv cameras
 * (cams: nv x 18).  The per-view sum is taken in pixel order. */
/* View scores (Sec. IV-A eq. (7)) as sums over pixels, per pixel p:
 *   mode 0: the rendered trace proxy U(p) = sum_i u_i a_i T_i;
 *   mode 1: the binary-J trace, the same sum with the Jacobian replaced by
 *           its sparsity pattern: sum of u_i over the Gaussians i that
 *           contribute to p (pass the alpha_min test, before termination). */
int rtgo_score(int64_t n, const double *means, const double *ls, const double *q,
               const double *o, const double *colors, const double *unc,
               const double *cams, int nv, const double *set, int tw, int th, int mode, double *scores)
{
    ogauss g;
    gauss_from(&g, n, means, ls, q, o, colors, unc);
    for (int v = 0; v < nv; v++) {
        oview V;
        if (view_setup(&V, &g, cams + 18 * v, set)) return -1;
        V.ev_a = 0.0;
        V.ev_t = 0.0;
        otiles T;
        if (tiles_build(&V, tw, th, &T)) return -1;
        int W = V.c.w;
        int64_t P = (int64_t)W * V.c.h;
        double *row = (double *)calloc((size_t)P, sizeof(double));
        if (!row) return -1;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t pix = 0; pix < P; pix++) {
            int u = (int)(pix % W), vv = (int)(pix / W);
            int64_t t = (int64_t)(vv / th) * T.ntx + u / tw;
            opix r;
            composite(&V, T.items + T.start[t], T.start[t + 1] - T.start[t], u, vv, NULL, 0, &r);
            row[pix] = mode ? r.ub : r.out[5];
        }
        double s = 0.0;
        for (int64_t p = 0; p < P; p++) s += row[p];
        scores[v] = s;
        free(row);
        tiles_free(&T);
        view_free(&V);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint                                                                  */
/* ------------------------------------------------------------------------ */

/* Per visible Gaussian, gradient with respect to its screen-space quantities:
 * mean2d (2), conic xx/xy/yy (3, xy counted once as a parameter that appears
 * twice in the quadratic form), opacity, colour (3), camera depth. */
#define O2D 10

typedef struct {
    int64_t pos;
    double alpha, T, G;
    int clamped;
    double dx, dy;
} ocontrib;

/* Marks, at a pixel holding near-threshold decisions, every Gaussian that
 * contributes under one of the decision sets the forward pass considers (the
 * primary one and each alternative of up to two flipped decisions) or whose
 * own decision is near its threshold: only their per-pixel gradient terms
 * depend on the decisions.  With more than two decisions, every candidate
 * whose alpha reaches the lower edge of the alpha_min band is marked. */
static void mark_touched(const oview *V, const int64_t *list, int64_t len, int u, int v, int32_t *touched)
{
    opix r;
    composite(V, list, len, u, v, NULL, 0, &r);
    int ne = r.nevents;
    if (ne > 2) {
        for (int64_t k = 0; k < len; k++) {
            double a, G, dx, dy;
            int cl;
            alpha_at(V, list[k], (double)u, (double)v, &a, &G, &cl, &dx, &dy);
            if (a >= V->s.alpha_min * (1.0 - V->ev_a)) {
#pragma omp atomic write
                touched[list[k]] = 1;
            }
        }
        return;
    }
    oevent ev[2];
    for (int e = 0; e < ne; e++) {
        ev[e] = r.ev[e];
#pragma omp atomic write
        touched[list[ev[e].pos]] = 1;
    }
    /* decision sets: bit e of `set` flips event e */
    for (int set = 0; set < (1 << ne); set++) {
        oevent f[2];
        int nf = 0;
        for (int e = 0; e < ne; e++)
            if (set & (1 << e)) f[nf++] = ev[e];
        double T = 1.0;
        for (int64_t k = 0; k < len; k++) {
            int64_t i = list[k];
            double a, G, dx, dy;
            int cl;
            alpha_at(V, i, (double)u, (double)v, &a, &G, &cl, &dx, &dy);
            int skip = a < V->s.alpha_min;
            if (nf && forced(f, nf, (int)k, 0)) skip = !skip;
            if (skip) continue;
            double Tn = T * (1.0 - a);
            int stop = Tn < V->s.T_min;
            if (nf && forced(f, nf, (int)k, 1)) stop = !stop;
            if (stop) break;
#pragma omp atomic write
            touched[i] = 1;
            T = Tn;
        }
    }
}

/* Reverse mode of one pixel given upstream gradients g[6] for r, g, b,
 * depth, alpha, uncertainty.  acc2d is indexed by Gaussian.  When touched is
 * not NULL and the pixel holds a near-threshold decision (the event bands of
 * the forward pass), every candidate whose alpha at the pixel reaches the
 * lower edge of the alpha_min band is marked in touched[]: the gradient of
 * each such Gaussian may legitimately follow another decision set there. */
static void pixel_adjoint(const oview *V, const int64_t *list, int64_t len, int u, int v,
                          const double g6[6], double *acc2d, ocontrib *buf, int32_t *touched)
{
    const double *col = V->g.colors, *unc = V->g.uncert;
    int64_t N = V->g.n;
    double T = 1.0;
    int64_t m = 0;
    int event = 0;
    for (int64_t k = 0; k < len; k++) {
        int64_t i = list[k];
        double a, G, dx, dy;
        int cl;
        alpha_at(V, i, (double)u, (double)v, &a, &G, &cl, &dx, &dy);
        if (fabs(a - V->s.alpha_min) <= V->ev_a * V->s.alpha_min) event = 1;
        if (a < V->s.alpha_min) continue;
        double Tn = T * (1.0 - a);
        if (fabs(Tn - V->s.T_min) <= V->ev_t * V->s.T_min) event = 1;
        if (Tn < V->s.T_min) break;
        buf[m].pos = i;
        buf[m].alpha = a;
        buf[m].T = T;
        buf[m].G = G;
        buf[m].clamped = cl;
        buf[m].dx = dx;
        buf[m].dy = dy;
        m++;
        T = Tn;
    }
    if (event && touched) mark_touched(V, list, len, u, v, touched);
    /* suffix sums S_ch = sum_{j > i} v_j w_j */
    double S[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = m - 1; k >= 0; k--) {
        int64_t i = buf[k].pos;
        double a = buf[k].alpha, Ti = buf[k].T, w = a * Ti;
        double val[6] = {col[i], col[N + i], col[2 * N + i], V->P[i].depth, 1.0, unc[i]};
        double da = 0.0;
        for (int ch = 0; ch < 6; ch++) da += g6[ch] * (val[ch] * Ti - S[ch] / (1.0 - a));
        double *G2 = acc2d + (size_t)i * O2D;
        G2[6] += g6[0] * w;
        G2[7] += g6[1] * w;
        G2[8] += g6[2] * w;
        G2[9] += g6[3] * w;
        for (int ch = 0; ch < 6; ch++) S[ch] += val[ch] * w;
        if (!buf[k].clamped) {
            double o = V->g.opacity[i];
            double Gv = buf[k].G;
            G2[5] += da * Gv;           /* d alpha / d o = G */
            double dG = da * o;         /* d alpha / d G = o */
            double dpow = -0.5 * Gv * dG; /* G = exp(-power / 2) */
            double dx = buf[k].dx, dy = buf[k].dy;
            const double *Q = V->P[i].con;
            G2[2] += dpow * dx * dx;
            G2[3] += dpow * 2.0 * dx * dy;
            G2[4] += dpow * dy * dy;
            double ddx = dpow * (2.0 * Q[0] * dx + 2.0 * Q[1] * dy);
            double ddy = dpow * (2.0 * Q[1] * dx + 2.0 * Q[2] * dy);
            G2[0] -= ddx; /* delta = p - mean2d */
            G2[1] -= ddy;
        }
    }
}

/* Chain rule from the screen-space gradient of one Gaussian to its
 * parameters (mean, log-scale, raw quaternion, opacity, colour); adds into
 * the output arrays. */
static void project_adjoint(const oview *V, int64_t i, const double *G2,
                            double *gm, double *gls, double *gq, double *go, double *gc)
{
    const oproj *p = &V->P[i];
    const ocam *c = &V->c;
    int64_t N = V->g.n;
    go[i] += G2[5];
    gc[i] += G2[6];
    gc[N + i] += G2[7];
    gc[2 * N + i] += G2[8];

    /* conic (parameters xx, xy, yy) -> full symmetric matrix gradient */
    double GQ[4] = {G2[2], 0.5 * G2[3], 0.5 * G2[3], G2[4]};
    double Q[4] = {p->con[0], p->con[1], p->con[1], p->con[2]};
    /* G_Sigma = -Q G_Q Q */
    double tmp[4], GS[4];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) tmp[a * 2 + b] = GQ[a * 2 + 0] * Q[0 * 2 + b] + GQ[a * 2 + 1] * Q[1 * 2 + b];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) GS[a * 2 + b] = -(Q[a * 2 + 0] * tmp[0 * 2 + b] + Q[a * 2 + 1] * tmp[1 * 2 + b]);

    double tx = p->t[0], ty = p->t[1], tz = p->t[2];
    double fx = c->fx, fy = c->fy;
    double gt[3] = {0.0, 0.0, 0.0};
    if (V->s.iso) {
        /* Sigma_aa = (f_a r / t_z)^2 + eps2d: d/dlog r = 2 (Sigma_aa - eps2d),
         * d/dt_z = -2 (Sigma_aa - eps2d) / t_z; Sigma_xy = 0 is constant */
        double gsum = GS[0] * (p->cov[0] - V->s.eps2d) + GS[3] * (p->cov[2] - V->s.eps2d);
        gls[i] += 2.0 * gsum;
        gt[2] += -2.0 * gsum / tz;
        gt[0] += G2[0] * fx / tz;
        gt[2] += G2[0] * (-fx * tx / (tz * tz));
        gt[1] += G2[1] * fy / tz;
        gt[2] += G2[1] * (-fy * ty / (tz * tz));
        gt[2] += G2[9];
        const double *R = c->R;
        for (int a = 0; a < 3; a++)
            gm[a * N + i] += R[a * 3 + 0] * gt[0] + R[a * 3 + 1] * gt[1] + R[a * 3 + 2] * gt[2];
        return;
    }

    const double *J = p->J, *Sc = p->Sc;
    /* G_Sc = J^T G_S J (3x3) */
    double GSc[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int r = 0; r < 2; r++)
                for (int s = 0; s < 2; s++) acc += J[r * 3 + a] * GS[r * 2 + s] * J[s * 3 + b];
            GSc[a * 3 + b] = acc;
        }
    /* G_J = 2 G_S J Sc (2x3) */
    double GJ[6];
    for (int r = 0; r < 2; r++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int s = 0; s < 2; s++)
                for (int k = 0; k < 3; k++) acc += GS[r * 2 + s] * J[s * 3 + k] * Sc[k * 3 + b];
            GJ[r * 3 + b] = 2.0 * acc;
        }
    /* camera-frame mean */
    gt[2] += GJ[0] * (-fx / (tz * tz));
    gt[0] += GJ[2] * (-fx / (tz * tz));
    gt[2] += GJ[2] * (2.0 * fx * tx / (tz * tz * tz));
    gt[2] += GJ[4] * (-fy / (tz * tz));
    gt[1] += GJ[5] * (-fy / (tz * tz));
    gt[2] += GJ[5] * (2.0 * fy * ty / (tz * tz * tz));
    gt[0] += G2[0] * fx / tz;
    gt[2] += G2[0] * (-fx * tx / (tz * tz));
    gt[1] += G2[1] * fy / tz;
    gt[2] += G2[1] * (-fy * ty / (tz * tz));
    gt[2] += G2[9]; /* depth image: d_i = t_z */
    const double *R = c->R;
    for (int a = 0; a < 3; a++) gm[a * N + i] += R[a * 3 + 0] * gt[0] + R[a * 3 + 1] * gt[1] + R[a * 3 + 2] * gt[2];

    /* G_Sw = R G_Sc R^T */
    double t2[9], GSw[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += GSc[a * 3 + k] * R[b * 3 + k];
            t2[a * 3 + b] = acc;
        }
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += R[a * 3 + k] * t2[k * 3 + b];
            GSw[a * 3 + b] = acc;
        }
    /* Sw = M M^T, M = Rq diag(s): G_M = 2 G_Sw M */
    const double *Rq = p->Rq, *s = p->s;
    double GM[9];
    for (int a = 0; a < 3; a++)
        for (int k = 0; k < 3; k++) {
            double acc = 0.0;
            for (int b = 0; b < 3; b++) acc += GSw[a * 3 + b] * Rq[b * 3 + k] * s[k];
            GM[a * 3 + k] = 2.0 * acc;
        }
    double GR[9];
    for (int k = 0; k < 3; k++) {
        double gs = 0.0;
        for (int a = 0; a < 3; a++) {
            gs += GM[a * 3 + k] * Rq[a * 3 + k];
            GR[a * 3 + k] = GM[a * 3 + k] * s[k];
        }
        gls[k * N + i] += gs * s[k];
    }
    /* rotation entries -> normalised quaternion */
    double w = p->qn[0], x = p->qn[1], y = p->qn[2], z = p->qn[3];
    double gw = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    /* R00 = 1 - 2(y^2 + z^2) */
    gy += GR[0] * (-4.0 * y); gz += GR[0] * (-4.0 * z);
    /* R01 = 2(xy - wz) */
    gw += GR[1] * (-2.0 * z); gx += GR[1] * (2.0 * y); gy += GR[1] * (2.0 * x); gz += GR[1] * (-2.0 * w);
    /* R02 = 2(xz + wy) */
    gw += GR[2] * (2.0 * y); gx += GR[2] * (2.0 * z); gy += GR[2] * (2.0 * w); gz += GR[2] * (2.0 * x);
    /* R10 = 2(xy + wz) */
    gw += GR[3] * (2.0 * z); gx += GR[3] * (2.0 * y); gy += GR[3] * (2.0 * x); gz += GR[3] * (2.0 * w);
    /* R11 = 1 - 2(x^2 + z^2) */
    gx += GR[4] * (-4.0 * x); gz += GR[4] * (-4.0 * z);
    /* R12 = 2(yz - wx) */
    gw += GR[5] * (-2.0 * x); gx += GR[5] * (-2.0 * w); gy += GR[5] * (2.0 * z); gz += GR[5] * (2.0 * y);
    /* R20 = 2(xz - wy) */
    gw += GR[6] * (-2.0 * y); gx += GR[6] * (2.0 * z); gy += GR[6] * (-2.0 * w); gz += GR[6] * (2.0 * x);
    /* R21 = 2(yz + wx) */
    gw += GR[7] * (2.0 * x); gx += GR[7] * (2.0 * w); gy += GR[7] * (2.0 * z); gz += GR[7] * (2.0 * y);
    /* R22 = 1 - 2(x^2 + y^2) */
    gx += GR[8] * (-4.0 * x); gy += GR[8] * (-4.0 * y);
    /* q_hat = q / |q|:  dq = (g - q_hat (q_hat . g)) / |q| */
    double dot = w * gw + x * gx + y * gy + z * gz;
    double inv = 1.0 / p->qnorm;
    gq[0 * N + i] += (gw - w * dot) * inv;
    gq[1 * N + i] += (gx - x * dot) * inv;
    gq[2 * N + i] += (gy - y * dot) * inv;
    gq[3 * N + i] += (gz - z * dot) * inv;
}

/* Gradient of sum_p sum_ch gimg_ch(p) * image_ch(p) for one camera, added
 * into gm (3N), gls (3N), gq (4N), go (N), gc (3N).  gimg: planar
 * r, g, b, depth, alpha, uncertainty (6 x H x W); a NULL plane means zero.
 * Optional g2d (N x 10) receives the screen-space gradients; optional
 * touched (N) is set to 1 for the Gaussians that may contribute at a pixel
 * holding a near-threshold decision, i.e. within the relative bands ev_a of
 * alpha_min or ev_t of T_min (never cleared here). */
int rtgo_adjoint(int64_t n, const double *means, const double *ls, const double *q,
                 const double *o, const double *colors, const double *unc,
                 const double *cam, const double *set, int tw, int th,
                 const double *g_rgb, const double *g_depth, const double *g_alpha,
                 const double *g_unc, double *gm, double *gls, double *gq, double *go,
                 double *gc, double *g2d, int32_t *touched, double ev_a, double ev_t)
{
    ogauss g;
    gauss_from(&g, n, means, ls, q, o, colors, unc);
    oview V;
    if (view_setup(&V, &g, cam, set)) return -1;
    V.ev_a = ev_a;
    V.ev_t = ev_t;
    otiles T;
    if (tiles_build(&V, tw, th, &T)) return -1;
    int W = V.c.w, H = V.c.h;
    int64_t P = (int64_t)W * H;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nth * (size_t)(n > 0 ? n : 1) * O2D, sizeof(double));
    if (!acc) return -1;
    int64_t maxlen = 0;
    int64_t nt = (int64_t)T.ntx * T.nty;
    for (int64_t t = 0; t < nt; t++)
        if (T.start[t + 1] - T.start[t] > maxlen) maxlen = T.start[t + 1] - T.start[t];
#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = acc + (size_t)tid * (size_t)n * O2D;
        ocontrib *buf = (ocontrib *)malloc(sizeof(ocontrib) * (size_t)(maxlen > 0 ? maxlen : 1));
#pragma omp for schedule(static)
        for (int64_t pix = 0; pix < P; pix++) {
            int u = (int)(pix % W), v = (int)(pix / W);
            double g6[6];
            g6[0] = g_rgb ? g_rgb[pix] : 0.0;
            g6[1] = g_rgb ? g_rgb[P + pix] : 0.0;
            g6[2] = g_rgb ? g_rgb[2 * P + pix] : 0.0;
            g6[3] = g_depth ? g_depth[pix] : 0.0;
            g6[4] = g_alpha ? g_alpha[pix] : 0.0;
            g6[5] = g_unc ? g_unc[pix] : 0.0;
            if (g6[0] == 0.0 && g6[1] == 0.0 && g6[2] == 0.0 && g6[3] == 0.0 && g6[4] == 0.0 && g6[5] == 0.0)
                continue;
            int64_t t = (int64_t)(v / th) * T.ntx + u / tw;
            pixel_adjoint(&V, T.items + T.start[t], T.start[t + 1] - T.start[t], u, v, g6, mine, buf, touched);
        }
        free(buf);
    }
    /* fixed-order reduction of the per-thread screen-space gradients */
    for (int tid = 1; tid < nth; tid++) {
        double *src = acc + (size_t)tid * (size_t)n * O2D;
        for (int64_t k = 0; k < n * O2D; k++) acc[k] += src[k];
    }
    if (g2d)
        for (int64_t k = 0; k < n * O2D; k++) g2d[k] = acc[k];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        if (!V.P[i].valid) continue;
        project_adjoint(&V, i, acc + (size_t)i * O2D, gm, gls, gq, go, gc);
    }
    free(acc);
    tiles_free(&T);
    view_free(&V);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Paper-literal view utility (Sec. IV-B eq. (8), thresholds of Sec. IV-C)  */
/* ------------------------------------------------------------------------ */

/* Thresholds for the high / low uncertainty sets: mean(u) -/+ k std(u)
 * (population standard deviation), summed in index order. */
void rtgo_thresholds(int64_t n, const double *u, double k, double *lo, double *hi)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += u[i];
    double mean = n > 0 ? s / (double)n : 0.0;
    double ss = 0.0;
    for (int64_t i = 0; i < n; i++) ss += (u[i] - mean) * (u[i] - mean);
    double sd = n > 0 ? sqrt(ss / (double)n) : 0.0;
    *lo = mean - k * sd;
    *hi = mean + k * sd;
}

/* Binary visibility v(x, g) of Sec. IV-B: the Gaussian's mean is in the
 * camera's field of view - camera depth in (z_near, range] (the perception
 * range; no occlusion test) and projected mean inside the image,
 * 0 <= mu_2D,x <= W - 1 and 0 <= mu_2D,y <= H - 1 (pixel-centre convention). */
static int fov_visible(const double *mu, const ocam *c, double z_near, double range)
{
    if (!isfinite(mu[0]) || !isfinite(mu[1]) || !isfinite(mu[2])) return 0;
    double dx = mu[0] - c->T[0], dy = mu[1] - c->T[1], dz = mu[2] - c->T[2];
    const double *R = c->R;
    double tx = (dx * R[0] + dy * R[3]) + dz * R[6];
    double ty = (dx * R[1] + dy * R[4]) + dz * R[7];
    double tz = (dx * R[2] + dy * R[5]) + dz * R[8];
    if (!(tz > z_near) || !(tz <= range)) return 0;
    double mx = c->fx * tx / tz + c->cx;
    double my = c->fy * ty / tz + c->cy;
    return mx >= 0.0 && mx <= (double)(c->w - 1) && my >= 0.0 && my <= (double)(c->h - 1);
}

/* For each of nv cameras: n_high = |{g in FOV : u_g > hi}|, n_low = |{g in
 * FOV : u_g < lo}|, sum_u = sum of u_g over the FOV (the "-sum" variant of
 * Sec. V-A), xi = n_high - lambda n_low (eq. (8)). */
int rtgo_view_utility(int64_t n, const double *means, const double *u, const double *cams, int nv,
                      double z_near, double range, double lo, double hi, double lambda,
                      int64_t *n_high, int64_t *n_low, double *sum_u, double *xi)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < nv; v++) {
        ocam c;
        read_cam(cams + 18 * v, &c);
        int64_t nh = 0, nl = 0;
        double su = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double mu[3] = {means[i], means[n + i], means[2 * n + i]};
            if (!fov_visible(mu, &c, z_near, range)) continue;
            if (u[i] > hi) nh++;
            if (u[i] < lo) nl++;
            su += u[i];
        }
        n_high[v] = nh;
        n_low[v] = nl;
        sum_u[v] = su;
        xi[v] = (double)nh - lambda * (double)nl;
    }
    return 0;
}

/* Trajectory selection of Sec. IV-B eq. (10): trajectory t is evaluated by
 * the sum of the view utilities xi of its states x_t(l tau / L), l = 0..L,
 * which are xi[off[t]] .. xi[off[t+1] - 1] here (summed in that order), and
 * the trajectory of highest total is chosen; among equal totals the first.
 * util (nullable) receives every total.  Returns the chosen index, -1 when
 * n_traj < 1. */
int rtgo_traj_select(int n_traj, const double *xi, const int32_t *off, double *util)
{
    int best = -1;
    double best_val = 0.0;
    for (int t = 0; t < n_traj; t++) {
        double total = 0.0;
        for (int32_t l = off[t]; l < off[t + 1]; l++) total += xi[l];
        if (util) util[t] = total;
        if (best < 0 || total > best_val) {
            best = t;
            best_val = total;
        }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Uncertainty bookkeeping and region utility (Sec. IV-A, IV-B, IV-C)      */
/* ------------------------------------------------------------------------ */

/* Per-Gaussian uncertainty after a map update: the magnitude of the change
 * of its mean, ||mu_k - mu_{k-1}||_2 (squared when `squared`, the -sq
 * variant of Sec. V-A); a Gaussian whose mean did not change in this update
 * (all three components equal) keeps its previous value u_prev.  Means are
 * planar 3 x n.  The displacement is formed in binary64 as
 * sqrt((dx dx + dy dy) + dz dz) and returned in binary64 (callers round). */
void rtgo_uncertainty_update(int64_t n, const double *prev, const double *cur, const double *u_prev,
                             int squared, double *u_out)
{
    for (int64_t i = 0; i < n; i++) {
        double dx = cur[i] - prev[i];
        double dy = cur[n + i] - prev[n + i];
        double dz = cur[2 * n + i] - prev[2 * n + i];
        if (dx == 0.0 && dy == 0.0 && dz == 0.0) {
            u_out[i] = u_prev[i];
            continue;
        }
        double s2 = (dx * dx + dy * dy) + dz * dz;
        u_out[i] = squared ? s2 : sqrt(s2);
    }
}

/* Grid of the region utility of Sec. IV-B (size from Sec. IV-C): the enclosing box [lo, hi)
 * (box = lo xyz, hi xyz) is partitioned into cuboids of edge `size`,
 * dims[a] = ceil((hi_a - lo_a) / size) per axis. */
int rtgo_region_grid(const double *box, double size, int *dims)
{
    if (!(size > 0.0)) return -1;
    for (int a = 0; a < 3; a++) {
        double e = (box[3 + a] - box[a]) / size;
        if (!(e > 0.0) || e > 1e6) return -1;
        dims[a] = (int)ceil(e);
    }
    return 0;
}

/* Region utility Omega_k of Sec. IV-B (high-level planner; the 2.5 m size is
 * set in Sec. IV-C): region (ix, iy, iz), index ix + nx (iy + ny iz),
 * holds the Gaussians whose mean lies in [lo + i size, lo + (i + 1) size) on
 * every axis (i = floor((mu_a - lo_a) / size) evaluated in binary64); means
 * outside the grid belong to no region.  count = M_k, sum = sum of u over the
 * region (index order), mean = Omega_k = sum / M_k (0 for an empty region). */
int rtgo_region_utility(int64_t n, const double *means, const double *u, const double *box, double size,
                        int64_t *count, double *sum, double *mean)
{
    int d[3];
    if (rtgo_region_grid(box, size, d)) return -1;
    int64_t nr = (int64_t)d[0] * d[1] * d[2];
    for (int64_t r = 0; r < nr; r++) {
        count[r] = 0;
        sum[r] = 0.0;
    }
    for (int64_t i = 0; i < n; i++) {
        int idx[3], inside = 1;
        for (int a = 0; a < 3; a++) {
            double f = floor((means[(int64_t)a * n + i] - box[a]) / size);
            if (!(f >= 0.0) || !(f < (double)d[a])) { inside = 0; break; }
            idx[a] = (int)f;
        }
        if (!inside) continue;
        int64_t r = idx[0] + (int64_t)d[0] * (idx[1] + (int64_t)d[1] * idx[2]);
        count[r]++;
        sum[r] += u[i];
    }
    for (int64_t r = 0; r < nr; r++) mean[r] = count[r] ? sum[r] / (double)count[r] : 0.0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Collision checking (Sec. IV-B, trajectory planner, Collision Checking)   */
/* ------------------------------------------------------------------------ */

/* Each test point is a sphere of radius r_robot; each Gaussian's radius is
 * its principal axis r_i = exp(max_k log_scale_k), scaled by lambda_g.  The
 * point collides when its distance to some Gaussian's mean is below
 * gamma_i = r_robot + lambda_g r_i, decided in binary64 as
 * (dx^2 + dy^2) + dz^2 < gamma_i^2.  clearance = min_i (||p - mu_i|| -
 * lambda_g r_i), so the point collides exactly when clearance < r_robot.
 * Gaussians with non-finite mean or log-scales are ignored; with none left,
 * clearance = +inf.  points and means planar (3 x n_points, 3 x n). */
void rtgo_collision(int64_t n, const double *means, const double *ls, int64_t np, const double *pts,
                    double r_robot, double lambda_g, int32_t *collide, double *clearance)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < np; j++) {
        double px = pts[j], py = pts[np + j], pz = pts[2 * np + j];
        int hit = 0;
        double best = INFINITY;
        for (int64_t i = 0; i < n; i++) {
            double mx = means[i], my = means[n + i], mz = means[2 * n + i];
            double l0 = ls[i], l1 = ls[n + i], l2 = ls[2 * n + i];
            if (!isfinite(mx) || !isfinite(my) || !isfinite(mz) || !isfinite(l0) || !isfinite(l1) ||
                !isfinite(l2))
                continue;
            double lm = l0 > l1 ? l0 : l1;
            lm = lm > l2 ? lm : l2;
            double r = exp(lm);
            double dx = px - mx, dy = py - my, dz = pz - mz;
            double d2 = (dx * dx + dy * dy) + dz * dz;
            double g = r_robot + lambda_g * r;
            if (d2 < g * g) hit = 1;
            double c = sqrt(d2) - lambda_g * r;
            if (c < best) best = c;
        }
        collide[j] = hit;
        clearance[j] = best;
    }
}
