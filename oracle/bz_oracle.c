/*
 * bz_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of the Bezier Splatting
 * rasterizer ("Bezier Splatting for Fast and Differentiable Vector Graphics
 * Rendering", arXiv 2503.16424).  It exists to check the HIP library; nothing
 * in the product path links, loads or calls it.  It shares no code, header,
 * table or constant with the HIP sources.
 *
 * What it computes, in the paper's order:
 *   sampling   Sec. 3.3: Bernstein form of a cubic (Eq. bezier / bezier1), K
 *              uniform parameters per row (Eq. sampling), the paired closed
 *              structure with R interpolated rows (Eq. for P^(k)_j and
 *              B^interp), scales from neighbour distances (Eq. sigma) and the
 *              tangent angle (Eq. rotation);
 *   forward    Sec. 3.4: alpha = o exp(-1/2 d^T Sigma^-1 d) (Eq. rasterization2),
 *              Sigma = (RS)(RS)^T (Eq. RSSR / rot_scale), front-to-back
 *              alpha blending C = sum c_i alpha_i prod_{j<i}(1-alpha_j);
 *   backward   the derivative of that forward pass, pixel by pixel in reverse
 *              contributor order, then the chain rule through the sampling
 *              to control points, stroke widths, colours and opacities.
 *
 * Readings where the paper is silent (all are plain parameters here):
 *   cubic segments (M = 3); global parameter u_k = k/(K-1) across the S
 *   segments of a composite curve, segment index floor(kS/(K-1)) capped at
 *   S-1 computed in integers; sigma^2 = |Delta|^2/rho^2 + sigma0^2 (isotropic
 *   dilation keeps the closed-curve endpoints, where neighbouring rows meet,
 *   non-singular); forward/backward differences at the last column / row;
 *   unit tangent (1,0) for a zero-length neighbour chord (atan2(0,0) = 0);
 *   truncated kernel Gt = (G - g_min)_+ / (1 - g_min); alpha clamped at
 *   alpha_max; a pixel stops after the contributor that brings T below T_min
 *   (the contributor is included); background composited with T_final; pixel
 *   (x, y) has its centre at (x + 1/2, y + 1/2).
 *
 * Culling: a Gaussian can only reach pixels whose centre lies in the support
 * ellipse 1/2 d^T Q d <= -ln(g_min), whose axis-aligned bounding box has
 * half-extents sqrt(-2 ln(g_min) Sigma_xx), sqrt(-2 ln(g_min) Sigma_yy).  Pixels
 * outside the box (padded) have G <= g_min and contribute exactly zero, so
 * skipping them changes nothing.  The `brute` flag disables the culling.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_MEM (-2)

/* ------------------------------------------------------------------------ */
/* Curve geometry (Sec. 3.2-3.3)                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int kind;          /* 0 open, 1 closed */
    int S, K, R;       /* segments, samples per row, interior rows */
    const double *P;   /* control points, [n_ctrl][2] */
    const double *tau; /* R+2 interpolation weights */
} curve_t;

/* Cubic Bernstein basis B_j^3(t), Eq. bezier1 with M = 3. */
static void bernstein3(double t, double B[4]) {
    double u = 1.0 - t;
    B[0] = u * u * u;
    B[1] = 3.0 * u * u * t;
    B[2] = 3.0 * u * t * t;
    B[3] = t * t * t;
}

/* Column k of a row: segment s and local parameter t (u_k = k/(K-1) spread
 * over S segments; integer arithmetic decides the segment). */
static void column_param(int k, int K, int S, int *s_out, double *t_out) {
    int s = (k * S) / (K - 1);
    if (s > S - 1) s = S - 1;
    *s_out = s;
    *t_out = (double)(k * S - s * (K - 1)) / (double)(K - 1);
}

/* Control point j (0..3S) of row r.  Open: the stroke's own points.  Closed:
 * boundary A is row 0, boundary B (sharing A's first and last point) is row
 * R+1, row r interpolates the control points with weight tau_r (Sec. 3.3). */
static void row_ctrl(const curve_t *c, int r, int j, double out[2]) {
    int m = 3 * c->S;
    if (c->kind == 0) {
        out[0] = c->P[2 * j];
        out[1] = c->P[2 * j + 1];
        return;
    }
    double ax = c->P[2 * j], ay = c->P[2 * j + 1];
    double bx, by;
    if (j == 0 || j == m) {
        bx = ax;
        by = ay;
    } else {
        bx = c->P[2 * (m + j)];       /* B interior points follow A's m+1 points */
        by = c->P[2 * (m + j) + 1];
    }
    double t = c->tau[r];
    out[0] = (1.0 - t) * ax + t * bx;
    out[1] = (1.0 - t) * ay + t * by;
}

/* Sample point X_{r,k} (Eq. bezier evaluated at the row's control points). */
static void sample_point(const curve_t *c, int r, int k, double X[2]) {
    int s;
    double t, B[4];
    column_param(k, c->K, c->S, &s, &t);
    bernstein3(t, B);
    X[0] = 0.0;
    X[1] = 0.0;
    for (int j = 0; j < 4; ++j) {
        double p[2];
        row_ctrl(c, r, 3 * s + j, p);
        X[0] += B[j] * p[0];
        X[1] += B[j] * p[1];
    }
}

static int rows_of(const curve_t *c) { return c->kind == 1 ? c->R + 2 : 1; }

/* Per-Gaussian geometry: mean, squared scales (dilated), unit tangent. */
typedef struct {
    double mu[2];
    double sx2, sy2;
    double cs, sn;       /* unit tangent (cos theta, sin theta) */
    double delta[2];     /* along-row neighbour difference */
    double delta_y[2];   /* across-row neighbour difference (closed) */
    double v[2];         /* central difference used for the tangent */
    int ka, kb;          /* delta = X[r][ka] - X[r][kb] */
    int ra, rb;          /* delta_y = X[ra][k] - X[rb][k] */
    int kp, km;          /* v = X[r][kp] - X[r][km] */
    int seg;             /* segment of column k */
} geom_t;

static void gaussian_geom(const curve_t *c, double width, int r, int k, double rho,
                          double sigma0_sq, geom_t *g) {
    int K = c->K;
    double X[2], A[2], B[2];
    double t;
    column_param(k, K, c->S, &g->seg, &t);
    sample_point(c, r, k, X);
    g->mu[0] = X[0];
    g->mu[1] = X[1];
    /* Eq. sigma, x: distance to the next point along the row; the last
     * column uses the previous point (nearest available neighbour). */
    if (k < K - 1) { g->ka = k + 1; g->kb = k; } else { g->ka = K - 1; g->kb = K - 2; }
    sample_point(c, r, g->ka, A);
    sample_point(c, r, g->kb, B);
    g->delta[0] = A[0] - B[0];
    g->delta[1] = A[1] - B[1];
    g->sx2 = (g->delta[0] * g->delta[0] + g->delta[1] * g->delta[1]) / (rho * rho) + sigma0_sq;
    /* Eq. sigma, y: distance to the same column of the next row (closed);
     * the stroke width for open curves. */
    if (c->kind == 1) {
        int R1 = c->R + 1;
        if (r < R1) { g->ra = r + 1; g->rb = r; } else { g->ra = R1; g->rb = R1 - 1; }
        sample_point(c, g->ra, k, A);
        sample_point(c, g->rb, k, B);
        g->delta_y[0] = A[0] - B[0];
        g->delta_y[1] = A[1] - B[1];
        g->sy2 = (g->delta_y[0] * g->delta_y[0] + g->delta_y[1] * g->delta_y[1]) / (rho * rho)
                 + sigma0_sq;
    } else {
        g->ra = g->rb = 0;
        g->delta_y[0] = g->delta_y[1] = 0.0;
        g->sy2 = width * width + sigma0_sq;
    }
    /* Eq. rotation: angle of X_{k+1} - X_{k-1}, one-sided at the ends. */
    g->kp = k + 1 < K ? k + 1 : K - 1;
    g->km = k - 1 >= 0 ? k - 1 : 0;
    sample_point(c, r, g->kp, A);
    sample_point(c, r, g->km, B);
    g->v[0] = A[0] - B[0];
    g->v[1] = A[1] - B[1];
    double nv = sqrt(g->v[0] * g->v[0] + g->v[1] * g->v[1]);
    if (nv > 0.0) {
        g->cs = g->v[0] / nv;
        g->sn = g->v[1] / nv;
    } else {
        g->cs = 1.0;
        g->sn = 0.0;
    }
}

/* Q = Sigma^-1 = R diag(1/sx2, 1/sy2) R^T (Eq. RSSR, rot_scale). */
static void conic_of(const geom_t *g, double Q[3]) {
    double a = 1.0 / g->sx2, b = 1.0 / g->sy2;
    Q[0] = g->cs * g->cs * a + g->sn * g->sn * b;
    Q[1] = g->cs * g->sn * (a - b);
    Q[2] = g->sn * g->sn * a + g->cs * g->cs * b;
}

static void load_curve(int i, const int32_t *kind, const int32_t *nseg, const int32_t *ks,
                       const int32_t *rs, const double *ctrl, const int32_t *ctrl_off,
                       const double *tau, const int32_t *tau_off, curve_t *c) {
    c->kind = kind[i];
    c->S = nseg[i];
    c->K = ks[i];
    c->R = c->kind == 1 ? rs[i] : 0;
    c->P = ctrl + 2 * (int64_t)ctrl_off[i];
    c->tau = tau + tau_off[i];
}

static int check_curves(int n, const int32_t *kind, const int32_t *nseg, const int32_t *ks,
                        const int32_t *rs, const int32_t *ctrl_off, const int32_t *tau_off,
                        const int32_t *opa_off, const int32_t *rank) {
    char *seen = (char *)calloc(n > 0 ? n : 1, 1);
    if (!seen) return ORC_ERR_MEM;
    int bad = 0;
    for (int i = 0; i < n && !bad; ++i) {
        int S = nseg[i], K = ks[i], R = kind[i] == 1 ? rs[i] : 0;
        int need_ctrl = kind[i] == 1 ? 6 * S : 3 * S + 1;
        int nopa = opa_off[i + 1] - opa_off[i];
        if ((kind[i] != 0 && kind[i] != 1) || S < 1 || K < 2 || R < 0) bad = 1;
        else if (ctrl_off[i + 1] - ctrl_off[i] != need_ctrl) bad = 1;
        else if (tau_off[i + 1] - tau_off[i] < R + 2) bad = 1;
        else if (nopa != 1 && nopa != S) bad = 1;
        else if (rank[i] < 0 || rank[i] >= n || seen[rank[i]]) bad = 1;
        else seen[rank[i]] = 1;
    }
    free(seen);
    return bad ? ORC_ERR_ARG : ORC_OK;
}

/* Number of Gaussians of the scene. */
int64_t orc_count_gaussians(int n, const int32_t *kind, const int32_t *ks, const int32_t *rs) {
    int64_t t = 0;
    for (int i = 0; i < n; ++i) t += (int64_t)ks[i] * (kind[i] == 1 ? rs[i] + 2 : 1);
    return t;
}

/*
 * Sampling.  Gaussians are emitted in draw order: curves by ascending rank
 * (rank 0 is drawn in front), then row-major (r, k) inside a curve.
 * Outputs, each of length n_gauss (= orc_count_gaussians):
 *   mu[2], conic[3] = (Qxx, Qxy, Qyy), sx2, sy2, tangent[2], opac, color[3],
 *   curve id, row r, column k, opacity slot (index into the curve's opacities).
 */
int orc_sample(int n, const int32_t *kind, const int32_t *nseg, const int32_t *ks,
               const int32_t *rs, const double *ctrl, const int32_t *ctrl_off, const double *tau,
               const int32_t *tau_off, const double *stroke_w, const double *color,
               const double *opacity, const int32_t *opa_off, const int32_t *rank, double rho,
               double sigma0_sq, double *mu, double *conic, double *sx2, double *sy2,
               double *tangent, double *opac, double *col_out, int32_t *curve_out,
               int32_t *row_out, int32_t *colk_out, int32_t *slot_out) {
    if (n < 0 || !(rho > 0.0) || !(sigma0_sq >= 0.0)) return ORC_ERR_ARG;
    int st = check_curves(n, kind, nseg, ks, rs, ctrl_off, tau_off, opa_off, rank);
    if (st) return st;
    int32_t *by_rank = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    if (!by_rank || !start) { free(by_rank); free(start); return ORC_ERR_MEM; }
    for (int i = 0; i < n; ++i) by_rank[rank[i]] = i;
    start[0] = 0;
    for (int p = 0; p < n; ++p) {
        int i = by_rank[p];
        start[p + 1] = start[p] + (int64_t)ks[i] * (kind[i] == 1 ? rs[i] + 2 : 1);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int p = 0; p < n; ++p) {
        int i = by_rank[p];
        curve_t c;
        load_curve(i, kind, nseg, ks, rs, ctrl, ctrl_off, tau, tau_off, &c);
        int nopa = opa_off[i + 1] - opa_off[i];
        int64_t g = start[p];
        for (int r = 0; r < rows_of(&c); ++r) {
            for (int k = 0; k < c.K; ++k, ++g) {
                geom_t ge;
                gaussian_geom(&c, stroke_w[i], r, k, rho, sigma0_sq, &ge);
                double Q[3];
                conic_of(&ge, Q);
                mu[2 * g] = ge.mu[0];
                mu[2 * g + 1] = ge.mu[1];
                conic[3 * g] = Q[0];
                conic[3 * g + 1] = Q[1];
                conic[3 * g + 2] = Q[2];
                if (sx2) sx2[g] = ge.sx2;
                if (sy2) sy2[g] = ge.sy2;
                if (tangent) { tangent[2 * g] = ge.cs; tangent[2 * g + 1] = ge.sn; }
                int slot = nopa == c.S ? ge.seg : 0;
                opac[g] = opacity[opa_off[i] + slot];
                for (int ch = 0; ch < 3; ++ch) col_out[3 * g + ch] = color[3 * i + ch];
                if (curve_out) curve_out[g] = i;
                if (row_out) row_out[g] = r;
                if (colk_out) colk_out[g] = k;
                if (slot_out) slot_out[g] = slot;
            }
        }
    }
    free(by_rank);
    free(start);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Forward and backward blending (Sec. 3.4)                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    const double *mu, *conic, *opac, *color;
    int W, H;
    double bg[3];
    double g_min, alpha_max, t_min;
    int brute;
    /* per-Gaussian pixel ranges (inclusive), from the support bounding box */
    int32_t *x0, *x1, *y0, *y1;
} blend_t;

/* Support bounding box in pixel indices.  Sigma = Q^-1; the ellipse
 * 1/2 d^T Q d <= P has half-extents sqrt(2 P Sigma_xx), sqrt(2 P Sigma_yy).
 * Padded by one pixel: the box only needs to contain the support. */
static int setup_ranges(blend_t *b) {
    int64_t n = b->n;
    b->x0 = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    b->x1 = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    b->y0 = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    b->y1 = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    if (!b->x0 || !b->x1 || !b->y0 || !b->y1) return ORC_ERR_MEM;
    double P = -log(b->g_min);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        if (b->brute) {
            b->x0[g] = 0; b->x1[g] = b->W - 1; b->y0[g] = 0; b->y1[g] = b->H - 1;
            continue;
        }
        double qa = b->conic[3 * g], qb = b->conic[3 * g + 1], qc = b->conic[3 * g + 2];
        double det = qa * qc - qb * qb;
        double mx = b->mu[2 * g], my = b->mu[2 * g + 1];
        int ok = det > 0.0 && qa > 0.0 && isfinite(mx) && isfinite(my) && isfinite(det);
        if (!ok) { b->x0[g] = 1; b->x1[g] = 0; b->y0[g] = 1; b->y1[g] = 0; continue; }
        double hx = sqrt(2.0 * P * qc / det), hy = sqrt(2.0 * P * qa / det);
        /* pixel x has centre x + 1/2 */
        double fx0 = floor(mx - hx - 0.5) - 1.0, fx1 = ceil(mx + hx - 0.5) + 1.0;
        double fy0 = floor(my - hy - 0.5) - 1.0, fy1 = ceil(my + hy - 0.5) + 1.0;
        if (fx0 < 0) fx0 = 0;
        if (fy0 < 0) fy0 = 0;
        if (fx1 > b->W - 1) fx1 = b->W - 1;
        if (fy1 > b->H - 1) fy1 = b->H - 1;
        if (fx0 > fx1 || fy0 > fy1) { b->x0[g] = 1; b->x1[g] = 0; b->y0[g] = 1; b->y1[g] = 0; continue; }
        b->x0[g] = (int32_t)fx0; b->x1[g] = (int32_t)fx1;
        b->y0[g] = (int32_t)fy0; b->y1[g] = (int32_t)fy1;
    }
    return ORC_OK;
}

static void free_ranges(blend_t *b) {
    free(b->x0); free(b->x1); free(b->y0); free(b->y1);
}

/* One contributor of one pixel, as the reverse pass needs it. */
typedef struct {
    int64_t g;
    double alpha, G, T_before, dx, dy;
    int clamped;
} contrib_t;

typedef struct {
    double T, C[3];
    int done;
    int32_t n;          /* contributors so far */
    contrib_t *list;    /* only kept when the reverse pass needs it */
    int32_t cap;
    double margin;      /* smallest relative distance of a decision to its threshold */
} pix_t;

/* Relative distance of v from the threshold t of a comparison (|v - t| / t). */
static double rel_margin(double v, double t) {
    return fabs(v - t) / t;
}

/* Evaluate Gaussian g at pixel (x, y) and composite it (one step of the
 * front-to-back loop).  Returns 1 when the Gaussian contributed. */
static int blend_step(const blend_t *b, pix_t *px, int64_t g, int x, int y, int keep) {
    if (px->done) return 0;
    double dx = (x + 0.5) - b->mu[2 * g];
    double dy = (y + 0.5) - b->mu[2 * g + 1];
    const double *Q = b->conic + 3 * g;
    double p = 0.5 * (Q[0] * dx * dx + 2.0 * Q[1] * dx * dy + Q[2] * dy * dy);
    double G = exp(-p);
    /* decision margins: the support test G > g_min, the clamp a_raw > alpha_max
       and the stop T < t_min, each as a relative distance to its threshold */
    double m = rel_margin(G, b->g_min);
    if (m < px->margin) px->margin = m;
    if (!(G > b->g_min)) return 0;                          /* outside the truncated support */
    double a_raw = b->opac[g] * (G - b->g_min) / (1.0 - b->g_min);
    m = rel_margin(a_raw, b->alpha_max);
    if (m < px->margin) px->margin = m;
    int clamped = a_raw > b->alpha_max;
    double alpha = clamped ? b->alpha_max : a_raw;
    if (keep) {
        if (px->n == px->cap) {
            int32_t nc = px->cap ? 2 * px->cap : 16;
            contrib_t *nl = (contrib_t *)realloc(px->list, sizeof(contrib_t) * nc);
            if (!nl) abort();
            px->list = nl;
            px->cap = nc;
        }
        contrib_t *e = &px->list[px->n];
        e->g = g; e->alpha = alpha; e->G = G; e->T_before = px->T;
        e->dx = dx; e->dy = dy; e->clamped = clamped;
    }
    for (int ch = 0; ch < 3; ++ch) px->C[ch] += alpha * px->T * b->color[3 * g + ch];
    px->T = px->T * (1.0 - alpha);
    px->n += 1;
    if (b->t_min > 0.0) {
        m = rel_margin(px->T, b->t_min);
        if (m < px->margin) px->margin = m;
    }
    if (px->T < b->t_min) px->done = 1;                     /* include, then stop */
    return 1;
}

/* Candidate Gaussians of row y, in draw order (CSR over rows). */
typedef struct {
    int64_t *start;   /* [H+1] */
    int64_t *ids;
} rows_t;

static int build_rows(const blend_t *b, int ya, int yb, rows_t *rw) {
    int H = b->H;
    rw->start = (int64_t *)calloc(H + 2, sizeof(int64_t));
    if (!rw->start) return ORC_ERR_MEM;
    for (int64_t g = 0; g < b->n; ++g) {
        int lo = b->y0[g] > ya ? b->y0[g] : ya, hi = b->y1[g] < yb - 1 ? b->y1[g] : yb - 1;
        for (int y = lo; y <= hi; ++y) rw->start[y + 1]++;
    }
    for (int y = 0; y <= H; ++y) rw->start[y + 1] += rw->start[y];
    rw->ids = (int64_t *)malloc(sizeof(int64_t) * (rw->start[H] > 0 ? rw->start[H] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (H + 1));
    if (!rw->ids || !fill) { free(fill); return ORC_ERR_MEM; }
    memcpy(fill, rw->start, sizeof(int64_t) * (H + 1));
    for (int64_t g = 0; g < b->n; ++g) {
        int lo = b->y0[g] > ya ? b->y0[g] : ya, hi = b->y1[g] < yb - 1 ? b->y1[g] : yb - 1;
        for (int y = lo; y <= hi; ++y) rw->ids[fill[y]++] = g;
    }
    free(fill);
    return ORC_OK;
}

/* Backward of one pixel: walk its contributors last to first.
 * A is the normalised colour composited behind the current contributor,
 * starting at the background; dC/dalpha_i = T_i (c_i - A_i). */
static void pixel_backward(const blend_t *b, const pix_t *px, const double gbar[3],
                           double *dg /* [n][9] */) {
    double A[3] = {b->bg[0], b->bg[1], b->bg[2]};
    for (int32_t i = px->n - 1; i >= 0; --i) {
        const contrib_t *e = &px->list[i];
        int64_t g = e->g;
        const double *c = b->color + 3 * g;
        double *o = dg + 9 * g;
        double abar = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            o[6 + ch] += e->alpha * e->T_before * gbar[ch];
            abar += e->T_before * (c[ch] - A[ch]) * gbar[ch];
        }
        for (int ch = 0; ch < 3; ++ch) A[ch] = e->alpha * c[ch] + (1.0 - e->alpha) * A[ch];
        if (e->clamped) continue;                             /* alpha = alpha_max: flat */
        double scale = 1.0 / (1.0 - b->g_min);
        o[5] += abar * (e->G - b->g_min) * scale;             /* d alpha / d o */
        double pbar = -abar * b->opac[g] * e->G * scale;      /* d alpha / d p */
        const double *Q = b->conic + 3 * g;
        /* p = 1/2 (Qxx dx^2 + 2 Qxy dx dy + Qyy dy^2), d = q - mu */
        o[0] += -pbar * (Q[0] * e->dx + Q[1] * e->dy);
        o[1] += -pbar * (Q[1] * e->dx + Q[2] * e->dy);
        o[2] += pbar * 0.5 * e->dx * e->dx;
        o[3] += pbar * e->dx * e->dy;
        o[4] += pbar * 0.5 * e->dy * e->dy;
    }
}

static void setup_blend(blend_t *b, int64_t n, const double *mu, const double *conic,
                        const double *opac, const double *color, int W, int H, const double *bg,
                        double g_min, double alpha_max, double t_min, int brute) {
    memset(b, 0, sizeof(*b));
    b->n = n; b->mu = mu; b->conic = conic; b->opac = opac; b->color = color;
    b->W = W; b->H = H;
    b->bg[0] = bg[0]; b->bg[1] = bg[1]; b->bg[2] = bg[2];
    b->g_min = g_min; b->alpha_max = alpha_max; b->t_min = t_min; b->brute = brute;
}

static int check_opts(int W, int H, double g_min, double alpha_max, double t_min) {
    if (W <= 0 || H <= 0) return ORC_ERR_ARG;
    if (!(g_min > 0.0 && g_min < 1.0)) return ORC_ERR_ARG;
    if (!(alpha_max > 0.0 && alpha_max <= 1.0)) return ORC_ERR_ARG;
    if (!(t_min >= 0.0 && t_min < 1.0)) return ORC_ERR_ARG;
    return ORC_OK;
}

/*
 * Forward render of rows [ya, yb) (pass 0, H for the whole frame), and, when
 * d_image is given, the backward pass of the same rows.
 *   image   [3][H][W]  (rows outside [ya, yb) untouched)
 *   t_final [H][W], n_contrib [H][W]
 *   d_gauss [n][9] accumulated: (mu_x, mu_y, Qxx, Qxy, Qyy, o, r, g, b)
 *   counters[0] = contributing (pixel, Gaussian) pairs, [1] = pairs inside the
 *   bounding boxes that were tested, [2] = pixels that terminated early.
 *   margin [H][W] (may be NULL): per pixel, the smallest relative distance
 *   |v - t| / t of any decision the pixel took to its threshold t: G > g_min
 *   (every tested pair), alpha_raw > alpha_max and T < t_min (contributors).
 *   A small margin marks a pixel where a lower-precision evaluation may take
 *   the other branch; the truncated kernel, the clamp and include-then-stop
 *   keep every such flip's effect on the image of the order of the margin
 *   (or at most t_min for the stop).
 */
int orc_render(int64_t n, const double *mu, const double *conic, const double *opac,
               const double *color, int W, int H, const double *bg, double g_min,
               double alpha_max, double t_min, int ya, int yb, int brute, double *image,
               double *t_final, int32_t *n_contrib, const double *d_image, double *d_gauss,
               int64_t *counters, double *margin) {
    int st = check_opts(W, H, g_min, alpha_max, t_min);
    if (st) return st;
    if (ya < 0) ya = 0;
    if (yb > H || yb <= 0) yb = H;
    blend_t b;
    setup_blend(&b, n, mu, conic, opac, color, W, H, bg, g_min, alpha_max, t_min, brute);
    st = setup_ranges(&b);
    if (st) { free_ranges(&b); return st; }
    rows_t rw = {0, 0};
    st = build_rows(&b, ya, yb, &rw);
    if (st) { free_ranges(&b); free(rw.start); free(rw.ids); return st; }
    int keep = d_image != NULL && d_gauss != NULL;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double **acc = NULL;
    if (keep) {
        acc = (double **)calloc(nthreads, sizeof(double *));
        for (int t = 0; t < nthreads; ++t) {
            acc[t] = (double *)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
            if (!acc[t]) abort();
        }
    }
    int64_t c0 = 0, c1 = 0, c2 = 0;
#pragma omp parallel reduction(+ : c0, c1, c2)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        pix_t *row = (pix_t *)calloc(W, sizeof(pix_t));
        if (!row) abort();
#pragma omp for schedule(dynamic, 1)
        for (int y = ya; y < yb; ++y) {
            for (int x = 0; x < W; ++x) {
                row[x].T = 1.0;
                row[x].C[0] = row[x].C[1] = row[x].C[2] = 0.0;
                row[x].done = 0;
                row[x].n = 0;
                row[x].margin = INFINITY;
            }
            /* Every pixel sees the row's candidates in draw order. */
            for (int64_t q = rw.start[y]; q < rw.start[y + 1]; ++q) {
                int64_t g = rw.ids[q];
                for (int x = b.x0[g]; x <= b.x1[g]; ++x) {
                    if (row[x].done) continue;
                    c1++;
                    c0 += blend_step(&b, &row[x], g, x, y, keep);
                }
            }
            for (int x = 0; x < W; ++x) {
                pix_t *px = &row[x];
                size_t pi = (size_t)y * W + x;
                for (int ch = 0; ch < 3; ++ch)
                    image[(size_t)ch * H * W + pi] = px->C[ch] + px->T * b.bg[ch];
                if (t_final) t_final[pi] = px->T;
                if (n_contrib) n_contrib[pi] = px->n;
                if (margin) margin[pi] = px->margin;
                c2 += px->done;
                if (keep) {
                    double gbar[3] = {d_image[pi], d_image[(size_t)H * W + pi],
                                      d_image[(size_t)2 * H * W + pi]};
                    pixel_backward(&b, px, gbar, acc[tid]);
                }
            }
        }
        for (int x = 0; x < W; ++x) free(row[x].list);
        free(row);
    }
    if (keep) {
        for (int t = 0; t < nthreads; ++t) {
            for (int64_t i = 0; i < 9 * n; ++i) d_gauss[i] += acc[t][i];
            free(acc[t]);
        }
        free(acc);
    }
    if (counters) { counters[0] = c0; counters[1] = c1; counters[2] = c2; }
    free(rw.start);
    free(rw.ids);
    free_ranges(&b);
    return ORC_OK;
}

/* Forward of an arbitrary list of pixels (each pixel scans every Gaussian,
 * culled by its bounding box).  Outputs per pixel: rgb[3], T, contributor count. */
int orc_render_pixels(int64_t n, const double *mu, const double *conic, const double *opac,
                      const double *color, int W, int H, const double *bg, double g_min,
                      double alpha_max, double t_min, int npix, const int32_t *px,
                      const int32_t *py, double *rgb, double *T, int32_t *ncontrib) {
    int st = check_opts(W, H, g_min, alpha_max, t_min);
    if (st) return st;
    blend_t b;
    setup_blend(&b, n, mu, conic, opac, color, W, H, bg, g_min, alpha_max, t_min, 0);
    st = setup_ranges(&b);
    if (st) { free_ranges(&b); return st; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < npix; ++i) {
        int x = px[i], y = py[i];
        pix_t p;
        memset(&p, 0, sizeof(p));
        p.T = 1.0;
        p.margin = INFINITY;
        if (x >= 0 && x < W && y >= 0 && y < H) {
            for (int64_t g = 0; g < n && !p.done; ++g) {
                if (x < b.x0[g] || x > b.x1[g] || y < b.y0[g] || y > b.y1[g]) continue;
                blend_step(&b, &p, g, x, y, 0);
            }
        }
        for (int ch = 0; ch < 3; ++ch) rgb[3 * i + ch] = p.C[ch] + p.T * b.bg[ch];
        T[i] = p.T;
        ncontrib[i] = p.n;
    }
    free_ranges(&b);
    return ORC_OK;
}

/*
 * Depth complexity per screen tile of tw x th pixels (row-major tiles):
 *   depth_contrib[t]: distinct curves with at least one Gaussian that
 *       contributes (G > g_min before the pixel stopped) to a pixel of tile t;
 *   depth_support[t]: distinct curves with at least one Gaussian whose support
 *       bounding box (the culling box of the forward pass) reaches tile t.
 * curve[g] is the curve index of Gaussian g (0 .. n_curves-1).  The forward
 * pass is re-run tile by tile, pixel by pixel in draw order.
 */
int orc_tile_depth(int64_t n, const double *mu, const double *conic, const double *opac,
                   const int32_t *curve, int n_curves, int W, int H, double g_min,
                   double alpha_max, double t_min, int tw, int th, int32_t *depth_contrib,
                   int32_t *depth_support) {
    int st = check_opts(W, H, g_min, alpha_max, t_min);
    if (st) return st;
    if (tw <= 0 || th <= 0 || n_curves < 0) return ORC_ERR_ARG;
    for (int64_t g = 0; g < n; ++g)
        if (curve[g] < 0 || curve[g] >= n_curves) return ORC_ERR_ARG;
    static const double no_color[3] = {0.0, 0.0, 0.0};
    blend_t b;
    setup_blend(&b, n, mu, conic, opac, no_color, W, H, no_color, g_min, alpha_max, t_min, 0);
    /* blend_step reads a colour per Gaussian: give it zeros */
    double *zeros = (double *)calloc((size_t)(n > 0 ? n : 1) * 3, sizeof(double));
    if (!zeros) return ORC_ERR_MEM;
    b.color = zeros;
    st = setup_ranges(&b);
    if (st) { free_ranges(&b); free(zeros); return st; }
    int tx_n = (W + tw - 1) / tw, ty_n = (H + th - 1) / th;
    /* candidates per tile row, in draw order */
    int64_t *start = (int64_t *)calloc(ty_n + 1, sizeof(int64_t));
    if (!start) { free_ranges(&b); free(zeros); return ORC_ERR_MEM; }
    for (int64_t g = 0; g < n; ++g)
        if (b.y0[g] <= b.y1[g] && b.x0[g] <= b.x1[g])
            for (int ty = b.y0[g] / th; ty <= b.y1[g] / th; ++ty) start[ty + 1]++;
    for (int ty = 0; ty < ty_n; ++ty) start[ty + 1] += start[ty];
    int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (start[ty_n] > 0 ? start[ty_n] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (ty_n + 1));
    if (!ids || !fill) {
        free(ids); free(fill); free(start); free_ranges(&b); free(zeros);
        return ORC_ERR_MEM;
    }
    memcpy(fill, start, sizeof(int64_t) * (ty_n + 1));
    for (int64_t g = 0; g < n; ++g)
        if (b.y0[g] <= b.y1[g] && b.x0[g] <= b.x1[g])
            for (int ty = b.y0[g] / th; ty <= b.y1[g] / th; ++ty) ids[fill[ty]++] = g;
    free(fill);
#pragma omp parallel
    {
        int32_t *seen_c = (int32_t *)malloc(sizeof(int32_t) * (n_curves > 0 ? n_curves : 1));
        int32_t *seen_s = (int32_t *)malloc(sizeof(int32_t) * (n_curves > 0 ? n_curves : 1));
        pix_t *px = (pix_t *)calloc((size_t)tw * th, sizeof(pix_t));
        if (!seen_c || !seen_s || !px) abort();
        for (int c = 0; c < n_curves; ++c) seen_c[c] = seen_s[c] = -1;
#pragma omp for schedule(dynamic, 1)
        for (int t = 0; t < tx_n * ty_n; ++t) {
            int ty = t / tx_n, tx = t - ty * tx_n;
            int xa = tx * tw, xb = xa + tw - 1, ya = ty * th, yb = ya + th - 1;
            if (xb > W - 1) xb = W - 1;
            if (yb > H - 1) yb = H - 1;
            for (int i = 0; i < tw * th; ++i) {
                px[i].T = 1.0;
                px[i].done = 0;
                px[i].n = 0;
                px[i].margin = INFINITY;
            }
            int32_t dc = 0, ds = 0;
            for (int64_t q = start[ty]; q < start[ty + 1]; ++q) {
                int64_t g = ids[q];
                if (b.x1[g] < xa || b.x0[g] > xb || b.y1[g] < ya || b.y0[g] > yb) continue;
                int c = curve[g];
                if (seen_s[c] != t) { seen_s[c] = t; ds++; }
                int x0 = b.x0[g] > xa ? b.x0[g] : xa, x1 = b.x1[g] < xb ? b.x1[g] : xb;
                int y0 = b.y0[g] > ya ? b.y0[g] : ya, y1 = b.y1[g] < yb ? b.y1[g] : yb;
                for (int y = y0; y <= y1; ++y)
                    for (int x = x0; x <= x1; ++x)
                        if (blend_step(&b, &px[(y - ya) * tw + (x - xa)], g, x, y, 0) &&
                            seen_c[c] != t) {
                            seen_c[c] = t;
                            dc++;
                        }
            }
            depth_contrib[t] = dc;
            depth_support[t] = ds;
        }
        free(seen_c);
        free(seen_s);
        free(px);
    }
    free(ids);
    free(start);
    free_ranges(&b);
    free(zeros);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Chain rule from per-Gaussian gradients to curve parameters               */
/* ------------------------------------------------------------------------ */

/*
 * d_gauss [n_gauss][9] in draw order (as produced by orc_render) ->
 *   d_ctrl [n_ctrl][2], d_width [n], d_color [n][3], d_opacity [n_opa].
 * Per Gaussian (r, k): Q(a = 1/sx2, b = 1/sy2, cos, sin) with
 *   Qxx = c^2 a + s^2 b, Qxy = c s (a - b), Qyy = s^2 a + c^2 b;
 * sx2 = |Delta|^2/rho^2 + s0, sy2 = |Delta_y|^2/rho^2 + s0 (closed) or
 * w^2 + s0 (open); (c, s) = v/|v|; mu = X_{r,k}.  The gradients of the sample
 * points X then flow to the control points through the Bernstein weights and
 * the row interpolation weights (1 - tau_r, tau_r).
 */
int orc_chain(int n, const int32_t *kind, const int32_t *nseg, const int32_t *ks,
              const int32_t *rs, const double *ctrl, const int32_t *ctrl_off, const double *tau,
              const int32_t *tau_off, const double *stroke_w, const int32_t *opa_off,
              const int32_t *rank, double rho, double sigma0_sq, const double *d_gauss,
              double *d_ctrl, double *d_width, double *d_color, double *d_opacity) {
    if (n < 0 || !(rho > 0.0)) return ORC_ERR_ARG;
    int32_t *by_rank = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    if (!by_rank || !start) { free(by_rank); free(start); return ORC_ERR_MEM; }
    for (int i = 0; i < n; ++i) by_rank[rank[i]] = i;
    start[0] = 0;
    for (int p = 0; p < n; ++p) {
        int i = by_rank[p];
        start[p + 1] = start[p] + (int64_t)ks[i] * (kind[i] == 1 ? rs[i] + 2 : 1);
    }
    int st = ORC_OK;
#pragma omp parallel for schedule(dynamic, 4)
    for (int p = 0; p < n; ++p) {
        int i = by_rank[p];
        curve_t c;
        load_curve(i, kind, nseg, ks, rs, ctrl, ctrl_off, tau, tau_off, &c);
        int rows = rows_of(&c), K = c.K, m = 3 * c.S;
        double *Xbar = (double *)calloc((size_t)rows * K * 2, sizeof(double));
        if (!Xbar) abort();
        int nopa = opa_off[i + 1] - opa_off[i];
        double wbar = 0.0, cbar[3] = {0, 0, 0};
        int64_t g = start[p];
        for (int r = 0; r < rows; ++r) {
            for (int k = 0; k < K; ++k, ++g) {
                const double *dg = d_gauss + 9 * g;
                geom_t ge;
                gaussian_geom(&c, stroke_w[i], r, k, rho, sigma0_sq, &ge);
                double a = 1.0 / ge.sx2, b = 1.0 / ge.sy2, cs = ge.cs, sn = ge.sn;
                double Qxx_b = dg[2], Qxy_b = dg[3], Qyy_b = dg[4];
                double abar = Qxx_b * cs * cs + Qxy_b * cs * sn + Qyy_b * sn * sn;
                double bbar = Qxx_b * sn * sn - Qxy_b * cs * sn + Qyy_b * cs * cs;
                double cbar_t = Qxx_b * 2.0 * cs * a + Qxy_b * sn * (a - b) + Qyy_b * 2.0 * cs * b;
                double sbar_t = Qxx_b * 2.0 * sn * b + Qxy_b * cs * (a - b) + Qyy_b * 2.0 * sn * a;
                double sx2bar = -abar * a * a;
                double sy2bar = -bbar * b * b;
                /* mean */
                double *X0 = Xbar + 2 * ((size_t)r * K + k);
                X0[0] += dg[0];
                X0[1] += dg[1];
                /* along-row scale */
                double f = 2.0 * sx2bar / (rho * rho);
                double *Xa = Xbar + 2 * ((size_t)r * K + ge.ka);
                double *Xb = Xbar + 2 * ((size_t)r * K + ge.kb);
                Xa[0] += f * ge.delta[0]; Xa[1] += f * ge.delta[1];
                Xb[0] -= f * ge.delta[0]; Xb[1] -= f * ge.delta[1];
                /* across-row scale */
                if (c.kind == 1) {
                    double fy = 2.0 * sy2bar / (rho * rho);
                    double *Ya = Xbar + 2 * ((size_t)ge.ra * K + k);
                    double *Yb = Xbar + 2 * ((size_t)ge.rb * K + k);
                    Ya[0] += fy * ge.delta_y[0]; Ya[1] += fy * ge.delta_y[1];
                    Yb[0] -= fy * ge.delta_y[0]; Yb[1] -= fy * ge.delta_y[1];
                } else {
                    wbar += 2.0 * stroke_w[i] * sy2bar;
                }
                /* tangent h = v/|v|: vbar = (hbar - h (h . hbar)) / |v| */
                double nv = sqrt(ge.v[0] * ge.v[0] + ge.v[1] * ge.v[1]);
                if (nv > 0.0) {
                    double hd = cs * cbar_t + sn * sbar_t;
                    double vb0 = (cbar_t - cs * hd) / nv, vb1 = (sbar_t - sn * hd) / nv;
                    double *Vp = Xbar + 2 * ((size_t)r * K + ge.kp);
                    double *Vm = Xbar + 2 * ((size_t)r * K + ge.km);
                    Vp[0] += vb0; Vp[1] += vb1;
                    Vm[0] -= vb0; Vm[1] -= vb1;
                }
                /* opacity and colour */
                int slot = nopa == c.S ? ge.seg : 0;
                d_opacity[opa_off[i] + slot] += dg[5];
                for (int ch = 0; ch < 3; ++ch) cbar[ch] += dg[6 + ch];
            }
        }
        /* sample points -> control points */
        double *dP = d_ctrl + 2 * (int64_t)ctrl_off[i];
        for (int r = 0; r < rows; ++r) {
            for (int k = 0; k < K; ++k) {
                int s;
                double t, B[4];
                column_param(k, K, c.S, &s, &t);
                bernstein3(t, B);
                const double *xb = Xbar + 2 * ((size_t)r * K + k);
                for (int j = 0; j < 4; ++j) {
                    int jj = 3 * s + j;
                    double gx = B[j] * xb[0], gy = B[j] * xb[1];
                    if (c.kind == 0) {
                        dP[2 * jj] += gx;
                        dP[2 * jj + 1] += gy;
                    } else {
                        double tr = c.tau[r];
                        if (jj == 0 || jj == m) {
                            dP[2 * jj] += gx;          /* shared endpoint: both weights */
                            dP[2 * jj + 1] += gy;
                        } else {
                            dP[2 * jj] += (1.0 - tr) * gx;
                            dP[2 * jj + 1] += (1.0 - tr) * gy;
                            dP[2 * (m + jj)] += tr * gx;
                            dP[2 * (m + jj) + 1] += tr * gy;
                        }
                    }
                }
            }
        }
        d_width[i] += wbar;
        for (int ch = 0; ch < 3; ++ch) d_color[3 * i + ch] += cbar[ch];
        free(Xbar);
    }
    free(by_rank);
    free(start);
    return st;
}

/* Threads the following calls use (OpenMP); n < 1 leaves it unchanged. */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
