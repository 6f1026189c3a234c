/*
 * Drives every entry point of the FP64 oracle (oracle/bz_oracle.c) on a small
 * procedural scene, for a build with AddressSanitizer, UndefinedBehavior-
 * Sanitizer and LeakSanitizer (see tests/test_oracle_sanitizers.py).  Test
 * infrastructure: it checks the oracle's memory and arithmetic hygiene, not
 * its values (the pin tests do that).
 *
 * Scene: open strokes of 1 and 3 segments (one and three opacities), closed
 * curves with interior rows, a curve whose control points coincide (zero-length
 * chords and tangents), curves reaching past the canvas edges; ragged canvas
 * size.  Then the error paths: a rank that is not a permutation, a curve with
 * K < 2, bad options.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t orc_count_gaussians(int n, const int32_t *kind, const int32_t *ks, const int32_t *rs);
int orc_sample(int n, const int32_t *kind, const int32_t *nseg, const int32_t *ks,
               const int32_t *rs, const double *ctrl, const int32_t *ctrl_off, const double *tau,
               const int32_t *tau_off, const double *stroke_w, const double *color,
               const double *opacity, const int32_t *opa_off, const int32_t *rank, double rho,
               double sigma0_sq, double *mu, double *conic, double *sx2, double *sy2,
               double *tangent, double *opac, double *col_out, int32_t *curve_out,
               int32_t *row_out, int32_t *colk_out, int32_t *slot_out);
int orc_render(int64_t n, const double *mu, const double *conic, const double *opac,
               const double *color, int W, int H, const double *bg, double g_min,
               double alpha_max, double t_min, int ya, int yb, int brute, double *image,
               double *t_final, int32_t *n_contrib, const double *d_image, double *d_gauss,
               int64_t *counters, double *margin);
int orc_render_pixels(int64_t n, const double *mu, const double *conic, const double *opac,
                      const double *color, int W, int H, const double *bg, double g_min,
                      double alpha_max, double t_min, int npix, const int32_t *px,
                      const int32_t *py, double *rgb, double *T, int32_t *ncontrib);
int orc_tile_depth(int64_t n, const double *mu, const double *conic, const double *opac,
                   const int32_t *curve, int n_curves, int W, int H, double g_min,
                   double alpha_max, double t_min, int tw, int th, int32_t *depth_contrib,
                   int32_t *depth_support);
int orc_chain(int n, const int32_t *kind, const int32_t *nseg, const int32_t *ks,
              const int32_t *rs, const double *ctrl, const int32_t *ctrl_off, const double *tau,
              const int32_t *tau_off, const double *stroke_w, const int32_t *opa_off,
              const int32_t *rank, double rho, double sigma0_sq, const double *d_gauss,
              double *d_ctrl, double *d_width, double *d_color, double *d_opacity);
void orc_set_threads(int n);

static uint64_t lcg = 12345;
static double urand(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) / 9007199254740992.0;
}

#define NC 9
#define CHECK(x) do { if (!(x)) { fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); return 1; } } while (0)

int main(void) {
    const int W = 53, H = 37;
    int32_t kind[NC], nseg[NC], ks[NC], rs[NC], ctrl_off[NC + 1], tau_off[NC + 1], opa_off[NC + 1],
        rank[NC];
    double ctrl[2 * 64 * NC], tau[32 * NC], stroke_w[NC], color[3 * NC], opacity[4 * NC];
    ctrl_off[0] = tau_off[0] = opa_off[0] = 0;
    for (int i = 0; i < NC; ++i) {
        const int closed = i % 3 == 0;
        kind[i] = closed;
        nseg[i] = closed ? 1 : (i % 2 ? 3 : 1);
        ks[i] = 6 + i;
        rs[i] = closed ? 2 + i % 3 : 0;
        const int npts = closed ? 6 * nseg[i] : 3 * nseg[i] + 1;
        const double cx = -5.0 + urand() * (W + 10), cy = -5.0 + urand() * (H + 10);
        const double L = 4.0 + 20.0 * urand();
        for (int j = 0; j < npts; ++j) {
            double *p = ctrl + 2 * (ctrl_off[i] + j);
            if (i == 4) {                      /* coincident points: zero-length chords */
                p[0] = cx;
                p[1] = cy;
            } else {
                p[0] = cx + L * (urand() - 0.5);
                p[1] = cy + L * (urand() - 0.5);
            }
        }
        ctrl_off[i + 1] = ctrl_off[i] + npts;
        const int nt = closed ? rs[i] + 2 : 2;
        for (int r = 0; r < nt; ++r) tau[tau_off[i] + r] = (double)r / (nt - 1);
        tau_off[i + 1] = tau_off[i] + nt;
        stroke_w[i] = closed ? 0.0 : 1.0 + 3.0 * urand();
        for (int c = 0; c < 3; ++c) color[3 * i + c] = urand();
        const int no = (!closed && nseg[i] == 3) ? 3 : 1;
        for (int k = 0; k < no; ++k) opacity[opa_off[i] + k] = 0.3 + 0.7 * urand();
        opa_off[i + 1] = opa_off[i] + no;
        rank[i] = (i * 4) % NC;              /* a permutation (4 and 9 are coprime) */
    }
    const int64_t ng = orc_count_gaussians(NC, kind, ks, rs);
    CHECK(ng > 0);
    double *mu = malloc(sizeof(double) * 2 * ng), *conic = malloc(sizeof(double) * 3 * ng);
    double *sx2 = malloc(sizeof(double) * ng), *sy2 = malloc(sizeof(double) * ng);
    double *tangent = malloc(sizeof(double) * 2 * ng), *opac = malloc(sizeof(double) * ng);
    double *col = malloc(sizeof(double) * 3 * ng);
    int32_t *curve = malloc(sizeof(int32_t) * ng), *row = malloc(sizeof(int32_t) * ng);
    int32_t *colk = malloc(sizeof(int32_t) * ng), *slot = malloc(sizeof(int32_t) * ng);
    CHECK(orc_sample(NC, kind, nseg, ks, rs, ctrl, ctrl_off, tau, tau_off, stroke_w, color,
                     opacity, opa_off, rank, 2.0, 0.3, mu, conic, sx2, sy2, tangent, opac, col,
                     curve, row, colk, slot) == 0);
    const double bg[3] = {1.0, 0.5, 0.25};
    double *image = malloc(sizeof(double) * 3 * W * H), *t_final = malloc(sizeof(double) * W * H);
    double *margin = malloc(sizeof(double) * W * H), *d_image = malloc(sizeof(double) * 3 * W * H);
    double *d_gauss = calloc((size_t)9 * ng, sizeof(double));
    int32_t *n_contrib = malloc(sizeof(int32_t) * W * H);
    int64_t counters[4];
    for (int64_t i = 0; i < 3 * W * H; ++i) d_image[i] = urand() - 0.5;
    for (int threads = 1; threads <= 3; threads += 2) {
        orc_set_threads(threads);
        for (int brute = 0; brute < 2; ++brute) {
            CHECK(orc_render(ng, mu, conic, opac, col, W, H, bg, 1.0 / 255, 0.99, 1e-6, 0, H, brute,
                             image, t_final, n_contrib, d_image, d_gauss, counters, margin) == 0);
            CHECK(orc_render(ng, mu, conic, opac, col, W, H, bg, 1.0 / 255, 0.99, 1e-6, 5, 11, brute,
                             image, t_final, n_contrib, NULL, NULL, counters, NULL) == 0);
        }
    }
    int32_t px[5] = {0, W - 1, 7, -3, W}, py[5] = {0, H - 1, 9, 2, 4};
    double rgb[15], T[5];
    int32_t nc[5];
    CHECK(orc_render_pixels(ng, mu, conic, opac, col, W, H, bg, 1.0 / 255, 0.99, 1e-6, 5, px, py,
                            rgb, T, nc) == 0);
    const int tx = (W + 7) / 8, ty = (H + 7) / 8;
    int32_t *dc = malloc(sizeof(int32_t) * tx * ty), *ds = malloc(sizeof(int32_t) * tx * ty);
    CHECK(orc_tile_depth(ng, mu, conic, opac, curve, NC, W, H, 1.0 / 255, 0.99, 1e-6, 8, 8, dc,
                         ds) == 0);
    double *d_ctrl = calloc((size_t)2 * ctrl_off[NC], sizeof(double));
    double d_width[NC], d_color[3 * NC], d_opacity[4 * NC];
    CHECK(orc_chain(NC, kind, nseg, ks, rs, ctrl, ctrl_off, tau, tau_off, stroke_w, opa_off, rank,
                    2.0, 0.3, d_gauss, d_ctrl, d_width, d_color, d_opacity) == 0);
    for (int i = 0; i < 2 * ctrl_off[NC]; ++i) CHECK(isfinite(d_ctrl[i]));
    /* error paths */
    int32_t bad_rank[NC];
    memcpy(bad_rank, rank, sizeof(rank));
    bad_rank[1] = bad_rank[0];
    CHECK(orc_sample(NC, kind, nseg, ks, rs, ctrl, ctrl_off, tau, tau_off, stroke_w, color,
                     opacity, opa_off, bad_rank, 2.0, 0.3, mu, conic, sx2, sy2, tangent, opac, col,
                     curve, row, colk, slot) != 0);
    int32_t bad_k[NC];
    memcpy(bad_k, ks, sizeof(ks));
    bad_k[2] = 1;
    CHECK(orc_sample(NC, kind, nseg, bad_k, rs, ctrl, ctrl_off, tau, tau_off, stroke_w, color,
                     opacity, opa_off, rank, 2.0, 0.3, mu, conic, sx2, sy2, tangent, opac, col,
                     curve, row, colk, slot) != 0);
    CHECK(orc_render(ng, mu, conic, opac, col, 0, H, bg, 1.0 / 255, 0.99, 1e-6, 0, H, 0, image,
                     t_final, n_contrib, NULL, NULL, counters, NULL) != 0);
    CHECK(orc_render(ng, mu, conic, opac, col, W, H, bg, 1.5, 0.99, 1e-6, 0, H, 0, image, t_final,
                     n_contrib, NULL, NULL, counters, NULL) != 0);
    curve[0] = NC;
    CHECK(orc_tile_depth(ng, mu, conic, opac, curve, NC, W, H, 1.0 / 255, 0.99, 1e-6, 8, 8, dc,
                         ds) != 0);
    free(mu); free(conic); free(sx2); free(sy2); free(tangent); free(opac); free(col);
    free(curve); free(row); free(colk); free(slot); free(image); free(t_final); free(margin);
    free(d_image); free(d_gauss); free(n_contrib); free(dc); free(ds); free(d_ctrl);
    printf("oracle driver: %lld Gaussians, %lld contributing pairs\n", (long long)ng,
           (long long)counters[0]);
    return 0;
}
