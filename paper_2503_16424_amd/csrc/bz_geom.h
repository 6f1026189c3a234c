// bz_geom.h -- per-curve sample geometry on the device (Sec. 3.3).
//
// One wave handles one curve.  The wave first evaluates the cubic Bernstein
// form (Eq. bezier, bezier1) at the K uniform parameters of the two boundary
// rows (open curves have one row) in double precision and keeps them in LDS;
// the interior rows of a closed curve are the tau_r blends of the boundary
// samples, which by linearity equal the samples of the blended control points
// of Sec. 3.3.  Each lane then derives its Gaussians' means, neighbour
// differences (Eq. sigma) and tangent chords (Eq. rotation) from LDS.
#pragma once

#include "bz_internal.h"

namespace bz {

struct CurveView {
    int id;          // curve index
    int kind;        // BZ_OPEN / BZ_CLOSED
    int S, K, R;     // segments, samples per row, interior rows (0 for open)
    int rows;        // 1 or R+2
    int nopa;        // 1 or S
    int64_t g0;      // first Gaussian
    const float *P;  // control points
    const float *tau;
    float width;
};

__device__ inline CurveView load_curve_view(const bz_curves &c, int p) {
    CurveView v;
    int i = c.order[p];
    v.id = i;
    v.kind = c.kind[i];
    v.S = c.nseg[i];
    v.K = c.k_samples[i];
    v.R = v.kind == BZ_CLOSED ? c.r_interior[i] : 0;
    v.rows = v.kind == BZ_CLOSED ? v.R + 2 : 1;
    v.nopa = c.opa_off[i + 1] - c.opa_off[i];
    v.g0 = c.gauss_off[p];
    v.P = c.ctrl + 2 * (int64_t)c.ctrl_off[i];
    v.tau = c.tau + c.tau_off[i];
    v.width = c.stroke_w[i];
    return v;
}

// View of curve i by its index (draw position unknown: g0 = 0).
__device__ inline CurveView load_curve_by_id(const bz_curves &c, int i) {
    CurveView v;
    v.id = i;
    v.kind = c.kind[i];
    v.S = c.nseg[i];
    v.K = c.k_samples[i];
    v.R = v.kind == BZ_CLOSED ? c.r_interior[i] : 0;
    v.rows = v.kind == BZ_CLOSED ? v.R + 2 : 1;
    v.nopa = c.opa_off[i + 1] - c.opa_off[i];
    v.g0 = 0;
    v.P = c.ctrl + 2 * (int64_t)c.ctrl_off[i];
    v.tau = c.tau + c.tau_off[i];
    v.width = c.stroke_w[i];
    return v;
}

// Column k of a row: segment s = min(floor(kS/(K-1)), S-1) in integers and the
// local parameter t in [0, 1] of that segment.
__device__ inline void column_param(int k, int K, int S, int &s, double &t) {
    s = (k * S) / (K - 1);
    if (s > S - 1) s = S - 1;
    t = (double)(k * S - s * (K - 1)) / (double)(K - 1);
}

__device__ inline void bernstein3(double t, double B[4]) {
    double u = 1.0 - t;
    B[0] = u * u * u;
    B[1] = 3.0 * u * u * t;
    B[2] = 3.0 * u * t * t;
    B[3] = t * t * t;
}

// Control point jj (0..3S) of boundary A or B of a closed curve (B shares A's
// endpoints; its interior points follow A's 3S+1 points in storage).
__device__ inline double2 ctrl_point(const CurveView &v, bool boundary_b, int jj) {
    int m = 3 * v.S;
    int idx = (boundary_b && jj != 0 && jj != m) ? m + jj : jj;
    return make_double2((double)v.P[2 * idx], (double)v.P[2 * idx + 1]);
}

// Copy a closed curve's row weights into LDS (rows <= 256) and point the view
// at the copy; sample_at reads them for every sample point.
__device__ inline void stage_tau(CurveView &v, float *s_tau, int lane, int nlanes) {
    if (v.kind != BZ_CLOSED) return;
    for (int r = lane; r < v.rows; r += nlanes) s_tau[r] = v.tau[r];
    v.tau = s_tau;
}

// Boundary samples XA[k] (and XB[k] for closed curves) into LDS.
__device__ inline void boundary_samples(const CurveView &v, double2 *XA, double2 *XB, int lane,
                                        int nlanes) {
    for (int k = lane; k < v.K; k += nlanes) {
        int s;
        double t, B[4];
        column_param(k, v.K, v.S, s, t);
        bernstein3(t, B);
        double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
        for (int j = 0; j < 4; ++j) {
            double2 a = ctrl_point(v, false, 3 * s + j);
            ax += B[j] * a.x;
            ay += B[j] * a.y;
            if (v.kind == BZ_CLOSED) {
                double2 b = ctrl_point(v, true, 3 * s + j);
                bx += B[j] * b.x;
                by += B[j] * b.y;
            }
        }
        XA[k] = make_double2(ax, ay);
        if (v.kind == BZ_CLOSED) XB[k] = make_double2(bx, by);
    }
}

// Sample k of boundary A (or B) evaluated directly (no LDS).
__device__ inline double2 boundary_point(const CurveView &v, bool boundary_b, int k) {
    int s;
    double t, B[4];
    column_param(k, v.K, v.S, s, t);
    bernstein3(t, B);
    double x = 0.0, y = 0.0;
    for (int j = 0; j < 4; ++j) {
        const double2 p = ctrl_point(v, boundary_b, 3 * s + j);
        x += B[j] * p.x;
        y += B[j] * p.y;
    }
    return make_double2(x, y);
}

// Sample point X_{r,k}.
__device__ inline double2 sample_at(const CurveView &v, const double2 *XA, const double2 *XB,
                                    int r, int k) {
    double2 a = XA[k];
    if (v.kind != BZ_CLOSED) return a;
    double t = (double)v.tau[r];
    double2 b = XB[k];
    return make_double2((1.0 - t) * a.x + t * b.x, (1.0 - t) * a.y + t * b.y);
}

// 1/x and 1/sqrt(x): for positive normal finite x the hardware estimate
// (relative error near 2^-22) refined by two Newton steps, each of which
// squares the relative error, so the result is within an ulp or two of the
// double quotient, far cheaper than the IEEE division and square root
// sequences; anything else (zero, subnormal, infinite, NaN) takes those.
constexpr double kMinNormal = 2.2250738585072014e-308;
constexpr double kMaxFinite = 1.7976931348623157e308;
__device__ inline double rcp_f64(double x) {
    if (!(x >= kMinNormal && x <= kMaxFinite)) return 1.0 / x;
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ inline double rsqrt_f64(double x) {
    if (!(x >= kMinNormal && x <= kMaxFinite)) return 1.0 / sqrt(x);
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    return y * fma(-hx * y, y, 1.5);
}

struct Geom {
    double2 mu;
    double sx2, sy2;       // dilated squared scales
    double cs, sn;         // unit tangent
    double2 d_along;       // X[r][ka] - X[r][kb]
    double2 d_across;      // X[ra][k] - X[rb][k] (closed)
    double2 v;             // X[r][kp] - X[r][km]
    double nv;             // |v|
    int ka, kb, ra, rb, kp, km;
    int seg;
};

// Geometry of Gaussian (r, k): Eq. sigma with the nearest-neighbour rule at
// the last column / row, Eq. rotation one-sided at the row ends, unit tangent
// (1, 0) when the chord has zero length.
__device__ inline void gauss_geom(const CurveView &v, const double2 *XA, const double2 *XB, int r,
                                  int k, double inv_rho2, double s0, Geom &g) {
    int K = v.K;
    double t;
    column_param(k, K, v.S, g.seg, t);
    // The stencils use at most the point, its row neighbours and one row
    // neighbour: each is evaluated once (the same values as evaluating them
    // per use).
    g.mu = sample_at(v, XA, XB, r, k);
    const double2 Xl = k > 0 ? sample_at(v, XA, XB, r, k - 1) : g.mu;
    const double2 Xr = k < K - 1 ? sample_at(v, XA, XB, r, k + 1) : g.mu;
    if (k < K - 1) { g.ka = k + 1; g.kb = k; } else { g.ka = K - 1; g.kb = K - 2; }
    const double2 A = k < K - 1 ? Xr : g.mu, B = k < K - 1 ? g.mu : Xl;   // X[r][ka], X[r][kb]
    g.d_along = make_double2(A.x - B.x, A.y - B.y);
    g.sx2 = (g.d_along.x * g.d_along.x + g.d_along.y * g.d_along.y) * inv_rho2 + s0;
    if (v.kind == BZ_CLOSED) {
        int R1 = v.R + 1;
        if (r < R1) { g.ra = r + 1; g.rb = r; } else { g.ra = R1; g.rb = R1 - 1; }
        const double2 Y = sample_at(v, XA, XB, r < R1 ? r + 1 : r - 1, k);
        const double2 P = r < R1 ? Y : g.mu, Q = r < R1 ? g.mu : Y;      // X[ra][k], X[rb][k]
        g.d_across = make_double2(P.x - Q.x, P.y - Q.y);
        g.sy2 = (g.d_across.x * g.d_across.x + g.d_across.y * g.d_across.y) * inv_rho2 + s0;
    } else {
        g.ra = g.rb = 0;
        g.d_across = make_double2(0.0, 0.0);
        double w = (double)v.width;
        g.sy2 = w * w + s0;
    }
    g.kp = k + 1 < K ? k + 1 : K - 1;
    g.km = k > 0 ? k - 1 : 0;
    const double2 Pp = k + 1 < K ? Xr : g.mu, Pm = k > 0 ? Xl : g.mu;   // X[r][kp], X[r][km]
    g.v = make_double2(Pp.x - Pm.x, Pp.y - Pm.y);
    const double nv2 = g.v.x * g.v.x + g.v.y * g.v.y;
    if (nv2 > 0.0) {
        const double inv = rsqrt_f64(nv2);
        g.nv = nv2 * inv;
        g.cs = g.v.x * inv;
        g.sn = g.v.y * inv;
    } else {
        g.nv = 0.0;
        g.cs = 1.0;
        g.sn = 0.0;
    }
}

}  // namespace bz
