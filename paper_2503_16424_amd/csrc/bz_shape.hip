// bz_shape.hip -- per-curve shape terms: area, draw order by area, Xing loss.
//
// Area (Sec. 3.3, depth from area).  A closed curve encloses the region
// between its boundaries A and B; its area is the shoelace sum of the
// polygon A_0 .. A_{K-1}, B_{K-2} .. B_1 of boundary samples (the sampling
// grid of the Gaussians), taken relative to A_0.  An open stroke covers its
// polyline length times its width.  One wave per curve, FP64 samples and
// sums (the areas of a 2048-pixel canvas span eight decades).
//
// Draw order.  Curves sorted by area, smallest in front, ties by index (a
// stable LSD radix sort on the float bits of the non-negative areas, the
// binning's sort kernels; for a batch a second stable pass on the canvas
// index keeps every canvas's curves together), then the first Gaussian of
// every draw position by an exclusive scan of the per-curve Gaussian counts.  Everything stays on
// the device, so the order can follow the curves every step.
//
// Xing loss (Sec. 3.5, the convexity term of LIVE).  Per cubic segment
// P0..P3 of a closed curve's boundaries: D1 = [cross(P1-P0, P2-P1) >= 0] (the
// turn at the first inner point), D2 = cross(P1-P0, P3-P2) / (|P1-P0||P3-P2|)
// (sine from the first control edge to the last); the segment costs
// D1 max(0, -D2) + (1 - D1) max(0, D2): a last edge that turns against the
// first turn (an S bend or a loop) is penalised.  One thread per curve; its
// gradient goes to the curve's own control points, so no atomics.
#include "bz_geom.h"

namespace bz {

namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

__device__ inline double cross2(double2 a, double2 b) { return a.x * b.y - a.y * b.x; }
__device__ inline double2 sub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__global__ __launch_bounds__(64) void k_area(bz_curves c, float *__restrict__ area) {
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    const CurveView v = load_curve_by_id(c, i);
    const bool closed = v.kind == BZ_CLOSED;
    const double2 o = boundary_point(v, false, 0);
    double acc = 0.0;
    for (int k = lane; k < v.K - 1; k += 64) {
        const double2 a0 = boundary_point(v, false, k), a1 = boundary_point(v, false, k + 1);
        if (closed) {
            const double2 b0 = boundary_point(v, true, k), b1 = boundary_point(v, true, k + 1);
            acc += cross2(sub2(a0, o), sub2(a1, o)) - cross2(sub2(b0, o), sub2(b1, o));
        } else {
            const double2 d = sub2(a1, a0);
            acc += sqrt(d.x * d.x + d.y * d.y);
        }
    }
    acc = wave_sum_d(acc);
    if (lane == 0) area[i] = (float)(closed ? 0.5 * fabs(acc) : acc * (double)v.width);
}

// keys: float bits of the area (non-negative floats order as their bits;
// NaN goes last), values: curve index.
__global__ void k_area_keys(const float *area, int n, uint32_t *keys, uint32_t *vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float a = area[i];
    keys[i] = isnan(a) ? 0xffffffffu : __float_as_uint(fmaxf(a, 0.f));
    vals[i] = (uint32_t)i;
}

// Second key of a batch's order: the canvas of the curve at each position.
__global__ void k_canvas_keys(const bz_canvas *cv, int n_canvas, const uint32_t *vals, int n,
                              uint32_t *keys) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    keys[p] = (uint32_t)batch_find(cv, n_canvas, (int64_t)vals[p],
                                   [](const bz_canvas &r) { return (int64_t)r.curve_off; });
}

__global__ void k_order_counts(bz_curves c, const uint32_t *vals, int32_t *order, uint32_t *cnt) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= c.n_curves) return;
    const int i = (int)vals[p];
    order[p] = i;
    const int rows = c.kind[i] == BZ_CLOSED ? c.r_interior[i] + 2 : 1;
    cnt[p] = (uint32_t)(rows * c.k_samples[i]);
}

__global__ void k_widen(const uint32_t *offs, int n, int64_t *gauss_off) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) gauss_off[p] = (int64_t)offs[p];
}

__global__ void k_zero1(float *p) {
    if (threadIdx.x == 0) p[0] = 0.f;
}

__global__ __launch_bounds__(256) void k_xing(bz_curves c, float weight, float *loss,
                                              float *d_ctrl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (i < c.n_curves && c.kind[i] == BZ_CLOSED) {
        const CurveView v = load_curve_by_id(c, i);
        const int m = 3 * v.S;
        float *g = d_ctrl + 2 * (int64_t)c.ctrl_off[i];
        for (int b = 0; b < 2; ++b) {
            for (int s = 0; s < v.S; ++s) {
                double2 P[4];
                int idx[4];
                for (int j = 0; j < 4; ++j) {
                    const int jj = 3 * s + j;
                    P[j] = ctrl_point(v, b == 1, jj);
                    idx[j] = (b == 1 && jj != 0 && jj != m) ? m + jj : jj;
                }
                const double2 e1 = sub2(P[1], P[0]), e2 = sub2(P[2], P[1]), e3 = sub2(P[3], P[2]);
                const double n1 = sqrt(e1.x * e1.x + e1.y * e1.y);
                const double n3 = sqrt(e3.x * e3.x + e3.y * e3.y);
                if (!(n1 > 0.0 && n3 > 0.0)) continue;
                const bool d1 = cross2(e1, e2) >= 0.0;
                const double d2 = cross2(e1, e3) / (n1 * n3);
                const double f = d1 ? (d2 < 0.0 ? -d2 : 0.0) : (d2 > 0.0 ? d2 : 0.0);
                if (f == 0.0) continue;
                l += f;
                const double dfd = d1 ? -1.0 : 1.0;               // d f / d D2 where f > 0
                // d D2 / d e1, d D2 / d e3
                const double inv = 1.0 / (n1 * n3);
                const double g1x = (e3.y * inv - d2 * e1.x / (n1 * n1)) * dfd * weight;
                const double g1y = (-e3.x * inv - d2 * e1.y / (n1 * n1)) * dfd * weight;
                const double g3x = (-e1.y * inv - d2 * e3.x / (n3 * n3)) * dfd * weight;
                const double g3y = (e1.x * inv - d2 * e3.y / (n3 * n3)) * dfd * weight;
                g[2 * idx[1]] += (float)g1x;
                g[2 * idx[1] + 1] += (float)g1y;
                g[2 * idx[0]] -= (float)g1x;
                g[2 * idx[0] + 1] -= (float)g1y;
                g[2 * idx[3]] += (float)g3x;
                g[2 * idx[3] + 1] += (float)g3y;
                g[2 * idx[2]] -= (float)g3x;
                g[2 * idx[2] + 1] -= (float)g3y;
            }
        }
    }
    if (loss) {
        __shared__ double part[4];
        double s = wave_sum_d(l);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0)
            atomicAdd(loss, (float)(weight * (part[0] + part[1] + part[2] + part[3])));
    }
}

}  // namespace

// Workspace of the draw-order pipeline (bytes), 256-byte aligned pieces.
struct OrderLayout {
    int64_t keys, vals, keys2, vals2, hist, part, status, total;
};

OrderLayout order_layout(int64_t n) {
    OrderLayout L;
    int64_t off = 0, m = n > 0 ? n : 1;
    L.keys = off;
    off = align256(off + 4 * m);
    L.vals = off;
    off = align256(off + 4 * m);
    L.keys2 = off;
    off = align256(off + 4 * m);
    L.vals2 = off;
    off = align256(off + 4 * m);
    L.hist = off;
    off = align256(off + 4 * 256 * sort_hist_blocks(m));
    L.part = off;
    off = align256(off + 8 * sort_part_elems(m));
    L.status = off;
    off = align256(off + 16);
    L.total = off;
    return L;
}

int64_t order_workspace_bytes(int64_t n_curves) { return order_layout(n_curves).total; }

hipError_t launch_area(const bz_curves &c, float *area, hipStream_t s) {
    if (c.n_curves > 0) hipLaunchKernelGGL(k_area, dim3(c.n_curves), dim3(64), 0, s, c, area);
    return hipGetLastError();
}

hipError_t launch_area_order(const bz_curves &c, const bz_batch *batch, float *area,
                             int32_t *order, int64_t *gauss_off, void *ws, hipStream_t s) {
    const int n = c.n_curves;
    if (n == 0) return hipGetLastError();
    OrderLayout L = order_layout(n);
    char *w = (char *)ws;
    uint32_t *keys = (uint32_t *)(w + L.keys), *vals = (uint32_t *)(w + L.vals);
    uint32_t *keys2 = (uint32_t *)(w + L.keys2), *vals2 = (uint32_t *)(w + L.vals2);
    uint32_t *hist = (uint32_t *)(w + L.hist);
    uint64_t *part = (uint64_t *)(w + L.part);
    int64_t *status = (int64_t *)(w + L.status);
    hipLaunchKernelGGL(k_area, dim3(n), dim3(64), 0, s, c, area);
    const unsigned nb = (unsigned)cdiv(n, 256);
    hipLaunchKernelGGL(k_area_keys, dim3(nb), dim3(256), 0, s, (const float *)area, n, keys, vals);
    hipError_t e = sort_pairs_u32(keys, vals, keys2, vals2, n, 32, hist, part, status, s);
    if (e != hipSuccess) return e;
    if (batch) {      // stable by canvas on top: canvas-major, area inside each canvas
        hipLaunchKernelGGL(k_canvas_keys, dim3(nb), dim3(256), 0, s, batch->canvas,
                           batch->n_canvas, (const uint32_t *)vals, n, keys);
        e = sort_pairs_u32(keys, vals, keys2, vals2, n, 16, hist, part, status, s);
        if (e != hipSuccess) return e;
    }
    // after the sort keys2 / vals2 are free: counts and offsets
    hipLaunchKernelGGL(k_order_counts, dim3(nb), dim3(256), 0, s, c, (const uint32_t *)vals,
                       order, keys2);
    e = exclusive_scan_u32(keys2, vals2, n, part, gauss_off + n, status, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_widen, dim3(nb), dim3(256), 0, s, (const uint32_t *)vals2, n, gauss_off);
    return hipGetLastError();
}

hipError_t launch_xing(const bz_curves &c, float weight, float *loss, float *d_ctrl,
                       hipStream_t s) {
    if (loss) hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, s, loss);
    if (c.n_curves > 0)
        hipLaunchKernelGGL(k_xing, dim3((unsigned)cdiv(c.n_curves, 256)), dim3(256), 0, s, c,
                           weight, loss, d_ctrl);
    return hipGetLastError();
}

}  // namespace bz
