// bz_sample.hip -- curves -> 2D Gaussians (Sec. 3.3).
//
// One workgroup per curve, in draw order.  The boundary
// rows are evaluated once per curve in double precision (LDS), every lane then
// emits Gaussians (r, k) of the curve: mean in double, split into a float
// high part and a float low part; squared scales from the neighbour distances
// of Eq. sigma plus the dilation sigma0^2; the covariance of Eq. RSSR (R =
// [c -s; s c], S = diag(sx, sy)) kept in its principal frame as e = (c, s) / sx
// and k = sx / sy, Sigma^-1 = e e^T + k^2 e_perp e_perp^T.  Records
// of one curve are contiguous; a wave stages its 64 records of a round in LDS
// and writes them as three contiguous 1 KB stores.  With kBin the kernel also
// does the binning's counting pass (Sec. 3.4): each Gaussian's tile rectangle
// and count, from the record values it stores, so the binning need not read
// the records back; on the bucketed path, instead of the count, the pairs per
// (bucket of 256 tile keys, emission block): a wave's 64 Gaussians fall in at
// most two emission blocks, so it adds its pairs up in LDS and sends each
// non-zero sum with one global atomic.
#include "bz_geom.h"

namespace bz {

// Wave-level barrier with LDS ordering (the wave's own slice only).
__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool kBin>
__global__ __launch_bounds__(kCurveThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_sample(bz_curves c, double inv_rho2, double s0,
                                               float4 *__restrict__ rec, BinCount bc,
                                               const bz_canvas *__restrict__ cv, int n_canvas,
                                               int W, int H) {
    extern __shared__ double2 lds_xy[];
    __shared__ float s_tau[256];
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    CurveView v = load_curve_view(c, p);
    stage_tau(v, s_tau, lane, kCurveThreads);
    double2 *XA = lds_xy;
    double2 *XB = lds_xy + c.max_k;
    boundary_samples(v, XA, XB, lane, kCurveThreads);
    __syncthreads();

    const float *col = c.color + 3 * (int64_t)v.id;
    const float cr = col[0], cg = col[1], cb = col[2];
    const float *opa = c.opacity + c.opa_off[v.id];
    const float cid = __int_as_float(v.id);
    const int n = v.rows * v.K;
    int txc = bc.tiles_x;
    uint32_t tbase = 0;
    if (kBin && cv) {   // the canvas holding the curve (and all its Gaussians)
        const int ci = batch_find(cv, n_canvas, v.g0, [](const bz_canvas &r) { return r.gauss_off; });
        W = cv[ci].width;
        H = cv[ci].height;
        txc = cv[ci].tiles_x;
        tbase = (uint32_t)cv[ci].tile_off;
    }
    // bucketed path: the wave's pairs per (emission block of the round's first
    // Gaussian + part, bucket) at hbw[part * n_buckets + bucket], in the dynamic
    // LDS after the boundary rows
    const bool bucketed = kBin && bc.bucket != nullptr;
    const int nbk = bc.n_buckets;
    bool nonfinite = false;
    // A wave emits 64 consecutive Gaussians per round: their 48-byte records
    // meet in the wave's LDS slice and leave as three 1 KB contiguous stores
    // (written straight, lane l's three 16-byte pieces would be 48 bytes apart).
    __shared__ float4 s_rec[kCurveThreads / 64][3 * 64];
    const int w = lane >> 6, l = lane & 63;
    float4 *my = s_rec[w];
    uint32_t *hbw = reinterpret_cast<uint32_t *>(lds_xy + 2 * c.max_k) + w * 2 * nbk;
    for (int base = 64 * w; base < n; base += kCurveThreads) {
        const int idx = base + l;
        const int64_t eb0 = (v.g0 + base) / kEmitBlock;
        if (bucketed) {
            for (int i = l; i < 2 * nbk; i += 64) hbw[i] = 0u;
            wave_sync_lds();
        }
        if (idx < n) {
            int r = idx / v.K, k = idx - r * v.K;
            Geom g;
            gauss_geom(v, XA, XB, r, k, inv_rho2, s0, g);
            // 1 / sx and sx / sy (scales are positive: sigma0^2 > 0, or the
            // caller's degenerate input gives inf / nan, which binning flags)
            const double isx = rsqrt_f64(g.sx2);
            const double kk = g.sx2 * isx * rsqrt_f64(g.sy2);
            float hx = (float)g.mu.x, hy = (float)g.mu.y;
            float lx = (float)(g.mu.x - (double)hx), ly = (float)(g.mu.y - (double)hy);
            float o = opa[v.nopa == v.S ? g.seg : 0];
            const float4 m = make_float4(hx, hy, lx, ly);
            const float4 q = make_float4((float)(g.cs * isx), (float)(g.sn * isx), (float)kk, o);
            my[3 * l + 0] = m;
            my[3 * l + 1] = q;
            my[3 * l + 2] = make_float4(cr, cg, cb, cid);
            if (kBin) {
                ushort4 rc;
                bool finite;
                // bucketed path: each row's span of keys to its buckets
                uint32_t *hb = hbw + (int)((v.g0 + idx) / kEmitBlock - eb0) * nbk;
                const uint32_t cnt = tile_rect(
                    m, q, W, H, bc.inv_tw, bc.inv_th, bc.th, bc.two_p, rc, finite,
                    [&](int ty, int c0, int c1) {
                        if (!bucketed) return;
                        const uint32_t k0 = tbase + (uint32_t)ty * (uint32_t)txc + (uint32_t)c0;
                        for_key_buckets(k0, (uint32_t)(c1 - c0 + 1),
                                        [&](uint32_t h, uint32_t c) { atomicAdd(&hb[h], c); });
                    });
                if (bc.counts) bc.counts[v.g0 + idx] = cnt;
                bc.rects[v.g0 + idx] = rc;
                nonfinite |= !finite;
            }
        }
        if (bucketed) {
            wave_sync_lds();
            for (int i = l; i < 2 * nbk; i += 64) {
                const uint32_t c = hbw[i];
                if (c) {
                    const int part = i >= nbk ? 1 : 0;
                    const int h = i - part * nbk;
                    atomicAdd(&bc.bucket[(int64_t)h * bc.n_eblk + eb0 + part], c);
                }
            }
        }
        wave_sync_lds();
        const int valid = 3 * (n - base < 64 ? n - base : 64);   // float4s of this round
        float4 *out = rec + 3 * (v.g0 + base);
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (j * 64 + l < valid) out[j * 64 + l] = my[j * 64 + l];
        wave_sync_lds();
    }
    if (kBin && __builtin_amdgcn_ballot_w64(nonfinite) && l == 0)
        atomicOr((unsigned long long *)&bc.status[1], (unsigned long long)Status::kNonFinite);
}

hipError_t launch_sample(const bz_curves &c, const bz_opts &o, float *rec, const BinCount *bc,
                         hipStream_t s) {
    if (c.n_curves == 0) return hipSuccess;
    size_t lds = 2 * sizeof(double2) * (size_t)c.max_k;
    if (bc && bc->bucket)      // per wave: two emission blocks' bucket sums
        lds += sizeof(uint32_t) * 2 * (size_t)bc->n_buckets * (kCurveThreads / 64);
    double rho = (double)o.rho;
    const bz_canvas *cv = o.batch ? o.batch->canvas : nullptr;
    const int ncv = o.batch ? o.batch->n_canvas : 0;
    if (bc)
        hipLaunchKernelGGL(k_sample<true>, dim3(c.n_curves), dim3(kCurveThreads), lds, s, c,
                           1.0 / (rho * rho), (double)o.sigma0_sq, reinterpret_cast<float4 *>(rec),
                           *bc, cv, ncv, o.width, o.height);
    else
        hipLaunchKernelGGL(k_sample<false>, dim3(c.n_curves), dim3(kCurveThreads), lds, s, c,
                           1.0 / (rho * rho), (double)o.sigma0_sq, reinterpret_cast<float4 *>(rec),
                           BinCount{}, cv, ncv, o.width, o.height);
    return hipGetLastError();
}

}  // namespace bz
