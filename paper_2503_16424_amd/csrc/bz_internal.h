// bz_internal.h -- private declarations of libbz (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bz.h"

namespace bz {

// Gaussian record: three float4 per Gaussian (see bz_gaussians in bz.h).
constexpr int kRecF4 = 3;

// Per-Gaussian gradient planes (see bz_grads in bz.h).
constexpr int kGradPlanes = 9;

// Wave size of gfx950.
constexpr int kWave = 64;

// Wave minimum and maximum of one unsigned value per lane, wave-uniform: an
// inclusive DPP scan (row shifts of 1, 2, 4 and 8 lanes, then row_bcast 15
// and 31 across rows) with the operation's identity where a lane has no
// source, read from the last lane.
template <int CTRL, int ROWS>
__device__ inline uint32_t dpp_or_u32(uint32_t identity, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)x, CTRL, ROWS, 0xF, false);
}
template <bool kMax>
__device__ inline uint32_t wave_extreme_u32(uint32_t v) {
    const uint32_t id = kMax ? 0u : 0xffffffffu;
    auto op = [](uint32_t a, uint32_t b) { return kMax ? (a > b ? a : b) : (a < b ? a : b); };
    v = op(v, dpp_or_u32<0x111, 0xF>(id, v));
    v = op(v, dpp_or_u32<0x112, 0xF>(id, v));
    v = op(v, dpp_or_u32<0x114, 0xF>(id, v));
    v = op(v, dpp_or_u32<0x118, 0xF>(id, v));
    v = op(v, dpp_or_u32<0x142, 0xA>(id, v));
    v = op(v, dpp_or_u32<0x143, 0xC>(id, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ inline uint32_t wave_min_u32(uint32_t v) { return wave_extreme_u32<false>(v); }
__device__ inline uint32_t wave_max_u32(uint32_t v) { return wave_extreme_u32<true>(v); }

// Quads: every wave owns one 8x8 block of pixels; tiles are made of quads.
constexpr int kQuad = 8;

// Largest number of segments per curve handled by the per-curve kernels.
constexpr int kMaxSeg = 4;

// Threads of the per-curve kernels (one workgroup per curve).
constexpr int kCurveThreads = 256;

// Curves of at most this many Gaussians run the per-curve backward as one-wave
// workgroups.
constexpr int kSmallCurve = 64;

// log2(e)
constexpr float kLog2e = 1.4426950408889634f;

// Relative slack on the support threshold used by the culling tests.  Culling
// only needs to be conservative: every pixel whose float32 kernel value exceeds
// g_min must survive both the tile bound and the per-wave quad test.
constexpr float kCullSlackQuad = 1.001f;   // on the quadratic-form threshold
constexpr float kCullSlackBox = 1.0012f;   // on the bounding-box half extents
constexpr float kCullPadBox = 0.02f;       // px added to the half extents

struct Status {
    static constexpr int64_t kOverflow = 1;
    static constexpr int64_t kNonFinite = 2;
    static constexpr int64_t kListMismatch = 4;   // set with kOverflow: lists invalid
};

// ---------------------------------------------------------------------------
// host launchers implemented in the .hip files
// ---------------------------------------------------------------------------
struct BinCount;
// bc non-null: sampling also writes every Gaussian's tile count and rectangle
// (what the binning's counting pass would write).
hipError_t launch_sample(const bz_curves &c, const bz_opts &o, float *rec, const BinCount *bc,
                         hipStream_t s);
hipError_t launch_bin(const float *rec, int64_t n_gauss, const bz_opts &o, const bz_bins &b,
                      hipStream_t s);
// bz_sample_bin: binning with its counting pass done by the sampler.
hipError_t launch_sample_bin(const bz_curves &c, const bz_opts &o, float *rec,
                             const bz_bins &b, hipStream_t s);
// The L2 loss gradient the forward can write with the image (loss may be null).
struct L2Out {
    const float *target;
    float *d_image;
    float *loss;
    float scale;
};
// st == nullptr: the forward writes only the image; the backward recomputes
// the blend state per tile.  l2 == nullptr: no loss gradient.
hipError_t launch_fwd(const float *rec, const bz_bins &b, const bz_opts &o, float *image,
                      const bz_pixstate *st, const L2Out *l2, hipStream_t s);
hipError_t launch_bwd_gauss(const float *rec, int64_t n_gauss, const bz_bins &b,
                            const bz_opts &o, const float *d_image, const bz_pixstate *st,
                            float *d_gauss, hipStream_t s);
hipError_t launch_bwd_curves(const bz_curves &c, const bz_opts &o, const float *d_gauss,
                             const bz_grads &gr, hipStream_t s);
hipError_t launch_l2(const float *image, const float *target, int64_t n, float scale,
                     float *d_image, float *loss, hipStream_t s);
hipError_t launch_area(const bz_curves &c, float *area, hipStream_t s);
hipError_t launch_area_order(const bz_curves &c, const bz_batch *batch, float *area,
                             int32_t *order, int64_t *gauss_off, void *ws, hipStream_t s);
hipError_t launch_xing(const bz_curves &c, float weight, float *loss, float *d_ctrl,
                       hipStream_t s);
int64_t order_workspace_bytes(int64_t n_curves);

// Sorting helpers of bz_bin.hip, reused by the draw-order pipeline.
// sort_pairs_u32: stable LSD radix sort of n (key, value) pairs on the low
// key_bits bits (16 or 32: an even number of 8-bit passes, so the result
// ends in keys/vals);
// hist: uint32 [256 * sort_hist_blocks(n)], part: uint64 [sort_part_elems(n)],
// status: int64 [2] scratch.
int64_t sort_hist_blocks(int64_t n);
int64_t sort_part_elems(int64_t n);
hipError_t sort_pairs_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2,
                          int64_t n, int key_bits, uint32_t *hist, uint64_t *part, int64_t *status,
                          hipStream_t s);
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint64_t *part,
                              int64_t *total_out, int64_t *status, hipStream_t s);

// Workspace layout of bz_bin (bytes); shared by bz_workspace_size and the launcher.
struct BinLayout {
    int64_t n_tiles = 0;
    int key_bits = 0;
    int passes = 0;
    int64_t hist_blocks = 0;      // radix blocks for cap_pairs
    int64_t off_counts = 0;       // uint32 [n_gauss]      per-Gaussian tile count -> offsets
    int64_t off_rects = 0;        // uint16x4 [n_gauss]    tile rectangles
    int64_t off_keys_a = 0;       // uint32 [cap]
    int64_t off_keys_b = 0;       // uint32 [cap]
    int64_t off_vals_b = 0;       // uint32 [cap]
    int64_t off_hist = 0;         // uint32 [radix][hist_blocks]
    int64_t off_part = 0;         // uint64 partial sums of the scans
    int64_t off_counters = 0;     // uint32 [4] at offset 0: tile counters of the persistent
                                  // blend kernels ([0] forward, [1] backward)
    // Bucketed path (fused): pairs are emitted straight into buckets of 256
    // consecutive tile keys, then sorted inside each bucket by the low key byte.
    bool fused = false;
    int64_t n_buckets = 0;        // ceil(n_tiles / 256)
    int64_t n_eblk = 0;           // emission blocks of kEmitBlock Gaussians
    int64_t seg_blocks = 0;       // radix blocks of the in-bucket pass: cap / 4096 + n_buckets
    int64_t off_bucket = 0;       // uint32 [n_buckets][n_eblk] pairs -> first position
    int64_t off_packed = 0;       // uint32 [cap] low key byte << 24 | Gaussian, bucket by bucket
    int64_t off_seg = 0;          // uint32 [2][n_buckets + 1] bucket starts, first radix block
    int64_t off_hseg = 0;         // uint32 [seg_blocks][256] digit counts -> positions
    int64_t total = 0;
};
// Gaussians per emission block of the bucketed path (one workgroup).
constexpr int kEmitBlock = 64;
// The bucketed path's limits: bucket indices fit a byte (n_tiles <= 2^16) and
// a Gaussian index fits the 24 bits below the key byte.
inline bool bin_fused(const bz_opts &o, int64_t n_gauss, int64_t n_tiles) {
    return o.bin_sort == 0 && n_tiles <= 65536 && n_gauss < (int64_t(1) << 24);
}
BinLayout bin_layout(const bz_opts &o, int64_t n_gauss, int64_t cap_pairs);

inline int64_t tiles_x(const bz_opts &o) { return (o.width + o.tile_w - 1) / o.tile_w; }
inline int64_t tiles_y(const bz_opts &o) { return (o.height + o.tile_h - 1) / o.tile_h; }
// Tiles of the canvas, or of all canvases of a batch.
inline int64_t num_tiles(const bz_opts &o) {
    return o.batch ? o.batch->n_tiles : tiles_x(o) * tiles_y(o);
}

// Canvas of an index inside a batch: the last c whose offset (read by off)
// is <= i, over the n_canvas + 1 records (empty canvases are skipped).
template <typename Off>
__host__ __device__ inline int batch_find(const bz_canvas *cv, int n_canvas, int64_t i, Off off) {
    int lo = 0, hi = n_canvas - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off(cv[mid]) <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// LDS of the per-curve backward: boundary samples (2 x double2 per column),
// Bernstein weights and segment per column, then, from a 16-byte boundary,
// the four per-Gaussian stencil terms (float2 each; the sample-point
// gradients overwrite the first).
__host__ __device__ inline int64_t stage2_terms_offset(int64_t max_k) {
    return (2 * 16 * max_k + 16 * max_k + 4 * max_k + 15) & ~int64_t(15);
}
inline int64_t stage2_lds_bytes(int64_t max_k, int64_t max_gauss) {
    return stage2_terms_offset(max_k) + 4 * 8 * max_gauss;
}

// Shape of a Gaussian record: e = (cos t, sin t) / sigma_x along the tangent
// and k = sigma_x / sigma_y (dilated scales), so that
//   d^T Sigma^-1 d = (e . d)^2 + k^2 (e_perp . d)^2,  e_perp = (-e.y, e.x),
// a sum of two squares: no cancellation for elongated Gaussians, where the
// expanded form Qxx dx^2 + 2 Qxy dx dy + Qyy dy^2 loses its value to rounding.
// The conic entries follow from the same identity.
__host__ __device__ inline void shape_conic(float ex, float ey, float k, float &qxx, float &qxy,
                                            float &qyy) {
    const float k2 = k * k;
    qxx = fmaf(k2 * ey, ey, ex * ex);
    qxy = ex * ey * (1.f - k2);
    qyy = fmaf(k2 * ex, ex, ey * ey);
}

// Support of a Gaussian record (mean hi + lo, shape (e, k), opacity) for the
// tile lists: the truncated support 1/2 d^T Sigma^-1 d <= two_p / 2, inflated
// (radius^2 x kCullSlackBox^2, kCullPadBox px) so that float rounding anywhere
// in the pipeline cannot drop a pixel whose kernel value exceeds g_min.
// Sigma = sigma_x^2 t t^T + sigma_y^2 n n^T is formed from (e, k) as sums of
// positive terms: Sigma_xx = (e.x^2 + e.y^2 / k^2) / |e|^4, Sigma_yy likewise,
// Sigma_xy = e.x e.y (1 - 1/k^2) / |e|^4, det = 1 / (k^2 |e|^4).  At a row
// offset dy the ellipse spans x = mx + a dy +- sqrt((r2 - dy^2 / Sigma_yy) D),
// a = Sigma_xy / Sigma_yy, D = det / Sigma_yy; over a band of rows its right
// edge peaks at dy = dys = Sigma_xy sqrt(r2 / Sigma_xx) (the ellipse's
// rightmost point) and its left edge at -dys.  The reciprocals and square
// roots are the hardware ones (about one ulp), far inside the inflation.
struct Support {
    float mx, my;            // mean
    float a, D, isyy, dys;   // row geometry (see above)
    float r2;                // inflated radius^2
    int px0, px1, py0, py1;  // bounding box of the support in pixels, on the canvas
};

// The support of a record; false when it reaches no pixel of the W x H canvas
// or the shape is degenerate.  finite: mean, shape and opacity are finite.
__device__ inline bool support_of(float4 m, float4 q, int W, int H, float two_p, Support &s,
                                  bool &finite) {
    // no contraction: counting and emission must take the same operations
#pragma clang fp contract(off)
    s.mx = m.x + m.z;
    s.my = m.y + m.w;
    const float e2 = q.x * q.x + q.y * q.y;
    finite = isfinite(s.mx) && isfinite(s.my) && isfinite(q.x) && isfinite(q.y) &&
             isfinite(q.z) && isfinite(q.w);
    if (!(finite && e2 > 0.f && q.z > 0.f && isfinite(e2))) return false;
    const float ik2 = __builtin_amdgcn_rcpf(q.z * q.z);
    const float ie4 = __builtin_amdgcn_rcpf(e2 * e2);
    const float sxx = fmaf(q.y * q.y, ik2, q.x * q.x) * ie4;
    const float syy = fmaf(q.x * q.x, ik2, q.y * q.y) * ie4;
    const float sxy = q.x * q.y * (1.f - ik2) * ie4;
    const float det = ik2 * ie4;
    if (!(isfinite(sxx) && isfinite(syy) && isfinite(det) && sxx > 0.f && syy > 0.f)) return false;
    s.r2 = two_p * (kCullSlackBox * kCullSlackBox);
    s.isyy = __builtin_amdgcn_rcpf(syy);
    s.a = sxy * s.isyy;
    s.D = det * s.isyy;
    s.dys = sxy * __builtin_amdgcn_sqrtf(s.r2 * __builtin_amdgcn_rcpf(sxx));
    const float hx = __builtin_amdgcn_sqrtf(two_p * sxx) * kCullSlackBox + kCullPadBox;
    const float hy = __builtin_amdgcn_sqrtf(two_p * syy) * kCullSlackBox + kCullPadBox;
    // pixel x covers centre x + 1/2
    const float fx0 = fmaxf(ceilf(s.mx - hx - 0.5f), 0.f);
    const float fx1 = fminf(floorf(s.mx + hx - 0.5f), (float)(W - 1));
    const float fy0 = fmaxf(ceilf(s.my - hy - 0.5f), 0.f);
    const float fy1 = fminf(floorf(s.my + hy - 0.5f), (float)(H - 1));
    if (!(fx0 <= fx1 && fy0 <= fy1)) return false;
    s.px0 = (int)fx0;
    s.px1 = (int)fx1;
    s.py0 = (int)fy0;
    s.py1 = (int)fy1;
    return true;
}

// Pixel columns [x0, x1] of the support over pixel rows [ya, yb] (inside its
// box); x1 < x0 when it reaches none of them.
__device__ inline void support_cols(const Support &s, int ya, int yb, int &x0, int &x1) {
#pragma clang fp contract(off)
    const float da = (float)ya + 0.5f - s.my, db = (float)yb + 0.5f - s.my;
    const float dr = fminf(fmaxf(s.dys, da), db), dl = fminf(fmaxf(-s.dys, da), db);
    const float hr = __builtin_amdgcn_sqrtf(fmaxf(s.r2 - dr * dr * s.isyy, 0.f) * s.D);
    const float hl = __builtin_amdgcn_sqrtf(fmaxf(s.r2 - dl * dl * s.isyy, 0.f) * s.D);
    const float xr = fmaf(s.a, dr, s.mx) + hr + kCullPadBox;
    const float xl = fmaf(s.a, dl, s.mx) - hl - kCullPadBox;
    x0 = max(s.px0, (int)fmaxf(ceilf(xl - 0.5f), -1.f));
    x1 = min(s.px1, (int)fminf(floorf(xr - 0.5f), 65535.f));
}

// Tile of pixel p (a whole number below 2^16): (p + 1/2) / t lies at least
// 1 / (2t) from a whole number, far beyond the float error of the product,
// so truncating it gives p / t exactly.  inv_t = 1 / tile side.
__device__ inline int tile_of(int p, float inv_t) { return (int)(((float)p + 0.5f) * inv_t); }

// Tile columns [c0, c1] of tile row ty (of height th) that the support
// reaches; c1 < c0 when none.
__device__ inline void support_row(const Support &s, int ty, int th, float inv_tw, int &c0,
                                   int &c1) {
    const int ya = max(ty * th, s.py0), yb = min(ty * th + th - 1, s.py1);
    int x0, x1;
    support_cols(s, ya, yb, x0, x1);
    c0 = tile_of(x0, inv_tw);
    c1 = x0 <= x1 ? tile_of(x1, inv_tw) : c0 - 1;
}

// Tile rows of a record's support: rc = (x0, y0, x1, y1) the tile rectangle
// of its bounding box ((1, 1, 0, 0) when it reaches no pixel), and the
// number of (tile, Gaussian) pairs: the sum over the rectangle's tile rows of
// the tile columns the support itself reaches there (support_row), which
// leaves out the corners of the box that an elongated, rotated Gaussian never
// touches.  finite: the record is finite.  on_row(ty, c0, c1) receives every
// row whose span is not empty.
template <typename F>
__device__ inline uint32_t tile_rect(float4 m, float4 q, int W, int H, float inv_tw,
                                     float inv_th, int th, float two_p, ushort4 &rc,
                                     bool &finite, F on_row) {
    Support s;
    rc = make_ushort4(1, 1, 0, 0);
    if (!support_of(m, q, W, H, two_p, s, finite)) return 0u;
    const int ty0 = tile_of(s.py0, inv_th), ty1 = tile_of(s.py1, inv_th);
    rc = make_ushort4(tile_of(s.px0, inv_tw), ty0, tile_of(s.px1, inv_tw), ty1);
    uint32_t n = 0;
    for (int ty = ty0; ty <= ty1; ++ty) {
        int c0, c1;
        support_row(s, ty, th, inv_tw, c0, c1);
        if (c1 >= c0) {
            n += (uint32_t)(c1 - c0 + 1);
            on_row(ty, c0, c1);
        }
    }
    return n;
}
__device__ inline uint32_t tile_rect(float4 m, float4 q, int W, int H, float inv_tw,
                                     float inv_th, int th, float two_p, ushort4 &rc,
                                     bool &finite) {
    return tile_rect(m, q, W, H, inv_tw, inv_th, th, two_p, rc, finite, [](int, int, int) {});
}

// Where sampling writes the tile counts and rectangles for the binning that
// follows it (bz_sample_bin): the binning workspace's arrays, the tile shape
// and the support constant.
struct BinCount {
    uint32_t *counts;      // per-Gaussian tile counts (two-pass radix path), or null
    ushort4 *rects;
    int64_t *status;
    float inv_tw, inv_th;
    int th;
    float two_p;
    // bucketed path: pairs per (key bucket, emission block), added to
    // bucket[h * n_eblk + g / kEmitBlock]; null on the radix path
    uint32_t *bucket;
    int64_t n_eblk;
    int n_buckets;
    int tiles_x;           // tiles per row of the canvas (single canvas)
};

// The key buckets (key >> 8) a tile-row span of keys [k0, k0 + w) falls in,
// with the part in each: f(h, count).
template <typename F>
__device__ inline void for_key_buckets(uint32_t k0, uint32_t w, F f) {
    const uint32_t k1 = k0 + w;
    for (uint32_t k = k0; k < k1;) {
        const uint32_t h = k >> 8;
        const uint32_t e = min(k1, (h + 1u) << 8);
        f(h, e - k);
        k = e;
    }
}

// Visit masks: one plane per 8x8 quad of a tile; a plane holds, for every tile,
// ceil(len/64) words starting at word start/64 + tile (see visit_word).
inline int64_t visit_words_per_plane(const bz_opts &o, int64_t cap_pairs) {
    return cap_pairs / 64 + num_tiles(o) + 2;
}
inline int64_t visit_words(const bz_opts &o, int64_t cap_pairs) {
    return (int64_t)(o.tile_w / 8) * (o.tile_h / 8) * visit_words_per_plane(o, cap_pairs);
}

}  // namespace bz
