// bz_api.hip -- the C ABI of libbz: host-side validation and launches.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "bz_internal.h"

using namespace bz;

// Binning workspace of bz_sample_bin_static: a fixed device array that every
// call on a device shares.  In host code `scratch` names a host-side stand-in,
// not the device memory: the device address comes from hipGetSymbolAddress
// (static_scratch below), once per device.
static __device__ __align__(256) unsigned char scratch[BZ_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call there (with that device current) and kept for later calls.
bz_status static_scratch(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BZ_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BZ_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BZ_OK;
}

// Per-curve limits of the per-curve kernels (LDS sizes).
constexpr int kMaxK = 1024;
constexpr int kMaxR = 254;
constexpr int64_t kMaxLdsBytes = 152 * 1024;   // dynamic LDS of the per-curve kernels (160 KB per CU on gfx950, static use ~2 KB)

bool finite_pos(float v) { return isfinite(v) && v > 0.f; }

bz_status check_opts(const bz_opts *o) {
    if (!o) return BZ_ERR_ARG;
    if (o->width < 1 || o->height < 1 || o->width > 32768 || o->height > 32768) return BZ_ERR_ARG;
    if (o->tile_w < 8 || o->tile_h < 8 || o->tile_w % 8 || o->tile_h % 8) return BZ_ERR_ARG;
    int64_t tp = (int64_t)o->tile_w * o->tile_h;
    if (tp < 64 || tp > 1024) return BZ_ERR_ARG;
    if (!finite_pos(o->rho) || !isfinite(o->sigma0_sq) || o->sigma0_sq < 0.f) return BZ_ERR_ARG;
    if (!(o->g_min > 0.f && o->g_min < 1.f)) return BZ_ERR_ARG;
    if (!(o->alpha_max > 0.f && o->alpha_max <= 1.f)) return BZ_ERR_ARG;
    if (!(o->t_min >= 0.f && o->t_min < 1.f)) return BZ_ERR_ARG;
    for (int c = 0; c < 3; ++c)
        if (!isfinite(o->bg[c])) return BZ_ERR_ARG;
    if (o->persistent != 0 && o->persistent != 1) return BZ_ERR_ARG;
    if (o->bin_sort != 0 && o->bin_sort != 1) return BZ_ERR_ARG;
    if (o->batch) {
        const bz_batch *bt = o->batch;
        if (bt->n_canvas < 1 || !bt->canvas || bt->n_tiles < bt->n_canvas || bt->n_pixels < 1 ||
            bt->n_gauss < 0)
            return BZ_ERR_ARG;
    }
    if (num_tiles(*o) > (int64_t(1) << 24)) return BZ_ERR_UNSUPPORTED;
    return BZ_OK;
}

bz_status check_curves(const bz_curves *c) {
    if (!c || c->n_curves < 0 || c->n_gauss < 0) return BZ_ERR_ARG;
    if (c->n_gauss >= (int64_t(1) << 32)) return BZ_ERR_UNSUPPORTED;
    if (c->n_curves == 0) return c->n_gauss == 0 ? BZ_OK : BZ_ERR_ARG;
    if (!c->kind || !c->nseg || !c->k_samples || !c->r_interior || !c->ctrl || !c->ctrl_off ||
        !c->tau || !c->tau_off || !c->stroke_w || !c->color || !c->opacity || !c->opa_off ||
        !c->order || !c->gauss_off)
        return BZ_ERR_ARG;
    if (c->max_k < 2 || c->max_k > kMaxK || c->max_gauss_per_curve < 2) return BZ_ERR_ARG;
    return BZ_OK;
}

bz_status check_bins(const bz_bins *b, const bz_opts *o, int64_t n_gauss, bool need_ws) {
    if (!b || !b->ids || !b->ranges || !b->status) return BZ_ERR_ARG;
    if (b->cap_pairs < 0 || b->cap_pairs >= (int64_t(1) << 32)) return BZ_ERR_ARG;
    if (need_ws) {
        if (!b->workspace || ((uintptr_t)b->workspace & 255)) return BZ_ERR_ARG;
        if (b->workspace_bytes < bin_layout(*o, n_gauss, b->cap_pairs).total)
            return BZ_ERR_CAPACITY;
    }
    return BZ_OK;
}

bz_status launched(hipError_t e) { return e == hipSuccess ? BZ_OK : BZ_ERR_HIP; }

// The blend calls of a persistent launch keep their tile counters at the start
// of the bin workspace.
bz_status check_persistent(const bz_bins *b, const bz_opts *o) {
    if (!o->persistent) return BZ_OK;
    if (!b->workspace || ((uintptr_t)b->workspace & 255) || b->workspace_bytes < 256)
        return BZ_ERR_ARG;
    return BZ_OK;
}

int64_t stage2_lds(const bz_curves *c) {
    return stage2_lds_bytes(c->max_k, c->max_gauss_per_curve);
}

}  // namespace

extern "C" {

const char *bz_status_str(bz_status s) {
    switch (s) {
        case BZ_OK: return "ok";
        case BZ_ERR_ARG: return "invalid argument";
        case BZ_ERR_CAPACITY: return "buffer too small";
        case BZ_ERR_HIP: return "HIP launch failed";
        case BZ_ERR_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

bz_status bz_layout_host(int32_t n, const int32_t *kind, const int32_t *nseg,
                         const int32_t *k_samples, const int32_t *r_interior,
                         const int32_t *ctrl_off, const int32_t *tau_off,
                         const int32_t *opa_off, const int32_t *rank, int32_t *order,
                         int64_t *gauss_off, int32_t *max_gauss, int32_t *max_k) {
    if (n < 0 || !gauss_off) return BZ_ERR_ARG;
    if (n > 0 && (!kind || !nseg || !k_samples || !r_interior || !ctrl_off || !tau_off ||
                  !opa_off || !rank || !order))
        return BZ_ERR_ARG;
    if (n > 0 && (ctrl_off[0] != 0 || tau_off[0] != 0 || opa_off[0] != 0)) return BZ_ERR_ARG;
    std::vector<char> seen((size_t)n, 0);
    std::vector<int64_t> per((size_t)n, 0);
    int32_t mg = 0, mk = 0;
    bz_status unsupported = BZ_OK;
    for (int32_t i = 0; i < n; ++i) {
        int S = nseg[i], K = k_samples[i];
        bool closed = kind[i] == BZ_CLOSED;
        if (kind[i] != BZ_OPEN && !closed) return BZ_ERR_ARG;
        if (S < 1 || K < 2) return BZ_ERR_ARG;
        int R = closed ? r_interior[i] : 0;
        if (R < 0) return BZ_ERR_ARG;
        if (S > kMaxSeg || K > kMaxK || R > kMaxR) unsupported = BZ_ERR_UNSUPPORTED;
        int64_t need_ctrl = closed ? 6 * (int64_t)S : 3 * (int64_t)S + 1;
        if ((int64_t)ctrl_off[i + 1] - ctrl_off[i] != need_ctrl) return BZ_ERR_ARG;
        if ((int64_t)tau_off[i + 1] - tau_off[i] < R + 2) return BZ_ERR_ARG;
        int nopa = opa_off[i + 1] - opa_off[i];
        if (nopa != 1 && nopa != S) return BZ_ERR_ARG;
        if (rank[i] < 0 || rank[i] >= n || seen[(size_t)rank[i]]) return BZ_ERR_ARG;
        seen[(size_t)rank[i]] = 1;
        order[rank[i]] = i;
        int64_t ng = (int64_t)K * (closed ? R + 2 : 1);
        per[(size_t)i] = ng;
        if (ng > mg) mg = (int32_t)(ng > 0x7fffffff ? 0x7fffffff : ng);
        if (K > mk) mk = K;
    }
    gauss_off[0] = 0;
    for (int32_t p = 0; p < n; ++p) gauss_off[p + 1] = gauss_off[p] + per[(size_t)order[p]];
    if (max_gauss) *max_gauss = mg;
    if (max_k) *max_k = mk;
    if (unsupported != BZ_OK) return unsupported;
    if (stage2_lds_bytes(mk, mg) > kMaxLdsBytes) return BZ_ERR_UNSUPPORTED;
    return BZ_OK;
}

bz_status bz_num_tiles(const bz_opts *o, int64_t *n_tiles) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if (!n_tiles) return BZ_ERR_ARG;
    *n_tiles = num_tiles(*o);
    return BZ_OK;
}

bz_status bz_batch_layout(const bz_opts *o, int32_t n, const int32_t *size, const float *bg,
                          const int64_t *gauss_off, const int32_t *curve_off, bz_canvas *canvas,
                          bz_batch *batch) {
    if (!o || n < 1 || !size || !gauss_off || !curve_off || !canvas || !batch) return BZ_ERR_ARG;
    if (o->tile_w < 8 || o->tile_h < 8 || o->tile_w % 8 || o->tile_h % 8) return BZ_ERR_ARG;
    if (gauss_off[0] != 0 || curve_off[0] != 0) return BZ_ERR_ARG;
    int64_t tile = 0, pix = 0;
    for (int32_t c = 0; c < n; ++c) {
        const int32_t W = size[2 * c], H = size[2 * c + 1];
        if (W < 1 || H < 1 || W > 32768 || H > 32768) return BZ_ERR_ARG;
        if (gauss_off[c + 1] < gauss_off[c] || curve_off[c + 1] < curve_off[c]) return BZ_ERR_ARG;
        bz_canvas &r = canvas[c];
        memset(&r, 0, sizeof(r));
        r.width = W;
        r.height = H;
        r.tiles_x = (W + o->tile_w - 1) / o->tile_w;
        r.tiles_y = (H + o->tile_h - 1) / o->tile_h;
        r.tile_off = tile;
        r.pix_off = pix;
        r.gauss_off = gauss_off[c];
        r.curve_off = curve_off[c];
        for (int k = 0; k < 3; ++k) {
            r.bg[k] = bg ? bg[3 * c + k] : o->bg[k];
            if (!isfinite(r.bg[k])) return BZ_ERR_ARG;
        }
        tile += (int64_t)r.tiles_x * r.tiles_y;
        pix += (int64_t)W * H;
    }
    bz_canvas &end = canvas[n];
    memset(&end, 0, sizeof(end));
    end.tile_off = tile;
    end.pix_off = pix;
    end.gauss_off = gauss_off[n];
    end.curve_off = curve_off[n];
    batch->n_canvas = n;
    batch->n_tiles = tile;
    batch->n_pixels = pix;
    batch->n_gauss = gauss_off[n];
    if (tile > (int64_t(1) << 24)) return BZ_ERR_UNSUPPORTED;
    return BZ_OK;
}

bz_status bz_visit_words(const bz_opts *o, int64_t cap_pairs, int64_t *words) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if (!words || cap_pairs < 0 || cap_pairs >= (int64_t(1) << 32)) return BZ_ERR_ARG;
    *words = visit_words(*o, cap_pairs);
    return BZ_OK;
}

bz_status bz_workspace_size(const bz_opts *o, int64_t n_gauss, int64_t cap_pairs, int64_t *bytes) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if (!bytes || n_gauss < 0 || cap_pairs < 0 || cap_pairs >= (int64_t(1) << 32))
        return BZ_ERR_ARG;
    *bytes = bin_layout(*o, n_gauss, cap_pairs).total;
    return BZ_OK;
}

bz_status bz_sample(const bz_curves *c, const bz_opts *o, bz_gaussians *g, hipStream_t s) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if ((st = check_curves(c)) != BZ_OK) return st;
    if (!g || (c->n_gauss > 0 && !g->rec)) return BZ_ERR_ARG;
    if ((uintptr_t)g->rec & 15) return BZ_ERR_ARG;
    if (g->cap < c->n_gauss) return BZ_ERR_CAPACITY;
    if (c->n_curves > 0 && 2 * 16 * (int64_t)c->max_k > kMaxLdsBytes) return BZ_ERR_UNSUPPORTED;
    (void)hipGetLastError();
    g->n = c->n_gauss;
    return launched(launch_sample(*c, *o, g->rec, nullptr, s));
}

// Arguments of bz_sample_bin other than the bin workspace.
static bz_status check_sample_bin(const bz_curves *c, const bz_opts *o, const bz_gaussians *g,
                                  const bz_bins *b) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if ((st = check_curves(c)) != BZ_OK) return st;
    if (!g || (c->n_gauss > 0 && !g->rec)) return BZ_ERR_ARG;
    if ((uintptr_t)g->rec & 15) return BZ_ERR_ARG;
    if (g->cap < c->n_gauss) return BZ_ERR_CAPACITY;
    if (c->n_curves > 0 && 2 * 16 * (int64_t)c->max_k > kMaxLdsBytes) return BZ_ERR_UNSUPPORTED;
    if (c->n_gauss >= (int64_t(1) << 32)) return BZ_ERR_UNSUPPORTED;
    if (o->batch && o->batch->n_gauss != c->n_gauss) return BZ_ERR_ARG;
    return check_bins(b, o, c->n_gauss, false);
}

bz_status bz_sample_bin(const bz_curves *c, const bz_opts *o, bz_gaussians *g, bz_bins *b,
                        hipStream_t s) {
    bz_status st = check_sample_bin(c, o, g, b);
    if (st != BZ_OK) return st;
    if ((st = check_bins(b, o, c->n_gauss, true)) != BZ_OK) return st;
    (void)hipGetLastError();
    g->n = c->n_gauss;
    return launched(launch_sample_bin(*c, *o, g->rec, *b, s));
}

bz_status bz_sample_bin_static(const bz_curves *c, const bz_opts *o, bz_gaussians *g,
                               bz_bins *b, hipStream_t s) {
    bz_status st = check_sample_bin(c, o, g, b);
    if (st != BZ_OK) return st;
    // sizes first, on the host: nothing touches the device for a call that
    // cannot fit
    if (bin_layout(*o, c->n_gauss, b->cap_pairs).total > (int64_t)BZ_STATIC_SCRATCH_BYTES)
        return BZ_ERR_CAPACITY;
    void *ws = nullptr;
    if ((st = static_scratch(&ws)) != BZ_OK) return st;
    bz_bins bs = *b;
    bs.workspace = ws;
    bs.workspace_bytes = BZ_STATIC_SCRATCH_BYTES;
    (void)hipGetLastError();
    g->n = c->n_gauss;
    return launched(launch_sample_bin(*c, *o, g->rec, bs, s));
}

bz_status bz_bin(const bz_gaussians *g, const bz_opts *o, bz_bins *b, hipStream_t s) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if (!g || g->n < 0 || g->n > g->cap || (g->n > 0 && !g->rec)) return BZ_ERR_ARG;
    if (g->n >= (int64_t(1) << 32)) return BZ_ERR_UNSUPPORTED;
    if (o->batch && o->batch->n_gauss != g->n) return BZ_ERR_ARG;
    if ((st = check_bins(b, o, g->n, true)) != BZ_OK) return st;
    (void)hipGetLastError();
    return launched(launch_bin(g->rec, g->n, *o, *b, s));
}

// Blend state: absent (recomputed by the backward), or complete and large enough.
static bz_status check_state(const bz_pixstate *state, const bz_opts *o, const bz_bins *b) {
    if (!state) return BZ_OK;
    if (!state->t_final || !state->n_last || !state->visit) return BZ_ERR_ARG;
    if (state->visit_words < visit_words(*o, b->cap_pairs)) return BZ_ERR_CAPACITY;
    return BZ_OK;
}

bz_status bz_render_fwd(const bz_gaussians *g, const bz_bins *b, const bz_opts *o, float *image,
                        bz_pixstate *state, hipStream_t s) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if (!g || g->n < 0 || (g->n > 0 && !g->rec)) return BZ_ERR_ARG;
    if ((st = check_bins(b, o, g->n, false)) != BZ_OK) return st;
    if (!image) return BZ_ERR_ARG;
    if ((st = check_state(state, o, b)) != BZ_OK) return st;
    if ((st = check_persistent(b, o)) != BZ_OK) return st;
    (void)hipGetLastError();
    return launched(launch_fwd(g->rec, *b, *o, image, state, nullptr, s));
}

bz_status bz_render_fwd_l2(const bz_gaussians *g, const bz_bins *b, const bz_opts *o, float *image,
                           bz_pixstate *state, const float *target, float scale, float *d_image,
                           float *loss, hipStream_t s) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if (!g || g->n < 0 || (g->n > 0 && !g->rec)) return BZ_ERR_ARG;
    if ((st = check_bins(b, o, g->n, false)) != BZ_OK) return st;
    if (!image || !target || !d_image || d_image == image) return BZ_ERR_ARG;
    if (!isfinite(scale)) return BZ_ERR_ARG;
    if ((st = check_state(state, o, b)) != BZ_OK) return st;
    if ((st = check_persistent(b, o)) != BZ_OK) return st;
    (void)hipGetLastError();
    const L2Out l2 = {target, d_image, loss, scale};
    return launched(launch_fwd(g->rec, *b, *o, image, state, &l2, s));
}

bz_status bz_render_bwd_gauss(const bz_gaussians *g, const bz_bins *b, const bz_opts *o,
                              const float *d_image, const bz_pixstate *state, float *d_gauss,
                              hipStream_t s) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if (!g || g->n < 0 || (g->n > 0 && (!g->rec || !d_gauss))) return BZ_ERR_ARG;
    if ((st = check_bins(b, o, g->n, false)) != BZ_OK) return st;
    if (!d_image) return BZ_ERR_ARG;
    if ((st = check_state(state, o, b)) != BZ_OK) return st;
    if ((st = check_persistent(b, o)) != BZ_OK) return st;
    if (!(o->alpha_max < 1.f)) return BZ_ERR_UNSUPPORTED;
    (void)hipGetLastError();
    return launched(launch_bwd_gauss(g->rec, g->n, *b, *o, d_image, state, d_gauss, s));
}

bz_status bz_render_bwd_curves(const bz_curves *c, const bz_opts *o, const float *d_gauss,
                               bz_grads *gr, hipStream_t s) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if ((st = check_curves(c)) != BZ_OK) return st;
    if (!gr) return BZ_ERR_ARG;
    if (c->n_curves > 0 &&
        (!d_gauss || !gr->d_ctrl || !gr->d_width || !gr->d_color || !gr->d_opacity))
        return BZ_ERR_ARG;
    if (c->n_curves > 0 && stage2_lds(c) > kMaxLdsBytes) return BZ_ERR_UNSUPPORTED;
    (void)hipGetLastError();
    return launched(launch_bwd_curves(*c, *o, d_gauss, *gr, s));
}

bz_status bz_render_bwd(const bz_curves *c, const bz_gaussians *g, const bz_bins *b,
                        const bz_opts *o, const float *d_image, const bz_pixstate *state,
                        bz_grads *gr, hipStream_t s) {
    bz_status st = check_opts(o);
    if (st != BZ_OK) return st;
    if ((st = check_curves(c)) != BZ_OK) return st;
    if (!g || g->n != c->n_gauss) return BZ_ERR_ARG;
    if (!gr || (c->n_curves > 0 && !gr->d_gauss)) return BZ_ERR_ARG;
    if ((st = bz_render_bwd_gauss(g, b, o, d_image, state, gr->d_gauss, s)) != BZ_OK) return st;
    return bz_render_bwd_curves(c, o, gr->d_gauss, gr, s);
}

bz_status bz_curve_area(const bz_curves *c, float *area, hipStream_t s) {
    bz_status st = check_curves(c);
    if (st != BZ_OK) return st;
    if (c->n_curves > 0 && !area) return BZ_ERR_ARG;
    (void)hipGetLastError();
    return launched(launch_area(*c, area, s));
}

bz_status bz_area_order_workspace(int32_t n, int64_t *bytes) {
    if (n < 0 || !bytes) return BZ_ERR_ARG;
    *bytes = order_workspace_bytes(n);
    return BZ_OK;
}

bz_status bz_area_order(const bz_curves *c, const bz_opts *o, float *area, int32_t *order,
                        int64_t *gauss_off, void *ws, int64_t ws_bytes, hipStream_t s) {
    bz_status st = check_curves(c);
    if (st != BZ_OK) return st;
    const bz_batch *batch = o ? o->batch : nullptr;
    if (batch && (batch->n_canvas < 1 || batch->n_canvas > 65535 || !batch->canvas))
        return BZ_ERR_ARG;
    if (c->n_curves > 0 && (!area || !order || !gauss_off || !ws)) return BZ_ERR_ARG;
    if (c->n_curves > 0 && ((uintptr_t)ws & 255)) return BZ_ERR_ARG;
    if (ws_bytes < order_workspace_bytes(c->n_curves)) return BZ_ERR_CAPACITY;
    (void)hipGetLastError();
    return launched(launch_area_order(*c, batch, area, order, gauss_off, ws, s));
}

bz_status bz_xing_loss(const bz_curves *c, float weight, float *loss, float *d_ctrl,
                       hipStream_t s) {
    bz_status st = check_curves(c);
    if (st != BZ_OK) return st;
    if (!isfinite(weight) || (c->n_curves > 0 && !d_ctrl)) return BZ_ERR_ARG;
    (void)hipGetLastError();
    return launched(launch_xing(*c, weight, loss, d_ctrl, s));
}

bz_status bz_l2_grad(const float *image, const float *target, int64_t n, float scale,
                     float *d_image, float *loss, hipStream_t s) {
    if (n < 0 || (n > 0 && (!image || !target || !d_image))) return BZ_ERR_ARG;
    if (!isfinite(scale)) return BZ_ERR_ARG;
    (void)hipGetLastError();
    return launched(launch_l2(image, target, n, scale, d_image, loss, s));
}

}  // extern "C"
