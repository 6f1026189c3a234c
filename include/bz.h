/*
 * bz.h -- C ABI of libbz, the MI355X (gfx950) rasterizer of Bezier Splatting
 * ("Bezier Splatting for Fast and Differentiable Vector Graphics Rendering",
 * arXiv 2503.16424).
 *
 * Problem statement (Sec. 3.5, "Training objective"): curves are laid on a
 * canvas, rendered by a differentiable rasterizer into an image, and optimised
 * through gradients of any image loss.  The library provides that rasterizer:
 *
 *   bz_sample      curves -> 2D Gaussians                    (Sec. 3.3)
 *   bz_bin         Gaussians -> per-tile lists in draw order (Sec. 3.4, tile pipeline);
 *                  bz_sample_bin does both in one call
 *   bz_render_fwd  per-tile front-to-back alpha blending     (Sec. 3.4, blending sum)
 *   bz_render_bwd  reverse-order gradients to Gaussians, then to curve
 *                  control points, widths, colours, opacities
 *   bz_l2_grad     the L2 loss gradient of an image          (Sec. 3.5); also fused
 *                  into the forward as bz_render_fwd_l2
 *
 * Conventions shared by every call:
 *  - Pointers inside the structs and the image/gradient pointers are DEVICE
 *    pointers owned by the caller; functions marked "host" take host pointers.
 *    The library never allocates or frees memory and keeps no global state,
 *    except the fixed device array of bz_sample_bin_static (see there).
 *  - Every device call is asynchronous and ordered on the caller's stream; no
 *    call synchronises.  The return code reports argument errors (BZ_ERR_ARG,
 *    BZ_ERR_UNSUPPORTED) detected on the host before anything is launched, and
 *    launch errors (BZ_ERR_HIP).  Data-dependent failures (tile-list overflow,
 *    non-finite Gaussians) are reported through the device status words of
 *    bz_bins, never silently.
 *  - Coordinates are pixels; pixel (x, y) has its centre at (x + 1/2, y + 1/2).
 *    Images are planar float32 [3][height][width].
 *  - Colours and opacities are activated values in [0, 1]; gradients are with
 *    respect to exactly the values passed in.
 *  - Calls on distinct buffers may run concurrently on different streams.
 */
#ifndef BZ_H
#define BZ_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BZ_OK = 0,
    BZ_ERR_ARG = -1,          /* invalid argument (null pointer, bad size, bad option) */
    BZ_ERR_CAPACITY = -2,     /* a host-known size exceeds a caller buffer */
    BZ_ERR_HIP = -3,          /* kernel launch failed */
    BZ_ERR_UNSUPPORTED = -4   /* valid but outside what the library supports */
} bz_status;

/* Kind of a curve (Sec. 3.2). */
#define BZ_OPEN 0     /* stroke: S cubic segments, 3S+1 control points, a width */
#define BZ_CLOSED 1   /* paired boundaries A, B sharing endpoints: 6S points, filled */

/* One canvas of a batch: many canvases of different sizes share one tile
 * space, one tile-list sort and one launch per stage.  Filled on the host by
 * bz_batch_layout and copied to the device by the caller.
 *   tile_off  : first global tile of the canvas (its tiles are row-major)
 *   pix_off   : first pixel: the canvas's image is image + 3*pix_off, planar
 *               [3][height][width]; per-pixel state starts at pix_off
 *   gauss_off : first Gaussian; the canvas's curves are consecutive in draw
 *               order, so its Gaussians are [gauss_off, next gauss_off).
 *   curve_off : first curve (by index) of the canvas; its curves are
 *               consecutive by index too. */
typedef struct {
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    int64_t tile_off, pix_off, gauss_off;
    float bg[3];
    int32_t curve_off;
} bz_canvas;

/* A batch of canvases.  canvas: device array of n_canvas + 1 records, the last
 * one holding the totals (tile_off = n_tiles, pix_off = n_pixels, gauss_off =
 * n_gauss).  n_tiles, n_pixels, n_gauss: host copies of the totals. */
typedef struct {
    int32_t n_canvas;
    int64_t n_tiles, n_pixels, n_gauss;
    const bz_canvas *canvas;
} bz_batch;

/* Rendering options (host struct, passed by pointer, read during the call). */
typedef struct {
    int32_t width, height;   /* canvas in pixels, 1..32768 each */
    float bg[3];             /* background colour composited with T_final */
    float rho;               /* density constant of Eq. sigma (> 0); 2.0 */
    float sigma0_sq;         /* isotropic screen dilation added to both squared
                                scales, px^2 (>= 0); 0.3 */
    float g_min;             /* kernel truncation: Gt = (G - g_min)_+/(1 - g_min),
                                0 < g_min < 1; 1/255 */
    float alpha_max;         /* alpha clamp, (0, 1]; 0.99 */
    float t_min;             /* a pixel stops after the contributor that brings its
                                transmittance below t_min, [0, 1); 1e-6 */
    int32_t tile_w, tile_h;  /* binning tile: multiples of 8, product 64..1024.
                                Results do not depend on the tile shape. */
    int32_t persistent;      /* tuning: 0 = one workgroup per tile; 1 = the blend
                                kernels run as many workgroups as fit on the GPU at
                                once, each taking tiles from a counter in
                                bz_bins.workspace.  Results do not depend on it. */
    int32_t bin_sort;        /* tuning: 0 = automatic: with at most 65,536 tiles and
                                fewer than 2^24 Gaussians, pairs are emitted straight
                                into buckets of 256 consecutive tiles and sorted
                                inside each bucket by one radix pass; otherwise, and
                                with 1, the (tile, Gaussian) pairs take a two-pass
                                radix sort on the tile.  Results do not depend on it;
                                the workspace size does. */
    const bz_batch *batch;   /* NULL: one canvas of width x height with bg.  Else
                                the canvases of the batch (host struct; width,
                                height and bg above are then unused). */
} bz_opts;

/* Curve set, structure of arrays on the device.
 *
 *   kind[i], nseg[i] = S (1..4), k_samples[i] = K (2..1024), r_interior[i] = R
 *   (0..254, closed only; ignored for open curves).
 *   ctrl[ctrl_off[i] .. ctrl_off[i+1]) : float2 control points.  Open: 3S+1
 *       points.  Closed: boundary A's 3S+1 points, then boundary B's 3S-1
 *       interior points (B shares A's first and last point).
 *   tau[tau_off[i] ..]: R+2 row interpolation weights of a closed curve,
 *       tau[0] = 0 and tau[R+1] = 1 (Sec. 3.3, rows sampled from a normalised CDF).
 *   stroke_w[i]  : stroke width of an open curve (sigma_y before dilation).
 *   color[i][3]  : RGB.
 *   opacity[opa_off[i] .. opa_off[i+1]) : 1 value, or S values (one per segment).
 *   order[p]     : the curve drawn at position p (p = 0 in front); a permutation.
 *   gauss_off[p] : first Gaussian of the curve drawn at position p; the curve has
 *       K (open) or K*(R+2) (closed) Gaussians; gauss_off[n_curves] = n_gauss.
 *   order and gauss_off are produced on the host by bz_layout_host.
 *   max_gauss_per_curve: the largest per-curve Gaussian count (from bz_layout_host).
 */
typedef struct {
    int32_t n_curves;
    int64_t n_gauss;
    int32_t max_gauss_per_curve;
    int32_t max_k;
    const int32_t *kind, *nseg, *k_samples, *r_interior;
    const float *ctrl;
    const int32_t *ctrl_off;
    const float *tau;
    const int32_t *tau_off;
    const float *stroke_w;
    const float *color;
    const float *opacity;
    const int32_t *opa_off;
    const int32_t *order;
    const int64_t *gauss_off;
} bz_curves;

/* Gaussians, one 48-byte record (12 floats) per Gaussian in draw order:
 *   [0..1]  mean, high float part (x, y)
 *   [2..3]  mean, low part: mean = hi + lo to ~2^-48 relative (the mean is
 *           computed in double precision)
 *   [4..6]  shape (e.x, e.y, k) in the covariance's principal frame (Eq. RSSR):
 *           e = (cos t, sin t) / sigma_x with (cos t, sin t) the unit tangent of
 *           Eq. rotation, k = sigma_x / sigma_y (dilated scales), so that
 *           Q = Sigma^-1 = e e^T + k^2 e' e'^T with e' = (-e.y, e.x), and
 *           p = 1/2 d^T Q d = 1/2 ((e . d)^2 + k^2 (e' . d)^2), d = pixel - mean.
 *           (A sum of squares keeps p accurate in float32 for elongated
 *           Gaussians, where the expanded conic form cancels.)
 *   [7]     opacity o
 *   [8..10] colour
 *   [11]    curve id (int32 bit pattern)
 * rec must be 16-byte aligned and hold cap records; n is the number of valid
 * records (set by bz_sample). */
typedef struct {
    int64_t cap;
    int64_t n;
    float *rec;
} bz_gaussians;

/* Tile lists.  ids[ranges[2t] .. ranges[2t+1]) are the Gaussians whose support
 * may reach a pixel of tile t (row-major tiles), in increasing draw order.
 * status (device, 4 x int64): [0] pairs required by the last bz_bin,
 * [1] flags: bit 0 = the lists are invalid (ids capacity exceeded, or bit 2)
 * and the render calls fill the image with NaN, bit 1 = non-finite Gaussian
 * skipped, bit 2 = a Gaussian's emitted tiles disagreed with its count (an
 * internal consistency check; never expected).
 * workspace: device scratch of bz_workspace_size bytes, 256-byte aligned. */
typedef struct {
    int64_t cap_pairs;       /* capacity of ids, < 2^32 */
    uint32_t *ids;
    uint32_t *ranges;        /* [n_tiles][2] */
    void *workspace;
    int64_t workspace_bytes;
    int64_t *status;
} bz_bins;

/* Forward state kept for the reverse pass (blend state).  The render calls
 * take a NULL state instead: the forward then writes only the image and the
 * reverse pass recomputes the state tile by tile (one extra front-to-back
 * sweep without colour, no per-pixel memory).  Both calls of one step must
 * agree: a NULL-state forward is followed by a NULL-state backward.
 * t_final, n_last: [height][width].  n_last bounds the tile-list positions of the
 *   pixel's contributors: for a pixel whose blend stopped (T below t_min) it is
 *   1 + the position of the contributor that stopped it; otherwise the end of
 *   the last 64-entry batch that contributed to the pixel's 8x8 block (capped
 *   at the list length).  Every entry before it with G > g_min contributed to
 *   the pixel and no entry at or after it did.
 * n_contrib (optional, may be NULL): contributors per pixel, [height][width].
 * visit: per 8x8 pixel block and per 64-entry batch of its tile list, the bit
 *   mask of entries that contributed to at least one pixel of the block; the
 *   reverse pass visits only those.  visit_words 64-bit words, at least what
 *   bz_visit_words reports for the same options and cap_pairs.  Written by
 *   bz_render_fwd, read by bz_render_bwd; no initialisation needed. */
typedef struct {
    float *t_final;
    uint32_t *n_last;
    uint32_t *n_contrib;
    uint64_t *visit;
    int64_t visit_words;
} bz_pixstate;

/* Gradients.  Per curve, same layouts as the inputs: d_ctrl [n_ctrl][2],
 * d_width [n_curves], d_color [n_curves][3], d_opacity [n_opa].  d_gauss is
 * required scratch and output: per-Gaussian gradients as 9 planes of n_gauss
 * floats: (mean x, mean y, Qxx, Qxy, Qyy, o, r, g, b), the conic entries being
 * those of p = 1/2 (Qxx dx^2 + 2 Qxy dx dy + Qyy dy^2).  bz_render_bwd overwrites
 * all of them (the caller need not zero them). */
typedef struct {
    float *d_ctrl, *d_width, *d_color, *d_opacity;
    float *d_gauss;
} bz_grads;

/* Host: validate a curve set's sizes and build order[] (inverse of rank,
 * rank 0 = front) and gauss_off[] (n_curves + 1 entries).  All pointers are
 * HOST pointers; ctrl_off, tau_off and opa_off have n_curves + 1 entries and
 * are checked against kind/S/R (3S+1 or 6S points, at least R+2 weights, 1 or
 * S opacities).  max_gauss and max_k (optional) receive the largest per-curve
 * Gaussian count and K.  Draw order: depth is assigned per curve (Sec. 3.3),
 * and inside a curve Gaussians follow row-major (r, k) order.
 * Returns BZ_ERR_ARG on any inconsistency, BZ_ERR_UNSUPPORTED for S > 4,
 * K > 1024, R > 254 or a curve whose Gaussians exceed the per-curve limit. */
bz_status bz_layout_host(int32_t n_curves, const int32_t *kind, const int32_t *nseg,
                         const int32_t *k_samples, const int32_t *r_interior,
                         const int32_t *ctrl_off, const int32_t *tau_off,
                         const int32_t *opa_off, const int32_t *rank, int32_t *order,
                         int64_t *gauss_off, int32_t *max_gauss, int32_t *max_k);

/* Host: bytes of workspace bz_bin needs for n_gauss Gaussians and cap_pairs pairs. */
bz_status bz_workspace_size(const bz_opts *opts, int64_t n_gauss, int64_t cap_pairs,
                            int64_t *bytes);

/* Host: number of tiles of the canvas (or of all canvases of opts->batch)
 * for the options' tile shape. */
bz_status bz_num_tiles(const bz_opts *opts, int64_t *n_tiles);

/* Host: lay out a batch of n_canvas canvases for the tile shape of opts.
 * size: [n_canvas][2] width, height (1..32768); bg: [n_canvas][3] or NULL (all
 * opts->bg); gauss_off: [n_canvas + 1] first Gaussian of every canvas and the
 * total, non-decreasing from 0; curve_off: [n_canvas + 1] first curve (by
 * index) of every canvas and the total, non-decreasing from 0.  Writes
 * canvas[0 .. n_canvas] (n_canvas + 1
 * records, all HOST memory) and batch->n_canvas, n_tiles, n_pixels, n_gauss
 * (batch->canvas is left for the caller to point at a device copy of the
 * records).
 * Tiles and pixels are numbered canvas by canvas. */
bz_status bz_batch_layout(const bz_opts *opts, int32_t n_canvas, const int32_t *size,
                          const float *bg, const int64_t *gauss_off, const int32_t *curve_off,
                          bz_canvas *canvas, bz_batch *batch);

/* Host: 64-bit words of bz_pixstate.visit for tile lists of cap_pairs entries. */
bz_status bz_visit_words(const bz_opts *opts, int64_t cap_pairs, int64_t *words);

/* Sec. 3.3: sample K Gaussians per row along every curve (one row for open
 * curves, R+2 rows for closed ones), scales from neighbour distances (Eq.
 * sigma), orientation from the neighbour chord (Eq. rotation), covariance
 * (Eq. RSSR) dilated by sigma0_sq, opacity per segment, colour per curve.
 * Writes g->rec[0 .. c->n_gauss) and sets g->n = c->n_gauss (host field);
 * requires g->cap >= c->n_gauss. */
bz_status bz_sample(const bz_curves *c, const bz_opts *opts, bz_gaussians *g,
                    hipStream_t stream);

/* bz_sample then bz_bin in one call: the sampler also writes each Gaussian's
 * tile rectangle and count (the binning's first pass, Sec. 3.4), so the
 * records are not read back for it.  Gaussians, tile lists, ranges and status
 * come out exactly as from the two calls; arguments and errors are theirs. */
bz_status bz_sample_bin(const bz_curves *c, const bz_opts *opts, bz_gaussians *g, bz_bins *b,
                        hipStream_t stream);

/* bz_sample_bin for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the binning workspace is a fixed device array inside the library,
 * BZ_STATIC_SCRATCH_BYTES (32 MiB) per GPU, held from the first call on a GPU
 * until the process ends; b->workspace and b->workspace_bytes are ignored.
 * Everything else (arguments, outputs, status words, errors) is bz_sample_bin's,
 * and the Gaussians, tile lists, ranges and status come out bit for bit as its.
 * Returns BZ_ERR_CAPACITY, before anything is launched, when the workspace
 * for c->n_gauss Gaussians and b->cap_pairs pairs (bz_workspace_size) exceeds
 * BZ_STATIC_SCRATCH_BYTES (size it with bz_workspace_size), and BZ_ERR_HIP if
 * the array's device address cannot be obtained.  The call allocates nothing.  The array needs no initialisation
 * (every byte the binning reads was written earlier in the same call); it keeps
 * the last call's contents.  All calls on one GPU share the array: calls that
 * overlap in time on one GPU (different streams, or host threads) race and
 * must be serialised by the caller.  Persistent blend launches still need the
 * 256 bytes of tile counters at bz_bins.workspace. */
#define BZ_STATIC_SCRATCH_BYTES (32 * 1024 * 1024)
bz_status bz_sample_bin_static(const bz_curves *c, const bz_opts *opts, bz_gaussians *g,
                               bz_bins *b, hipStream_t stream);

/* Sec. 3.4 tile pipeline: list each Gaussian in every tile its truncated
 * support (1/2 d^T Sigma^-1 d <= -ln g_min, slightly inflated) reaches, tile
 * row by tile row (the ellipse's span over the row's pixels, not its bounding
 * box), sort the (tile, Gaussian) pairs by tile keeping draw order, and write
 * per-tile ranges.  Uses b->workspace; reports through b->status. */
bz_status bz_bin(const bz_gaussians *g, const bz_opts *opts, bz_bins *b, hipStream_t stream);

/* Sec. 3.4 blending: per pixel, front to back over its tile's list,
 * alpha = min(alpha_max, o (G - g_min)_+/(1 - g_min)) with
 * G = exp(-1/2 d^T Q d) (Eq. rasterization2), C += alpha T c, T *= 1 - alpha,
 * stop after T < t_min, then C += T bg.  image: [3][H][W]; state: per-pixel
 * t_final, n_last (and optionally n_contrib) for bz_render_bwd, or NULL. */
bz_status bz_render_fwd(const bz_gaussians *g, const bz_bins *b, const bz_opts *opts,
                        float *image, bz_pixstate *state, hipStream_t stream);

/* bz_render_fwd and bz_l2_grad on its image in one pass (Sec. 3.4 blending,
 * Sec. 3.5 L2 term).  image and state come out exactly as bz_render_fwd writes
 * them; as each pixel is written, d_image = scale*(image - target) for its
 * three channels (bit for bit what bz_l2_grad writes), and loss[0] = sum of
 * (image - target)^2 over all pixels and channels (zeroed by the call; may be
 * NULL; the order of its float additions differs from bz_l2_grad's).  target
 * and d_image have the layout of image ([3][H][W], or a batch's canvases one
 * after another); d_image may be target itself but not image (BZ_ERR_ARG). */
bz_status bz_render_fwd_l2(const bz_gaussians *g, const bz_bins *b, const bz_opts *opts,
                           float *image, bz_pixstate *state, const float *target, float scale,
                           float *d_image, float *loss, hipStream_t stream);

/* Reverse pass.  Stage 1, per pixel, walks the contributors of the forward
 * pass last to first, recovering T before each one by division by (1 - alpha)
 * and carrying the colour composited behind it, and accumulates per-Gaussian
 * gradients into grads->d_gauss.  Stage 2, per curve, chains them through the
 * sampling of Sec. 3.3 to control points, widths, colours and opacities.
 * d_image: dL/dimage, [3][H][W].  c, g, b, opts and state must be those of the
 * forward pass; with state NULL the per-pixel state is recomputed per tile
 * (same results, one more sweep of the tile lists).  Requires alpha_max < 1
 * (the division recovering T).
 * Per-Gaussian sums use float atomics, so d_gauss and the curve gradients
 * vary in the last bits from run to run. */
bz_status bz_render_bwd(const bz_curves *c, const bz_gaussians *g, const bz_bins *b,
                        const bz_opts *opts, const float *d_image, const bz_pixstate *state,
                        bz_grads *grads, hipStream_t stream);

/* Stage 1 of bz_render_bwd alone: per-Gaussian gradients into d_gauss (9 planes
 * of g->n floats, overwritten), the derivative of the blending of Sec. 3.4.
 * For callers that want gradients with respect to the Gaussians themselves. */
bz_status bz_render_bwd_gauss(const bz_gaussians *g, const bz_bins *b, const bz_opts *opts,
                              const float *d_image, const bz_pixstate *state, float *d_gauss,
                              hipStream_t stream);

/* Stage 2 of bz_render_bwd alone: chain per-Gaussian gradients d_gauss (9
 * planes of c->n_gauss floats, as written by bz_render_bwd_gauss, possibly
 * modified by the caller) through the sampling of Sec. 3.3 into
 * grads->d_ctrl, d_width, d_color, d_opacity (overwritten; grads->d_gauss is
 * ignored).  Deterministic. */
bz_status bz_render_bwd_curves(const bz_curves *c, const bz_opts *opts, const float *d_gauss,
                               bz_grads *grads, hipStream_t stream);

/* Per-curve area (Sec. 3.3: depth follows curve area).  Closed curve: the
 * area of the polygon of its boundary samples A_0..A_{K-1}, B_{K-2}..B_1 (the
 * region between its two boundaries).  Open stroke: polyline length of its K
 * samples times its width.  area: float [n_curves], by curve index. */
bz_status bz_curve_area(const bz_curves *c, float *area, hipStream_t stream);

/* Host: workspace bytes of bz_area_order for n_curves curves. */
bz_status bz_area_order_workspace(int32_t n_curves, int64_t *bytes);

/* Draw order by area (Sec. 3.3): curves sorted by bz_curve_area, smallest in
 * front (position 0), equal areas by curve index.  With a batch (opts->batch;
 * opts may be NULL otherwise) the order is per canvas: canvas by canvas, by
 * area inside each, so every canvas keeps its range of draw positions.  Writes area [n_curves],
 * order [n_curves] (the curve at each position) and gauss_off [n_curves + 1]
 * (first Gaussian of every position), the fields bz_layout_host would fill
 * for that rank; order and gauss_off may be c->order and c->gauss_off
 * themselves (they are not read).  workspace: device, 256-byte aligned, of
 * bz_area_order_workspace bytes.  Runs entirely on the device. */
bz_status bz_area_order(const bz_curves *c, const bz_opts *opts, float *area, int32_t *order,
                        int64_t *gauss_off, void *workspace, int64_t workspace_bytes,
                        hipStream_t stream);

/* Xing loss (Sec. 3.5, the convexity term the paper takes from LIVE) of the
 * closed curves' boundary segments: per cubic segment P0..P3,
 * D1 = [cross(P1-P0, P2-P1) >= 0], D2 = cross(P1-P0, P3-P2)/(|P1-P0||P3-P2|),
 * cost D1 max(0, -D2) + (1 - D1) max(0, D2).  loss[0] (device, may be NULL) =
 * weight * sum of costs (overwritten); weight * d(sum)/d(control points) is
 * ADDED to d_ctrl ([n_ctrl][2], e.g. after bz_render_bwd).  Segments with a
 * zero-length first or last control edge cost 0. */
bz_status bz_xing_loss(const bz_curves *c, float weight, float *loss, float *d_ctrl,
                       hipStream_t stream);

/* Mean squared error loss of Sec. 3.5 (the L2 term): d_image = scale*(image - target)
 * elementwise over n floats, and loss[0] = sum (image - target)^2 accumulated
 * (loss is zeroed by the call; may be NULL). */
bz_status bz_l2_grad(const float *image, const float *target, int64_t n, float scale,
                     float *d_image, float *loss, hipStream_t stream);

/* Short description of a status code (static string). */
const char *bz_status_str(bz_status s);

#ifdef __cplusplus
}
#endif
#endif /* BZ_H */
