// bz_render.hip -- per-tile blending (Sec. 3.4) and its reverse pass.
//
// Work decomposition (forward and backward stage 1): one workgroup per tile,
// one wave per 8x8 pixel quad of the tile, one pixel per lane.  Waves are
// independent: each walks its tile's list in batches of 64 entries; lane j
// loads entry j's record, tests the entry's truncated support against the
// quad (exact minimum of the quadratic form over the quad's pixel centres),
// and writes the derived per-Gaussian constants into the wave's LDS slice.
// A ballot of the test gives the batch's mask; the wave then iterates only
// over the surviving entries, every lane reading the entry's constants from
// the same LDS address (three 16-byte reads), so pixels never spend ALU on
// Gaussians that cannot reach their quad.  A wave stops when all 64 of its pixels have terminated.  (In the
// backward the quads of a tile also share a sum table in LDS, so its waves
// meet at the tile's start and end.)
//
// Blocks are mapped to tiles XCD-contiguously: the dispatcher deals blocks
// round robin to the 8 XCDs, so block b serves tile (b % 8) * per + b / 8 and
// each XCD's L2 sees a compact band of neighbouring tiles, which share most
// of their Gaussians.
//
// The forward can also write the L2 loss gradient of Sec. 3.5 as it writes
// each pixel (k_fwd_l2), which spares the step a pass over the image.
//
// Stage 2 of the backward pass is per curve (one workgroup per curve: 64
// threads for curves of at most 64 Gaussians, 256 for larger ones; no
// atomics): it chains the per-Gaussian gradients through the sampling of
// Sec. 3.3.
#include "bz_geom.h"

namespace bz {

namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline int xcd_tile(int b, int per) { return (b & 7) * per + (b >> 3); }

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Minimum over the box [x0,x1]x[y0,y1] (offsets from the mean) of
// f(d) = qa dx^2 + 2 qb dx dy + qc dy^2, compared against thr.
__device__ inline bool box_hit(float x0, float x1, float y0, float y1, float qa, float qb,
                               float qc, float thr) {
    if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return true;
    float best = 3.0e38f;
    // hardware reciprocals: an error in the clamped edge point moves the value
    // of the quadratic form only to second order (the slack on thr covers it)
    float ia = __builtin_amdgcn_rcpf(qa), ic = __builtin_amdgcn_rcpf(qc);
    // vertical edges: dx fixed, minimise over dy
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        float dx = e ? x1 : x0;
        float dy = fminf(fmaxf(-qb * dx * ic, y0), y1);
        best = fminf(best, qa * dx * dx + 2.f * qb * dx * dy + qc * dy * dy);
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        float dy = e ? y1 : y0;
        float dx = fminf(fmaxf(-qb * dy * ia, x0), x1);
        best = fminf(best, qa * dx * dx + 2.f * qb * dx * dy + qc * dy * dy);
    }
    return best <= thr;
}

struct TileArgs {
    const float4 *rec;
    const uint32_t *ids;
    const uint32_t *ranges;
    const int64_t *status;
    int W, H, tile_w, tile_h, tiles_x, n_tiles, per_xcd, quads_x;
    float bg0, bg1, bg2;
    float g_min, alpha_max, t_min, inv_1mg, box_thr;
    float *image;
    float *t_final;
    uint32_t *n_last;
    uint32_t *n_contrib;
    uint64_t *visit;          // per (quad plane, tile batch) contribution masks
    int64_t words_per_plane;
    const bz_canvas *canvas;  // batch canvases (null: one canvas W x H)
    int n_canvas;
    uint32_t *counter;        // persistent launch: next tile (null: one workgroup per tile)
    int tab_cap;              // positions of the backward's per-tile sum table
    // backward
    const float *d_image;
    float *d_gauss;
    int64_t n_gauss;
    // forward with the L2 loss gradient: target, d_image out, loss sum, scale
    const float *l2_target;
    float *l2_grad;
    float *l2_loss;
    float l2_scale;
};

// Entry of the wave's LDS slice.  The shape as two scaled axis vectors: with
// e' = e sqrt(log2(e) / 2) and f = k e', the base-2 exponent of the kernel at
// offset d = pixel - mean is p2 = u^2 + w^2, u = e' . d, w = f x d (= f.x dy
// - f.y dx), a sum of two squares.  The mean is taken relative to the quad's
// first pixel centre (qx0, qy0): the record's mean is hi + lo and hi - qx0 is
// exact for any Gaussian near the quad, so the relative mean m' is rounded
// once, and a pixel's offset is its place in the quad l (0..7 in x and y)
// minus m'.
// - With u0 = e' . m' and w0 = f x m' staged, u = e' . l - u0 and
//   w = f x l - w0 cost two FMAs each and no offsets.
// - The reverse pass stages the same form relative to the tile centre (the
//   origin the per-tile sums of every quad share), with l the pixel centre
//   from it.  The conic gradient of entries past the tile's sum table needs
//   the offset d itself: d = M^-1 (u, w), M = [e'.x e'.y; -f.y f.x], whose
//   determinant e' . f = k |e'|^2 the record gives; 1 / det is staged.
struct Staged {
    float4 m;   // -u0, -w0, e'.x, e'.y
    float4 q;   // f.x, f.y, 1 / (e' . f) (reverse pass), o' = o / (1 - g_min)
    float4 c;   // r, g, b, o' * g_min
};

// sqrt(log2(e) / 2): scales the record's axis e so that the squares sum to p2.
constexpr float kHalfLog2eSqrt = 0.84932180028801907f;

// Load a record and compute its LDS constants.  q receives the record's shape
// (e.x, e.y, k, o).
template <bool kSweep>
__device__ inline void stage_record(const TileArgs &a, uint32_t id, float qx0, float qy0,
                                    Staged &st, float4 &q) {
    const float4 m = a.rec[3 * (int64_t)id];
    q = a.rec[3 * (int64_t)id + 1];
    const float4 c = a.rec[3 * (int64_t)id + 2];
    const float op = q.w * a.inv_1mg;
    const float ex = kHalfLog2eSqrt * q.x, ey = kHalfLog2eSqrt * q.y;
    const float fx = q.z * ex, fy = q.z * ey;
    const float mx = (m.x - qx0) + m.z, my = (m.y - qy0) + m.w;
    const float nu0 = -fmaf(ex, mx, ey * my);      // -(e' . m')
    const float nw0 = -fmaf(fx, my, -fy * mx);     // -(f x m')
    st.m = make_float4(nu0, nw0, ex, ey);
    st.q = make_float4(fx, fy, kSweep ? 0.f : 1.f / fmaf(ex, fx, ey * fy), op);
    st.c = make_float4(c.x, c.y, c.z, op * a.g_min);
}

// Load a tile-list entry, compute its LDS constants and test its support
// against the wave's 8x8 quad (first pixel centre qx0, qy0).
template <bool kSweep>
__device__ inline bool stage_entry(const TileArgs &a, uint32_t id, float qx0, float qy0,
                                   Staged &st) {
    float4 q;
    stage_record<kSweep>(a, id, qx0, qy0, st, q);
    // offsets of the quad's first pixel centre from the mean
    const float4 m = a.rec[3 * (int64_t)id];
    const float x0 = -((m.x - qx0) + m.z), y0 = -((m.y - qy0) + m.w);
    float qxx, qxy, qyy;
    shape_conic(q.x, q.y, q.z, qxx, qxy, qyy);
    return box_hit(x0, x0 + 7.f, y0, y0 + 7.f, qxx, qxy, qyy, a.box_thr);
}

// stage_entry for the reverse pass: the record staged relative to the tile
// centre (ox, oy), the quad's first pixel centre at (bx, by) from it.
__device__ inline bool stage_entry_bwd(const TileArgs &a, uint32_t id, float ox, float oy,
                                       float bx, float by, Staged &st) {
    float4 q;
    stage_record<false>(a, id, ox, oy, st, q);
    const float4 m = a.rec[3 * (int64_t)id];
    const float x0 = bx - ((m.x - ox) + m.z), y0 = by - ((m.y - oy) + m.w);
    float qxx, qxy, qyy;
    shape_conic(q.x, q.y, q.z, qxx, qxy, qyy);
    return box_hit(x0, x0 + 7.f, y0, y0 + 7.f, qxx, qxy, qyy, a.box_thr);
}

// Base-2 exponent p2 = (e' . d)^2 + (f x d)^2 of a staged entry at the
// pixel centre (lx, ly) from the staging origin; u = e' . d and w = f x d are
// returned for the gradient.
__device__ inline float exponent2(const Staged &st, float lx, float ly, float &u, float &w) {
    u = fmaf(st.m.z, lx, fmaf(st.m.w, ly, st.m.x));
    w = fmaf(st.q.x, ly, fmaf(-st.q.y, lx, st.m.y));
    return fmaf(u, u, w * w);
}

// The same without u and w (the front-to-back sweep).
__device__ inline float exponent2_sweep(const Staged &st, float lx, float ly) {
    float u, w;
    return exponent2(st, lx, ly, u, w);
}

// Word of the visit mask of batch k of tile t inside one quad plane: tile t's
// batches occupy [start_t / 64 + t, start_t / 64 + t + ceil(len_t / 64)), which
// never overlaps the next tile's range, so every word has one writer.
__device__ inline int64_t visit_word(uint32_t start, int tile) {
    return (int64_t)(start >> 6) + tile;
}

// Canvas geometry of a (wave-uniform) global tile.
struct TileGeo {
    int W, H;          // canvas size
    int tx, ty;        // tile coordinates inside the canvas
    int64_t pix0;      // first pixel of the canvas
    float bg0, bg1, bg2;
};

__device__ inline TileGeo tile_geo(const TileArgs &a, int tile) {
    TileGeo g;
    if (a.canvas) {
        const int c = batch_find(a.canvas, a.n_canvas, (int64_t)tile,
                                 [](const bz_canvas &r) { return r.tile_off; });
        const bz_canvas &cv = a.canvas[c];
        const int local = tile - (int)cv.tile_off;
        g.W = cv.width;
        g.H = cv.height;
        g.ty = local / cv.tiles_x;
        g.tx = local - g.ty * cv.tiles_x;
        g.pix0 = cv.pix_off;
        g.bg0 = cv.bg[0];
        g.bg1 = cv.bg[1];
        g.bg2 = cv.bg[2];
    } else {
        g.W = a.W;
        g.H = a.H;
        g.ty = tile / a.tiles_x;
        g.tx = tile - g.ty * a.tiles_x;
        g.pix0 = 0;
        g.bg0 = a.bg0;
        g.bg1 = a.bg1;
        g.bg2 = a.bg2;
    }
    return g;
}

// Tile loop of a launch: one tile per workgroup (XCD-contiguous), or, when
// the launch is persistent, tiles taken from a counter until they run out.
template <typename Body>
__device__ inline void for_tiles(const TileArgs &a, Body body) {
    if (!a.counter) {
        const int tile = xcd_tile(blockIdx.x, a.per_xcd);
        if (tile < a.n_tiles) body(tile);
        return;
    }
    __shared__ int s_next;
    for (;;) {
        __syncthreads();                        // the previous tile is done with LDS
        if (threadIdx.x == 0) s_next = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int tile = __builtin_amdgcn_readfirstlane(s_next);
        if (tile >= a.n_tiles) break;
        body(tile);
    }
}

// min(x, hi) for finite x and a wave-uniform hi, as one VALU instruction:
// fminf would canonicalise both operands first (IEEE mode), two more per use.
__device__ inline float min_amax(float x, float hi) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "s"(hi), "v"(x));
    return r;
}

// Per lane: bit `lane` of the wave-uniform mask m ? on : off, as one
// v_cndmask with m in scalar registers (a bool built from m would cost a shift,
// an and and a compare per lane).
__device__ inline float select_lanes(uint64_t m, float on, float off) {
    float r;
    asm("v_cndmask_b32_e64 %0, %2, %1, %3" : "=v"(r) : "v"(on), "v"(off), "s"(m));
    return r;
}
__device__ inline uint32_t select_lanes_u32(uint64_t m, uint32_t on, uint32_t off) {
    return __float_as_uint(select_lanes(m, __uint_as_float(on), __uint_as_float(off)));
}

// The backward's quad origin, re-read from LDS at every staging so that it
// occupies no register across the slot loop: the index is a zero the compiler
// cannot see through (one scalar move), so the read is not hoisted.
__device__ inline int opaque_zero() {
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

// Clear bit b of a wave-uniform mask: one scalar instruction (the compiler's
// mask & (mask - 1) or mask & ~(1 << b) take two or three).
__device__ inline void clear_bit(uint64_t &mask, int b) {
    asm("s_bitset0_b64 %0, %1" : "+s"(mask) : "s"(b));
}

// A wave-uniform float moved to a scalar register.
__device__ inline float uniform_f32(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// A staged record as three 16-byte LDS reads (the compiler splits the read
// around fields the sweep leaves unused, five LDS instructions), waited for
// in the same block; off is the record's LDS byte offset (the low 32 bits
// of a flat address into LDS).  The outputs are early-clobber: the address
// register must not be shared with a destination while later reads use it.
__device__ inline Staged read_staged_at(uint32_t off) {
    float4 m, q, c;
    asm volatile("ds_read_b128 %0, %3\n\t"
                 "ds_read_b128 %1, %3 offset:16\n\t"
                 "ds_read_b128 %2, %3 offset:32\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(m), "=&v"(q), "=&v"(c)       // early clobber: off is read by all three
                 : "v"(off)
                 : "memory");
    return Staged{m, q, c};
}

// LDS offset of entry b of a wave's staged slice (base: the slice's offset,
// held in a vector register) as one VALU multiply-add from the scalar index:
// the compiler's scalar multiply, add and move to a vector register cost two
// scalar instructions more per visited entry.
// The slice's offset in a vector register, produced once: an inline-asm
// value is kept in its register rather than moved back from a scalar one
// inside the loop.
__device__ inline uint32_t vector_copy(uint32_t v) {
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
    return r;
}
__device__ inline uint32_t staged_off(uint32_t base, int b) {
    uint32_t r;
    asm("v_mad_u32_u24 %0, %1, 48, %2" : "=v"(r) : "s"(b), "v"(base));
    return r;
}

// Result of a front-to-back sweep for one pixel.
struct Sweep {
    float T, C0, C1, C2;   // transmittance after the last contributor, colour sum
    uint32_t last;         // list positions the reverse pass must consider (see below)
    uint32_t cnt;          // contributors (kCount only)
};

// Front-to-back blend (Sec. 3.4) of one wave's 8x8 quad over tile-list
// positions [start, end): per batch of 64 entries, every lane stages one entry
// into the wave's LDS slice and box-tests it against the quad; the wave then
// visits the hits in list order.  Per pixel and hit: alpha = min(alpha_max,
// o (G - g_min) / (1 - g_min)) when G > g_min, colour += alpha T c, T *= 1 - alpha;
// a pixel stops after the first contributor that takes T below t_min, and the
// wave leaves when all its pixels have stopped.  sink(k, bits) receives, for
// batch k, the entries that changed at least one pixel of the quad.
//
// A pixel has stopped exactly when T < t_min (T never grows; lanes outside the
// canvas start at T = -1), so the wave keeps that set as one 64-bit mask.
// last: for a pixel that stopped, 1 + the list position of the contributor
// that stopped it; otherwise the end of the last batch that changed a pixel of
// the quad (capped at the list length).  Either way no entry at or beyond it
// contributed to the pixel, and every earlier entry with G > g_min did, which
// is all the reverse pass needs; recording it costs the loop nothing except
// when a pixel stops.
template <bool kColor, bool kCount, typename Sink>
__device__ inline Sweep fwd_sweep(const TileArgs &a, Staged *my, uint32_t start, uint32_t end,
                                  float lx, float ly, float qx0, float qy0, bool valid, int lane,
                                  Sink sink) {
    Sweep r = {valid ? 1.f : -1.f, 0.f, 0.f, 0.f, 0u, 0u};
    const float g_min = a.g_min, amax = a.alpha_max, tmin = a.t_min;
    uint64_t stopped = __builtin_amdgcn_ballot_w64(r.T < tmin);
    uint32_t k = 0, k_used = 0;
    const uint32_t my_off = vector_copy((uint32_t)(uintptr_t)my);   // LDS offset of the slice
    for (uint32_t base = start; base < end; base += 64, ++k) {
        const uint32_t j = base + lane;
        bool hit = false;
        if (j < end) {
            Staged st;
            hit = stage_entry<true>(a, a.ids[j], qx0, qy0, st);
            my[lane] = st;
        }
        uint64_t mask = __ballot(hit);
        // the batch's entries that change a pixel: every hit, less the
        // (rarer) ones that change none
        uint64_t vbits = mask;
        wave_lds_sync();
        while (mask) {
            const int b = __builtin_ctzll(mask);
            clear_bit(mask, b);
            const Staged st = read_staged_at(staged_off(my_off, b));
            const float G = __builtin_amdgcn_exp2f(-exponent2_sweep(st, lx, ly));
            // contributors: inside the support and not stopped, as a lane mask
            const uint64_t cm = __builtin_amdgcn_ballot_w64(G > g_min) & ~stopped;
            const float araw = fmaf(st.q.w, G, -st.c.w);
            const float al = select_lanes(cm, min_amax(araw, amax), 0.f);
            const float wgt = al * r.T;
            if (kColor) {
                r.C0 = fmaf(wgt, st.c.x, r.C0);
                r.C1 = fmaf(wgt, st.c.y, r.C1);
                r.C2 = fmaf(wgt, st.c.z, r.C2);
            }
            {
                // T (1 - alpha) as T - wgt, after wgt has used T: no copy of T
                _Pragma("clang fp contract(off)") r.T = r.T - wgt;
            }
            if (kCount) r.cnt = select_lanes_u32(cm, r.cnt + 1u, r.cnt);
            if (__builtin_expect(cm == 0, 0)) clear_bit(vbits, b);
            const uint64_t now = __builtin_amdgcn_ballot_w64(r.T < tmin);
            if (__builtin_expect(now != stopped, 0)) {     // some pixel stopped here
                r.last = select_lanes_u32(now & ~stopped, k * 64 + b + 1, r.last);
                stopped = now;
            }
        }
        if (vbits) k_used = k + 1;
        sink(k, vbits);
        if (stopped == ~0ull) break;
        wave_lds_sync();
    }
    r.last = select_lanes_u32(stopped, r.last, min(k_used * 64u, end - start));
    return r;
}

// Forward pass.  With kState the blend state the backward reads is written:
// T after the last contributor, a bound on its position, and per (quad, batch) the mask
// of entries that contributed; without it only the image.  With kL2, as each
// pixel is written, also the L2 loss gradient scale * (image - target) (the
// same float arithmetic as k_l2) and the lane's sum of squared errors in l2.
template <bool kState, bool kCount, bool kL2>
__device__ inline void fwd_tile(const TileArgs &a, int tile, float &l2) {
    extern __shared__ Staged s_stage[];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const TileGeo tg = tile_geo(a, tile);
    const int qx = w % a.quads_x, qy = w / a.quads_x;
    const int x0 = tg.tx * a.tile_w + qx * kQuad, y0 = tg.ty * a.tile_h + qy * kQuad;
    if (x0 >= tg.W || y0 >= tg.H) return;
    const int x = x0 + (lane & 7), y = y0 + (lane >> 3);
    const bool valid = x < tg.W && y < tg.H;
    const float lx = (float)(lane & 7), ly = (float)(lane >> 3);   // pixel - first pixel of the quad
    // wave-uniform: held in scalar registers
    const float qx0 = uniform_f32((float)x0 + 0.5f), qy0 = uniform_f32((float)y0 + 0.5f);
    Staged *my = s_stage + w * 64;

    const int64_t pix = tg.pix0 + (int64_t)y * tg.W + x;
    const int64_t plane = (int64_t)tg.W * tg.H;
    float *img = a.image + 2 * tg.pix0;     // canvas image: 3 planes from 3 * pix0
    if (a.status[1] & Status::kOverflow) {
        if (valid) {
            float nan = __int_as_float(0x7fc00000);
            img[pix] = nan;
            img[plane + pix] = nan;
            img[2 * plane + pix] = nan;
            if (kL2) {
                float *dimg = a.l2_grad + 2 * tg.pix0;
                dimg[pix] = nan;
                dimg[plane + pix] = nan;
                dimg[2 * plane + pix] = nan;
                l2 = nan;
            }
            if (kState) {
                a.t_final[pix] = nan;
                a.n_last[pix] = 0;
                if (kCount) a.n_contrib[pix] = 0;
            }
        }
        return;
    }
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    uint64_t *vis = kState ? a.visit + (int64_t)w * a.words_per_plane + visit_word(start, tile)
                           : nullptr;
    const Sweep r = fwd_sweep<true, kCount>(a, my, start, end, lx, ly, qx0, qy0, valid, lane,
                                            [&](uint32_t k, uint64_t bits) {
                                                if (kState && lane == 0) vis[k] = bits;
                                            });
    if (valid) {
        const float v0 = fmaf(r.T, tg.bg0, r.C0), v1 = fmaf(r.T, tg.bg1, r.C1),
                    v2 = fmaf(r.T, tg.bg2, r.C2);
        img[pix] = v0;
        img[plane + pix] = v1;
        img[2 * plane + pix] = v2;
        if (kL2) {
            const float *tgt = a.l2_target + 2 * tg.pix0;
            float *dimg = a.l2_grad + 2 * tg.pix0;
            const float e0 = v0 - tgt[pix], e1 = v1 - tgt[plane + pix],
                        e2 = v2 - tgt[2 * plane + pix];
            dimg[pix] = a.l2_scale * e0;
            dimg[plane + pix] = a.l2_scale * e1;
            dimg[2 * plane + pix] = a.l2_scale * e2;
            l2 = fmaf(e0, e0, fmaf(e1, e1, fmaf(e2, e2, l2)));
        }
        if (kState) {
            a.t_final[pix] = r.T;
            a.n_last[pix] = r.last;
            if (kCount) a.n_contrib[pix] = r.cnt;
        }
    }
}

// Forward pass.  With kState the blend state the backward reads is written:
// T after the last contributor, a bound on its position, and per (quad, batch) the mask
// of entries that contributed; without it only the image.
template <bool kState, bool kCount>
__global__ __launch_bounds__(1024) void k_fwd(TileArgs a) {
    float unused = 0.f;
    for_tiles(a, [&](int tile) { fwd_tile<kState, kCount, false>(a, tile, unused); });
}

// Sum over the wave's 64 lanes, wave-uniform: an inclusive DPP scan (row
// shifts of 1, 2, 4, 8 lanes with zeros shifted in, then row_bcast 15 and 31
// across rows), whose last lane holds the total.
template <int CTRL, int ROWS, bool BOUND>
__device__ inline float dpp_f32(float x) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, BOUND));
}
__device__ inline float wave_sum(float v) {
    v += dpp_f32<0x111, 0xF, true>(v);
    v += dpp_f32<0x112, 0xF, true>(v);
    v += dpp_f32<0x114, 0xF, true>(v);
    v += dpp_f32<0x118, 0xF, true>(v);
    v += dpp_f32<0x142, 0xA, false>(v);
    v += dpp_f32<0x143, 0xC, false>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// The forward with the L2 loss gradient.  Every lane sums its squared errors
// over the block's tiles; the block's waves add their sums in LDS and the last
// one out adds the block's total to the loss, one global atomic per block.
// Every wave of the block reaches the end exactly once (waves outside the
// canvas leave fwd_tile early, not the kernel).
template <bool kState, bool kCount>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_fwd_l2(TileArgs a) {
    __shared__ float s_loss;
    __shared__ int s_done;
    if (threadIdx.x == 0) {
        s_loss = 0.f;
        s_done = 0;
    }
    __syncthreads();
    float l2 = 0.f;
    for_tiles(a, [&](int tile) { fwd_tile<kState, kCount, true>(a, tile, l2); });
    if (!a.l2_loss) return;
    l2 = wave_sum(l2);
    if ((threadIdx.x & 63) == 0) {
        __hip_atomic_fetch_add(&s_loss, l2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int waves = (int)(blockDim.x >> 6);
        if (__hip_atomic_fetch_add(&s_done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) ==
            waves - 1) {
            const float total =
                __hip_atomic_load(&s_loss, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (total != 0.f) atomicAdd(a.l2_loss, total);
        }
    }
}

// Broadcast lane 0's 64-bit value as a wave-uniform (scalar) value.  The
// builtin returns a signed int: each half goes through uint32_t so that the
// low half is zero-extended, not sign-extended into the high word.
__device__ inline uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

template <int CTRL>
__device__ inline float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 CTRL, 0xF, 0xF, false));
}

// Exchange lanes 32..63 of x[i] with lanes 0..31 of y[i] (v_permlane32_swap),
// or the odd 16-lane rows of x[i] with the even rows of y[i]
// (v_permlane16_swap), for 8 register pairs.  Both registers of a pair are
// outputs of the instruction; the compiler builtins of this toolchain return
// the first one twice, so the instructions are written here with both
// operands read-write.  One s_nop 1 gives the two wait states a swap needs
// after a VALU write of its operands; the 8 swaps of a group do not depend on
// each other.
#define BZ_SWAP8(OP, x, y, o)                                                           \
    asm volatile("s_nop 1\n\t" OP " %0, %8\n\t" OP " %1, %9\n\t" OP " %2, %10\n\t" OP    \
                 " %3, %11\n\t" OP " %4, %12\n\t" OP " %5, %13\n\t" OP " %6, %14\n\t" OP \
                 " %7, %15"                                                             \
                 : "+v"(x[o + 0]), "+v"(x[o + 1]), "+v"(x[o + 2]), "+v"(x[o + 3]),       \
                   "+v"(x[o + 4]), "+v"(x[o + 5]), "+v"(x[o + 6]), "+v"(x[o + 7]),       \
                   "+v"(y[o + 0]), "+v"(y[o + 1]), "+v"(y[o + 2]), "+v"(y[o + 3]),       \
                   "+v"(y[o + 4]), "+v"(y[o + 5]), "+v"(y[o + 6]), "+v"(y[o + 7]))

// d[i] on the lanes of the banks in MASK (4-lane groups of a 16-lane row) =
// s[i] + s[i] read from the DPP partner lane (row_ror:8: lane ^ 8;
// row_half_mirror: lane ^ 7 inside 8 lanes), for 4 registers; lanes of the
// other banks keep d (OUT "+v") or are left undefined (OUT "=&v", early
// clobber: the block reads its inputs after writing outputs).  The wait
// states before the first DPP read of a freshly written register come first.
#define BZ_DPPADD4(OUT, CTRL, MASK, d, s, od, os)                                        \
    asm volatile("s_nop 1\n\t"                                                          \
                 "v_add_f32_dpp %0, %4, %4 " CTRL " row_mask:0xf bank_mask:" MASK "\n\t"  \
                 "v_add_f32_dpp %1, %5, %5 " CTRL " row_mask:0xf bank_mask:" MASK "\n\t"  \
                 "v_add_f32_dpp %2, %6, %6 " CTRL " row_mask:0xf bank_mask:" MASK "\n\t"  \
                 "v_add_f32_dpp %3, %7, %7 " CTRL " row_mask:0xf bank_mask:" MASK          \
                 : OUT(d[od + 0]), OUT(d[od + 1]), OUT(d[od + 2]), OUT(d[od + 3])        \
                 : "v"(s[os + 0]), "v"(s[os + 1]), "v"(s[os + 2]), "v"(s[os + 3]))

// d[i] (2 registers) on the banks in MASK = s[i] + s[i] of the DPP partner.
#define BZ_DPPADD2(OUT, CTRL, MASK, d, s, od, os)                                        \
    asm volatile("s_nop 1\n\t"                                                          \
                 "v_add_f32_dpp %0, %2, %2 " CTRL " row_mask:0xf bank_mask:" MASK "\n\t"  \
                 "v_add_f32_dpp %1, %3, %3 " CTRL " row_mask:0xf bank_mask:" MASK          \
                 : OUT(d[od + 0]), OUT(d[od + 1])                                        \
                 : "v"(s[os + 0]), "v"(s[os + 1]))

// Transposed reduction of 32 per-lane values over the 64 lanes: on return
// lanes 2i and 2i + 1 both hold the sum over all lanes of v[i].  Each level
// halves the values a lane holds by exchanging half of them with a partner
// lane: lanes l and l^32 (permlane32 swap), l^16 (permlane16 swap), l^8 (DPP
// row rotate by 8), l^7 (DPP half-row mirror), l^3 (DPP quad permute); bit b
// of the lane index decides which half a lane keeps, so after five levels
// lanes 2i and 2i + 1 hold index i, and a last DPP add over l^1 completes the
// sum.  Lanes l and l^8 differ in bit 1 of their bank, lanes l and l^7 in bit
// 0, so those two levels are pairs of bank-masked DPP adds (the lanes of a
// bank add the index they keep).  Works in place: v holds partial sums
// afterwards.
__device__ inline float reduce_scatter32(float (&v)[32], int lane) {
    BZ_SWAP8("v_permlane32_swap_b32", v, (v + 16), 0);
    BZ_SWAP8("v_permlane32_swap_b32", v, (v + 16), 8);
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] += v[i + 16];
    BZ_SWAP8("v_permlane16_swap_b32", v, (v + 8), 0);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] += v[i + 8];
    float w[4];
    BZ_DPPADD4("=&v", "row_ror:8", "0x3", w, v, 0, 0);
    BZ_DPPADD4("+v", "row_ror:8", "0xc", w, v, 0, 4);
    float u[2];
    BZ_DPPADD2("=&v", "row_half_mirror", "0x5", u, w, 0, 0);
    BZ_DPPADD2("+v", "row_half_mirror", "0xa", u, w, 0, 2);
    const bool b1 = lane & 2;
    const float keep = b1 ? u[1] : u[0], send = b1 ? u[0] : u[1];
    const float r = keep + dpp_f<0x1B>(send);      // quad_perm [3,2,1,0] (lane ^ 3)
    return r + dpp_f<0xB1>(r);                     // quad_perm [1,0,3,2] (lane ^ 1)
}

// Gaussians per reduction batch: 3 x 10 = 30 sums in 32 registers.  (Seven
// Gaussians in 64 registers cost fewer reduction instructions per sum, but the
// kernel then needs 96 registers and spills; the reverse pass waits on memory
// more than it issues arithmetic, and the smaller form, with more waves and no
// spills, runs it 30% faster.)
constexpr int kSlots = 3;
constexpr int kAcc = 32;
constexpr int kSums = 10;     // per-lane values of one Gaussian

// What a Gaussian's sums hold.  With f the alpha gradient, o' the scaled
// opacity, G = 2^-p2, p2 = u^2 + w^2 (u = e' . d, w = f x d, d = pixel - mean)
// and P = f o' G = -dL/dp (p = d^T Q d / 2, Q the conic):
//   dL/dmean = 2 ln 2 P (u e'.x - w f.y, u e'.y + w f.x)
//            = 2 ln 2 o' [A B; B C] sum(f G d),
//     A = e'.x^2 + f.y^2, B = e'.x e'.y - f.x f.y, C = e'.y^2 + f.x^2;
//   dL/dQ = -P (dx^2 / 2, dx dy, dy^2 / 2);  dL/do = f (G - g_min) / (1 - g_min);
//   dL/dcolour = alpha T g.
// Entries in the tile's LDS table add moments about the tile centre: with
// (x, y) the pixel centre relative to it, sums 0-9 are f G (1, x, y, x^2, x y,
// y^2), alpha T g (3) and f; the table's flush turns them into the planes with
// the record's mean and shape (sum(f G dx) = sum(f G x) - mx sum(f G), ...),
// which per pixel costs five products instead of eleven.  Entries past the
// table add the nine plane values directly (sums 0-8, the constant factors
// below applied after the reduction).
__device__ inline float plane_scale(int v, float inv_1mg) {
    return v < 2 ? 1.38629436112f : v == 3 ? -1.f : (v == 2 || v == 4) ? -0.5f : v == 5 ? inv_1mg : 1.f;
}

// Tile-list positions pooled in LDS by the backward.  With 16x16 tiles a
// block then takes 256 x 48 B of staging + 10 x 352 x 4 B of sums = 25.8 KiB,
// so six blocks share a CU's 160 KiB of LDS.  (Five blocks ran 5% slower; with
// half the positions more sums go to global atomics, 16% slower; a table sized
// to each tile shape's occupancy ran 8x8 and 16x8 tiles 4-9% slower and 16x32
// tiles 12% slower.)  The recomputing backward also keeps its batch masks in
// LDS; its table gives up their bytes (table_cap), so both forms hold the
// same LDS per block: 240 positions at 16x16, 6% faster than 352 at five
// blocks per CU.
constexpr int kTableCap = 352;

// Backward stage 1.  Each wave walks its tile list from the last entry any of
// its pixels used down to the first.  Per pixel and contributor (reverse
// order): T before it = T after / (1 - alpha); colour gradient alpha T g;
// alpha gradient T (c - A) . g with A the colour composited behind it (starts
// at the background, A <- alpha c + (1 - alpha) A; only A . g is carried);
// then, unless alpha was clamped, the opacity gradient and dL/dp = -alpha_bar
// o' G, which gives the mean gradient -dL/dp Q d and the conic gradient dL/dp
// (dx^2/2, dx dy, dy^2/2).  The per-lane values of three Gaussians are summed
// over the wave in one transposed reduction and added, with one atomic
// instruction, to the tile's LDS sum table (positions below its capacity) or
// straight to the per-Gaussian planes in HBM; the table is added to the planes
// when the tile is done.
//
// kRecompute: the blend state (T after the last contributor, the bound on its position and
// the per-batch contribution masks) is not read from memory but recomputed by
// a front-to-back sweep of the same quad (colour omitted), with the
// instruction sequence of the forward pass, so T and the positions are those
// the forward pass had.  The masks of the first kVisCap batches stay in LDS;
// later batches are staged whole and box-tested again (a superset of the
// contributors: the others add exact zeros).
constexpr int kVisCap = 128;

template <bool kRecompute>
__device__ inline void bwd_tile(const TileArgs &a, int tile) {
    // dynamic LDS: [waves][64] staged records, the sum table, and (kRecompute)
    // [waves][kVisCap] batch masks
    extern __shared__ Staged s_stage[];
    __shared__ uint32_t s_top[16];
    __shared__ float s_q0[16][2];      // the tile centre (same for every wave), read when staging
    const int nwaves = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const TileGeo tg = tile_geo(a, tile);
    const int qx = w % a.quads_x, qy = w / a.quads_x;
    const int x0 = tg.tx * a.tile_w + qx * kQuad, y0 = tg.ty * a.tile_h + qy * kQuad;
    const bool wave_on = x0 < tg.W && y0 < tg.H;         // quad inside the canvas
    const int x = x0 + (lane & 7), y = y0 + (lane >> 3);
    const bool valid = wave_on && x < tg.W && y < tg.H;
    const float lx = (float)(lane & 7), ly = (float)(lane >> 3);   // pixel - first pixel of the quad
    const float qx0 = (float)x0 + 0.5f, qy0 = (float)y0 + 0.5f;
    // The reverse pass measures from the tile centre (ox, oy): the moments the
    // quads of a tile add to one table need one origin.  (cx, cy): this pixel's
    // centre, (bx, by): the quad's first pixel centre, both relative to it.
    const float ox = (float)(tg.tx * a.tile_w) + 0.5f * (float)a.tile_w;
    const float oy = (float)(tg.ty * a.tile_h) + 0.5f * (float)a.tile_h;
    const float bx = qx0 - ox, by = qy0 - oy;
    const float cx = bx + lx, cy = by + ly;
    if (lane == 0) {
        s_q0[w][0] = ox;
        s_q0[w][1] = oy;
    }
    Staged *my = s_stage + w * 64;
    // LDS offset of the slice (the recomputing form, short of registers,
    // leaves its address arithmetic to the compiler)
    const uint32_t my_off = kRecompute ? (uint32_t)(uintptr_t)my
                                       : vector_copy((uint32_t)(uintptr_t)my);
    // Per-tile sums, plane-major [kSums][tab_cap], indexed by tile-list position:
    // the quads of a tile share most of their Gaussians, so their sums meet
    // here and leave the block with one global atomic per (Gaussian, plane).
    const int tab_cap = a.tab_cap;
    float *table = reinterpret_cast<float *>(s_stage + nwaves * 64);
    // kRecompute: per-wave batch masks after the table
    uint64_t *s_vis = reinterpret_cast<uint64_t *>(table + kSums * tab_cap) + w * kVisCap;

    const uint32_t start = a.ranges[2 * tile];
    const uint32_t len = a.ranges[2 * tile + 1] - start;
    const uint64_t *vis =
        kRecompute ? nullptr : a.visit + (int64_t)w * a.words_per_plane + visit_word(start, tile);
    const int64_t pix = tg.pix0 + (int64_t)y * tg.W + x;
    const int64_t plane = (int64_t)tg.W * tg.H;
    const float *dimg = a.d_image + 2 * tg.pix0;   // canvas planes from 3 * pix0
    uint32_t nl = 0;
    float T = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    if (kRecompute) {
        if (wave_on) {
            const Sweep r = fwd_sweep<false, false>(a, my, start, start + len, lx, ly, qx0, qy0,
                                                    valid, lane, [&](uint32_t k, uint64_t bits) {
                                                        if (lane == 0 && k < kVisCap) s_vis[k] = bits;
                                                    });
            nl = valid ? r.last : 0u;
            T = valid ? r.T : 0.f;
        }
        wave_lds_sync();
    } else if (valid) {
        nl = a.n_last[pix];
        T = a.t_final[pix];
    }
    if (valid) {
        g0 = dimg[pix];
        g1 = dimg[plane + pix];
        g2 = dimg[2 * plane + pix];
    }
    // A (the colour composited behind, from the background forward) enters the
    // gradient only through A . g, so that scalar is what the pass carries:
    // A <- alpha c + (1 - alpha) A gives A.g <- alpha (c.g) + (1 - alpha) A.g.
    float Ag = fmaf(tg.bg0, g0, fmaf(tg.bg1, g1, tg.bg2 * g2));
    uint32_t top = wave_max_u32(nl);   // wave-uniform
    top = top < len ? top : len;
    if (lane == 0) s_top[w] = top;
    __syncthreads();
    uint32_t top_block = 0;
    for (int i = 0; i < nwaves; ++i) top_block = max(top_block, s_top[i]);
    const int tab_n = (int)(top_block < (uint32_t)tab_cap ? top_block : (uint32_t)tab_cap);
    for (int i = threadIdx.x; i < kSums * tab_n; i += blockDim.x) {
        const int v = i / tab_n;
        table[v * tab_cap + (i - v * tab_n)] = 0.f;
    }
    __syncthreads();

    const float g_min = a.g_min, amax = a.alpha_max, inv_1mg = a.inv_1mg;
    const int64_t ng = a.n_gauss;
    // sum index of this lane after the reduction (lanes 2i and 2i + 1 hold
    // sum i; the even one stores it)
    const int my_o = lane >> 1;
    const bool my_store = (lane & 1) == 0;
    const int my_v = my_o % kSums, my_s = my_o / kSums;
    uint32_t slot_pos[kSlots];
#pragma unroll
    for (int i = 0; i < kSlots; ++i) slot_pos[i] = 0;

    // Batches are visited last to first; inside a batch, entries from the
    // highest position down.  Only entries whose bit the forward pass set (at
    // least one pixel of this quad used them) are staged and visited.
    // batch counter (32-bit: its test k > 0 runs on the scalar unit every slot)
    int32_t k = wave_on ? (int32_t)(((uint64_t)top + 63) / 64) : 0;
    uint64_t mask = 0;
    uint32_t lo = 0;

    // Slots not refilled in a round only feed sums that are never stored.
    float acc[kAcc];
#pragma unroll
    for (int i = 0; i < kAcc; ++i) acc[i] = 0.f;
    while (true) {
        int filled = 0;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            if (mask == 0) {
                // the next batch with entries to visit, walking down
                while (k > 0) {
                    --k;
                    lo = (uint32_t)k * 64;
                    // only entries of this tile's list can be visited
                    const uint32_t avail = len - lo;
                    const uint64_t in_list = avail >= 64 ? ~0ull : ((1ull << avail) - 1ull);
                    uint64_t vm;
                    if (!kRecompute || k < kVisCap) {
                        const uint64_t vraw = kRecompute ? s_vis[k] : vis[k];
                        vm = uniform_u64(vraw) & in_list;
                        if (vm != 0) {
                            wave_lds_sync();
                            if ((vm >> lane) & 1ull) {
                                const uint32_t id = a.ids[start + lo + lane];
                                Staged st;
                                float4 q;
                                const float *q0 = s_q0[w + opaque_zero()];
                                stage_record<false>(a, id, q0[0], q0[1], st, q);
                                my[lane] = st;
                            }
                            wave_lds_sync();
                        }
                    } else {
                        wave_lds_sync();
                        bool hit = false;
                        if ((uint32_t)lane < avail) {
                            const uint32_t id = a.ids[start + lo + lane];
                            Staged st;
                            const float *q0 = s_q0[w + opaque_zero()];
                            hit = stage_entry_bwd(a, id, q0[0], q0[1], bx, by, st);
                            my[lane] = st;
                        }
                        vm = __ballot(hit) & in_list;
                        wave_lds_sync();
                    }
                    mask = vm;
                    if (mask != 0) break;
                }
                if (mask == 0) break;      // the list is done: the slots from s stay empty
            }
            {
                const int b = 63 - __builtin_clzll(mask);
                clear_bit(mask, b);
                const Staged st = kRecompute ? read_staged_at(my_off + 48u * (uint32_t)b)
                                             : read_staged_at(staged_off(my_off, b));
                const uint32_t pos = lo + (uint32_t)b;
                float u, w;
                const float G = __builtin_amdgcn_exp2f(-exponent2(st, cx, cy, u, w));
                const bool c = pos < nl && G > g_min;
                const float araw = fmaf(st.q.w, G, -st.c.w);
                const bool shaped = c && araw <= amax;       // alpha not clamped
                const float acl = min_amax(araw, amax);
                const float al = c ? acl : 0.f;
                const float Tb = T * __builtin_amdgcn_rcpf(1.f - al);
                const float wgt = al * Tb;
                const float cg = fmaf(st.c.x, g0, fmaf(st.c.y, g1, st.c.z * g2));
                const float e = cg - Ag;                     // (c - A) . g
                const float abar = c ? Tb * e : 0.f;
                Ag = fmaf(al, e, Ag);
                T = Tb;
                const float f = shaped ? abar : 0.f;
                // f G and f straight into their moment registers (the
                // positions past the table overwrite the first and
                // ignore the tenth), so neither needs a copy
                acc[kSums * s + 0] = f * G;
                acc[kSums * s + 9] = f;
                const float fG = acc[kSums * s + 0];
                acc[kSums * s + 6] = wgt * g0;
                acc[kSums * s + 7] = wgt * g1;
                acc[kSums * s + 8] = wgt * g2;
                if (pos < (uint32_t)tab_cap) {
                    // moments about the tile centre (wave-uniform branch)
                    const float fGx = fG * cx, fGy = fG * cy;
                    acc[kSums * s + 1] = fGx;
                    acc[kSums * s + 2] = fGy;
                    acc[kSums * s + 3] = fGx * cx;
                    acc[kSums * s + 4] = fGx * cy;
                    acc[kSums * s + 5] = fGy * cy;
                } else {
                    // the planes without their constant factors (plane_scale);
                    // the offset d = M^-1 (u, w)
                    const float dx = (st.q.x * u - st.m.w * w) * st.q.z;
                    const float dy = fmaf(st.q.y, u, st.m.z * w) * st.q.z;
                    const float P = fG * st.q.w;             // -dL/dp
                    const float Pdx = P * dx, Pdy = P * dy;
                    acc[kSums * s + 0] = P * fmaf(u, st.m.z, -w * st.q.y);
                    acc[kSums * s + 1] = P * fmaf(u, st.m.w, w * st.q.x);
                    acc[kSums * s + 2] = Pdx * dx;
                    acc[kSums * s + 3] = Pdx * dy;
                    acc[kSums * s + 4] = Pdy * dy;
                    acc[kSums * s + 5] = fmaf(-g_min, f, fG);    // f (G - g_min)
                    // acc[kSums * s + 9] is not stored for these
                    // positions: the reduction sums each index on its own
                }
                slot_pos[s] = pos;
                filled = s + 1;
            }
        }
        if (filled == 0) break;
        // the registers past kSums * kSlots feed only sums that are never
        // stored: setting them here keeps them out of the registers live
        // across the slot loop
#pragma unroll
        for (int i = kSums * kSlots; i < kAcc; ++i) acc[i] = 0.f;
        const float r = reduce_scatter32(acc, lane);
        uint32_t my_pos = slot_pos[0];
#pragma unroll
        for (int i = 1; i < kSlots; ++i) my_pos = my_s == i ? slot_pos[i] : my_pos;
        if (my_store && my_s < filled) {
            if (my_pos < (uint32_t)tab_cap)
                atomicAdd(&table[my_v * tab_cap + my_pos], r);
            else if (my_v < kGradPlanes)
                atomicAdd(a.d_gauss + (int64_t)my_v * ng + a.ids[start + my_pos],
                          r * plane_scale(my_v, inv_1mg));
        }
    }
    __syncthreads();
    // the table's moments to the nine planes, one position per thread
    for (int p = threadIdx.x; p < tab_n; p += blockDim.x) {
        float S[kSums];
        bool any = false;
#pragma unroll
        for (int v = 0; v < kSums; ++v) {
            S[v] = table[v * tab_cap + p];
            any |= S[v] != 0.f;
        }
        if (!any) continue;
        const uint32_t id = a.ids[start + p];
        const float4 m = a.rec[3 * (int64_t)id];
        const float4 q = a.rec[3 * (int64_t)id + 1];
        const float mx = (m.x - ox) + m.z, my = (m.y - oy) + m.w;   // mean - tile centre
        const float ex = kHalfLog2eSqrt * q.x, ey = kHalfLog2eSqrt * q.y;
        const float fx = q.z * ex, fy = q.z * ey;
        const float op = q.w * inv_1mg;
        // sums over the tile's pixels of f G (dx, dy, dx^2, dx dy, dy^2), d = pixel - mean
        const float sx = fmaf(-mx, S[0], S[1]), sy = fmaf(-my, S[0], S[2]);
        const float sxx = fmaf(-mx, S[1] + sx, S[3]);
        const float sxy = fmaf(-mx, sy, fmaf(-my, S[1], S[4]));
        const float syy = fmaf(-my, S[2] + sy, S[5]);
        const float A = fmaf(ex, ex, fy * fy), B = fmaf(ex, ey, -fx * fy),
                    C = fmaf(ey, ey, fx * fx);
        const float k2 = 1.38629436112f * op;        // 2 ln 2 o'
        float out[kGradPlanes];
        out[0] = k2 * fmaf(A, sx, B * sy);
        out[1] = k2 * fmaf(B, sx, C * sy);
        out[2] = -0.5f * op * sxx;
        out[3] = -op * sxy;
        out[4] = -0.5f * op * syy;
        out[5] = fmaf(-g_min, S[9], S[0]) * inv_1mg;
        out[6] = S[6];
        out[7] = S[7];
        out[8] = S[8];
#pragma unroll
        for (int v = 0; v < kGradPlanes; ++v)
            if (out[v] != 0.f) atomicAdd(a.d_gauss + (int64_t)v * ng + id, out[v]);
    }
}

// Held to 80 VGPRs (six waves per SIMD; it needs 77, without spills), which
// matches the six blocks per CU its LDS allows: the pass waits on memory
// (records, tile ids, atomics) for a large part of its time, so resident waves
// count more than instruction count.
template <bool kRecompute>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_bwd_tiles(
    TileArgs a) {
    if (a.status[1] & Status::kOverflow) return;         // whole grid
    for_tiles(a, [&](int tile) { bwd_tile<kRecompute>(a, tile); });
}

__global__ void k_zero(float *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.f;
}

// Stage 2: one workgroup per curve.  Per Gaussian (r, k) the gradients of
// (mean, Q, o, colour) are chained to the sample points of its stencil:
//   Q = R diag(a, b) R^T, a = 1/sx2, b = 1/sy2, (c, s) = v/|v|,
//   sx2 = |X[r][ka]-X[r][kb]|^2/rho^2 + s0, sy2 = |X[ra][k]-X[rb][k]|^2/rho^2 + s0
//   (closed) or w^2 + s0 (open), mean = X[r][k].
// Each Gaussian stores its four stencil terms (mean, along-row, across-row,
// tangent) in LDS; every sample point then gathers the terms that reference
// it (the exact inverse of the stencil's index rules), so no atomics are
// needed and the result is deterministic.  The sample-point gradients then go
// to the control points: X[r][k] = sum_j B_j(t_k) ((1-tau_r) A_{3s+j} + tau_r B_{3s+j}).
// The boundary samples are evaluated in double precision (coordinates of
// thousands of pixels) and only their differences along each boundary and
// from boundary A to B are kept, rounded to float (differences of a pixel):
// a row's differences are blends of those, and the chain itself is float.
//
// NT threads per curve.  Two launches split the curves by size: those of at
// most kSmallCurve Gaussians (open strokes) run as one-wave workgroups with
// LDS sized for them, the others with kCurveThreads threads; each launch
// skips the other's curves.  lk and lg are the K and Gaussian capacities the
// dynamic LDS is laid out for.
// Eight waves per SIMD (at most 64 VGPRs; 49 used): the stage waits on
// latency, and at seven it ran 5% slower.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_bwd_curves(bz_curves c, int lk, int lg, double inv_rho2,
                                                   double s0, const float *__restrict__ d_gauss,
                                                   int64_t ng, float *__restrict__ d_ctrl,
                                                   float *__restrict__ d_width,
                                                   float *__restrict__ d_color,
                                                   float *__restrict__ d_opacity) {
    extern __shared__ double2 lds_xy[];
    __shared__ float s_tau[256];
    __shared__ float s_red[NT / 64][8];
    __shared__ float s_cp[2][3 * kMaxSeg + 1][2];
    const int p = blockIdx.x;
    const bool small = c.gauss_off[p + 1] - c.gauss_off[p] <= kSmallCurve;
    if (small != (NT == kWave)) return;   // the other launch's curve
    const int lane = threadIdx.x;          // thread of the curve's workgroup
    CurveView v = load_curve_view(c, p);
    stage_tau(v, s_tau, lane, NT);
    // [K] column differences of the boundary samples: DA[k] = XA[k+1] - XA[k],
    // DB[k] likewise, and W[k] = XB[k] - XA[k] (closed), in the boundary
    // samples' space (2 x double2 per column)
    float2 *DA = reinterpret_cast<float2 *>(lds_xy);
    float2 *DB = DA + lk;
    float2 *Wd = DB + lk;
    float4 *Bw = reinterpret_cast<float4 *>(lds_xy + 2 * lk);          // [K] Bernstein weights
    int *Bs = reinterpret_cast<int *>(Bw + lk);                        // [K] segment of column k
    float2 *Tm = reinterpret_cast<float2 *>(reinterpret_cast<char *>(lds_xy) +
                                            stage2_terms_offset(lk));  // mean term, then Xbar
    float2 *Tf = Tm + lg;                                              // along-row term
    float2 *Th = Tf + lg;                                              // across-row term
    float2 *Tv = Th + lg;                                              // tangent term
    float2 *Xbar = Tm;                                                 // [rows*K]
    const bool closed = v.kind == BZ_CLOSED;
    // The boundary samples in double precision, one per thread, in the space
    // of the terms (written only after the next barrier; 32 K <= 32 lg
    // bytes), and each column's segment and Bernstein weights beside them;
    // then the differences, rounded once.
    {
        double2 *P = reinterpret_cast<double2 *>(Tm);    // [A's K][B's K]
        const int nb = closed ? 2 : 1;
        for (int i = lane; i < (nb + 1) * v.K; i += NT) {
            if (i < nb * v.K) {
                const bool bb = i >= v.K;
                P[i] = boundary_point(v, bb, bb ? i - v.K : i);
            } else {
                const int k = i - nb * v.K;
                int s;
                double t, B[4];
                column_param(k, v.K, v.S, s, t);
                bernstein3(t, B);
                Bw[k] = make_float4((float)B[0], (float)B[1], (float)B[2], (float)B[3]);
                Bs[k] = s;
            }
        }
        __syncthreads();
        for (int k = lane; k < v.K; k += NT) {
            const double2 a0 = P[k], a1 = k + 1 < v.K ? P[k + 1] : a0;
            DA[k] = make_float2((float)(a1.x - a0.x), (float)(a1.y - a0.y));
            if (closed) {
                const double2 b0 = P[v.K + k], b1 = k + 1 < v.K ? P[v.K + k + 1] : b0;
                DB[k] = make_float2((float)(b1.x - b0.x), (float)(b1.y - b0.y));
                Wd[k] = make_float2((float)(b0.x - a0.x), (float)(b0.y - a0.y));
            }
        }
    }
    const int n = v.rows * v.K;
    __syncthreads();

    float wbar = 0.f, cb0 = 0.f, cb1 = 0.f, cb2 = 0.f;
    float ob[kMaxSeg] = {0.f, 0.f, 0.f, 0.f};
    const float rho2f = (float)inv_rho2;
    const int K = v.K, R1 = v.R + 1;
    // (r, k) of idx = lane + i*NT advance by (NT / K, NT % K) per pass.
    const int rstep = NT / K, kstep = NT - rstep * K;
    const int r0 = lane / K, k0 = lane - r0 * K;
    for (int idx = lane, r = r0, k = k0; idx < n; idx += NT) {
        float dg[kGradPlanes];
#pragma unroll
        for (int q = 0; q < kGradPlanes; ++q) dg[q] = d_gauss[q * ng + v.g0 + idx];
        // stencil (Eq. sigma with nearest-neighbour ends, Eq. rotation).  Row
        // r's samples are (1 - tau_r) XA + tau_r XB, so its differences along
        // the row are the same blend of DA and DB, and across rows
        // (tau_ra - tau_rb) W.
        const int kb = k < K - 1 ? k : K - 2;              // ka = kb + 1
        const int km = k > 0 ? k - 1 : 0;                  // kp = km + 1 or km + 2
        const bool two = k > 0 && k < K - 1;
        const float tr = closed ? v.tau[r] : 0.f, t1 = 1.f - tr;
        float dax = DA[kb].x, day = DA[kb].y;
        float vx = DA[km].x, vy = DA[km].y;
        if (two) {
            vx += DA[km + 1].x;
            vy += DA[km + 1].y;
        }
        float dyx = 0.f, dyy = 0.f, sy2;
        if (closed) {
            float bx = DB[km].x, by = DB[km].y;
            if (two) {
                bx += DB[km + 1].x;
                by += DB[km + 1].y;
            }
            vx = fmaf(tr, bx, t1 * vx);
            vy = fmaf(tr, by, t1 * vy);
            dax = fmaf(tr, DB[kb].x, t1 * dax);
            day = fmaf(tr, DB[kb].y, t1 * day);
            const int ra = r < R1 ? r + 1 : R1, rb = r < R1 ? r : R1 - 1;
            const float dt = v.tau[ra] - v.tau[rb];
            dyx = dt * Wd[k].x;
            dyy = dt * Wd[k].y;
            sy2 = (dyx * dyx + dyy * dyy) * rho2f + (float)s0;
        } else {
            sy2 = v.width * v.width + (float)s0;
        }
        const float sx2 = (dax * dax + day * day) * rho2f + (float)s0;
        const float nv2 = vx * vx + vy * vy;
        const float inv_nv = nv2 > 0.f ? __frsqrt_rn(nv2) : 0.f;
        const float cs = nv2 > 0.f ? vx * inv_nv : 1.f, sn = nv2 > 0.f ? vy * inv_nv : 0.f;
        const float ia = __builtin_amdgcn_rcpf(sx2), ib = __builtin_amdgcn_rcpf(sy2);
        const float qxx = dg[2], qxy = dg[3], qyy = dg[4];
        const float abar = qxx * cs * cs + qxy * cs * sn + qyy * sn * sn;
        const float bbar = qxx * sn * sn - qxy * cs * sn + qyy * cs * cs;
        const float cbar_t = qxx * 2.f * cs * ia + qxy * sn * (ia - ib) + qyy * 2.f * cs * ib;
        const float sbar_t = qxx * 2.f * sn * ib + qxy * cs * (ia - ib) + qyy * 2.f * sn * ia;
        const float f = 2.f * (-abar * ia * ia) * rho2f;
        const float sy2bar = -bbar * ib * ib;
        Tm[idx] = make_float2(dg[0], dg[1]);
        Tf[idx] = make_float2(f * dax, f * day);
        if (closed) {
            const float h = 2.f * sy2bar * rho2f;
            Th[idx] = make_float2(h * dyx, h * dyy);
        } else {
            wbar += 2.f * v.width * sy2bar;
        }
        if (nv2 > 0.f) {
            const float hd = cs * cbar_t + sn * sbar_t;
            Tv[idx] = make_float2((cbar_t - cs * hd) * inv_nv, (sbar_t - sn * hd) * inv_nv);
        } else {
            Tv[idx] = make_float2(0.f, 0.f);
        }
        const int slot = v.nopa == v.S ? Bs[k] : 0;
#pragma unroll
        for (int q = 0; q < kMaxSeg; ++q)
            if (q == slot) ob[q] += dg[5];
        cb0 += dg[6];
        cb1 += dg[7];
        cb2 += dg[8];
        k += kstep;
        r += rstep;
        if (k >= K) { k -= K; ++r; }
    }
    __syncthreads();
    // Gather: the terms each sample point (r, k) receives.
    //  along  +Tf(j) where ka(j) = k: j = k-1 (k >= 1), and j = K-1 when k = K-1
    //         -Tf(j) where kb(j) = k: j = k (k < K-1), and j = K-1 when k = K-2
    //  tangent+Tv(j) where kp(j) = k: j = k-1 (k >= 1), and j = K-1 when k = K-1
    //         -Tv(j) where km(j) = k: j = k+1 (k < K-1), and j = 0 when k = 0
    //  across +Th(i) where ra(i) = r: i = r-1 (r >= 1), and i = R+1 when r = R+1
    //         -Th(i) where rb(i) = r: i = r (r <= R), and i = R+1 when r = R
    // Xbar overwrites Tm in place: a point reads only its own mean term.
    for (int idx = lane, r = r0, k = k0; idx < n; idx += NT) {
        const int row = idx - k;
        const float2 x = Tm[idx];
        float ax = 0.f, ay = 0.f;
        if (k >= 1) { ax += Tf[row + k - 1].x + Tv[row + k - 1].x; ay += Tf[row + k - 1].y + Tv[row + k - 1].y; }
        if (k == K - 1) { ax += Tf[row + K - 1].x + Tv[row + K - 1].x; ay += Tf[row + K - 1].y + Tv[row + K - 1].y; }
        if (k < K - 1) { ax -= Tf[row + k].x + Tv[row + k + 1].x; ay -= Tf[row + k].y + Tv[row + k + 1].y; }
        if (k == K - 2) { ax -= Tf[row + K - 1].x; ay -= Tf[row + K - 1].y; }
        if (k == 0) { ax -= Tv[row].x; ay -= Tv[row].y; }
        if (closed) {
            if (r >= 1) { ax += Th[idx - K].x; ay += Th[idx - K].y; }
            if (r == R1) { ax += Th[idx].x; ay += Th[idx].y; }
            if (r <= R1 - 1) { ax -= Th[idx].x; ay -= Th[idx].y; }
            if (r == R1 - 1) { ax -= Th[idx + K].x; ay -= Th[idx + K].y; }
        }
        Xbar[idx] = make_float2(x.x + ax, x.y + ay);
        k += kstep;
        r += rstep;
        if (k >= K) { k -= K; ++r; }
    }

    // per-curve sums: wave reduction, then across the workgroup's waves
    wbar = wave_sum(wbar);
    cb0 = wave_sum(cb0);
    cb1 = wave_sum(cb1);
    cb2 = wave_sum(cb2);
#pragma unroll
    for (int q = 0; q < kMaxSeg; ++q) ob[q] = wave_sum(ob[q]);
    if ((lane & 63) == 0) {
        float *sr = s_red[lane >> 6];
        sr[0] = wbar; sr[1] = cb0; sr[2] = cb1; sr[3] = cb2;
#pragma unroll
        for (int q = 0; q < kMaxSeg; ++q) sr[4 + q] = ob[q];
    }
    __syncthreads();
    if (lane == 0) {
        for (int wv = 1; wv < NT / 64; ++wv) {
            wbar += s_red[wv][0]; cb0 += s_red[wv][1]; cb1 += s_red[wv][2]; cb2 += s_red[wv][3];
#pragma unroll
            for (int q = 0; q < kMaxSeg; ++q) ob[q] += s_red[wv][4 + q];
        }
        d_width[v.id] = closed ? 0.f : wbar;
        d_color[3 * v.id] = cb0;
        d_color[3 * v.id + 1] = cb1;
        d_color[3 * v.id + 2] = cb2;
        float *dop = d_opacity + c.opa_off[v.id];
#pragma unroll
        for (int q = 0; q < kMaxSeg; ++q)
            if (q < v.nopa) dop[q] = ob[q];
    }

    // Control points, in two deterministic steps.  (1) Thread (k, coord) sums
    // column k of Xbar over the rows three ways: all rows (open curves and the
    // endpoints a closed curve's boundaries share), weighted by 1 - tau_r (A's
    // interior points) and by tau_r (B's interior points); the sums go to LDS
    // over Tf..Tv (dead by now; 24 K bytes fit in their 24 rows*K).  (2) Thread
    // (point jj, coord, boundary) adds B_{jj - 3 s_k}(t_k) times those sums
    // over the columns k in order.
    const int m = 3 * v.S;
    float *colsum = reinterpret_cast<float *>(Tf);      // [K][coord][3]
    __syncthreads();   // every Xbar written, every T* read
    for (int t = lane; t < 2 * K; t += NT) {
        const int coord = t & 1, kk = t >> 1;
        float sall = 0.f, sa = 0.f, sb = 0.f;
        for (int rr = 0; rr < v.rows; ++rr) {
            const float2 xb2 = Xbar[rr * K + kk];
            const float xb = coord ? xb2.y : xb2.x;
            const float tr = closed ? v.tau[rr] : 0.f;
            sall += xb;
            sa = fmaf(1.f - tr, xb, sa);
            sb = fmaf(tr, xb, sb);
        }
        float *o = colsum + 3 * t;
        o[0] = sall;
        o[1] = sa;
        o[2] = sb;
    }
    __syncthreads();
    for (int t = lane; t < 4 * (m + 1); t += NT) {
        const int coord = t & 1, which = (t >> 1) & 1, jj = t >> 2;
        // which 1 (B's interior points) exists only for closed curves
        if (which == 1 && (!closed || jj == 0 || jj == m)) continue;
        const int pick = !closed || jj == 0 || jj == m ? 0 : 1 + which;
        float sum = 0.f;
        for (int kk = 0; kk < K; ++kk) {
            const int i = jj - 3 * Bs[kk];
            if (i < 0 || i > 3) continue;
            const float4 B = Bw[kk];
            const float w = i == 0 ? B.x : i == 1 ? B.y : i == 2 ? B.z : B.w;
            sum = fmaf(w, colsum[3 * (2 * kk + coord) + pick], sum);
        }
        s_cp[which][jj][coord] = sum;
    }
    __syncthreads();
    const int nstore = closed ? 2 * m : m + 1;
    float *out = d_ctrl + 2 * (int64_t)c.ctrl_off[v.id];
    for (int t = lane; t < 2 * nstore; t += NT) {
        const int coord = t & 1, j = t >> 1;
        const int which = j <= m ? 0 : 1;       // A (or open) points, then B's interior
        const int jj = j <= m ? j : j - m;
        out[t] = s_cp[which][jj][coord];
    }
}

__global__ void k_loss_zero(float *loss) {
    if (threadIdx.x == 0) loss[0] = 0.f;
}

__global__ __launch_bounds__(256) void k_l2(const float *__restrict__ img,
                                            const float *__restrict__ tgt, int64_t n, float scale,
                                            float *__restrict__ d, float *loss) {
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    float acc = 0.f;
    // four elements per load where all three arrays are 16-byte aligned
    const bool vec = ((reinterpret_cast<uintptr_t>(img) | reinterpret_cast<uintptr_t>(tgt) |
                       reinterpret_cast<uintptr_t>(d)) & 15) == 0;
    const int64_t n4 = vec ? n / 4 : 0;
    for (int64_t i = t0; i < n4; i += stride) {
        const float4 a = reinterpret_cast<const float4 *>(img)[i];
        const float4 b = reinterpret_cast<const float4 *>(tgt)[i];
        const float4 e = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
        reinterpret_cast<float4 *>(d)[i] = make_float4(scale * e.x, scale * e.y, scale * e.z,
                                                       scale * e.w);
        acc = fmaf(e.x, e.x, fmaf(e.y, e.y, fmaf(e.z, e.z, fmaf(e.w, e.w, acc))));
    }
    for (int64_t i = 4 * n4 + t0; i < n; i += stride) {
        const float e = img[i] - tgt[i];
        d[i] = scale * e;
        acc = fmaf(e, e, acc);
    }
    if (loss) {
        __shared__ float s_part[4];
        acc = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(loss, s_part[0] + s_part[1] + s_part[2] + s_part[3]);
    }
}

__global__ void k_counter_reset(uint32_t *counter) {
    if (threadIdx.x == 0) counter[0] = 0u;
}

// Workgroups of a persistent launch: as many as are resident on the device at
// once (occupancy of this kernel and block shape x compute units), at most
// one per tile.  Host queries only (nothing is enqueued), so the launch can be
// captured in a graph.
int persistent_grid(const void *kernel, int threads, size_t lds, int n_tiles) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, lds) != hipSuccess)
        return n_tiles;
    const int64_t blocks = (int64_t)(cus > 0 ? cus : 1) * (per > 0 ? per : 1);
    return blocks < n_tiles ? (int)blocks : n_tiles;
}

// Launch a blend kernel over all tiles: one workgroup per tile, or persistent
// workgroups behind a counter that is cleared first (by a kernel, so that the
// sequence can be captured in a graph).
template <typename K>
void launch_tiles(K kernel, TileArgs &a, const bz_bins &b, const bz_opts &o, int which,
                  int threads, size_t lds, hipStream_t s) {
    if (o.persistent && a.n_tiles > 0) {
        uint32_t *counters = (uint32_t *)b.workspace;     // BinLayout::off_counters == 0
        a.counter = counters + which;
        hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, s, a.counter);
        int grid = persistent_grid(reinterpret_cast<const void *>(kernel), threads, lds,
                                   a.n_tiles);
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, s, a);
    } else {
        a.counter = nullptr;
        hipLaunchKernelGGL(kernel, dim3(8 * a.per_xcd), dim3(threads), lds, s, a);
    }
}

TileArgs tile_args(const float *rec, const bz_bins &b, const bz_opts &o) {
    TileArgs a = {};
    a.rec = (const float4 *)rec;
    a.ids = b.ids;
    a.ranges = b.ranges;
    a.status = b.status;
    a.W = o.width;
    a.H = o.height;
    if (o.batch) {
        a.canvas = o.batch->canvas;
        a.n_canvas = o.batch->n_canvas;
    }
    a.tile_w = o.tile_w;
    a.tile_h = o.tile_h;
    a.tiles_x = (int)tiles_x(o);
    a.n_tiles = (int)num_tiles(o);
    a.per_xcd = (int)cdiv(a.n_tiles, 8);
    a.quads_x = o.tile_w / kQuad;
    a.bg0 = o.bg[0];
    a.bg1 = o.bg[1];
    a.bg2 = o.bg[2];
    a.g_min = o.g_min;
    a.alpha_max = o.alpha_max;
    a.t_min = o.t_min;
    a.inv_1mg = 1.0f / (1.0f - o.g_min);
    a.box_thr = 2.0f * (-logf(o.g_min)) * kCullSlackQuad;
    a.words_per_plane = visit_words_per_plane(o, b.cap_pairs);
    return a;
}

}  // namespace

hipError_t launch_fwd(const float *rec, const bz_bins &b, const bz_opts &o, float *image,
                      const bz_pixstate *st, const L2Out *l2, hipStream_t s) {
    TileArgs a = tile_args(rec, b, o);
    a.image = image;
    int threads = o.tile_w * o.tile_h;
    size_t lds = sizeof(Staged) * (size_t)threads;
    if (l2) {
        a.l2_target = l2->target;
        a.l2_grad = l2->d_image;
        a.l2_loss = l2->loss;
        a.l2_scale = l2->scale;
        if (l2->loss) hipLaunchKernelGGL(k_loss_zero, dim3(1), dim3(64), 0, s, l2->loss);
    }
    if (st) {
        a.t_final = st->t_final;
        a.n_last = st->n_last;
        a.n_contrib = st->n_contrib;
        a.visit = st->visit;
    }
    const bool count = st && st->n_contrib;
    if (l2) {
        if (!st)
            launch_tiles(k_fwd_l2<false, false>, a, b, o, 0, threads, lds, s);
        else if (count)
            launch_tiles(k_fwd_l2<true, true>, a, b, o, 0, threads, lds, s);
        else
            launch_tiles(k_fwd_l2<true, false>, a, b, o, 0, threads, lds, s);
    } else {
        if (!st)
            launch_tiles(k_fwd<false, false>, a, b, o, 0, threads, lds, s);
        else if (count)
            launch_tiles(k_fwd<true, true>, a, b, o, 0, threads, lds, s);
        else
            launch_tiles(k_fwd<true, false>, a, b, o, 0, threads, lds, s);
    }
    return hipGetLastError();
}

// Sum-table positions of a backward block whose batch masks take vis_bytes of
// LDS (0 for the stored blend state): kTableCap less those bytes, in whole
// multiples of 16 positions, at least 128.
int table_cap(size_t vis_bytes) {
    const int64_t per16 = (int64_t)(sizeof(float) * kSums * 16);
    const int64_t cut = ((int64_t)vis_bytes + per16 - 1) / per16 * 16;
    return kTableCap - cut < 128 ? 128 : (int)(kTableCap - cut);
}

hipError_t launch_bwd_gauss(const float *rec, int64_t n_gauss, const bz_bins &b,
                            const bz_opts &o, const float *d_image, const bz_pixstate *st,
                            float *d_gauss, hipStream_t s) {
    int64_t nz = (int64_t)kGradPlanes * n_gauss;
    if (nz > 0) {
        int64_t blocks = cdiv(nz, 256);
        if (blocks > 16384) blocks = 16384;
        hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, d_gauss, nz);
    }
    TileArgs a = tile_args(rec, b, o);
    a.d_image = d_image;
    a.d_gauss = d_gauss;
    a.n_gauss = n_gauss;
    int threads = o.tile_w * o.tile_h;
    const size_t vis = st ? 0 : sizeof(uint64_t) * kVisCap * (size_t)(threads / 64);
    a.tab_cap = table_cap(vis);
    size_t lds = sizeof(Staged) * (size_t)threads + vis + sizeof(float) * kSums * (size_t)a.tab_cap;
    if (st) {
        a.t_final = st->t_final;
        a.n_last = st->n_last;
        a.visit = st->visit;
        launch_tiles(k_bwd_tiles<false>, a, b, o, 1, threads, lds, s);
    } else {
        launch_tiles(k_bwd_tiles<true>, a, b, o, 1, threads, lds, s);
    }
    return hipGetLastError();
}

hipError_t launch_bwd_curves(const bz_curves &c, const bz_opts &o, const float *d_gauss,
                             const bz_grads &gr, hipStream_t s) {
    if (c.n_curves == 0) return hipSuccess;
    const double rho = (double)o.rho, inv_rho2 = 1.0 / (rho * rho), s0 = (double)o.sigma0_sq;
    if (c.max_gauss_per_curve > kSmallCurve) {
        const size_t lds = stage2_lds_bytes(c.max_k, c.max_gauss_per_curve);
        hipLaunchKernelGGL(k_bwd_curves<kCurveThreads>, dim3(c.n_curves), dim3(kCurveThreads),
                           lds, s, c, c.max_k, c.max_gauss_per_curve, inv_rho2, s0, d_gauss,
                           c.n_gauss, gr.d_ctrl, gr.d_width, gr.d_color, gr.d_opacity);
    }
    // a small curve has K <= its Gaussian count <= kSmallCurve
    const int lk = c.max_k < kSmallCurve ? c.max_k : kSmallCurve;
    const int lg = c.max_gauss_per_curve < kSmallCurve ? c.max_gauss_per_curve : kSmallCurve;
    hipLaunchKernelGGL(k_bwd_curves<kWave>, dim3(c.n_curves), dim3(kWave), stage2_lds_bytes(lk, lg),
                       s, c, lk, lg, inv_rho2, s0, d_gauss, c.n_gauss, gr.d_ctrl, gr.d_width,
                       gr.d_color, gr.d_opacity);
    return hipGetLastError();
}

hipError_t launch_l2(const float *image, const float *target, int64_t n, float scale,
                     float *d_image, float *loss, hipStream_t s) {
    if (loss) hipLaunchKernelGGL(k_loss_zero, dim3(1), dim3(64), 0, s, loss);
    if (n > 0) {
        // every workgroup adds its partial loss to one word: more than ~256 of
        // them and those same-address atomics, not HBM, set the time (at
        // 2048x2048: 27 us with 256, 33 with 1024, 62 with 4096)
        int64_t blocks = cdiv(n, 4 * 256);
        if (blocks > 256) blocks = 256;
        hipLaunchKernelGGL(k_l2, dim3(blocks), dim3(256), 0, s, image, target, n, scale, d_image,
                           loss);
    }
    return hipGetLastError();
}

}  // namespace bz
