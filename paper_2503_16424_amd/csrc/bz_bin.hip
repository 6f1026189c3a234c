// bz_bin.hip -- tile lists of the splatting pipeline (Sec. 3.4).
//
// 1. count : per Gaussian, the tiles its truncated support
//            1/2 d^T Sigma^-1 d <= -ln g_min (slightly inflated) reaches: the
//            tile rows of its bounding box on the canvas, and in each row the
//            tile columns the ellipse itself spans over that row's pixels
//            (tile_rect) -> tile rectangle and number of tiles.
// 2. scan  : exclusive scan of the counts -> pair offsets; the total is the pair
//            count (status[0]); more than cap_pairs sets the overflow flag and
//            every later stage of this call does nothing.
// 3. emit  : (tile, Gaussian) pairs, Gaussians in draw order, row by row with
//            the same per-row spans the count used.
// 4. sort  : stable LSD radix sort on the tile id only (8-bit digits, LDS
//            ranking with wave ballots, LDS staging so that the scattered
//            writes leave a block as contiguous runs).  Stability keeps the
//            draw order inside every tile.
// 5. ranges: first/last position of every tile in the sorted list.
//
// With at most 65,536 tiles and fewer than 2^24 Gaussians (bin_fused) steps
// 2-5 take a shorter route: the count also adds each Gaussian's pairs per
// (bucket of 256 consecutive tile keys, emission block of kEmitBlock
// Gaussians); the scan of those counts places every block's part of every
// bucket; the emission writes the pairs straight into their bucket, in draw
// order; and one stable radix pass on the low key byte inside each bucket
// finishes the lists, whose ranges then follow from that pass's scanned digit
// counts.  Same lists, one pass over the pairs fewer and no sorted keys.
//
// Sizes that depend on the data (the pair count) stay on the device: the
// grids are sized for the capacity and idle blocks exit, so a call never
// waits for the host.
#include "bz_internal.h"

namespace bz {

namespace {

constexpr int kBlk = 256;
constexpr int kItems = 16;
constexpr int kTile = kBlk * kItems;  // 4096 elements per block
constexpr int kRadix = 256;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

__device__ inline int lds_pad(int i) { return i + (i >> 5); }

// Block-wide exclusive scan of one 64-bit value per thread (256 threads).
__device__ inline uint64_t block_excl_scan(uint64_t v, uint64_t *s_wave, uint64_t &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t t = __shfl_up(x, d, 64);
        if (lane >= d) x += t;
    }
    if (lane == 63) s_wave[w] = x;
    __syncthreads();
    uint64_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlk / 64; ++i) {
        uint64_t s = s_wave[i];
        if (i < w) before += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + x - v;
}

// Exclusive prefix over the wave of one value per lane; total in *tot.
// Inclusive scan with DPP: within each 16-lane row by shifts of 1, 2, 4 and
// 8 lanes (zeros shifted in), then row 0's total into row 1 and row 2's into
// row 3 (row_bcast:15), then lane 31's (rows 0-1) into rows 2 and 3
// (row_bcast:31); lanes a row mask leaves out add the old value 0.
template <int CTRL, int ROWS, bool BOUND>
__device__ inline uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xF, BOUND);
}
__device__ inline uint32_t wave_excl_scan(uint32_t v, uint32_t &tot) {
    uint32_t x = v;
    x += dpp_u32<0x111, 0xF, true>(x);     // row_shr:1
    x += dpp_u32<0x112, 0xF, true>(x);     // row_shr:2
    x += dpp_u32<0x114, 0xF, true>(x);     // row_shr:4
    x += dpp_u32<0x118, 0xF, true>(x);     // row_shr:8
    x += dpp_u32<0x142, 0xA, false>(x);    // row_bcast:15 into rows 1 and 3
    x += dpp_u32<0x143, 0xC, false>(x);    // row_bcast:31 into rows 2 and 3
    tot = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
    return x - v;
}

__device__ inline void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// canvas (W x H) of Gaussian g: the single canvas, or its batch canvas
__device__ inline void gauss_canvas(const bz_canvas *cv, int n_canvas, int64_t g, int &W, int &H,
                                    int &tiles_x, uint32_t &tile_base) {
    if (!cv) return;
    const int c = batch_find(cv, n_canvas, g, [](const bz_canvas &r) { return r.gauss_off; });
    W = cv[c].width;
    H = cv[c].height;
    tiles_x = cv[c].tiles_x;
    tile_base = (uint32_t)cv[c].tile_off;
}

// One thread per Gaussian; on the bucketed path (bucket != null) each wave is
// one emission block, whose pairs per key bucket it adds up in LDS.
__global__ __launch_bounds__(256) void k_count(const float4 *__restrict__ rec, int64_t n, int W,
                                               int H, int tiles_x, float inv_tw, float inv_th,
                                               int th, float two_p,
                                               const bz_canvas *__restrict__ cv, int n_canvas,
                                               uint32_t *__restrict__ counts,
                                               ushort4 *__restrict__ rects,
                                               uint32_t *__restrict__ bucket, int nbk,
                                               int64_t n_eblk, int64_t *status) {
    static_assert(kEmitBlock == 64, "one emission block per wave");
    __shared__ uint32_t s_hb[4][256];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *hb = s_hb[wv];
    if (bucket) {
        for (int i = lane; i < nbk; i += 64) hb[i] = 0u;
        wave_lds_fence();
    }
    if (g < n) {
        int txc = tiles_x;
        uint32_t tbase = 0;
        gauss_canvas(cv, n_canvas, g, W, H, txc, tbase);
        ushort4 rc;
        bool finite;
        const uint32_t cnt = tile_rect(rec[3 * g], rec[3 * g + 1], W, H, inv_tw, inv_th, th,
                                       two_p, rc, finite, [&](int ty, int c0, int c1) {
                                           if (!bucket) return;
                                           const uint32_t k0 = tbase + (uint32_t)ty * (uint32_t)txc +
                                                               (uint32_t)c0;
                                           for_key_buckets(k0, (uint32_t)(c1 - c0 + 1),
                                                           [&](uint32_t h, uint32_t c) {
                                                               atomicAdd(&hb[h], c);
                                                           });
                                       });
        if (!finite)
            atomicOr((unsigned long long *)&status[1], (unsigned long long)Status::kNonFinite);
        if (counts) counts[g] = cnt;
        rects[g] = rc;
    }
    if (bucket) {
        wave_lds_fence();
        const int64_t eb = g / kEmitBlock;
        if (eb < n_eblk)
            for (int i = lane; i < nbk; i += 64) bucket[(int64_t)i * n_eblk + eb] = hb[i];
    }
}

// --- device-wide exclusive scan of uint32 (64-bit partials) ---------------

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                     uint64_t *__restrict__ part) {
    __shared__ uint64_t s_wave[kBlk / 64];
    int64_t base = (int64_t)blockIdx.x * kTile;
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        int64_t e = base + j * kBlk + threadIdx.x;
        if (e < n) s += in[e];
    }
    uint64_t tot;
    block_excl_scan(s, s_wave, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Block b: exclusive scan of its kTile values, plus the carry-in of the blocks
// before it, which it adds up from their partials itself.  The last block also
// writes the grand total to total_out (may be null) and raises the overflow
// flag when it exceeds cap.
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *in, uint32_t *out, int64_t n,
                                                    const uint64_t *__restrict__ part,
                                                    int64_t *total_out, int64_t cap,
                                                    int64_t *status) {
    __shared__ uint32_t s_v[kTile + kTile / 32];
    __shared__ uint64_t s_wave[kBlk / 64];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    // the block's values and the partials before it are loaded kU at a time
    // with no wait between the loads: one memory latency instead of one per
    // partial a thread adds
    uint32_t x[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t e = base + j * kBlk + threadIdx.x;
        x[j] = e < n ? in[e] : 0u;
    }
    constexpr int kU = 8;
    const int64_t nprev = blockIdx.x;
    uint64_t c = 0;
    int64_t i = threadIdx.x;
    for (; i + (kU - 1) * kBlk < nprev; i += kU * kBlk) {
        uint64_t p[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) p[u] = part[i + u * kBlk];
#pragma unroll
        for (int u = 0; u < kU; ++u) c += p[u];
    }
    {
        uint64_t p[kU - 1];
#pragma unroll
        for (int u = 0; u < kU - 1; ++u) p[u] = i + u * kBlk < nprev ? part[i + u * kBlk] : 0ull;
#pragma unroll
        for (int u = 0; u < kU - 1; ++u) c += p[u];
    }
    uint64_t carry;
    block_excl_scan(c, s_wave, carry);
#pragma unroll
    for (int j = 0; j < kItems; ++j) s_v[lds_pad(j * kBlk + threadIdx.x)] = x[j];
    __syncthreads();
    uint32_t v[kItems];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        v[j] = s_v[lds_pad(threadIdx.x * kItems + j)];
        s += v[j];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan(s, s_wave, tot) + carry;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        s_v[lds_pad(threadIdx.x * kItems + j)] = (uint32_t)ex;
        ex += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        int li = j * kBlk + threadIdx.x;
        int64_t e = base + li;
        if (e < n) out[e] = s_v[lds_pad(li)];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0 && total_out) {
        *total_out = (int64_t)(carry + tot);
        if ((int64_t)(carry + tot) > cap)
            atomicOr((unsigned long long *)&status[1], (unsigned long long)Status::kOverflow);
    }
}

hipError_t scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint64_t *part,
                    int64_t *total_out, int64_t cap, int64_t *status, hipStream_t s) {
    int64_t nb = cdiv(n, kTile);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlk), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlk), 0, s, in, out, n,
                       (const uint64_t *)part, total_out, cap, status);
    return hipGetLastError();
}

// --- pair emission ---------------------------------------------------------

// Pair emission, one wave per 64 consecutive Gaussians, which own one
// contiguous output range (their scan offsets are consecutive).  Their tile
// rows are taken as (Gaussian, row) items, kRowChunk at a time: every item's
// span of tile columns (support_row: the same function of the same record
// bits as the count, so the widths add up to the counts exactly) and an
// exclusive scan of the widths give each row its place; the wave then writes
// the chunk's output range, consecutive lanes on consecutive positions, each
// finding its row by binary search.  In a batch the key is the global
// tile: the canvas's first tile + its local tile.  Every Gaussian's last row
// must end where its range ends; otherwise the lists are marked invalid
// (never expected), and nothing downstream reads them.  Any position left
// unwritten then holds the key one past the last tile, which sorts after
// every real tile and no range covers.
constexpr int kEmitG = 64;        // Gaussians per wave
constexpr int kRowChunk = 256;    // row items per round

__global__ __launch_bounds__(64) void k_emit(const float4 *__restrict__ rec,
                                             const uint32_t *__restrict__ offs,
                                             const ushort4 *__restrict__ rects, int64_t n, int W,
                                             int H, int tiles_x, float inv_tw, int th,
                                             float two_p, const bz_canvas *__restrict__ cv,
                                             int n_canvas, uint32_t end_key,
                                             uint32_t *__restrict__ keys,
                                             uint32_t *__restrict__ vals,
                                             const int64_t *status) {
    __shared__ uint32_t s_rows[kEmitG + 1];   // exclusive prefix of tile rows per Gaussian
    __shared__ uint32_t s_off[kEmitG + 1];    // pair offsets (the last: the wave's end)
    __shared__ Support s_sup[kEmitG];         // each Gaussian's support, computed once
    __shared__ uint32_t s_key0[kEmitG];       // key of tile (0, first row of its rectangle)
    __shared__ uint16_t s_ty0[kEmitG];        // first tile row of its rectangle
    __shared__ int s_tx[kEmitG];              // tiles per row of its canvas
    __shared__ uint32_t s_item_off[kRowChunk + 1];
    __shared__ uint32_t s_item_key[kRowChunk];  // key of the row's first tile
    __shared__ uint8_t s_item_g[kRowChunk];     // Gaussian of the row (in the wave)
    if (status[1] & Status::kOverflow) return;
    const int64_t g0 = (int64_t)blockIdx.x * kEmitG;
    const int nb = (int)(n - g0 < kEmitG ? n - g0 : kEmitG);
    const int t = threadIdx.x;
    uint32_t my_rows = 0;
    if (t < nb) {
        const int64_t g = g0 + t;
        const ushort4 rc = rects[g];
        s_off[t] = offs[g];
        int Wc = W, Hc = H, txc = tiles_x;
        uint32_t base = 0;
        gauss_canvas(cv, n_canvas, g, Wc, Hc, txc, base);
        Support sp;
        bool finite;
        // the count's function on the same record bits; a Gaussian without
        // support has the empty rectangle and no rows
        if (rc.x <= rc.z && rc.y <= rc.w &&
            support_of(rec[3 * g], rec[3 * g + 1], Wc, Hc, two_p, sp, finite)) {
            my_rows = (uint32_t)(rc.w - rc.y + 1);
            s_sup[t] = sp;
            s_key0[t] = base + (uint32_t)rc.y * (uint32_t)txc;
            s_ty0[t] = rc.y;
            s_tx[t] = txc;
        }
    }
    uint32_t nrows;
    s_rows[t] = wave_excl_scan(my_rows, nrows);
    if (t == 0) {
        s_rows[kEmitG] = nrows;
        s_off[nb] = g0 + nb < n ? offs[g0 + nb] : (uint32_t)status[0];
    }
    wave_lds_fence();
    uint32_t out = s_off[0];                   // next output position
    for (uint32_t c0 = 0; c0 < nrows; c0 += kRowChunk) {
        const uint32_t ci = nrows - c0 < (uint32_t)kRowChunk ? nrows - c0 : (uint32_t)kRowChunk;
        // the round's rows (four per lane, consecutive): span of tile columns, width
        uint32_t wsum = 0;
        uint32_t wid[kRowChunk / 64];
#pragma unroll
        for (int j = 0; j < kRowChunk / 64; ++j) {
            const uint32_t it = (uint32_t)t * (kRowChunk / 64) + j;
            wid[j] = 0;
            if (it < ci) {
                const uint32_t r = c0 + it;
                // last Gaussian whose first row <= r (lanes past nb hold
                // nrows > r, so the search needs no bound)
                int lo = 0;
#pragma unroll
                for (int step = kEmitG / 2; step >= 1; step >>= 1)
                    if (s_rows[lo + step] <= r) lo += step;
                const int dr = (int)(r - s_rows[lo]);
                int cl, ch;
                support_row(s_sup[lo], (int)s_ty0[lo] + dr, th, inv_tw, cl, ch);
                wid[j] = ch >= cl ? (uint32_t)(ch - cl + 1) : 0u;
                s_item_key[it] = s_key0[lo] + (uint32_t)dr * (uint32_t)s_tx[lo] + (uint32_t)cl;
                s_item_g[it] = (uint8_t)lo;
                wsum += wid[j];
            }
        }
        uint32_t cnt;
        uint32_t ex = wave_excl_scan(wsum, cnt);
#pragma unroll
        for (int j = 0; j < kRowChunk / 64; ++j) {
            const uint32_t it = (uint32_t)t * (kRowChunk / 64) + j;
            if (it < ci) s_item_off[it] = ex;
            ex += wid[j];
        }
        // the slots past the chunk's last row hold cnt (> every pair index),
        // so the pair search below needs no bound
        for (uint32_t it = ci + t; it <= (uint32_t)kRowChunk; it += 64) s_item_off[it] = cnt;
        wave_lds_fence();
#pragma unroll
        for (int j = 0; j < kRowChunk / 64; ++j) {
            const uint32_t it = (uint32_t)t * (kRowChunk / 64) + j;
            if (it < ci) {
                const int gl = s_item_g[it];
                if (c0 + it + 1 == s_rows[gl + 1] && out + s_item_off[it + 1] != s_off[gl + 1])
                    atomicOr((unsigned long long *)&status[1],
                             (unsigned long long)(Status::kOverflow | Status::kListMismatch));
            }
        }
        // consecutive lanes on consecutive positions (coalesced stores), each
        // finding its row by binary search
        for (uint32_t i = t; i < cnt; i += 64) {
            int lo = 0;                        // last row item whose offset <= i
#pragma unroll
            for (int step = kRowChunk / 2; step >= 1; step >>= 1)
                if (s_item_off[lo + step] <= i) lo += step;
            const uint32_t o = out + i;
            const int gl = s_item_g[lo];
            // only inside the Gaussian's own range (the counts agree, so this holds)
            if (o >= s_off[gl] && o < s_off[gl + 1]) {
                keys[o] = s_item_key[lo] + (i - s_item_off[lo]);
                vals[o] = (uint32_t)(g0 + gl);
            }
        }
        out += cnt;
        wave_lds_fence();
    }
    // positions of the wave's range no row filled
    for (uint32_t o = out + t; o < s_off[nb]; o += 64) {
        keys[o] = end_key;
        vals[o] = (uint32_t)(g0 + nb - 1);
    }
}

// --- stable LSD radix sort on tile ids --------------------------------------
//
// A block owns kTile consecutive elements; inside it wave w owns the kWaveItems
// elements [w kWaveItems, (w + 1) kWaveItems) and takes them 64 at a time, in
// order, lane l holding element 64 j + l of round j.  The lanes of a round that
// share a digit find each other with one ballot per digit bit; the lowest of
// them adds the group's size to the wave's count of that digit (an LDS word no
// other lane of the round touches).  So every element learns its rank among the
// wave's elements of its digit, in element order, without block barriers.

constexpr int kWaveItems = kItems * 64;

// Lanes of the wave whose digit equals this lane's (valid lanes only).  Per
// bit, a lane keeps the lanes whose bit agrees with its own: with m all ones
// where the bit is set, peers &= ~(ballot ^ m) on each 32-bit half, one
// three-input bit operation (v_bitop3_b32) per half.
__device__ inline uint64_t digit_peers(bool valid, uint32_t d, int nbits) {
    const uint64_t vb = __ballot(valid);
    uint32_t lo = (uint32_t)vb, hi = (uint32_t)(vb >> 32);
    for (int b = 0; b < nbits; ++b) {
        const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);   // bit b, sign-extended
        const uint64_t bal = __ballot(m != 0u);
        lo &= ~((uint32_t)bal ^ m);
        hi &= ~((uint32_t)(bal >> 32) ^ m);
    }
    return valid ? (((uint64_t)hi << 32) | lo) : 0ull;
}

// Per-block digit counts in LDS (atomics: cheaper here than grouping the lanes
// of a digit with ballots first, which the scatter needs for its ranks anyway;
// adding runs of equal digits at once took 3 us off each pass).
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                    const int64_t *status, int shift, int nbits,
                                                    uint32_t *__restrict__ hist,
                                                    int64_t hist_blocks) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t n = (status[1] & Status::kOverflow) ? 0 : status[0];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const uint32_t mask = (1u << nbits) - 1u;
    if (base < n) {
        // thread t counts keys [16t, 16t + 16) of the block, adding each run of
        // equal digits with one atomic (neighbouring pairs often share a digit)
        const int64_t e0 = base + (int64_t)threadIdx.x * kItems;
        uint32_t run_d = 0u, run_c = 0u;
        auto count = [&](uint32_t key) {
            const uint32_t d = (key >> shift) & mask;
            if (d != run_d && run_c) {
                atomicAdd(&h[run_d], run_c);
                run_c = 0u;
            }
            run_d = d;
            ++run_c;
        };
        if (e0 + kItems <= n) {
            const uint4 *p = reinterpret_cast<const uint4 *>(keys + e0);   // 64-byte aligned
#pragma unroll
            for (int v = 0; v < kItems / 4; ++v) {
                const uint4 k4 = p[v];
                count(k4.x);
                count(k4.y);
                count(k4.z);
                count(k4.w);
            }
        } else {
            for (int j = 0; j < kItems; ++j)
                if (e0 + j < n) count(keys[e0 + j]);
        }
        if (run_c) atomicAdd(&h[run_d], run_c);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * hist_blocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_radix_scatter(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
    uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
    const uint32_t *__restrict__ hist_scanned, int64_t hist_blocks, const int64_t *status,
    int shift, int nbits) {
    __shared__ uint32_t s_keys[kTile];
    __shared__ uint32_t s_vals[kTile];
    __shared__ uint32_t s_prefix[kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    __shared__ uint32_t s_wrun[kBlk / 64][kRadix];   // per-wave digit counts, then bases
    __shared__ uint64_t s_wave[kBlk / 64];

    if (status[1] & Status::kOverflow) return;
    const int64_t n = status[0];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base >= n) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t dmask = (1u << nbits) - 1u;
    const int cnt = (int)(n - base < kTile ? n - base : kTile);

#pragma unroll
    for (int q = 0; q < kBlk / 64; ++q) s_wrun[q][tid] = 0;
    __syncthreads();

    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t *run = s_wrun[w];
    uint32_t key[kItems], val[kItems], rank[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int li = w * kWaveItems + j * 64 + lane;
        const bool valid = li < cnt;
        key[j] = valid ? keys_in[base + li] : 0u;
        val[j] = valid ? vals_in[base + li] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int li = w * kWaveItems + j * 64 + lane;
        const bool valid = li < cnt;
        const uint32_t d = (key[j] >> shift) & dmask;
        const uint64_t peers = digit_peers(valid, d, nbits);
        // the wave's LDS accesses execute in order: this round reads the
        // counts the previous round's group leaders wrote
        const uint32_t before = valid ? run[d] : 0u;
        rank[j] = before + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) run[d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        // digit tid: bases of the four waves, then the block's prefix
        uint32_t t = 0;
#pragma unroll
        for (int q = 0; q < kBlk / 64; ++q) {
            const uint32_t c = s_wrun[q][tid];
            s_wrun[q][tid] = t;
            t += c;
        }
        uint64_t tot;
        s_prefix[tid] = (uint32_t)block_excl_scan(t, s_wave, tot);
        s_gbase[tid] = hist_scanned[(int64_t)tid * hist_blocks + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int li = w * kWaveItems + j * 64 + lane;
        if (li < cnt) {
            const uint32_t d = (key[j] >> shift) & dmask;
            const uint32_t slot = s_prefix[d] + run[d] + rank[j];
            s_keys[slot] = key[j];
            s_vals[slot] = val[j];
        }
    }
    __syncthreads();
    for (int i = tid; i < cnt; i += kBlk) {
        const uint32_t k = s_keys[i];
        const uint32_t d = (k >> shift) & dmask;
        const uint32_t pos = s_gbase[d] + (uint32_t)i - s_prefix[d];
        keys_out[pos] = k;
        vals_out[pos] = s_vals[i];
    }
}

// Start of a binning: the status words (pair count, flags) and every tile's
// range cleared, in one launch.
__global__ void k_bin_clear(int64_t *status, uint32_t *ranges, int64_t n_ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_ranges) ranges[i] = 0u;
    if (i < 2) status[i] = 0;
}

// First and one-past-last position of every tile: thread t looks at the
// kRangeItems keys from kRangeItems t and the key after them.
constexpr int kRangeItems = 8;

__global__ __launch_bounds__(256) void k_ranges(const uint32_t *__restrict__ keys,
                                                const int64_t *status, int64_t cap,
                                                uint32_t n_tiles, uint32_t *__restrict__ ranges) {
    if (status[1] & Status::kOverflow) return;
    const int64_t n0 = status[0];
    const int64_t n = n0 < cap ? n0 : cap;
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeItems;
    if (i0 >= n) return;
    uint32_t k[kRangeItems + 1];
    if (i0 + kRangeItems <= n && (i0 & 3) == 0) {
        const uint4 a = *reinterpret_cast<const uint4 *>(keys + i0);
        const uint4 b = *reinterpret_cast<const uint4 *>(keys + i0 + 4);
        k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w;
        k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
    } else {
#pragma unroll
        for (int j = 0; j < kRangeItems; ++j) k[j] = i0 + j < n ? keys[i0 + j] : ~0u;
    }
    k[kRangeItems] = i0 + kRangeItems < n ? keys[i0 + kRangeItems] : ~0u;
    const uint32_t prev = i0 > 0 ? keys[i0 - 1] : ~0u;
#pragma unroll
    for (int j = 0; j < kRangeItems; ++j) {
        const int64_t i = i0 + j;
        if (i >= n || k[j] >= n_tiles) break;      // keys past the last tile: no range
        if ((j == 0 ? prev : k[j - 1]) != k[j]) ranges[2 * (int64_t)k[j]] = (uint32_t)i;
        if (k[j + 1] != k[j]) ranges[2 * (int64_t)k[j] + 1] = (uint32_t)(i + 1);
    }
}

__global__ void k_set_count(int64_t *status, int64_t n) {
    if (threadIdx.x == 0) {
        status[0] = n;
        status[1] = 0;
    }
}

// --- bucketed path ----------------------------------------------------------

// Start of a bucketed binning with Gaussians: the status words and the
// (bucket, emission block) counts cleared, in one launch (the in-bucket pass
// writes every tile's range itself).  16 bytes per thread (the table starts
// on a 256-byte boundary), then the last n % 4 words.
__global__ void k_bucket_clear(int64_t *status, uint32_t *bucket, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n4 = n >> 2;
    if (i < n4) reinterpret_cast<uint4 *>(bucket)[i] = make_uint4(0u, 0u, 0u, 0u);
    if (i < (n & 3)) bucket[4 * n4 + i] = 0u;
    if (i < 2) status[i] = 0;
}


// Bucketed emission.  A bucket's pairs form one contiguous segment of the
// packed array, emission block 0's first, then block 1's, ...: the scanned
// (bucket, block) counts, bucket-major, give each block its place.  One wave
// per emission block of kEmitBlock (= kEmitG = 64) Gaussians (kEmitWaves per
// workgroup).  The pairs are generated as in k_emit: (Gaussian, row) items,
// kBkChunk at a time, each row's span by support_row (the count's function
// of the same record bits), and consecutive lanes on consecutive pairs of the
// chunk (Gaussian-major, i.e. draw order), each finding its row by counting
// the marked first pairs of the rows at or before it (a bitmap per chunk; a
// binary search in chunks of more than kStartBits pairs); a row item finds
// its Gaussian the same way from the Gaussians' first items.  A pair's place
// is its bucket's running position in the block's part (LDS) plus the lanes
// of the round before it with the same bucket, found with one ballot per bit
// of the bucket's index relative to the block's first bucket (as the radix
// scatter ranks digits); so each bucket keeps draw order, and a row whose
// keys straddle two buckets needs nothing special.  LDS per wave is what
// limits the waves a CU holds, so the supports are kept as 32 bytes and the
// bucket arrays are sized for the buckets there are (64 or 256).  A pair is packed as (key & 255) << 24 | Gaussian.  Every bucket's
// total must equal the count's; otherwise the lists are marked invalid (never
// expected), and no lane writes outside the block's part of a bucket.
// Neighbouring blocks' parts of a bucket are neighbours in memory, so blocks
// are dealt to the XCDs in contiguous runs (the dispatcher sends workgroup w to
// XCD w % 8): the parts meet in one L2.
constexpr int kEmitWaves = 1;
constexpr int kStartBits = 2048;   // pairs of a chunk whose rows a bitmap marks
constexpr int kBkChunk = 128;   // row items per chunk

// A support as the bucketed emission keeps it in LDS: the float row geometry
// and the pixel box in 16 bits (a canvas side is at most 32768 pixels); r2
// depends on the options alone and is recomputed as the support computes it.
struct SupportLds {
    float mx, my, a, D, isyy, dys;
    uint16_t px0, px1, py0, py1;
};

__device__ inline SupportLds pack_support(const Support &s) {
    return SupportLds{s.mx, s.my, s.a, s.D, s.isyy, s.dys, (uint16_t)s.px0, (uint16_t)s.px1,
                      (uint16_t)s.py0, (uint16_t)s.py1};
}

__device__ inline Support unpack_support(const SupportLds &p, float r2) {
    Support s;
    s.mx = p.mx;
    s.my = p.my;
    s.a = p.a;
    s.D = p.D;
    s.isyy = p.isyy;
    s.dys = p.dys;
    s.r2 = r2;
    s.px0 = p.px0;
    s.px1 = p.px1;
    s.py0 = p.py0;
    s.py1 = p.py1;
    return s;
}

// Segment table of the in-bucket pass, written by one wave (the first of the
// emission, which runs after the counts' scan and before the pass):
// seg[s] = first position of bucket s, seg[nbk + 1 + s] = its first radix
// block (ceil(len / kTile) blocks per bucket), entry nbk of each = the end.
// Lane l takes buckets 4 l .. 4 l + 3 (nbk <= 256).
__device__ inline void segment_table(const uint32_t *__restrict__ bucket, int nbk,
                                     int64_t n_eblk, uint32_t total, int lane,
                                     uint32_t *__restrict__ seg) {
    uint32_t S[4], nb[4], sum = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = 4 * lane + i;
        S[i] = t < nbk ? bucket[(int64_t)t * n_eblk] : total;
        const uint32_t S1 = t + 1 < nbk ? bucket[(int64_t)(t + 1) * n_eblk] : total;
        nb[i] = t < nbk ? (S1 - S[i] + kTile - 1) / kTile : 0u;
        sum += nb[i];
    }
    uint32_t tot;
    uint32_t P = wave_excl_scan(sum, tot);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = 4 * lane + i;
        if (t <= nbk) {
            seg[t] = S[i];
            seg[nbk + 1 + t] = P;
        }
        P += nb[i];
    }
    if (nbk == 4 * 64 && lane == 63) {
        seg[nbk] = total;
        seg[2 * nbk + 1] = P;
    }
}

// kMaxBk: at least the number of buckets (the LDS of a wave's bucket parts)
template <int kMaxBk>
__global__ __launch_bounds__(64 * kEmitWaves) void k_emit_bucketed(
    const float4 *__restrict__ rec, const ushort4 *__restrict__ rects, int64_t n, int W, int H,
    int tiles_x, float inv_tw, int th, float two_p, const bz_canvas *__restrict__ cv,
    int n_canvas, const uint32_t *__restrict__ bucket, int nbk, int64_t n_eblk,
    uint32_t *__restrict__ packed, uint32_t *__restrict__ seg, int64_t *status) {
    static_assert(kEmitBlock == kEmitG, "one emission block per wave");
    __shared__ uint32_t s_rows[kEmitWaves][kEmitG + 1];   // exclusive prefix of tile rows
    __shared__ SupportLds s_sup[kEmitWaves][kEmitG];
    __shared__ uint32_t s_key0[kEmitWaves][kEmitG];      // key of tile (first row, column 0)
    __shared__ uint16_t s_ty0[kEmitWaves][kEmitG];
    __shared__ uint16_t s_tx[kEmitWaves][kEmitG];
    // rows with pairs: (first pair in the chunk, first key | Gaussian << 16),
    // one 8-byte read for a pair's row (keys are below 2^16 on this path)
    __shared__ uint2 s_item[kEmitWaves][kBkChunk + 1];
    __shared__ __align__(8) uint32_t s_start[kEmitWaves][kStartBits / 32];
    __shared__ uint8_t s_nzg[kEmitWaves][kEmitG];        // Gaussians with rows, in order
    __shared__ uint32_t s_gstart[kEmitWaves][kBkChunk / 32], s_gpref[kEmitWaves][kBkChunk / 32];
    // a bucket's next position in this block's part, and the part's end
    __shared__ uint2 s_pe[kEmitWaves][kMaxBk];   // (pos, end), one 8-byte read
    if (status[1] & Status::kOverflow) return;
    const int t = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (blockIdx.x == 0 && wv == 0) segment_table(bucket, nbk, n_eblk, (uint32_t)status[0], t, seg);
    const int64_t per = (n_eblk + 8 * kEmitWaves - 1) / (8 * kEmitWaves);   // workgroups per XCD
    const int64_t eb = ((int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3)) * kEmitWaves + wv;
    if (eb >= n_eblk) return;                        // whole wave
    const int64_t g0 = eb * kEmitG;
    const int nb = (int)(n - g0 < kEmitG ? n - g0 : kEmitG);
    const uint32_t total = (uint32_t)status[0];
    const int64_t nflat = (int64_t)nbk * n_eblk;
    uint32_t my_rows = 0, hlo = 0xffffffffu, hhi = 0;
    if (t < nb) {
        const int64_t g = g0 + t;
        const ushort4 rc = rects[g];
        int Wc = W, Hc = H, txc = tiles_x;
        uint32_t tbase = 0;
        gauss_canvas(cv, n_canvas, g, Wc, Hc, txc, tbase);
        Support sp;
        bool finite;
        if (rc.x <= rc.z && rc.y <= rc.w &&
            support_of(rec[3 * g], rec[3 * g + 1], Wc, Hc, two_p, sp, finite)) {
            my_rows = (uint32_t)(rc.w - rc.y + 1);
            s_sup[wv][t] = pack_support(sp);
            s_key0[wv][t] = tbase + (uint32_t)rc.y * (uint32_t)txc;
            s_ty0[wv][t] = rc.y;
            s_tx[wv][t] = (uint16_t)txc;
            // the keys of its pairs lie in [key(first row, rc.x), key(last row, rc.z)]
            hlo = (tbase + (uint32_t)rc.y * (uint32_t)txc + rc.x) >> 8;
            hhi = (tbase + (uint32_t)rc.w * (uint32_t)txc + rc.z) >> 8;
        }
    }
    uint32_t nrows;
    const uint32_t row0 = wave_excl_scan(my_rows, nrows);   // this lane's first row item
    s_rows[wv][t] = row0;
    if (t == 0) s_rows[wv][kEmitG] = nrows;
    // the Gaussians with rows, compacted in order
    const bool has_rows = my_rows != 0u;
    const uint64_t nzm = __ballot(has_rows);
    if (has_rows)
        s_nzg[wv][__builtin_amdgcn_mbcnt_hi((uint32_t)(nzm >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)nzm, 0u))] =
            (uint8_t)t;
    const uint32_t hl = wave_min_u32(hlo);
    if (hl == 0xffffffffu) return;                   // no pairs in this block
    const uint32_t span = wave_max_u32(my_rows ? hhi : 0u) - hl;   // buckets hl .. hl + span
    int nbits = 0;
    while (nbits < 8 && (1u << nbits) <= span) ++nbits;
    nbits = __builtin_amdgcn_readfirstlane(nbits);     // wave-uniform: a scalar loop
    // this block's part of each of its buckets (first position, size), stored
    // in LDS once the first chunk's rows are done, which hides the loads
    auto fetch_parts = [&]() {
        for (uint32_t i = t; i <= span; i += 64) {
            const int64_t fi = (int64_t)(hl + i) * n_eblk + eb;
            const uint32_t a = bucket[fi];
            s_pe[wv][i] = make_uint2(a, fi + 1 < nflat ? bucket[fi + 1] : total);
        }
    };
    const uint64_t lt = (t == 0) ? 0ull : (~0ull >> (64 - t));
    const int th_ = th;
    const float r2 = two_p * (kCullSlackBox * kCullSlackBox);   // as support_of sets it
    for (uint32_t c0 = 0; c0 < nrows; c0 += kBkChunk) {
        const uint32_t ci = nrows - c0 < (uint32_t)kBkChunk ? nrows - c0 : (uint32_t)kBkChunk;
        // A row item's Gaussian: mark the first items of the Gaussians with
        // rows that start in the chunk; the item's Gaussian is the
        // (carry + marks at or before it)-th of them, carry the number that
        // start before the chunk.
        if (t < kBkChunk / 32) s_gstart[wv][t] = 0u;
        wave_lds_fence();
        if (has_rows && row0 >= c0 && row0 - c0 < (uint32_t)kBkChunk)
            atomicOr(&s_gstart[wv][(row0 - c0) >> 5], 1u << ((row0 - c0) & 31));
        const uint32_t carry = (uint32_t)__popcll(__ballot(has_rows && row0 < c0));
        wave_lds_fence();
        {
            const uint32_t pc = t < kBkChunk / 32 ? (uint32_t)__popc(s_gstart[wv][t]) : 0u;
            uint32_t tot_pc;
            const uint32_t pref = wave_excl_scan(pc, tot_pc);
            if (t < kBkChunk / 32) s_gpref[wv][t] = pref;
        }
        wave_lds_fence();
        // this lane's kBkChunk / 64 items share one word of the marks
        const uint32_t it0 = (uint32_t)t * (kBkChunk / 64);
        const uint32_t mword = s_gstart[wv][it0 >> 5];
        const uint32_t mbase = carry + s_gpref[wv][it0 >> 5] - 1u;
        uint32_t wsum = 0, nzc = 0;
        uint32_t wid[kBkChunk / 64], ikey[kBkChunk / 64], ig[kBkChunk / 64];
#pragma unroll
        for (int j = 0; j < kBkChunk / 64; ++j) {
            const uint32_t it = it0 + j;
            wid[j] = 0;
            ikey[j] = 0;
            ig[j] = 0;
            if (it < ci) {
                const uint32_t r = c0 + it;
                // the last Gaussian with rows whose first row <= r
                const uint32_t upto = (2u << (it & 31)) - 1u;    // marks at or before it
                const int lo = s_nzg[wv][mbase + (uint32_t)__popc(mword & upto)];
                const int dr = (int)(r - s_rows[wv][lo]);
                int cl, ch;
                support_row(unpack_support(s_sup[wv][lo], r2), (int)s_ty0[wv][lo] + dr, th_,
                            inv_tw, cl, ch);
                wid[j] = ch >= cl ? (uint32_t)(ch - cl + 1) : 0u;
                ikey[j] = s_key0[wv][lo] + (uint32_t)dr * (uint32_t)s_tx[wv][lo] + (uint32_t)cl;
                ig[j] = (uint32_t)lo;
                wsum += wid[j];
                nzc += wid[j] != 0u;
            }
        }
        uint32_t cnt, nnz;
        uint32_t ex = wave_excl_scan(wsum, cnt);
        uint32_t rk = wave_excl_scan(nzc, nnz);
        // wave-uniform: the round loop and its branches run on the scalar unit
        cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)cnt);
        nnz = (uint32_t)__builtin_amdgcn_readfirstlane((int)nnz);
        // Rows with pairs, compacted in order (rank rk): their first key,
        // Gaussian and first pair.  A chunk of at most kStartBits pairs also
        // marks each such row's first pair in a bitmap, so a pair's row is
        // the number of marks at or before it, minus one; longer chunks
        // binary-search the first pairs.
        const bool use_bits = cnt <= (uint32_t)kStartBits;
        const uint32_t nwords = 2 * ((cnt + 63) / 64);
        if (use_bits)
            for (uint32_t q = t; q < nwords; q += 64) s_start[wv][q] = 0u;
        wave_lds_fence();
#pragma unroll
        for (int j = 0; j < kBkChunk / 64; ++j) {
            if (wid[j] != 0u) {
                s_item[wv][rk] = make_uint2(ex, ikey[j] | (ig[j] << 16));
                if (use_bits) atomicOr(&s_start[wv][ex >> 5], 1u << (ex & 31));
                ++rk;
            }
            ex += wid[j];
        }
        // the slots past the chunk's last row hold cnt (> every pair index),
        // so the pair search below needs no bound
        for (uint32_t it = nnz + t; it <= (uint32_t)kBkChunk; it += 64) s_item[wv][it].x = cnt;
        if (c0 == 0) fetch_parts();
        wave_lds_fence();
        // rounds of 64 consecutive pairs of the chunk, one per lane
        uint32_t seen = 0;                 // row marks before the round
        for (uint32_t r0 = 0; r0 < cnt; r0 += 64) {
            const uint32_t i = r0 + (uint32_t)t;
            const bool valid = i < cnt;
            int lo = 0;                        // row of pair i (compacted)
            if (use_bits) {
                // marks of pairs r0 .. r0 + 63 (words past the chunk are zero)
                const uint64_t m = *reinterpret_cast<const uint64_t *>(&s_start[wv][r0 >> 5]);
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                lo = (int)(seen + below + (uint32_t)((m >> t) & 1ull)) - 1;
                seen += (uint32_t)__popcll(m);
            } else {
#pragma unroll
                for (int step = kBkChunk / 2; step >= 1; step >>= 1)
                    if (s_item[wv][lo + step].x <= i) lo += step;
            }
            // lo is a row of the chunk for every lane (lanes past the last
            // pair too), so the reads need no guard; those lanes' values are
            // not used
            const uint2 item = s_item[wv][lo];
            const uint32_t key = (item.y & 0xffffu) + (i - item.x);
            const uint32_t gl = item.y >> 16;
            const uint32_t hr = valid ? (key >> 8) - hl : 0u;
            const uint64_t peers = digit_peers(valid, hr, nbits);
            // the wave's LDS accesses execute in order: this round reads the
            // counts the previous round's group leaders wrote
            const uint2 pe = s_pe[wv][hr];
            const uint32_t before = pe.x;
            const uint32_t pos = before + (uint32_t)__popcll(peers & lt);
            if (valid && (peers & lt) == 0) s_pe[wv][hr].x = before + (uint32_t)__popcll(peers);
            if (valid && pos < pe.y)
                packed[pos] = ((key & 255u) << 24) | (uint32_t)(g0 + gl);
        }
        wave_lds_fence();
    }
    // every bucket of the block filled exactly
    for (uint32_t i = t; i <= span; i += 64)
        if (s_pe[wv][i].x != s_pe[wv][i].y)
            atomicOr((unsigned long long *)&status[1],
                     (unsigned long long)(Status::kOverflow | Status::kListMismatch));
}

// Segment of radix block b (b < P[nbk]): the last s with P[s] <= b (buckets
// without pairs own no block).
__device__ inline int seg_find(const uint32_t *P, int nbk, uint32_t b) {
    int lo = 0, hi = nbk - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// A radix block of the in-bucket pass: its segment, its first element and
// count, and the index of its digit-0 count in hseg.
struct SegBlock {
    uint32_t pos0, cnt;
    int64_t h0;        // hseg index of (segment, digit 0, this block)
    uint32_t nbs;      // blocks of the segment (stride between digits)
    bool real;
};

__device__ inline SegBlock seg_block(const uint32_t *s_S, const uint32_t *s_P, int nbk, uint32_t b) {
    SegBlock r;
    r.real = b < s_P[nbk];
    if (!r.real) {
        r.pos0 = r.cnt = r.nbs = 0;
        r.h0 = (int64_t)b * kRadix;
        return r;
    }
    const int s = seg_find(s_P, nbk, b);
    const uint32_t j = b - s_P[s];
    r.nbs = s_P[s + 1] - s_P[s];
    r.pos0 = s_S[s] + j * (uint32_t)kTile;
    r.cnt = min((uint32_t)kTile, s_S[s + 1] - r.pos0);
    r.h0 = (int64_t)kRadix * s_P[s] + j;
    return r;
}

__device__ inline void load_seg(const uint32_t *seg, int nbk, uint32_t *s_S, uint32_t *s_P) {
    for (int i = threadIdx.x; i <= nbk; i += blockDim.x) {
        s_S[i] = seg[i];
        s_P[i] = seg[nbk + 1 + i];
    }
}

// Digit counts of one radix block of the in-bucket pass (low key byte).
__global__ __launch_bounds__(256) void k_seg_hist(const uint32_t *__restrict__ packed,
                                                  const uint32_t *__restrict__ seg, int nbk,
                                                  const int64_t *status,
                                                  uint32_t *__restrict__ hseg) {
    __shared__ uint32_t h[kRadix];
    __shared__ uint32_t s_S[kRadix + 1], s_P[kRadix + 1];
    if (status[1] & Status::kOverflow) return;
    const int t = threadIdx.x;
    load_seg(seg, nbk, s_S, s_P);
    h[t] = 0u;
    __syncthreads();
    const SegBlock sb = seg_block(s_S, s_P, nbk, blockIdx.x);
    // consecutive pairs of a bucket are mostly consecutive keys: no runs of
    // equal digits to add at once, so one LDS atomic per pair
    for (uint32_t i = t; i < sb.cnt; i += kBlk) atomicAdd(&h[packed[sb.pos0 + i] >> 24], 1u);
    __syncthreads();
    hseg[sb.h0 + (int64_t)t * (sb.real ? sb.nbs : 1u)] = h[t];
}

// The in-bucket pass's scatter: ranks as in k_radix_scatter (digit = key
// byte), positions from the scanned hseg, and only the Gaussian leaves.
__global__ __launch_bounds__(256) void k_seg_scatter(const uint32_t *__restrict__ packed,
                                                     const uint32_t *__restrict__ seg, int nbk,
                                                     const uint32_t *__restrict__ hseg,
                                                     const int64_t *status,
                                                     uint32_t *__restrict__ ids) {
    __shared__ uint32_t s_keys[kTile];
    __shared__ uint32_t s_goff[kRadix];          // output position of a digit's slot 0
    __shared__ uint32_t s_wrun[kBlk / 64][kRadix];
    __shared__ uint64_t s_wave[kBlk / 64];
    __shared__ uint32_t s_S[kRadix + 1], s_P[kRadix + 1];
    if (status[1] & Status::kOverflow) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    load_seg(seg, nbk, s_S, s_P);
#pragma unroll
    for (int q = 0; q < kBlk / 64; ++q) s_wrun[q][tid] = 0;
    __syncthreads();
    const SegBlock sb = seg_block(s_S, s_P, nbk, blockIdx.x);
    if (!sb.real) return;                      // uniform over the block
    const int cnt = (int)sb.cnt;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t *run = s_wrun[w];
    uint32_t key[kItems], rank[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int li = w * kWaveItems + j * 64 + lane;
        key[j] = li < cnt ? packed[sb.pos0 + li] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int li = w * kWaveItems + j * 64 + lane;
        const bool valid = li < cnt;
        const uint32_t d = key[j] >> 24;
        const uint64_t peers = digit_peers(valid, d, 8);
        const uint32_t before = valid ? run[d] : 0u;
        rank[j] = before + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) run[d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        // digit tid: the block's count before it (prefix), then each wave's
        // first slot in the block's order and the output position of slot 0
        uint32_t c[kBlk / 64], tt = 0;
#pragma unroll
        for (int q = 0; q < kBlk / 64; ++q) {
            c[q] = s_wrun[q][tid];
            tt += c[q];
        }
        uint64_t tot;
        const uint32_t prefix = (uint32_t)block_excl_scan(tt, s_wave, tot);
        uint32_t r = prefix;
#pragma unroll
        for (int q = 0; q < kBlk / 64; ++q) {
            s_wrun[q][tid] = r;
            r += c[q];
        }
        s_goff[tid] = hseg[sb.h0 + (int64_t)tid * sb.nbs] - prefix;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int li = w * kWaveItems + j * 64 + lane;
        if (li < cnt) s_keys[run[key[j] >> 24] + rank[j]] = key[j];
    }
    __syncthreads();
    for (int i = tid; i < cnt; i += kBlk) {
        const uint32_t k = s_keys[i];
        ids[s_goff[k >> 24] + (uint32_t)i] = k & 0xffffffu;
    }
}

// Ranges of the bucketed path: tile t = 256 s + d starts where (segment s,
// digit d, first block) does in the scanned hseg and ends where digit d + 1
// starts (the segment's end for d = 255); an empty tile gets (0, 0).
__global__ void k_seg_ranges(const uint32_t *__restrict__ hseg, const uint32_t *__restrict__ seg,
                             int nbk, uint32_t n_tiles, const int64_t *status,
                             uint32_t *__restrict__ ranges) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    uint32_t a = 0, e = 0;
    if (!(status[1] & Status::kOverflow)) {
        const uint32_t s = t >> 8, d = t & 255u;
        const uint32_t P = seg[nbk + 1 + s], nbs = seg[nbk + 2 + s] - P;
        if (nbs == 0) {
            a = e = seg[s];
        } else {
            const int64_t h0 = (int64_t)kRadix * P;
            a = hseg[h0 + (int64_t)d * nbs];
            e = d < 255u ? hseg[h0 + (int64_t)(d + 1) * nbs] : seg[s + 1];
        }
        if (a == e) a = e = 0u;      // an empty tile: (0, 0), as the radix path leaves it
    }
    ranges[2 * (int64_t)t] = a;
    ranges[2 * (int64_t)t + 1] = e;
}

}  // namespace

int64_t sort_hist_blocks(int64_t n) { return cdiv(n > 0 ? n : 1, kTile); }
int64_t sort_part_elems(int64_t n) {
    const int64_t a = cdiv(n > 0 ? n : 1, kTile);
    const int64_t b = cdiv(kRadix * sort_hist_blocks(n), kTile);
    return a > b ? a : b;
}

hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint64_t *part,
                              int64_t *total_out, int64_t *status, hipStream_t s) {
    // cap = 2^62: the overflow test of the pair count never fires here
    return scan_u32(in, out, n, part, total_out, int64_t(1) << 62, status, s);
}

hipError_t sort_pairs_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2,
                          int64_t n, int key_bits, uint32_t *hist, uint64_t *part, int64_t *status,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (key_bits < 16 || key_bits > 32 || key_bits % 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(64), 0, s, status, n);
    const int64_t hb = sort_hist_blocks(n);
    const int passes = (key_bits + 7) / 8;
    uint32_t *kin = keys, *vin = vals, *kout = keys2, *vout = vals2;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const int nbits = key_bits - shift < 8 ? key_bits - shift : 8;
        hipLaunchKernelGGL(k_radix_hist, dim3(hb), dim3(kBlk), 0, s, kin, (const int64_t *)status,
                           shift, nbits, hist, hb);
        hipError_t e = scan_u32(hist, hist, kRadix * hb, part, nullptr, 0, status, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(hb), dim3(kBlk), 0, s, kin, vin, kout, vout,
                           (const uint32_t *)hist, hb, (const int64_t *)status, shift, nbits);
        uint32_t *tk = kin, *tv = vin;
        kin = kout;
        vin = vout;
        kout = tk;
        vout = tv;
    }
    return hipGetLastError();
}

BinLayout bin_layout(const bz_opts &o, int64_t n_gauss, int64_t cap) {
    BinLayout L;
    L.n_tiles = num_tiles(o);
    L.fused = bin_fused(o, n_gauss, L.n_tiles);
    if (L.fused) {
        const int64_t ng = n_gauss > 0 ? n_gauss : 1, cp = cap > 0 ? cap : 1;
        L.n_buckets = cdiv(L.n_tiles > 0 ? L.n_tiles : 1, 256);
        L.n_eblk = cdiv(ng, kEmitBlock);
        L.seg_blocks = cdiv(cp, kTile) + L.n_buckets;
        int64_t off = 0;
        L.off_counters = off;             // first, so that its place needs no sizes
        off = align256(off + 4 * 4);
        L.off_rects = off;
        off = align256(off + 8 * ng);
        L.off_bucket = off;
        off = align256(off + 4 * L.n_buckets * L.n_eblk);
        L.off_packed = off;
        off = align256(off + 4 * cp);
        L.off_seg = off;
        off = align256(off + 4 * 2 * (L.n_buckets + 1));
        L.off_hseg = off;
        off = align256(off + 4 * kRadix * L.seg_blocks);
        L.off_part = off;
        const int64_t pa = cdiv(L.n_buckets * L.n_eblk, kTile), pb = cdiv(kRadix * L.seg_blocks, kTile);
        off = align256(off + 8 * (pa > pb ? pa : pb));
        L.total = off;
        return L;
    }
    int bits = 0;
    while ((int64_t(1) << bits) <= L.n_tiles) ++bits;   // keys 0 .. n_tiles
    if (bits == 0) bits = 1;
    L.key_bits = bits;
    L.passes = (bits + 7) / 8;
    L.hist_blocks = cdiv(cap > 0 ? cap : 1, kTile);
    int64_t off = 0;
    L.off_counters = off;                 // first, so that its place needs no sizes
    off = align256(off + 4 * 4);
    L.off_counts = off;
    off = align256(off + 4 * (n_gauss > 0 ? n_gauss : 1));
    L.off_rects = off;
    off = align256(off + 8 * (n_gauss > 0 ? n_gauss : 1));
    L.off_keys_a = off;
    off = align256(off + 4 * (cap > 0 ? cap : 1));
    L.off_keys_b = off;
    off = align256(off + 4 * (cap > 0 ? cap : 1));
    L.off_vals_b = off;
    off = align256(off + 4 * (cap > 0 ? cap : 1));
    L.off_hist = off;
    off = align256(off + 4 * kRadix * L.hist_blocks);
    L.off_part = off;
    int64_t nparts = cdiv(n_gauss > 0 ? n_gauss : 1, kTile);
    int64_t nparts_h = cdiv(kRadix * L.hist_blocks, kTile);
    off = align256(off + 8 * (nparts > nparts_h ? nparts : nparts_h));
    L.total = off;
    return L;
}

namespace {

// The binning workspace's arrays (the path's own; the others are null).
struct BinBufs {
    BinLayout L;
    uint32_t *counts;
    ushort4 *rects;
    uint32_t *keys_a, *keys_b, *vals_b, *hist;
    uint64_t *part;
    uint32_t *bucket, *packed, *seg, *hseg;
};

BinBufs bin_bufs(const bz_opts &o, int64_t n, const bz_bins &b) {
    BinBufs u = {};
    u.L = bin_layout(o, n, b.cap_pairs);
    char *ws = (char *)b.workspace;
    if (u.L.fused) {
        u.rects = (ushort4 *)(ws + u.L.off_rects);
        u.bucket = (uint32_t *)(ws + u.L.off_bucket);
        u.packed = (uint32_t *)(ws + u.L.off_packed);
        u.seg = (uint32_t *)(ws + u.L.off_seg);
        u.hseg = (uint32_t *)(ws + u.L.off_hseg);
        u.part = (uint64_t *)(ws + u.L.off_part);
        return u;
    }
    u.counts = (uint32_t *)(ws + u.L.off_counts);
    u.rects = (ushort4 *)(ws + u.L.off_rects);
    u.keys_a = (uint32_t *)(ws + u.L.off_keys_a);
    u.keys_b = (uint32_t *)(ws + u.L.off_keys_b);
    u.vals_b = (uint32_t *)(ws + u.L.off_vals_b);
    u.hist = (uint32_t *)(ws + u.L.off_hist);
    u.part = (uint64_t *)(ws + u.L.off_part);
    return u;
}

float support_two_p(const bz_opts &o) { return 2.0f * (-logf(o.g_min)); }

// Status and ranges cleared: before anything of the call writes a flag.  The
// bucketed path's counts start at zero (they are added to).
void bin_prepare(const BinBufs &u, const bz_bins &b, int64_t n, hipStream_t s) {
    if (u.L.fused && n > 0) {
        const int64_t nf = u.L.n_buckets * u.L.n_eblk, nt = (nf >> 2) > 3 ? (nf >> 2) : 3;
        hipLaunchKernelGGL(k_bucket_clear, dim3(cdiv(nt, 256)), dim3(256), 0, s, b.status,
                           u.bucket, nf);
        return;
    }
    const int64_t nr = 2 * u.L.n_tiles;
    hipLaunchKernelGGL(k_bin_clear, dim3(cdiv(nr > 2 ? nr : 2, 256)), dim3(256), 0, s, b.status,
                       b.ranges, nr);
}

// Bucketed path, after the counts per (bucket, emission block): positions,
// emission into the buckets, the in-bucket radix pass, ranges.
hipError_t bin_finish_fused(const float *rec, const BinBufs &u, int64_t n, const bz_opts &o,
                            const bz_bins &b, hipStream_t s) {
    const BinLayout &L = u.L;
    const int nbk = (int)L.n_buckets;
    const bz_canvas *cv = o.batch ? o.batch->canvas : nullptr;
    const int ncv = o.batch ? o.batch->n_canvas : 0;
    hipError_t e = scan_u32(u.bucket, u.bucket, L.n_buckets * L.n_eblk, u.part, b.status,
                            b.cap_pairs, b.status, s);
    if (e != hipSuccess) return e;
    // a smaller bucket table in LDS when it fits: more waves per CU
    hipLaunchKernelGGL(nbk <= 64 ? k_emit_bucketed<64> : k_emit_bucketed<256>,
                       dim3(8 * cdiv(L.n_eblk, 8 * kEmitWaves)), dim3(64 * kEmitWaves), 0, s,
                       (const float4 *)rec, (const ushort4 *)u.rects, n, o.width, o.height,
                       (int)tiles_x(o), 1.0f / o.tile_w, o.tile_h, support_two_p(o), cv, ncv,
                       (const uint32_t *)u.bucket, nbk, L.n_eblk, u.packed, u.seg, b.status);
    hipLaunchKernelGGL(k_seg_hist, dim3(L.seg_blocks), dim3(kBlk), 0, s,
                       (const uint32_t *)u.packed, (const uint32_t *)u.seg, nbk,
                       (const int64_t *)b.status, u.hseg);
    e = scan_u32(u.hseg, u.hseg, kRadix * L.seg_blocks, u.part, nullptr, 0, b.status, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_scatter, dim3(L.seg_blocks), dim3(kBlk), 0, s,
                       (const uint32_t *)u.packed, (const uint32_t *)u.seg, nbk,
                       (const uint32_t *)u.hseg, (const int64_t *)b.status, b.ids);
    hipLaunchKernelGGL(k_seg_ranges, dim3(cdiv(L.n_tiles, 256)), dim3(256), 0, s,
                       (const uint32_t *)u.hseg, (const uint32_t *)u.seg, nbk,
                       (uint32_t)L.n_tiles, (const int64_t *)b.status, b.ranges);
    return hipGetLastError();
}

// From the per-Gaussian tile counts and rectangles: offsets, pairs, sort, ranges.
hipError_t bin_finish(const float *rec, const BinBufs &u, int64_t n, const bz_opts &o,
                      const bz_bins &b, hipStream_t s) {
    const BinLayout &L = u.L;
    const int tx = (int)tiles_x(o);
    const bz_canvas *cv = o.batch ? o.batch->canvas : nullptr;
    const int ncv = o.batch ? o.batch->n_canvas : 0;
    hipError_t e = scan_u32(u.counts, u.counts, n, u.part, b.status, b.cap_pairs, b.status, s);
    if (e != hipSuccess) return e;
    // The final radix pass must land in (keys_a, ids).
    bool even = (L.passes % 2) == 0;
    uint32_t *k0 = even ? u.keys_a : u.keys_b, *v0 = even ? b.ids : u.vals_b;
    hipLaunchKernelGGL(k_emit, dim3(cdiv(n, kEmitG)), dim3(kEmitG), 0, s, (const float4 *)rec,
                       u.counts, u.rects, n, o.width, o.height, tx, 1.0f / o.tile_w, o.tile_h,
                       support_two_p(o), cv, ncv, (uint32_t)L.n_tiles, k0, v0,
                       (const int64_t *)b.status);
    uint32_t *kin = k0, *vin = v0;
    for (int p = 0; p < L.passes; ++p) {
        int shift = 8 * p;
        int nbits = L.key_bits - shift < 8 ? L.key_bits - shift : 8;
        uint32_t *kout = (kin == u.keys_a) ? u.keys_b : u.keys_a;
        uint32_t *vout = (vin == b.ids) ? u.vals_b : b.ids;
        hipLaunchKernelGGL(k_radix_hist, dim3(L.hist_blocks), dim3(kBlk), 0, s, kin,
                           (const int64_t *)b.status, shift, nbits, u.hist, L.hist_blocks);
        e = scan_u32(u.hist, u.hist, kRadix * L.hist_blocks, u.part, nullptr, 0, b.status, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(L.hist_blocks), dim3(kBlk), 0, s, kin, vin, kout,
                           vout, (const uint32_t *)u.hist, L.hist_blocks,
                           (const int64_t *)b.status, shift, nbits);
        kin = kout;
        vin = vout;
    }
    hipLaunchKernelGGL(k_ranges, dim3(cdiv(cdiv(b.cap_pairs, kRangeItems), 256)), dim3(256), 0, s,
                       kin, (const int64_t *)b.status, b.cap_pairs, (uint32_t)L.n_tiles, b.ranges);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bin(const float *rec_f, int64_t n, const bz_opts &o, const bz_bins &b,
                      hipStream_t s) {
    const BinBufs u = bin_bufs(o, n, b);
    bin_prepare(u, b, n, s);
    if (n == 0) return hipGetLastError();
    const bz_canvas *cv = o.batch ? o.batch->canvas : nullptr;
    const int ncv = o.batch ? o.batch->n_canvas : 0;
    hipLaunchKernelGGL(k_count, dim3(cdiv(n, 256)), dim3(256), 0, s, (const float4 *)rec_f, n,
                       o.width, o.height, (int)tiles_x(o), 1.0f / o.tile_w, 1.0f / o.tile_h,
                       o.tile_h, support_two_p(o), cv, ncv, u.counts, u.rects, u.bucket,
                       (int)u.L.n_buckets, u.L.n_eblk, b.status);
    return u.L.fused ? bin_finish_fused(rec_f, u, n, o, b, s) : bin_finish(rec_f, u, n, o, b, s);
}

hipError_t launch_sample_bin(const bz_curves &c, const bz_opts &o, float *rec, const bz_bins &b,
                             hipStream_t s) {
    const int64_t n = c.n_gauss;
    const BinBufs u = bin_bufs(o, n, b);
    bin_prepare(u, b, n, s);
    if (n == 0) return hipGetLastError();
    const BinCount bc = {u.counts, u.rects, b.status, 1.0f / o.tile_w, 1.0f / o.tile_h, o.tile_h,
                         support_two_p(o), u.bucket, u.L.n_eblk, (int)u.L.n_buckets,
                         (int)tiles_x(o)};
    hipError_t e = launch_sample(c, o, rec, &bc, s);
    if (e != hipSuccess) return e;
    return u.L.fused ? bin_finish_fused(rec, u, n, o, b, s) : bin_finish(rec, u, n, o, b, s);
}

}  // namespace bz
