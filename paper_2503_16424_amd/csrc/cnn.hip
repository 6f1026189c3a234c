// cnn.hip -- BF16 implicit-GEMM convolutions on the gfx950 matrix cores.
//
// All three passes of a convolution are one GEMM C[m][n] = sum_k A[m][k] B[k][n]
// whose operands are gathered on the fly (no im2col buffer):
//
//   forward      m = output pixel, n = output channel, k = (dy, dx, in channel)
//                A = shifted input pixels, B = filters
//   input grad   m = input pixel,  n = in channel,     k = (dy, dx, out channel)
//                A = the output gradients that pixel fed, B = filters; one GEMM
//                per parity class of the input pixels modulo the stride, over
//                the taps that reach that class only
//   filter grad  m = out channel,  n = (dy, dx, in channel), k = output pixel
//                A = output gradients, B = shifted input pixels
//
// A workgroup (4 waves) computes a 64 x 64 tile of C in steps of 32 along k:
// the 256 threads gather the A and B slices (8 consecutive k per thread) into
// LDS with k contiguous, then each wave runs 2 x 2 v_mfma_f32_16x16x32_bf16 on
// its 32 x 32 quarter.  For that instruction lane l supplies row (l mod 16)
// of A and column (l mod 16) of B, each with the 8 k values 8 (l / 16) ..
// 8 (l / 16) + 7, and receives rows 4 (l / 16) .. 4 (l / 16) + 3 of column
// (l mod 16) of the 16 x 16 result.  The filter gradient splits its long k
// (all output pixels) over workgroups and adds the partial tiles with float
// atomics.
#include "bz_internal.h"
#include "../../include/bz_cnn.h"

namespace bz {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kLdsK = kBK + 8;          // row pitch in bf16 (80 bytes) against bank conflicts
// Filter gradient: output pixels per workgroup.  256 by default; 128 when
// 256 would leave fewer than 512 workgroups (small late layers).  Measured on
// the 256-patch training step: 1024 rows per workgroup ran the first layer's
// 256 workgroups at one per CU (140 us), 128 rows made its 1,728 outputs
// take too many float atomics (141 us); 256 gives 100 us.
constexpr int kSplitRows = 256, kSplitRowsSmall = 128, kSplitMinGroups = 512;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline __bf16 bf_bits(uint16_t u) { return __builtin_bit_cast(__bf16, u); }
__device__ inline float bf_to_f(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }

// float -> bfloat16 bits, round to nearest even (finite inputs; NaN stays NaN)
__device__ inline uint16_t f_to_bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct Shape {
    int n, h, w, c, k, r, s, p, ho, wo;
};

// Input pixel read by output pixel m through filter tap `tap`, or -1 (padding).
__device__ inline int in_pixel(const Shape &S, int m, int tap) {
    const int hw = (int)S.ho * S.wo;
    const int b = m / hw;
    const int rem = (int)(m - b * hw);
    const int oy = rem / S.wo, ox = rem - (rem / S.wo) * S.wo;
    const int ky = tap / S.r, kx = tap - (tap / S.r) * S.r;
    const int iy = oy * S.s - S.p + ky, ix = ox * S.s - S.p + kx;
    if (iy < 0 || ix < 0 || iy >= S.h || ix >= S.w) return -1;
    return (b * S.h + iy) * S.w + ix;
}

// Output pixel that input pixel m feeds through tap `tap`, or -1.
__device__ inline int out_pixel(const Shape &S, int m, int tap) {
    const int hw = (int)S.h * S.w;
    const int b = m / hw;
    const int rem = (int)(m - b * hw);
    const int iy = rem / S.w, ix = rem - (rem / S.w) * S.w;
    const int ky = tap / S.r, kx = tap - (tap / S.r) * S.r;
    const int ty = iy + S.p - ky, tx = ix + S.p - kx;
    if (ty < 0 || tx < 0 || ty % S.s || tx % S.s) return -1;
    const int oy = ty / S.s, ox = tx / S.s;
    if (oy >= S.ho || ox >= S.wo) return -1;
    return (b * S.ho + oy) * S.wo + ox;
}

enum Mode { kFwd = 0, kBwdData = 1, kBwdWeight = 2 };

struct GemmArgs {
    Shape S;
    int M, N, K;          // GEMM sizes
    const uint16_t *x;        // input activations (bf16)
    const uint16_t *w;        // filters (bf16)
    const float *dy;          // output gradients (f32)
    const float *bias;
    const uint16_t *mask;     // bwd data: zero where the layer input is <= 0
    int relu;
    float *out_f;             // fwd y, bwd-data dx, bwd-weight dw
    uint16_t *out_b;          // fwd y in bf16
    int k_chunk;          // bwd weight: k range per workgroup
    // bwd data, one parity class: rows are the input pixels (iy, ix) with
    // iy = cy, ix = cx (mod stride), hq x wq of them per image; only taps
    // ky = ky0, kx = kx0 (mod stride) reach them, nkx of them along x
    int cy, cx, hq, wq, ky0, kx0, nkx;
};

// Input pixel of class row m (input gradient).
__device__ inline int cls_pixel(const GemmArgs &g, int m) {
    if (g.S.s == 1) return m;                   // one class: every pixel
    const int hw = (int)g.hq * g.wq;
    const int b = m / hw;
    const int rem = (int)(m - b * hw);
    const int qy = rem / g.wq, qx = rem - (rem / g.wq) * g.wq;
    return (b * g.S.h + qy * g.S.s + g.cy) * g.S.w + qx * g.S.s + g.cx;
}

// Input gradient: the parity class of workgroup row z (cy = z / stride,
// cx = z mod stride), its GEMM rows M and its k extent K.
__device__ inline void set_class(GemmArgs &g, int z) {
    const Shape &S = g.S;
    const int st = S.s;
    g.cy = z / st;
    g.cx = z - (z / st) * st;
    g.hq = g.cy < S.h ? (S.h - g.cy + st - 1) / st : 0;
    g.wq = g.cx < S.w ? (S.w - g.cx + st - 1) / st : 0;
    g.ky0 = (g.cy + S.p) % st;
    g.kx0 = (g.cx + S.p) % st;
    const int nky = g.ky0 < S.r ? (S.r - g.ky0 + st - 1) / st : 0;
    const int nkx = g.kx0 < S.r ? (S.r - g.kx0 + st - 1) / st : 0;
    g.nkx = nkx > 0 ? nkx : 1;                  // no taps: K = 0, the class gets zeros
    g.M = (int)S.n * g.hq * g.wq;
    g.K = (int)nky * nkx * S.k;
}

// Filter tap of the class's j-th (ky, kx) pair (input gradient).
__device__ inline int cls_tap(const GemmArgs &g, int j) {
    if (g.S.s == 1) return j;                   // one class: every tap
    const int a = j / g.nkx, b = j - (j / g.nkx) * g.nkx;
    return (g.ky0 + a * g.S.s) * g.S.r + g.kx0 + b * g.S.s;
}

// Operand slices travel in two halves so that one k step's loads are in
// flight while the previous step multiplies: fetch_* issues the global loads
// into 8 raw 32-bit registers per thread, put_tiles converts them to BF16 and
// writes LDS after the next barrier.  Raw forms: BF16 vector (4 words of 2
// elements), FP32 (8 float bit patterns, rounded at put), BF16 element (8
// zero-extended halves).
enum RawKind { kRawBf16Vec = 0, kRawF32 = 1, kRawBf16 = 2 };

__device__ inline void raw_to_bf16(int kind, const uint32_t (&r)[8], uint16_t (&v)[8]) {
    if (kind == kRawBf16Vec) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = (uint16_t)r[i];
            v[2 * i + 1] = (uint16_t)(r[i] >> 16);
        }
    } else if (kind == kRawF32) {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = f_to_bf(__uint_as_float(r[j]));
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (uint16_t)r[j];
    }
}

// A[m][k .. k+7] and B[k .. k+7][n] for each mode, element by element (zeros
// outside the GEMM); FP32 output gradients stay FP32 (raw) until put.
template <int MODE>
__device__ inline void gather_a(const GemmArgs &g, int m, int k0, int kend,
                                uint32_t (&v)[8]) {
    const Shape &S = g.S;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = k0 + j;
        uint32_t u = 0;
        if (m < g.M && k < kend) {
            if (MODE == kFwd) {
                const int tap = (int)(k / S.c), ci = (int)(k - (int)tap * S.c);
                const int px = in_pixel(S, m, tap);
                if (px >= 0) u = g.x[px * S.c + ci];
            } else if (MODE == kBwdData) {
                const int j = (int)(k / S.k), co = (int)(k - (int)j * S.k);
                const int px = out_pixel(S, cls_pixel(g, m), cls_tap(g, j));
                if (px >= 0) u = __float_as_uint(g.dy[px * S.k + co]);
            } else {   // m = out channel, k = output pixel
                u = __float_as_uint(g.dy[k * S.k + m]);
            }
        }
        v[j] = u;
    }
}

template <int MODE>
__device__ inline void gather_b(const GemmArgs &g, int n, int k0, int kend,
                                uint32_t (&v)[8]) {
    const Shape &S = g.S;
    const int kf = (int)S.r * S.r * S.c;     // filter length per output channel
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = k0 + j;
        uint32_t u = 0;
        if (n < g.N && k < kend) {
            if (MODE == kFwd) {
                u = g.w[n * kf + k];
            } else if (MODE == kBwdData) {        // n = in channel, k = (tap, out channel)
                const int j = (int)(k / S.k), co = (int)(k - (int)j * S.k);
                u = g.w[(int)co * kf + (int)cls_tap(g, j) * S.c + n];
            } else {                              // n = (tap, in channel), k = output pixel
                const int tap = (int)(n / S.c), ci = (int)(n - (int)tap * S.c);
                const int px = in_pixel(S, k, tap);
                if (px >= 0) u = g.x[px * S.c + ci];
            }
        }
        v[j] = u;
    }
}

// Filter gradient, B without vector loads (input channels not a multiple of
// 8): B[k .. k+7][n] = the input channel of n at the pixel that output pixels
// k .. k+7 read through the tap of n.  The output pixels are consecutive, so
// the first one's (image, row, column) is divided out once and the others
// follow by stepping along the row (gather_b's element path divides for each).
__device__ inline void gather_b_wgrad(const GemmArgs &g, int n, int k0, int kend,
                                      uint32_t (&v)[8]) {
    const Shape &S = g.S;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = 0;
    if (n >= g.N || k0 >= kend) return;
    const int tap = (int)(n / S.c), ci = (int)(n - (int)tap * S.c);
    const int ky = tap / S.r, kx = tap - (tap / S.r) * S.r;
    const int hw = (int)S.ho * S.wo;
    int b = k0 / hw;
    const int rem = (int)(k0 - b * hw);
    int oy = rem / S.wo, ox = rem - (rem / S.wo) * S.wo;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (k0 + j < kend) {
            const int iy = oy * S.s - S.p + ky, ix = ox * S.s - S.p + kx;
            if (iy >= 0 && ix >= 0 && iy < S.h && ix < S.w)
                v[j] = g.x[((b * S.h + iy) * S.w + ix) * S.c + ci];
        }
        if (++ox == S.wo) {
            ox = 0;
            if (++oy == S.ho) {
                oy = 0;
                ++b;
            }
        }
    }
}

// 8 bf16 from a 16-byte aligned address (4 raw words), or zeros.
__device__ inline void fetch8_bf16(const uint16_t *p, bool ok, uint32_t (&r)[8]) {
    uint4 q = make_uint4(0, 0, 0, 0);
    if (ok) q = *reinterpret_cast<const uint4 *>(p);
    r[0] = q.x; r[1] = q.y; r[2] = q.z; r[3] = q.w;
    r[4] = r[5] = r[6] = r[7] = 0;
}

// 8 floats from a 32-byte aligned address (raw bits), or zeros.
__device__ inline void fetch8_f32(const float *p, bool ok, uint32_t (&r)[8]) {
    uint4 a = make_uint4(0, 0, 0, 0), b = a;
    if (ok) {
        a = reinterpret_cast<const uint4 *>(p)[0];
        b = reinterpret_cast<const uint4 *>(p)[1];
    }
    r[0] = a.x; r[1] = a.y; r[2] = a.z; r[3] = a.w;
    r[4] = b.x; r[5] = b.y; r[6] = b.z; r[7] = b.w;
}

// How each operand of a mode moves.  VA / VB: the operand's contiguous
// dimension holds whole groups of 8, so a thread moves 8 neighbours with one
// vector load: along k for operands stored k-contiguous (forward input and
// filters, input-gradient output gradients), along m or n otherwise (written
// transposed, "mn-major").  Else the element gather, k-major.
template <int MODE, bool VA>
struct OpA {
    static constexpr bool kMn = MODE == kBwdWeight && VA;
    static constexpr int kKind = (MODE == kFwd) ? (VA ? kRawBf16Vec : kRawBf16) : kRawF32;
};
template <int MODE, bool VB>
struct OpB {
    static constexpr bool kMn = (MODE == kBwdData || MODE == kBwdWeight) && VB;
    static constexpr int kKind = VB ? kRawBf16Vec : kRawBf16;
};

// Global loads of one k step's slices into registers.
template <int MODE, bool VA, bool VB>
__device__ inline void fetch_tiles(const GemmArgs &g, int m0, int n0, int k0,
                                   int kend, uint32_t (&ra)[8], uint32_t (&rb)[8]) {
    const Shape &S = g.S;
    const int t = threadIdx.x;
    const int lrow = t >> 2, lk = (t & 3) * 8;          // k-major slot: row, 8 k
    const int tk = t >> 3, tc = (t & 7) * 8;            // mn-major slot: k, 8 rows
    const int kf = (int)S.r * S.r * S.c;
    // ---- A ----
    if (MODE == kFwd && VA) {
        const int m = m0 + lrow, k = k0 + lk;
        const int tap = (int)(k / S.c), ci = (int)(k - (int)tap * S.c);
        const int px = (m < g.M && k < kend) ? in_pixel(S, m, tap) : -1;
        fetch8_bf16(g.x + (px >= 0 ? px * S.c + ci : 0), px >= 0, ra);
    } else if (MODE == kBwdData && VA) {
        const int m = m0 + lrow, k = k0 + lk;
        const int j = (int)(k / S.k), co = (int)(k - (int)j * S.k);
        const int px =
            (m < g.M && k < kend) ? out_pixel(S, cls_pixel(g, m), cls_tap(g, j)) : -1;
        fetch8_f32(g.dy + (px >= 0 ? px * S.k + co : 0), px >= 0, ra);
    } else if (MODE == kBwdWeight && VA) {              // A[co][pixel] = dy[pixel][co]
        const int k = k0 + tk, m = m0 + tc;
        const bool ok = k < kend && m < g.M;
        fetch8_f32(g.dy + (ok ? k * S.k + m : 0), ok, ra);
    } else {
        gather_a<MODE>(g, m0 + lrow, k0 + lk, kend, ra);
    }
    // ---- B ----
    if (MODE == kFwd && VB) {
        const int n = n0 + lrow, k = k0 + lk;
        const bool ok = n < g.N && k < kend;
        fetch8_bf16(g.w + (ok ? n * kf + k : 0), ok, rb);
    } else if (MODE == kBwdData && VB) {                // B[(tap, co)][ci] = w[co][tap][ci]
        const int k = k0 + tk, n = n0 + tc;
        const int j = (int)(k / S.k), co = (int)(k - (int)j * S.k);
        const bool ok = k < kend && n < g.N;
        fetch8_bf16(g.w + (ok ? (int)co * kf + (int)cls_tap(g, j) * S.c + n : 0), ok, rb);
    } else if (MODE == kBwdWeight && VB) {              // B[pixel][(tap, ci)] = x[shifted pixel][ci]
        const int k = k0 + tk, n = n0 + tc;
        const int tap = (int)(n / S.c), ci = (int)(n - (int)tap * S.c);
        const int px = (k < kend && n < g.N) ? in_pixel(S, k, tap) : -1;
        fetch8_bf16(g.x + (px >= 0 ? px * S.c + ci : 0), px >= 0, rb);
    } else if (MODE == kBwdWeight) {
        gather_b_wgrad(g, n0 + lrow, k0 + lk, kend, rb);
    } else {
        gather_b<MODE>(g, n0 + lrow, k0 + lk, kend, rb);
    }
}

// The fetched slices, rounded to BF16, into LDS (k contiguous in sA[m][.],
// sB[n][.]).
template <int MODE, bool VA, bool VB>
__device__ inline void put_tiles(const uint32_t (&ra)[8], const uint32_t (&rb)[8],
                                 uint16_t (*sA)[kLdsK], uint16_t (*sB)[kLdsK]) {
    const int t = threadIdx.x;
    const int lrow = t >> 2, lk = (t & 3) * 8;
    const int tk = t >> 3, tc = (t & 7) * 8;
    uint16_t v[8];
    raw_to_bf16(OpA<MODE, VA>::kKind, ra, v);
    if (OpA<MODE, VA>::kMn) {
#pragma unroll
        for (int j = 0; j < 8; ++j) sA[tc + j][tk] = v[j];
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) sA[lrow][lk + j] = v[j];
    }
    raw_to_bf16(OpB<MODE, VB>::kKind, rb, v);
    if (OpB<MODE, VB>::kMn) {
#pragma unroll
        for (int j = 0; j < 8; ++j) sB[tc + j][tk] = v[j];
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) sB[lrow][lk + j] = v[j];
    }
}

template <int MODE, bool VA, bool VB>
__global__ __launch_bounds__(256) void k_igemm(GemmArgs args) {
    __shared__ __align__(16) uint16_t sA[kBM][kLdsK];
    __shared__ __align__(16) uint16_t sB[kBN][kLdsK];
    GemmArgs g = args;
    if (MODE == kBwdData) set_class(g, (int)blockIdx.z);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = (int)blockIdx.x * kBM, n0 = (int)blockIdx.y * kBN;
    if (m0 >= g.M) return;                            // this class has fewer rows
    int kbeg = 0, kend = g.K;
    if (MODE == kBwdWeight) {
        kbeg = (int)blockIdx.z * g.k_chunk;
        kend = kbeg + g.k_chunk < g.K ? kbeg + g.k_chunk : g.K;
    }
    const int wm = wave >> 1, wn = wave & 1;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    uint32_t ra[8], rb[8];
    fetch_tiles<MODE, VA, VB>(g, m0, n0, kbeg, kend, ra, rb);
    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
        __syncthreads();                              // previous step's reads are done
        put_tiles<MODE, VA, VB>(ra, rb, sA, sB);
        __syncthreads();
        // the next step's loads fly while this one multiplies (past kend
        // they are masked off and give zeros)
        fetch_tiles<MODE, VA, VB>(g, m0, n0, k0 + kBK, kend, ra, rb);
        const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = bf_bits(sA[wm * 32 + i * 16 + r16][kq + j]);
#pragma unroll
            for (int jn = 0; jn < 2; ++jn) {
                bf16x8 b;
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = bf_bits(sB[wn * 32 + jn * 16 + r16][kq + j]);
                acc[i][jn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][jn], 0, 0, 0);
            }
        }
    }
    // epilogue: lane holds rows 4 (lane / 16) + e, column lane mod 16 of each block
    const int col = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jn = 0; jn < 2; ++jn)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm * 32 + i * 16 + rq + e;
                const int n = n0 + wn * 32 + jn * 16 + col;
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][jn][e];
                if (MODE == kFwd) {
                    if (g.bias) v += g.bias[n];
                    if (g.relu) v = fmaxf(v, 0.f);
                    if (g.out_f) g.out_f[m * g.N + n] = v;
                    if (g.out_b) g.out_b[m * g.N + n] = f_to_bf(v);
                } else if (MODE == kBwdData) {
                    const int px = cls_pixel(g, m);
                    if (g.mask && !(bf_to_f(g.mask[px * g.N + n]) > 0.f)) v = 0.f;
                    g.out_f[px * g.N + n] = v;
                } else {
                    atomicAdd(&g.out_f[m * g.N + n], v);
                }
            }
}

// Dispatch on which operands can move 8 at a time.
template <int MODE>
void launch_igemm(const GemmArgs &g, bool va, bool vb, dim3 grid, hipStream_t s) {
    if (va && vb)
        hipLaunchKernelGGL((k_igemm<MODE, true, true>), grid, dim3(256), 0, s, g);
    else if (va)
        hipLaunchKernelGGL((k_igemm<MODE, true, false>), grid, dim3(256), 0, s, g);
    else if (vb)
        hipLaunchKernelGGL((k_igemm<MODE, false, true>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_igemm<MODE, false, false>), grid, dim3(256), 0, s, g);
}

__global__ void k_fill0(float *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.f;
}

// db[o] = sum over output pixels of dy[.][o].  Workgroup (chunk, group): 64
// channels x 4 row phases over `chunk` rows, so each wave reads 64
// consecutive floats of a row; the phases meet in LDS and one atomic per
// channel adds the chunk's sum (db is cleared first).  The atomics of all
// workgroups meet on the few lines of db, so chunks are sized for about 256
// workgroups (bias_chunk): at 262,144 rows, chunks of 256 rows took 34 us,
// of 1024 rows 17 us.
inline int64_t bias_chunk(int64_t rows) {
    int64_t c = 256;
    while (c * 256 < rows) c *= 2;
    return c;
}

__global__ __launch_bounds__(256) void k_bias_grad(const float *__restrict__ dy, int64_t rows,
                                                   int64_t chunk, int k, float *db) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int o = blockIdx.y * 64 + tx;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = rows < r0 + chunk ? rows : r0 + chunk;
    // four independent sums keep four loads of each thread in flight
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (o < k) {
        int64_t r = r0 + ty;
        for (; r + 12 < r1; r += 16) {
            s0 += dy[r * k + o];
            s1 += dy[(r + 4) * k + o];
            s2 += dy[(r + 8) * k + o];
            s3 += dy[(r + 12) * k + o];
        }
        for (; r < r1; r += 4) s0 += dy[r * k + o];
    }
    const float s = (s0 + s1) + (s2 + s3);
    __shared__ float part[4][64];
    part[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && o < k) atomicAdd(&db[o], (part[0][tx] + part[1][tx]) + (part[2][tx] + part[3][tx]));
}

// The same for k a multiple of 4 up to 64 with 16-byte loads: lane l of a wave
// reads channels 4 (l % 16) .. +3 of row phase l / 16, so a wave covers four
// 256-byte rows per load and a workgroup 16 row phases.
__global__ __launch_bounds__(256) void k_bias_grad4(const float *__restrict__ dy, int64_t rows,
                                                    int64_t chunk, int k, float *db) {
    const int t = threadIdx.x, c4 = 4 * (t & 15), ph = t >> 4;     // 16 phases
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = rows < r0 + chunk ? rows : r0 + chunk;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
    if (c4 < k) {
        int64_t r = r0 + ph;
        for (; r + 16 < r1; r += 32) {
            const float4 u = *reinterpret_cast<const float4 *>(dy + r * k + c4);
            const float4 v = *reinterpret_cast<const float4 *>(dy + (r + 16) * k + c4);
            a.x += u.x; a.y += u.y; a.z += u.z; a.w += u.w;
            b.x += v.x; b.y += v.y; b.z += v.z; b.w += v.w;
        }
        for (; r < r1; r += 16) {
            const float4 u = *reinterpret_cast<const float4 *>(dy + r * k + c4);
            a.x += u.x; a.y += u.y; a.z += u.z; a.w += u.w;
        }
    }
    __shared__ float part[16][64];
    part[ph][c4] = a.x + b.x;
    part[ph][c4 + 1] = a.y + b.y;
    part[ph][c4 + 2] = a.z + b.z;
    part[ph][c4 + 3] = a.w + b.w;
    __syncthreads();
    if (t < k) {
        float s = 0.f;
#pragma unroll
        for (int p = 0; p < 16; ++p) s += part[p][t];
        atomicAdd(&db[t], s);
    }
}

// Filter and bias gradients of the first layer's shape: 3 x 3 filters, stride
// 1, padding 1, at most 3 input channels, 64 output channels, rows of 32
// pixels.  The generic split-K path spends most of its time in float atomics
// there (1,728 outputs per 256 output pixels, all meeting on 54 lines).
//
// One workgroup per image.  The image (h x 32 x C BF16) goes into LDS three
// times, shifted by kx = 0, 1, 2 columns and stored channel-planar with a zero
// border, so the 8 consecutive output pixels a lane feeds the matrix core
// through tap (ky, kx) and channel ci are one aligned 16-byte LDS read.  A
// wave takes whole output rows: a row of 32 pixels is one k step of
// C[co][(tap, ci)] += dy_row^T x shifted input row (4 x 2 blocks of
// v_mfma_f32_16x16x32_bf16), with the next row's dy loads in flight, and the
// bias gradient sums the same dy values in FP32.  The waves meet in LDS; one
// float atomic per output adds the image's share (dw and db are cleared
// first): 1,792 atomics per 1,024 pixels.
constexpr int kWg0Waves = 8;

inline bool wgrad_first_shape(const bz_conv &c) {
    return c.r == 3 && c.stride == 1 && c.pad == 1 && c.c >= 1 && c.c <= 3 && c.k == 64 &&
           c.w == 32 && c.h >= 1 && c.h <= 64;
}

inline size_t wgrad_first_lds(const bz_conv &c) {
    return (size_t)3 * (c.h + 2) * c.c * 32 * sizeof(uint16_t);
}

// dy of output row oy, pixels 8q .. 8q + 7, channels 16 mb + r (mb = 0..3)
__device__ inline void wgrad_first_row(const float *__restrict__ dy, int64_t row, int q, int r,
                                       float (&v)[4][8]) {
    const float *p = dy + (row * 32 + 8 * q) * 64 + r;
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) v[mb][j] = p[j * 64 + 16 * mb];
}

// Rows a wave has in flight at once (its rows are wave, wave + 8, ...).
constexpr int kWg0Rows = 4;

template <int C>
__global__ __launch_bounds__(64 * kWg0Waves) void k_wgrad_first(const float *__restrict__ dy,
                                                                const uint16_t *__restrict__ x,
                                                                int h, float *dw, float *db) {
    extern __shared__ __align__(16) uint16_t s_img[];    // [kx][h + 2][C][32]
    // each wave's result blocks, lane-major (the waves meet by plain sums:
    // LDS float atomics from eight waves took longer than the rows)
    __shared__ floatx4 s_part[kWg0Waves][8][64];
    __shared__ float s_bpart[kWg0Waves][64];
    constexpr int kThreads = 64 * kWg0Waves, kPitch = C * 32, kN = 9 * C;
    const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int rows = h + 2, plane = rows * kPitch;
    const int r = lane & 15, q = lane >> 4;
    // the first kWg0Rows rows of dy go in flight before the image is staged
    float v[kWg0Rows][4][8];
#pragma unroll
    for (int i = 0; i < kWg0Rows; ++i)
        if (wave + kWg0Waves * i < h) wgrad_first_row(dy, (int64_t)b * h + wave + kWg0Waves * i, q, r, v[i]);
    // clear the copies (their borders stay zero) and the sums
    for (int i = t; i < 3 * plane / 8; i += kThreads)
        reinterpret_cast<uint4 *>(s_img)[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    // s_img[kx][iy + 1][ci][ix + 1 - kx] = x[b][iy][ix][ci]: the image is
    // 64 h C bytes (a multiple of 16, as is its offset), 8 elements per load
    const uint4 *src = reinterpret_cast<const uint4 *>(x + (int64_t)b * h * 32 * C);
    for (int i = t; i < 4 * h * C; i += kThreads) {
        const uint4 u = src[i];
        const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = 8 * i + j;                        // (iy * 32 + ix) * C + ci
            const int px = e / C, ci = e - px * C;
            const int iy = px >> 5, ix = px & 31;
            const uint16_t u16 = (uint16_t)(w4[j >> 1] >> (16 * (j & 1)));
            uint16_t *d = s_img + (iy + 1) * kPitch + ci * 32 + ix + 1;
            if (ix < 31) d[0] = u16;                        // kx = 0
            d[plane - 1] = u16;                             // kx = 1
            if (ix > 0) d[2 * plane - 2] = u16;             // kx = 2
        }
    }
    __syncthreads();
    // B column n = 16 nb + r is (tap, ci) = (n / C, n mod C); lane q feeds
    // output pixels 8q .. 8q + 7 of the row.  Offset of row oy = 0, or -1
    // for the padding columns n >= 9C.
    int boff[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const int n = 16 * nb + r;
        boff[nb] = -1;
        if (n < kN) {
            const int tap = n / C, ci = n - tap * C, ky = tap / 3, kx = tap - 3 * ky;
            boff[nb] = (kx * rows + ky) * kPitch + ci * 32 + 8 * q;
        }
    }
    floatx4 acc[4][2];
    float bsum[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        bsum[mb] = 0.f;
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    for (int oy0 = wave; oy0 < h; oy0 += kWg0Waves * kWg0Rows) {
#pragma unroll
        for (int i = 0; i < kWg0Rows; ++i) {
            const int oy = oy0 + kWg0Waves * i;
            if (oy >= h) break;
            bf16x8 bv[2];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                bf16x8 z;
#pragma unroll
                for (int j = 0; j < 8; ++j) z[j] = bf_bits(0);
                bv[nb] = boff[nb] >= 0
                             ? *reinterpret_cast<const bf16x8 *>(s_img + boff[nb] + oy * kPitch)
                             : z;
            }
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                bf16x8 a;
                float sm = 0.f;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    a[j] = (__bf16)v[i][mb][j];             // v_cvt_pk_bf16_f32, nearest even
                    sm += v[i][mb][j];
                }
                bsum[mb] += sm;
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
                    acc[mb][nb] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv[nb], acc[mb][nb], 0, 0, 0);
            }
            // refill the slot with the row kWg0Rows ahead (images taller than
            // kWg0Waves * kWg0Rows rows)
            const int on = oy + kWg0Waves * kWg0Rows;
            if (on < h) wgrad_first_row(dy, (int64_t)b * h + on, q, r, v[i]);
        }
    }
    // lane holds C[16 mb + 4q + e][16 nb + r] in acc[mb][nb][e]
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) s_part[wave][2 * mb + nb][lane] = acc[mb][nb];
        float sm = bsum[mb];
        sm += __shfl_xor(sm, 16);
        sm += __shfl_xor(sm, 32);
        if (q == 0) s_bpart[wave][16 * mb + r] = sm;
    }
    __syncthreads();
    for (int o = t; o < 64 * kN + 64; o += kThreads) {
        float sum = 0.f;
        if (o < 64 * kN) {
            const int m = o / kN, n = o - m * kN;
            const int blk = 2 * (m >> 4) + (n >> 4), ln = 16 * ((m >> 2) & 3) + (n & 15), e = m & 3;
#pragma unroll
            for (int w = 0; w < kWg0Waves; ++w) sum += s_part[w][blk][ln][e];
            atomicAdd(&dw[o], sum);
        } else if (db) {
#pragma unroll
            for (int w = 0; w < kWg0Waves; ++w) sum += s_bpart[w][o - 64 * kN];
            atomicAdd(&db[o - 64 * kN], sum);
        }
    }
}

template <int C>
void launch_wgrad_first(const bz_conv &c, const float *dy, const uint16_t *x, float *dw,
                        float *db, hipStream_t s) {
    hipLaunchKernelGGL(k_wgrad_first<C>, dim3((unsigned)c.n), dim3(64 * kWg0Waves),
                       wgrad_first_lds(c), s, dy, x, c.h, dw, db);
}

__global__ void k_to_bf16(const float *src, uint16_t *dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = f_to_bf(src[i]);
}

__global__ void k_patches(const float *img, int W, int H, const int32_t *xy, int np, int side,
                          float fill, uint16_t *out) {
    const int64_t per = (int64_t)side * side * 3;
    const int64_t total = per * np;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        const int p = (int)(i / per);
        const int rem = (int)(i - (int64_t)p * per);
        const int ch = rem % 3, pix = rem / 3;
        const int x = xy[2 * p] + pix % side, y = xy[2 * p + 1] + pix / side;
        float v = fill;
        if (x >= 0 && y >= 0 && x < W && y < H) v = img[((int64_t)ch * H + y) * W + x];
        out[i] = f_to_bf(v);
    }
}

Shape shape_of(const bz_conv &c) {
    return Shape{c.n, c.h, c.w, c.c, c.k, c.r, c.stride, c.pad, c.ho, c.wo};
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_conv_fwd(const bz_conv &c, const uint16_t *x, const uint16_t *w,
                           const float *bias, int relu, float *y, uint16_t *yb, hipStream_t s) {
    GemmArgs g = {};
    g.S = shape_of(c);
    g.M = (int64_t)c.n * c.ho * c.wo;
    g.N = c.k;
    g.K = (int64_t)c.r * c.r * c.c;
    g.x = x;
    g.w = w;
    g.bias = bias;
    g.relu = relu;
    g.out_f = y;
    g.out_b = yb;
    dim3 grid((unsigned)cdiv(g.M, kBM), (unsigned)cdiv(g.N, kBN), 1);
    // A: 8 input channels per load (c % 8); B: 8 filter taps-channels per load (K % 8)
    launch_igemm<kFwd>(g, c.c % 8 == 0, g.K % 8 == 0 && c.c % 8 == 0, grid, s);
    return hipGetLastError();
}

hipError_t launch_conv_bwd_data(const bz_conv &c, const float *dy, const uint16_t *w,
                                const uint16_t *mask, float *dx, hipStream_t s) {
    // One GEMM per parity class of the input pixels (stride^2 of them, one
    // launch, blockIdx.z = class): a tap reaches input row iy only if
    // iy + pad - ky is a multiple of the stride, so each class gathers only its
    // own taps (for 3x3 stride 2: 1, 2, 2 or 4 of the 9) instead of zeros.
    GemmArgs g = {};
    g.S = shape_of(c);
    g.N = c.c;
    g.dy = dy;
    g.w = w;
    g.mask = mask;
    g.out_f = dx;
    const int st = c.stride;
    const int64_t rows = (int64_t)c.n * ((c.h + st - 1) / st) * ((c.w + st - 1) / st);  // class 0
    dim3 grid((unsigned)cdiv(rows, kBM), (unsigned)cdiv(g.N, kBN), (unsigned)(st * st));
    // A: 8 output channels of dy (k % 8); B: 8 input channels of a filter row (c % 8)
    launch_igemm<kBwdData>(g, c.k % 8 == 0, c.c % 8 == 0, grid, s);
    return hipGetLastError();
}

hipError_t launch_conv_bwd_weight(const bz_conv &c, const float *dy, const uint16_t *x,
                                  float *dw, float *db, hipStream_t s) {
    GemmArgs g = {};
    g.S = shape_of(c);
    g.M = c.k;
    g.N = (int64_t)c.r * c.r * c.c;
    g.K = (int64_t)c.n * c.ho * c.wo;
    g.dy = dy;
    g.x = x;
    g.out_f = dw;
    const int64_t tiles = cdiv(g.M, kBM) * cdiv(g.N, kBN);
    g.k_chunk = cdiv(g.K, kSplitRows) * tiles < kSplitMinGroups ? kSplitRowsSmall : kSplitRows;
    const int64_t nz = g.M * g.N;
    hipLaunchKernelGGL(k_fill0, dim3((unsigned)cdiv(nz, 256) < 4096 ? (unsigned)cdiv(nz, 256) : 4096),
                       dim3(256), 0, s, dw, nz);
    if (wgrad_first_shape(c) && ((uintptr_t)x & 15) == 0) {     // 16-byte image loads
        if (db)
            hipLaunchKernelGGL(k_fill0, dim3(1), dim3(256), 0, s, db, (int64_t)c.k);
        if (c.c == 1) launch_wgrad_first<1>(c, dy, x, dw, db, s);
        else if (c.c == 2) launch_wgrad_first<2>(c, dy, x, dw, db, s);
        else launch_wgrad_first<3>(c, dy, x, dw, db, s);
        return hipGetLastError();
    }
    dim3 grid((unsigned)cdiv(g.M, kBM), (unsigned)cdiv(g.N, kBN), (unsigned)cdiv(g.K, g.k_chunk));
    // A: 8 output channels of dy (k % 8); B: 8 input channels of a shifted pixel (c % 8)
    launch_igemm<kBwdWeight>(g, c.k % 8 == 0, c.c % 8 == 0, grid, s);
    if (db) {
        hipLaunchKernelGGL(k_fill0, dim3((unsigned)cdiv(c.k, 256)), dim3(256), 0, s, db,
                           (int64_t)c.k);
        // dy rows are 16-byte aligned when k % 4 == 0 (dy itself is)
        const int64_t chunk = bias_chunk(g.K);
        if (c.k % 4 == 0 && c.k <= 64 && ((uintptr_t)dy & 15) == 0)
            hipLaunchKernelGGL(k_bias_grad4, dim3((unsigned)cdiv(g.K, chunk)), dim3(256), 0, s,
                               dy, g.K, chunk, c.k, db);
        else
            hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)cdiv(g.K, chunk), (unsigned)cdiv(c.k, 64)),
                               dim3(256), 0, s, dy, g.K, chunk, c.k, db);
    }
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, uint16_t *dst, int64_t n, hipStream_t s) {
    if (n > 0) {
        int64_t b = cdiv(n, 256);
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s, src,
                           dst, n);
    }
    return hipGetLastError();
}

hipError_t launch_patches(const float *img, int W, int H, const int32_t *xy, int np, int side,
                          float fill, uint16_t *out, hipStream_t s) {
    int64_t total = (int64_t)side * side * 3 * np;
    if (total > 0) {
        int64_t b = cdiv(total, 256);
        hipLaunchKernelGGL(k_patches, dim3((unsigned)(b < 8192 ? b : 8192)), dim3(256), 0, s, img,
                           W, H, xy, np, side, fill, out);
    }
    return hipGetLastError();
}

}  // namespace bz

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace bz;

extern "C" {

bz_status bz_conv_shape(bz_conv *cv) {
    if (!cv) return BZ_ERR_ARG;
    if (cv->n < 1 || cv->h < 1 || cv->w < 1 || cv->c < 1 || cv->k < 1) return BZ_ERR_ARG;
    if (cv->r != 1 && cv->r != 3) return BZ_ERR_ARG;
    if (cv->stride < 1 || cv->stride > 4 || cv->pad < 0 || cv->pad >= cv->r) return BZ_ERR_ARG;
    const int64_t ho = ((int64_t)cv->h + 2 * cv->pad - cv->r) / cv->stride + 1;
    const int64_t wo = ((int64_t)cv->w + 2 * cv->pad - cv->r) / cv->stride + 1;
    if ((int64_t)cv->h + 2 * cv->pad < cv->r || (int64_t)cv->w + 2 * cv->pad < cv->r || ho < 1 ||
        wo < 1)
        return BZ_ERR_ARG;
    const int64_t lim = int64_t(1) << 30;      // index arithmetic stays in 32 bits
    if ((int64_t)cv->n * cv->h * cv->w * cv->c >= lim || (int64_t)cv->n * ho * wo * cv->k >= lim ||
        (int64_t)cv->k * cv->r * cv->r * cv->c >= lim)
        return BZ_ERR_UNSUPPORTED;
    cv->ho = (int32_t)ho;
    cv->wo = (int32_t)wo;
    return BZ_OK;
}

static bz_status check_conv(const bz_conv *cv) {
    if (!cv) return BZ_ERR_ARG;
    bz_conv c = *cv;
    bz_status st = bz_conv_shape(&c);
    if (st != BZ_OK) return st;
    if (c.ho != cv->ho || c.wo != cv->wo) return BZ_ERR_ARG;
    return BZ_OK;
}

static bz_status done(hipError_t e) { return e == hipSuccess ? BZ_OK : BZ_ERR_HIP; }

bz_status bz_conv_fwd(const bz_conv *cv, const uint16_t *x, const uint16_t *w, const float *bias,
                      int32_t relu, float *y, uint16_t *y_bf16, hipStream_t s) {
    bz_status st = check_conv(cv);
    if (st != BZ_OK) return st;
    if (!x || !w || (!y && !y_bf16) || (relu != 0 && relu != 1)) return BZ_ERR_ARG;
    (void)hipGetLastError();
    return done(launch_conv_fwd(*cv, x, w, bias, relu, y, y_bf16, s));
}

bz_status bz_conv_bwd_data(const bz_conv *cv, const float *dy, const uint16_t *w,
                           const uint16_t *x_mask, float *dx, hipStream_t s) {
    bz_status st = check_conv(cv);
    if (st != BZ_OK) return st;
    if (!dy || !w || !dx) return BZ_ERR_ARG;
    (void)hipGetLastError();
    return done(launch_conv_bwd_data(*cv, dy, w, x_mask, dx, s));
}

bz_status bz_conv_bwd_weight(const bz_conv *cv, const float *dy, const uint16_t *x, float *dw,
                             float *db, hipStream_t s) {
    bz_status st = check_conv(cv);
    if (st != BZ_OK) return st;
    if (!dy || !x || !dw) return BZ_ERR_ARG;
    (void)hipGetLastError();
    return done(launch_conv_bwd_weight(*cv, dy, x, dw, db, s));
}

bz_status bz_f32_to_bf16(const float *src, uint16_t *dst, int64_t n, hipStream_t s) {
    if (n < 0 || (n > 0 && (!src || !dst))) return BZ_ERR_ARG;
    (void)hipGetLastError();
    return done(launch_to_bf16(src, dst, n, s));
}

bz_status bz_extract_patches(const float *image, int32_t width, int32_t height, const int32_t *xy,
                             int32_t n_patch, int32_t side, float fill, uint16_t *out,
                             hipStream_t s) {
    if (width < 1 || height < 1 || n_patch < 0 || side < 1 || side > 4096) return BZ_ERR_ARG;
    if (n_patch > 0 && (!image || !xy || !out)) return BZ_ERR_ARG;
    if ((int64_t)side * side * 3 * n_patch >= (int64_t(1) << 40)) return BZ_ERR_UNSUPPORTED;
    (void)hipGetLastError();
    return done(launch_patches(image, width, height, xy, n_patch, side, fill, out, s));
}

}  // extern "C"
