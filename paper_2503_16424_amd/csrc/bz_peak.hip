// bz_peak.hip -- sustained device rates that the rasterizer's roofline is
// taken against: HBM copy, plain FP32 FMA, the two transcendentals of the
// blend loops (exp2, reciprocal), LDS broadcast reads and LDS float atomics
// with and without address conflicts.  Each kernel is a stream of one kind of
// instruction over independent chains, sized to fill every compute unit; the
// caller times the launch and bz_peak_work gives the work it did.
#include <hip/hip_runtime.h>

#include "../../include/bz_peak.h"

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;

__global__ __launch_bounds__(kThreads) void k_copy(const float4 *__restrict__ src,
                                                   float4 *__restrict__ dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        dst[i] = src[i];
}

// kind: 0 FMA, 1 exp2, 2 reciprocal.  The chains stay bounded: x -> x*b + c
// with b < 1, x -> 2^-x on [0, 1], x -> 1/x alternating between x and 1/x.
template <int kKind>
__global__ __launch_bounds__(kThreads) void k_alu(float *out, int iters, float b, float c) {
    float a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = 0.5f + 0.01f * (float)(threadIdx.x & 7) + 0.001f * i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
            if (kKind == 0) a[i] = fmaf(a[i], b, c);
            else if (kKind == 1) a[i] = __builtin_amdgcn_exp2f(-a[i]);
            else a[i] = __builtin_amdgcn_rcpf(a[i]);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i];
    if (s == 12345.678f) out[blockIdx.x] = s;   // keeps the chains alive
}

// LDS: kind 0 broadcast 16-byte reads (every lane of a wave the same address),
// 1 float atomic add with 64 distinct addresses per instruction (consecutive
// words, no bank conflict), 2 the same with every 4 lanes on one address,
// 3 every lane of the wave on one address.
template <int kKind>
__global__ __launch_bounds__(kThreads) void k_lds(float *out, int iters) {
    __shared__ float4 s4[512];
    float *s = reinterpret_cast<float *>(s4);
    for (int i = threadIdx.x; i < 2048; i += blockDim.x) s[i] = 1.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float acc = 0.f;
    if (kKind == 0) {
        // every word of each read is folded in with two 3-input XORs
        const uint4 *u4 = reinterpret_cast<const uint4 *>(s4);
        uint32_t x = 0;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                const uint4 r = u4[(w * 64 + ((it * kChains + i) & 63))];
                x = x ^ r.x ^ r.y;
                x = x ^ r.z ^ r.w;
            }
        }
        acc = __uint_as_float(x);
    } else {
        const int addr0 = kKind == 1 ? lane : kKind == 2 ? (lane >> 2) : 0;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kChains; ++i)
                __hip_atomic_fetch_add(&s[w * 512 + ((addr0 + 64 * i) & 511)], 1.0f,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        acc = s[threadIdx.x];
    }
    if (acc == 12345.678f) out[blockIdx.x] = acc;
}

int blocks_for(int64_t n, int64_t per_block, int64_t cap) {
    int64_t b = (n + per_block - 1) / per_block;
    return (int)(b < 1 ? 1 : b > cap ? cap : b);
}

}  // namespace

extern "C" {

bz_status bz_peak_work(int32_t kind, int64_t n, int32_t iters, double *work) {
    if (!work || n < 0 || iters < 0) return BZ_ERR_ARG;
    switch (kind) {
        case BZ_PEAK_COPY:
            *work = 2.0 * 16.0 * (double)(n / 16);   // bytes read + written
            return BZ_OK;
        case BZ_PEAK_FMA:
            *work = 2.0 * kChains * (double)iters * (double)n;   // flops (FMA = 2)
            return BZ_OK;
        case BZ_PEAK_EXP2:
        case BZ_PEAK_RCP:
            *work = (double)kChains * iters * (double)n;         // lane operations
            return BZ_OK;
        case BZ_PEAK_LDS_BCAST:
        case BZ_PEAK_LDS_ADD:
        case BZ_PEAK_LDS_ADD_4WAY:
        case BZ_PEAK_LDS_ADD_SAME:
            *work = (double)kChains * iters * (double)(n / 64);  // wave instructions
            return BZ_OK;
        default:
            return BZ_ERR_ARG;
    }
}

bz_status bz_peak_run(int32_t kind, int64_t n, int32_t iters, float *buf, int64_t buf_bytes,
                      hipStream_t stream) {
    if (!buf || n <= 0 || iters < 0) return BZ_ERR_ARG;
    if (kind == BZ_PEAK_COPY) {
        // buf holds the source and the destination, n bytes each
        if (buf_bytes < 2 * n || n % 16) return BZ_ERR_ARG;
        const int64_t n4 = n / 16;
        hipLaunchKernelGGL(k_copy, dim3(blocks_for(n4, kThreads, 256 * 64)), dim3(kThreads), 0,
                           stream, (const float4 *)buf, (float4 *)(buf) + n4, n4);
        return hipGetLastError() == hipSuccess ? BZ_OK : BZ_ERR_HIP;
    }
    // n threads, whole workgroups; buf receives one float per workgroup at most
    if (n % kThreads) return BZ_ERR_ARG;
    const int blocks = (int)(n / kThreads);
    if (buf_bytes < (int64_t)sizeof(float) * blocks) return BZ_ERR_ARG;
    switch (kind) {
        case BZ_PEAK_FMA:
            hipLaunchKernelGGL(k_alu<0>, dim3(blocks), dim3(kThreads), 0, stream, buf, iters,
                               0.999f, 1e-4f);
            break;
        case BZ_PEAK_EXP2:
            hipLaunchKernelGGL(k_alu<1>, dim3(blocks), dim3(kThreads), 0, stream, buf, iters,
                               0.f, 0.f);
            break;
        case BZ_PEAK_RCP:
            hipLaunchKernelGGL(k_alu<2>, dim3(blocks), dim3(kThreads), 0, stream, buf, iters,
                               0.f, 0.f);
            break;
        case BZ_PEAK_LDS_BCAST:
            hipLaunchKernelGGL(k_lds<0>, dim3(blocks), dim3(kThreads), 0, stream, buf, iters);
            break;
        case BZ_PEAK_LDS_ADD:
            hipLaunchKernelGGL(k_lds<1>, dim3(blocks), dim3(kThreads), 0, stream, buf, iters);
            break;
        case BZ_PEAK_LDS_ADD_4WAY:
            hipLaunchKernelGGL(k_lds<2>, dim3(blocks), dim3(kThreads), 0, stream, buf, iters);
            break;
        case BZ_PEAK_LDS_ADD_SAME:
            hipLaunchKernelGGL(k_lds<3>, dim3(blocks), dim3(kThreads), 0, stream, buf, iters);
            break;
        default:
            return BZ_ERR_ARG;
    }
    return hipGetLastError() == hipSuccess ? BZ_OK : BZ_ERR_HIP;
}

}  // extern "C"
