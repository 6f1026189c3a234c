/*
 * bz_peak.h -- C ABI of libbz's rate probes: the sustained device rates that
 * the rasterizer's roofline fractions are reported against (HBM copy, plain
 * FP32 FMA, the exp2 and reciprocal of the blend loops, LDS broadcast reads
 * and LDS float atomics).  Not part of the paper's method: measurement only.
 *
 * Each probe is one kernel launch of a single kind of instruction over
 * independent chains, sized to fill the device.  The caller times the launch
 * (e.g. with events on `stream`) and divides bz_peak_work's count by the time.
 */
#ifndef BZ_PEAK_H
#define BZ_PEAK_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "bz.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BZ_PEAK_COPY = 0,          /* n bytes read and n written (float4 loads/stores) */
    BZ_PEAK_FMA = 1,           /* v_fma_f32 chains; work in flops (an FMA counts 2) */
    BZ_PEAK_EXP2 = 2,          /* v_exp_f32 chains; work in lane operations */
    BZ_PEAK_RCP = 3,           /* v_rcp_f32 chains; work in lane operations */
    BZ_PEAK_LDS_BCAST = 4,     /* 16-byte LDS reads, one address per wave; work in wave instructions */
    BZ_PEAK_LDS_ADD = 5,       /* LDS float atomic add, 64 distinct conflict-free addresses */
    BZ_PEAK_LDS_ADD_4WAY = 6,  /* the same, every 4 lanes on one address */
    BZ_PEAK_LDS_ADD_SAME = 7   /* the same, all 64 lanes on one address */
};

/* Launch probe `kind` on `stream`.
 *   BZ_PEAK_COPY: n bytes (a multiple of 16) copied from the first half of buf
 *       to the second; buf (device, 16-byte aligned) holds buf_bytes >= 2n.
 *   other kinds: n threads (a multiple of 256), each running `iters` rounds
 *       of 8 independent operations; buf (device) receives nothing the caller
 *       needs but must hold n/256 floats.
 * Returns BZ_ERR_ARG on a bad kind or size, BZ_ERR_HIP if the launch fails. */
bz_status bz_peak_run(int32_t kind, int64_t n, int32_t iters, float *buf, int64_t buf_bytes,
                      hipStream_t stream);

/* Host: the work one bz_peak_run(kind, n, iters) does, in the unit its kind
 * states, into *work. */
bz_status bz_peak_work(int32_t kind, int64_t n, int32_t iters, double *work);

#ifdef __cplusplus
}
#endif
#endif /* BZ_PEAK_H */
