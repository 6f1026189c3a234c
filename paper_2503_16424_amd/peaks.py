"""Sustained device rates measured with libbz's rate probes (include/bz_peak.h).

Each probe is one launch of a single kind of instruction over independent
chains; it is timed with events on the current stream and its work (from
bz_peak_work) divided by the time.  The rates are what the rasterizer's
roofline fractions are also reported against, beside the published peaks.
"""
from __future__ import annotations

import ctypes as C

from . import bz

COPY, FMA, EXP2, RCP, LDS_BCAST, LDS_ADD, LDS_ADD_4WAY, LDS_ADD_SAME = range(8)
CUS, CLOCK_HZ = 256, 2.4e9


def _time(lib, kind, n, iters, buf, nbytes, reps):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(2):
        bz._check("bz_peak_run", lib.bz_peak_run(kind, n, iters, C.c_void_p(buf), nbytes,
                                                 C.c_void_p(stream)))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bz._check("bz_peak_run", lib.bz_peak_run(kind, n, iters, C.c_void_p(buf), nbytes,
                                                 C.c_void_p(stream)))
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    w = C.c_double(0.0)
    bz._check("bz_peak_work", lib.bz_peak_work(kind, n, iters, C.byref(w)))
    return w.value / sec


def measure(copy_mib: int = 512, threads: int = 1 << 20, reps: int = 5) -> dict:
    """Rates of every probe: HBM copy GB/s, FP32 FMA TFLOP/s, exp2 and
    reciprocal in lane operations per second and in FMA slots (how many FMAs
    one costs), LDS instructions per CU and cycle at the 2.4 GHz peak clock."""
    import torch
    lib = bz.load_library()
    n = copy_mib << 20
    buf = torch.empty(2 * n // 4, dtype=torch.float32, device="cuda")
    buf.fill_(1.0)
    out = {}
    out["copy_GBs"] = _time(lib, COPY, n, 0, buf.data_ptr(), 2 * n, reps) / 1e9
    del buf
    small = torch.empty(threads // 256 + 64, dtype=torch.float32, device="cuda")
    nb = small.numel() * 4
    fma = _time(lib, FMA, threads, 4096, small.data_ptr(), nb, reps)
    out["fma_TFLOPs"] = fma / 1e12
    for name, kind in (("exp2", EXP2), ("rcp", RCP)):
        r = _time(lib, kind, threads, 1024, small.data_ptr(), nb, reps)
        out[f"{name}_Gops"] = r / 1e9
        out[f"{name}_fma_slots"] = (fma / 2.0) / r
    per_cu_cycle = CUS * CLOCK_HZ
    for name, kind in (("lds_bcast_b128", LDS_BCAST), ("lds_add", LDS_ADD),
                       ("lds_add_4way", LDS_ADD_4WAY), ("lds_add_same", LDS_ADD_SAME)):
        iters = 64 if kind == LDS_ADD_SAME else 1024
        r = _time(lib, kind, threads, iters, small.data_ptr(), nb, reps)
        out[f"{name}_per_cu_cycle"] = r / per_cu_cycle
    return out


if __name__ == "__main__":
    import json
    print(json.dumps(measure(), indent=1))
