"""Launch-shape autotuner for the blend kernels.

The tile shape (tile_w x tile_h pixels = threads per workgroup, one 8x8 quad
per wave) and the launch form (one workgroup per tile, or persistent
workgroups taking tiles from a counter) change only speed, never results.
Which is fastest depends on the workload.  Smaller tiles list and stage a
Gaussian in more tiles; larger ones stage entries that fewer of their quads
need and leave more lanes idle at canvas edges; a persistent launch pays off
when tiles are many and cheap.  :func:`autotune` measures every candidate on
the actual workload, each as a recorded step graph, and returns the fastest.
``python -m paper_2503_16424_amd.autotune`` runs it on the 2048x2048,
20,000-curve workload.
"""
from __future__ import annotations

import itertools
import time
from dataclasses import replace

TILE_SHAPES = ((8, 8), (16, 8), (8, 16), (16, 16), (32, 8), (8, 32), (32, 16), (16, 32),
               (32, 32))


def candidates(shapes=TILE_SHAPES, persistent=(False, True)):
    return [dict(tile_w=w, tile_h=h, persistent=p) for (w, h), p in
            itertools.product(shapes, persistent)]


def time_graph(g, reps: int) -> float:
    """Milliseconds per replay of a recorded step (HIP events)."""
    import torch
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(scenes_or_scene, target, base=None, cands=None, reps: int = 5, log=None):
    """Time one graph-recorded fwd+bwd step per candidate launch shape.

    scenes_or_scene: a scene or a list of scenes (a batch); target: the L2
    target on the device in the rasterizer's image layout.  Returns
    (best options, [(candidate, ms per step), ...] in the order measured)."""
    import torch
    from . import bz
    from .graph import StepGraph
    base = base or bz.RenderOptions()
    table = []
    for c in (cands or candidates()):
        ro = replace(base, **c)
        t0 = time.perf_counter()
        r = bz.Rasterizer(scenes_or_scene, ro)
        g = StepGraph(r, target)
        ms = time_graph(g, reps)
        table.append((c, ms))
        if log:
            log(f"  tile {c['tile_w']}x{c['tile_h']} persistent={int(c['persistent'])}: "
                f"{ms:.3f} ms/step ({time.perf_counter() - t0:.1f} s to build and time)")
        del g, r
        torch.cuda.empty_cache()
    best = min(table, key=lambda t: t[1])[0]
    return replace(base, **best), table


def main(argv=None) -> int:
    """Every candidate on the 2048x2048, 20,000-curve workload (one GPU)."""
    import argparse

    import torch

    from . import scenes
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--reps", type=int, default=10, help="timed graph replays per candidate")
    a = ap.parse_args(argv)
    sc = scenes.paper_2048(0)
    tgt = torch.as_tensor(scenes.target_noise(1, sc.width, sc.height), device="cuda")
    best, _ = autotune(sc, tgt, reps=a.reps, log=lambda m: print(m, flush=True))
    print(f"best: tile {best.tile_w}x{best.tile_h} persistent={int(best.persistent)}", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
