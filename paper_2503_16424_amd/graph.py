"""One optimisation step as a single HIP graph launch.

A step of the rasterizer is a dozen small kernels (sampling, binning with its
scans and radix passes, blending, L2 gradient, both backward stages).  For
many small canvases - a batch - their launch overhead is a large part of the
step, so :class:`StepGraph` records the whole step once into a HIP graph
(through torch's graph capture, which owns the stream) and replays it with
one launch.  Nothing in libbz allocates or synchronises inside a step, and
every buffer it clears is cleared by a kernel, so the recorded step is the
eager step.

The pair buffer cannot grow inside a graph: it is sized eagerly (with slack)
before the capture, and :meth:`StepGraph.replay` can check the overflow flag
(which synchronises) and re-record after growing it.
"""
from __future__ import annotations


class StepGraph:
    """sample + bin + forward + L2 gradient (against ``target``) + backward of
    ``rast``, recorded once and replayed with one launch."""

    def __init__(self, rast, target, slack: float = 1.25, warmup: int = 2):
        self.rast, self.target, self.slack, self.warmup = rast, target, slack, warmup
        self.graph = None
        self.records = 0
        self._record()

    def _record(self):
        import torch
        r = self.rast
        r.render()                                   # eager: sizes the pair buffer
        need = r.pairs_required()
        if need * self.slack > r.cap_pairs:
            r._alloc_pairs(int(need * self.slack) + 1024)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(self.warmup):
                r.step(self.target)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            r.step(self.target)
        self.records += 1

    def replay(self, check: bool = False) -> bool:
        """Run the recorded step.  With ``check``, synchronise, and if the tile
        lists overflowed, grow the pair buffer, re-record and run again;
        returns True when that happened."""
        from . import bz
        self.graph.replay()
        if check and self.rast.flags() & bz.STATUS_OVERFLOW:
            self._record()
            self.graph.replay()
            return True
        return False
