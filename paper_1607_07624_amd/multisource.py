"""Batched multi-source, multi-wavelength pyramid sensing in one HIP graph.

Several guide stars (sources) are sensed at several wavelengths: one plan
per wavelength measures the same batch of source OPDs (the OPD in nm is
achromatic; the plan turns it into phase at its wavelength).  All the
pwfs_measure calls of a step are captured once into a HIP graph (through
torch's graph capture; the library launches only kernels on the caller's
stream, with no allocation, copy-engine work or host synchronisation while
timing is off) and replayed as one launch.  The graph reads the sources from
one static input buffer and writes one static slope buffer per wavelength.
"""
from __future__ import annotations

from ._lib import Plan


class MultiSourceSensor:
    def __init__(self, cfgs, n_sources: int, autotune: bool = True, reps: int = 3):
        import torch
        self._torch = torch
        P = cfgs[0].n_pupil
        if any(c.n_pupil != P for c in cfgs):
            raise ValueError("all wavelengths must share the pupil sampling")
        self.plans = [Plan(c, batch_max=n_sources) for c in cfgs]
        self.schedules = [p.autotune(n_sources, reps=reps) if autotune else None for p in self.plans]
        dev = torch.device("cuda", self.plans[0].device)
        self.n_sources = n_sources
        self.opd = torch.zeros((n_sources, P, P), device=dev)
        self.slopes = [torch.empty((n_sources, 2 * p.n_valid), device=dev) for p in self.plans]
        self.graph = None

    def measure_eager(self, out=None):
        """Same calls as the graph, launched one by one (into `out` or the static buffers)."""
        out = out or self.slopes
        for p, s in zip(self.plans, out):
            p.measure_into(self.opd, None, s)
        return out

    def capture(self):
        torch = self._torch
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.measure_eager()                     # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.measure_eager()
        self.graph = g
        return g

    def measure(self, opd=None):
        """Copy `opd` [n_sources, P, P] into the static input (if given) and replay."""
        if self.graph is None:
            self.capture()
        if opd is not None:
            self.opd.copy_(opd)
        self.graph.replay()
        return self.slopes

    def close(self):
        self.graph = None
        for p in self.plans:
            p.close()
