"""Batched iterations over many independent scans.

``BatchRunner`` keeps every job's object, probe, positions, measured data,
outputs and workspace on the device, builds one plan (persistent launches per
probe size, see ``Plan``) and can capture a whole iteration in one HIP graph:
the loss and gradients of every job, the advance of a device-side iteration
count and the Adam step on every object, whose bias correction reads that
count when it runs (adorym_adam_dev).  ``run_per_job`` is the plain form for
comparison: the same work as one ``loss_grad`` call per job.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import torch

from .api import Context, Geometry, Job, split_positions


@dataclasses.dataclass
class DeviceScan:
    geom: Geometry
    a: torch.Tensor            # current object estimate (delta or Re O)
    b: torch.Tensor
    probe: torch.Tensor
    corner: torch.Tensor
    shift: torch.Tensor
    i_meas: torch.Tensor
    m_a: torch.Tensor          # Adam moments of the object
    v_a: torch.Tensor
    m_b: torch.Tensor
    v_b: torch.Tensor


def simulate_measurements(ctx: Context, geom: Geometry, a_true, b_true, probe, corner, shift, photons_seed=None,
                          chunk=512):
    """Measured data for synthetic scans: the forward model at the truth,
    Poisson-sampled when ``photons_seed`` is given."""
    outs = []
    for s in range(0, corner.shape[0], chunk):
        outs.append(ctx.forward(geom, a_true, b_true, probe, corner[s:s + chunk], shift[s:s + chunk]))
    i_true = torch.cat(outs)
    if photons_seed is None:
        return i_true
    gen = torch.Generator(device=i_true.device)
    gen.manual_seed(int(photons_seed))
    return torch.poisson(i_true.clamp_min(0), generator=gen)


def to_device_scan(ctx: Context, scan, seed: int = 0) -> DeviceScan:
    dev = ctx.device
    t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    geom = Geometry.from_scan(scan)
    probe = t(scan.probe, torch.complex64)
    corner, shift = split_positions(t(scan.positions, torch.float64))
    a_true, b_true = t(scan.obj_a, torch.float32), t(scan.obj_b, torch.float32)
    im = simulate_measurements(ctx, geom, a_true, b_true, probe, corner, shift,
                               photons_seed=seed if scan.loss == "poisson" else None)
    a = t(scan.eval_obj_a, torch.float32) if scan.eval_obj_a is not None else torch.zeros_like(a_true)
    b = t(scan.eval_obj_b, torch.float32) if scan.eval_obj_b is not None else torch.zeros_like(b_true)
    z = torch.zeros_like
    return DeviceScan(geom, a, b, probe, corner, shift, im.contiguous(), z(a), z(a), z(b), z(b))


class BatchRunner:
    """One iteration = loss and gradients of every job + Adam on every object."""

    def __init__(self, ctx: Context, scans: List[DeviceScan], lr: float = 1e-7):
        self.ctx = ctx
        self.scans = scans
        self.lr = lr
        self.t = 0
        # the iteration count the Adam kernels read (advanced on the device)
        self.t_dev = torch.zeros(1, dtype=torch.int32, device=ctx.device)
        self.jobs = [Job(geom=s.geom, obj_a=s.a, obj_b=s.b, probe=s.probe, corner=s.corner, shift=s.shift,
                         i_meas=s.i_meas) for s in scans]
        self.plan = None
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    def build_plan(self):
        if self.plan is not None:
            self.plan.close()
        self.plan = self.ctx.plan(self.jobs)
        return self.plan

    def _adam(self):
        """Advance the device iteration count and take every object's Adam step."""
        self.t_dev.add_(1)
        for s, j in zip(self.scans, self.jobs):
            self.ctx.adam(s.a, j.out["g_a"], s.m_a, s.v_a, self.t_dev, lr=self.lr)
            self.ctx.adam(s.b, j.out["g_b"], s.m_b, s.v_b, self.t_dev, lr=self.lr)

    def step(self, adam: bool = True):
        """One batched iteration (eager launches)."""
        self.t += 1
        self.plan.run()
        if adam:
            self._adam()

    def capture(self, adam: bool = True):
        """Capture one iteration in one HIP graph: plan.run() (loss and
        gradients of every job) and, with ``adam``, the count's advance and
        every Adam step."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.plan.run()
            if adam:
                self._adam()
        self.graph = g
        self.graph_adam = adam
        return g

    def step_graph(self):
        """One iteration: one graph replay."""
        self.t += 1
        self.graph.replay()

    def run_per_job(self, adam: bool = True):
        """The plain form: one loss_grad call per job (its own launches)."""
        self.t += 1
        for s, j in zip(self.scans, self.jobs):
            self.ctx.loss_grad(s.geom, s.a, s.b, s.probe, s.corner, s.shift, s.i_meas, out=j.out,
                               workspace=j.workspace)
        if adam:
            self._adam()

    def positions(self) -> int:
        return sum(int(s.corner.shape[0]) for s in self.scans)

    def close(self):
        if self.plan is not None:
            self.plan.close()
            self.plan = None
