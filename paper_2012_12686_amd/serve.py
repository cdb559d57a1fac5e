"""Serving loop: reconstruction jobs of mixed sizes on one GPU.

Jobs arrive over time (e.g. a Poisson process).  Each job is a few
iterations of a reconstruction: per iteration one minibatch (or, for a tilt
series, one rotation angle) goes through the loss and gradient of the
multislice model, then Adam updates the job's object.  Everything a job
needs (object estimate, Adam moments, its measured data, positions, probe,
gradient buffers, workspace) is allocated on the device when it is admitted
and stays there until it finishes.

Continuous batching: the loop works in ticks.  A tick is one iteration of
every active job -- their loss and gradient evaluations go through one
batched plan (a persistent launch per probe size whose workgroups draw
positions of all jobs from one queue), so the jobs' work overlaps on the
device.  Jobs that arrive while a tick runs wait in a queue and are admitted
at the next tick boundary when both the HBM budget (their exact footprint)
and the slots allow: at most ``max_jobs`` jobs and ``max_positions``
positions per tick.  Finished jobs leave at tick boundaries.  Two ticks may
be in flight, so the host prepares tick t+1 while the device runs tick t.

Latency of an iteration = host time from enqueueing its tick to observing
the tick's completion event; queue wait = arrival to admission; job time =
arrival to the completion of its last iteration.

Tilt-series jobs (Sec. S1.D.2) rotate the object to the iteration's angle
(R), evaluate the loss on the rotated object, take the gradient back with
the exact transpose R^T and update the unrotated object.
"""
from __future__ import annotations

import dataclasses
import math
import sys
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from .api import Context, Geometry, Job, split_positions
from .batch import simulate_measurements


# ---------------------------------------------------------------------------
# Job types
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Template:
    """One job type: its geometry and synthetic inputs on the device (read-only).

    ``corner``/``shift``/``i_meas`` hold one block per step: minibatch k of a
    scan, or angle k of a tilt series (the same positions at every angle).
    Iteration ``it`` of a job uses step ``it % n_steps``.
    """

    name: str
    kind: str                   # "scan" | "tilt"
    geom: Geometry
    a0: torch.Tensor            # start point of the object estimate [S][Ly][Lx]
    b0: torch.Tensor
    probe: torch.Tensor         # complex64 [N][N]
    corner: torch.Tensor        # int32 [steps][B][2]
    shift: torch.Tensor         # float32 [steps][B][2]
    i_meas: torch.Tensor        # float32 [steps][B][N][N]
    angles: Tuple[float, ...] = ()   # tilt: rotation angle (radians) of each step
    lr: float = 1e-7

    @property
    def minibatch(self) -> int:
        return int(self.corner.shape[1])

    @property
    def n_steps(self) -> int:
        return int(self.corner.shape[0])


def scan_template(ctx: Context, scan, name: str, seed: int = 0, lr: float = 1e-7,
                  n_minibatches: Optional[int] = None) -> Template:
    """A scan job type: data simulated at the truth (Poisson-sampled when the
    scan counts photons), evaluated from the scan's evaluation point.
    Minibatches are contiguous blocks of a seeded permutation of the
    positions; a last partial block is dropped."""
    dev = ctx.device
    t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    geom = Geometry.from_scan(scan)
    a_true, b_true = t(scan.obj_a, torch.float32), t(scan.obj_b, torch.float32)
    probe_true = t(scan.probe, torch.complex64)
    c_true, s_true = split_positions(t(scan.positions, torch.float64))
    im = simulate_measurements(ctx, geom, a_true, b_true, probe_true, c_true, s_true,
                               photons_seed=seed if scan.loss == "poisson" else None)
    pos_eval = scan.eval_positions if scan.eval_positions is not None else scan.positions
    c_eval, s_eval = split_positions(t(pos_eval, torch.float64))
    bsz = scan.minibatch
    steps = len(scan.positions) // bsz
    if n_minibatches is not None:
        steps = min(steps, n_minibatches)
    perm = torch.as_tensor(np.random.default_rng(seed).permutation(len(scan.positions))[:steps * bsz],
                           device=dev)
    a0 = t(scan.eval_obj_a, torch.float32) if scan.eval_obj_a is not None else torch.zeros_like(a_true)
    b0 = t(scan.eval_obj_b, torch.float32) if scan.eval_obj_b is not None else torch.zeros_like(b_true)
    probe = t(scan.eval_probe, torch.complex64) if scan.eval_probe is not None else probe_true
    n = geom.n
    return Template(name=name, kind="scan", geom=geom, a0=a0.contiguous(), b0=b0.contiguous(),
                    probe=probe.contiguous(),
                    corner=c_eval[perm].reshape(steps, bsz, 2).contiguous(),
                    shift=s_eval[perm].reshape(steps, bsz, 2).contiguous(),
                    i_meas=im[perm].reshape(steps, bsz, n, n).contiguous(), lr=lr)


def tilt_template(ctx: Context, scan, angles: Sequence[float], name: str = "tilt", seed: int = 0,
                  lr: float = 1e-7) -> Template:
    """A tilt-series job type: the scan's positions at every angle; data of
    angle k simulated from the truth rotated by angles[k]."""
    dev = ctx.device
    t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    geom = Geometry.from_scan(scan)
    a_true, b_true = t(scan.obj_a, torch.float32), t(scan.obj_b, torch.float32)
    probe = t(scan.probe, torch.complex64)
    corner, shift = split_positions(t(scan.positions, torch.float64))
    ra, rb = torch.empty_like(a_true), torch.empty_like(b_true)
    ims = []
    for k, th in enumerate(angles):
        ctx.rotate(a_true, th, out=ra)
        ctx.rotate(b_true, th, out=rb)
        ims.append(simulate_measurements(ctx, geom, ra, rb, probe, corner, shift,
                                         photons_seed=(seed * 1000 + k) if scan.loss == "poisson" else None))
    del ra, rb
    steps = len(angles)
    a0 = t(scan.eval_obj_a, torch.float32) if scan.eval_obj_a is not None else torch.zeros_like(a_true)
    b0 = t(scan.eval_obj_b, torch.float32) if scan.eval_obj_b is not None else torch.zeros_like(b_true)
    return Template(name=name, kind="tilt", geom=geom, a0=a0.contiguous(), b0=b0.contiguous(),
                    probe=probe.contiguous(), corner=corner.expand(steps, -1, -1).contiguous(),
                    shift=shift.expand(steps, -1, -1).contiguous(), i_meas=torch.stack(ims).contiguous(),
                    angles=tuple(float(a) for a in angles), lr=lr)


# ---------------------------------------------------------------------------
# One admitted job
# ---------------------------------------------------------------------------

def job_work(tpl: Template, iterations: int) -> float:
    """Relative cost of a job for scheduling: voxels the multislice sweep
    visits over all its iterations (positions x slices x N^2, the FFT work
    per position being ~N^2 S log N), plus the tilt job's rotations and the
    Adam steps on the object, which touch every voxel of it."""
    g = tpl.geom
    s, ly, lx = tpl.a0.shape
    sweep = tpl.minibatch * g.n_slices * g.n * g.n * np.log2(g.n)
    per_voxel = (4 if tpl.kind == "tilt" else 0) + 2
    return float(iterations * (sweep + per_voxel * s * ly * lx))


def job_footprint(ctx: Context, tpl: Template, deterministic: bool = False) -> int:
    """Device bytes a job of this type holds while admitted (what ServedJob allocates)."""
    s, ly, lx = tpl.a0.shape
    vol = s * ly * lx * 4
    n, bsz = tpl.geom.n, tpl.minibatch
    geom = dataclasses.replace(tpl.geom, deterministic=deterministic)
    n_vol = 2 + 4 + 2                         # object, Adam moments, gradients
    if tpl.kind == "tilt":
        n_vol += 4                            # rotated object, gradients in the rotated frame
    data = tpl.corner.numel() * 4 + tpl.shift.numel() * 4 + tpl.i_meas.numel() * 4
    minibatch = bsz * 2 * 4 * 2 + bsz * n * n * 4
    outputs = 8 + n * n * 8 + bsz * 2 * 4
    return n_vol * vol + data + minibatch + outputs + ctx.workspace_size(geom, bsz)


class ServedJob:
    """Device state of one admitted job and its per-iteration steps."""

    def __init__(self, ctx: Context, tpl: Template, job_id: int, iterations: int, deterministic: bool = False):
        self.ctx, self.tpl, self.id, self.iterations = ctx, tpl, job_id, iterations
        self.geom = dataclasses.replace(tpl.geom, deterministic=deterministic)
        dev = ctx.device
        z = torch.zeros_like
        self.a, self.b = tpl.a0.clone(), tpl.b0.clone()
        self.m_a, self.v_a, self.m_b, self.v_b = z(self.a), z(self.a), z(self.b), z(self.b)
        self.g_a, self.g_b = torch.empty_like(self.a), torch.empty_like(self.b)
        # the job's own copy of its data
        self.corner_all, self.shift_all = tpl.corner.clone(), tpl.shift.clone()
        self.i_all = tpl.i_meas.clone()
        bsz, n = tpl.minibatch, tpl.geom.n
        # the current iteration's inputs: fixed addresses that a plan can keep
        self.corner = torch.empty((bsz, 2), dtype=torch.int32, device=dev)
        self.shift = torch.empty((bsz, 2), dtype=torch.float32, device=dev)
        self.i_meas = torch.empty((bsz, n, n), dtype=torch.float32, device=dev)
        if tpl.kind == "tilt":
            self.a_rot, self.b_rot = torch.empty_like(self.a), torch.empty_like(self.b)
            self.gr_a, self.gr_b = torch.empty_like(self.a), torch.empty_like(self.b)
            obj_a, obj_b, ga, gb = self.a_rot, self.b_rot, self.gr_a, self.gr_b
        else:
            obj_a, obj_b, ga, gb = self.a, self.b, self.g_a, self.g_b
        self.out = {"loss": torch.empty((), dtype=torch.float64, device=dev), "g_a": ga, "g_b": gb,
                    "g_probe": torch.empty_like(tpl.probe),
                    "g_shift": torch.empty((bsz, 2), dtype=torch.float32, device=dev)}
        self.workspace = ctx.workspace(self.geom, bsz)
        self.job = Job(geom=self.geom, obj_a=obj_a, obj_b=obj_b, probe=tpl.probe, corner=self.corner,
                       shift=self.shift, i_meas=self.i_meas, out=self.out, workspace=self.workspace)
        self.losses = torch.zeros(iterations, dtype=torch.float64, device=dev)
        self.enqueued = 0          # iterations enqueued
        self.completed = 0         # iterations whose tick completed

    @property
    def positions(self) -> int:
        return self.tpl.minibatch

    def pre(self):
        """Stage iteration `enqueued`'s inputs (and rotate the object for a tilt job)."""
        k = self.enqueued % self.tpl.n_steps
        self.corner.copy_(self.corner_all[k])
        self.shift.copy_(self.shift_all[k])
        self.i_meas.copy_(self.i_all[k])
        if self.tpl.kind == "tilt":
            th = self.tpl.angles[k]
            self.ctx.rotate(self.a, th, out=self.a_rot)
            self.ctx.rotate(self.b, th, out=self.b_rot)

    def evaluate(self):
        """The loss and gradient on their own (the per-job form)."""
        self.ctx.loss_grad(self.geom, self.job.obj_a, self.job.obj_b, self.tpl.probe, self.corner, self.shift,
                           self.i_meas, out=self.out, workspace=self.workspace)

    def post(self):
        """Gradient back to the object frame, Adam, record the loss."""
        it = self.enqueued
        if self.tpl.kind == "tilt":
            th = self.tpl.angles[it % self.tpl.n_steps]
            self.ctx.rotate(self.gr_a, th, transpose=True, out=self.g_a)
            self.ctx.rotate(self.gr_b, th, transpose=True, out=self.g_b)
        self.ctx.adam(self.a, self.g_a, self.m_a, self.v_a, it + 1, lr=self.tpl.lr)
        self.ctx.adam(self.b, self.g_b, self.m_b, self.v_b, it + 1, lr=self.tpl.lr)
        self.losses[it].copy_(self.out["loss"])
        self.enqueued += 1


# ---------------------------------------------------------------------------
# Admission
# ---------------------------------------------------------------------------

class Admission:
    """Admission control: HBM budget and slots (jobs, positions per tick)."""

    def __init__(self, budget_bytes: int, max_jobs: int = 16, max_positions: int = 2048):
        self.budget, self.max_jobs, self.max_positions = int(budget_bytes), int(max_jobs), int(max_positions)
        self.used = 0
        self.jobs = 0
        self.positions = 0

    def fits_ever(self, footprint: int) -> bool:
        return footprint <= self.budget

    def try_admit(self, footprint: int, positions: int) -> bool:
        if self.used + footprint > self.budget or self.jobs + 1 > self.max_jobs:
            return False
        if self.jobs > 0 and self.positions + positions > self.max_positions:
            return False
        self.used += footprint
        self.jobs += 1
        self.positions += positions
        return True

    def release(self, footprint: int, positions: int):
        self.used -= footprint
        self.jobs -= 1
        self.positions -= positions
        assert self.used >= 0 and self.jobs >= 0 and self.positions >= 0


@dataclasses.dataclass
class Request:
    arrival_s: float
    template: Template
    iterations: int = 20


@dataclasses.dataclass
class JobRecord:
    id: int
    template: str
    arrival_s: float
    admitted_s: float = math.nan
    finished_s: float = math.nan
    footprint: int = 0
    losses: Optional[np.ndarray] = None
    state: Optional[Dict[str, torch.Tensor]] = None


@dataclasses.dataclass
class _Tick:
    index: int
    t_enq: float
    event: torch.cuda.Event
    members: List[ServedJob]
    positions: int


class Server:
    """The request loop (see the module docstring).

    batched=True: one plan per set of active jobs (continuous batching in
    lockstep ticks);
    streams=n > 0: every admitted job iterates on its own schedule, on one of
    n streams, so jobs of different sizes overlap on the device without
    waiting for each other (continuous batching without lockstep);
    batched=False with max_jobs=1: the plain per-job form, one job at a time,
    each iteration its own loss_grad call.

    order="fifo" admits waiting jobs first come first served (a job that
    does not fit blocks the ones behind it); order="sjf" admits the waiting
    job with the least work (job_work) that fits first, so that short jobs
    are not held behind long ones.

    busy_jobs: with a deep queue (at least busy_queue jobs waiting) the slot
    limit rises from max_jobs to busy_jobs.  Each concurrent job slows the
    others, which stretches the long jobs that make up the tail of the job
    time; a queue that deep is where the extra overlap pays for itself.
    """

    def __init__(self, ctx: Context, budget_bytes: Optional[int] = None, max_jobs: int = 16,
                 max_positions: int = 2048, batched: bool = True, deterministic: bool = False,
                 keep_state: bool = False, inflight: int = 2, streams: int = 0, order: str = "fifo",
                 busy_jobs: Optional[int] = None, busy_queue: int = 4):
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(ctx.device)
            budget_bytes = int(0.8 * free)
        self.ctx = ctx
        self.adm = Admission(budget_bytes, max_jobs, max_positions)
        self.batched, self.deterministic, self.keep_state = batched, deterministic, keep_state
        self.inflight = max(1, inflight)
        self.streams = int(streams)
        if order not in ("fifo", "sjf"):
            raise ValueError("order must be 'fifo' or 'sjf'")
        self.order = order
        self.max_jobs = int(max_jobs)
        self.busy_jobs = int(busy_jobs) if busy_jobs is not None else self.max_jobs
        self.busy_queue = int(busy_queue)
        if self.busy_jobs < self.max_jobs or self.busy_queue < 1:
            raise ValueError("busy_jobs must be at least max_jobs and busy_queue at least 1")

    def _admit_next(self, waiting: List[int], requests, foot) -> Optional[int]:
        """Pop and return the next waiting request to admit, or None."""
        if not waiting:
            return None
        self.adm.max_jobs = self.busy_jobs if len(waiting) >= self.busy_queue else self.max_jobs
        if self.order == "fifo":
            i = waiting[0]
            if not self.adm.try_admit(foot[i], requests[i].template.minibatch):
                return None
            return waiting.pop(0)
        for i in sorted(waiting, key=lambda i: (job_work(requests[i].template, requests[i].iterations),
                                                requests[i].arrival_s)):
            if self.adm.try_admit(foot[i], requests[i].template.minibatch):
                waiting.remove(i)
                return i
        return None

    def run(self, requests: Sequence[Request], realtime: bool = True) -> dict:
        """Serve every request; arrivals follow ``arrival_s`` on the wall clock
        (realtime) or are all present at the start.  Returns the statistics
        and one JobRecord per request."""
        if self.streams > 0:
            return self._run_streams(requests, realtime)
        ctx = self.ctx
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival_s)
        records = [JobRecord(i, requests[i].template.name, requests[i].arrival_s) for i in range(len(requests))]
        foot = {}
        for i, r in enumerate(requests):
            foot[i] = job_footprint(ctx, r.template, self.deterministic)
            if not self.adm.fits_ever(foot[i]):
                raise ValueError(f"request {i} ({r.template.name}) needs {foot[i]} bytes, more than the "
                                 f"budget of {self.adm.budget}")
            records[i].footprint = foot[i]
        waiting: List[int] = []
        nxt = 0
        active: List[ServedJob] = []
        ticks: List[_Tick] = []
        latencies: List[float] = []
        plans: Dict[int, object] = {}
        plan_key: Optional[tuple] = None
        plan_id = -1
        plan_last_tick: Dict[int, int] = {}
        peak_used, peak_jobs, total_pos, n_ticks = 0, 0, 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0

        def complete(tick: _Tick):
            nonlocal total_pos
            tick.event.synchronize()
            t_done = now()
            latencies.extend([t_done - tick.t_enq] * len(tick.members))
            total_pos += tick.positions
            for j in tick.members:
                j.completed += 1
                if j.completed == j.iterations:
                    rec = records[j.id]
                    rec.finished_s = t_done
                    rec.losses = j.losses.cpu().numpy()
                    if self.keep_state:
                        rec.state = {"a": j.a, "b": j.b}
                    self.adm.release(foot[j.id], j.positions)
            # plans that no tick in flight uses any more
            for p in [p for p, last in plan_last_tick.items() if last <= tick.index and p != plan_id]:
                plans.pop(p).close()
                plan_last_tick.pop(p)

        while nxt < len(order) or waiting or active or ticks:
            t = now()
            while nxt < len(order) and (not realtime or requests[order[nxt]].arrival_s <= t):
                waiting.append(order[nxt])
                nxt += 1
            # admission in the server's order
            while True:
                i = self._admit_next(waiting, requests, foot)
                if i is None:
                    break
                r = requests[i]
                active.append(ServedJob(ctx, r.template, i, r.iterations, self.deterministic))
                records[i].admitted_s = now()
            peak_used = max(peak_used, self.adm.used)
            peak_jobs = max(peak_jobs, len(active))
            runnable = [j for j in active if j.enqueued < j.iterations]
            if not runnable:
                if ticks:
                    complete(ticks.pop(0))
                elif nxt < len(order):
                    time.sleep(max(0.0, min(0.05, requests[order[nxt]].arrival_s - now())))
                active = [j for j in active if j.completed < j.iterations]
                continue
            # one tick: an iteration of every runnable job
            if self.batched:
                key = tuple(j.id for j in runnable)
                if key != plan_key:
                    plan_id += 1
                    plans[plan_id] = ctx.plan([j.job for j in runnable])
                    plan_key = key
            t_enq = now()
            for j in runnable:
                j.pre()
            if self.batched:
                plans[plan_id].run()
                plan_last_tick[plan_id] = n_ticks
            else:
                for j in runnable:
                    j.evaluate()
            for j in runnable:
                j.post()
            ev = torch.cuda.Event()
            ev.record()
            ticks.append(_Tick(n_ticks, t_enq, ev, runnable, sum(j.positions for j in runnable)))
            n_ticks += 1
            # keep at most `inflight` ticks outstanding: wait for the older ones
            while len(ticks) >= self.inflight:
                complete(ticks.pop(0))
            active = [j for j in active if j.completed < j.iterations]
        for p in list(plans):
            plans.pop(p).close()
        wall = now()
        ctx.sync_error()
        return _stats(requests, records, latencies, n_ticks, wall, total_pos, peak_used, peak_jobs)

    def _run_streams(self, requests: Sequence[Request], realtime: bool) -> dict:
        """Each admitted job iterates as soon as its previous iteration is
        done, on one of `streams` streams (default priority), with up to
        `inflight` iterations enqueued per job."""
        ctx = self.ctx
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival_s)
        records = [JobRecord(i, requests[i].template.name, requests[i].arrival_s) for i in range(len(requests))]
        foot = {}
        for i, r in enumerate(requests):
            foot[i] = job_footprint(ctx, r.template, self.deterministic)
            if not self.adm.fits_ever(foot[i]):
                raise ValueError(f"request {i} ({r.template.name}) needs {foot[i]} bytes, more than the "
                                 f"budget of {self.adm.budget}")
            records[i].footprint = foot[i]
        pool = [torch.cuda.Stream(device=ctx.device) for _ in range(self.streams)]
        waiting: List[int] = []
        nxt = 0
        active: List[ServedJob] = []
        pending: Dict[int, List[Tuple[float, torch.cuda.Event]]] = {}
        latencies: List[float] = []
        peak_used, peak_jobs, total_pos, n_iters, rr = 0, 0, 0, 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while nxt < len(order) or waiting or active:
            t = now()
            while nxt < len(order) and (not realtime or requests[order[nxt]].arrival_s <= t):
                waiting.append(order[nxt])
                nxt += 1
            while True:
                i = self._admit_next(waiting, requests, foot)
                if i is None:
                    break
                r = requests[i]
                job = ServedJob(ctx, r.template, i, r.iterations, self.deterministic)
                job.stream = pool[rr % len(pool)]
                rr += 1
                ready = torch.cuda.Event()
                ready.record()                        # the job's buffers were filled on this stream
                job.stream.wait_event(ready)
                active.append(job)
                pending[job.id] = []
                records[i].admitted_s = now()
            peak_used = max(peak_used, self.adm.used)
            peak_jobs = max(peak_jobs, len(active))
            progressed = False
            for job in active:
                q = pending[job.id]
                while q and q[0][1].query():          # completed iterations
                    t_enq, _ = q.pop(0)
                    latencies.append(now() - t_enq)
                    job.completed += 1
                    total_pos += job.positions
                    progressed = True
                while job.enqueued < job.iterations and len(q) < self.inflight:
                    t_enq = now()
                    with torch.cuda.stream(job.stream):
                        job.pre()
                        job.evaluate()
                        job.post()
                        ev = torch.cuda.Event()
                        ev.record()
                    q.append((t_enq, ev))
                    n_iters += 1
                    progressed = True
            for job in [j for j in active if j.completed == j.iterations]:
                rec = records[job.id]
                rec.finished_s = now()
                rec.losses = job.losses.cpu().numpy()
                if self.keep_state:
                    rec.state = {"a": job.a, "b": job.b}
                self.adm.release(foot[job.id], job.positions)
                pending.pop(job.id)
            active = [j for j in active if j.completed < j.iterations]
            if not progressed:
                if not active and nxt < len(order):
                    time.sleep(max(0.0, min(0.05, requests[order[nxt]].arrival_s - now())))
                else:
                    time.sleep(50e-6)
        torch.cuda.synchronize()
        wall = now()
        ctx.sync_error()
        return _stats(requests, records, latencies, n_iters, wall, total_pos, peak_used, peak_jobs)


def _stats(requests, records, latencies, n_ticks, wall, total_pos, peak_used, peak_jobs) -> dict:
    """Throughput and latency figures of one run (ticks: ticks, or iterations in stream mode)."""
    lat = np.array(latencies) * 1e3
    waits = np.array([r.admitted_s - r.arrival_s for r in records]) * 1e3
    turn = np.array([r.finished_s - r.arrival_s for r in records]) * 1e3
    first = min(r.arrival_s for r in requests) if requests else 0.0
    return {
        "jobs": len(requests), "ticks": n_ticks, "wall_s": wall,
        "positions": total_pos, "positions_per_s": total_pos / max(wall - first, 1e-9),
        "p50_iter_ms": float(np.percentile(lat, 50)) if lat.size else math.nan,
        "p99_iter_ms": float(np.percentile(lat, 99)) if lat.size else math.nan,
        "p50_wait_ms": float(np.percentile(waits, 50)) if waits.size else math.nan,
        "p99_wait_ms": float(np.percentile(waits, 99)) if waits.size else math.nan,
        "p50_job_ms": float(np.percentile(turn, 50)) if turn.size else math.nan,
        "p99_job_ms": float(np.percentile(turn, 99)) if turn.size else math.nan,
        "peak_hbm_bytes": peak_used, "peak_jobs": peak_jobs, "records": records,
    }


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process (seeded exponential gaps), first at 0."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    return t - t[0]


# ---------------------------------------------------------------------------
# The serving workload: Poisson arrivals of 2D, 64-slice, 128-slice and tilt-series jobs
# ---------------------------------------------------------------------------

def build_templates(ctx: Context, tilt_angles: int = 20) -> Dict[str, Template]:
    """The four job types of the serving mix (synthetic inputs, see synth)."""
    import synth
    tpl = {
        "ptycho2d_n64": scan_template(ctx, synth.ptycho2d_n64(), "ptycho2d_n64", seed=11, lr=1e-3),
        "multislice_s64": scan_template(ctx, synth.multislice_n128_s64(), "multislice_s64", seed=12),
        "multislice_s128": scan_template(ctx, synth.multislice_n128_s128(), "multislice_s128", seed=13),
    }
    scan, angles = synth.tilt_job()
    # a job's 20 iterations visit 20 of the 90 angles, spread over 180 degrees
    idx = [(k * len(angles)) // tilt_angles for k in range(tilt_angles)]
    tpl["tilt"] = tilt_template(ctx, scan, [angles[i] for i in idx], "tilt", seed=14)
    torch.cuda.synchronize()
    return tpl


def serving_requests(templates: Dict[str, Template], n_jobs: int, rate: float, seed: int = 5,
                     iterations: int = 20) -> List[Request]:
    rng = np.random.default_rng(seed)
    names = list(templates)          # job types in the dict's insertion order
    kinds = rng.integers(0, len(names), size=n_jobs)
    times = poisson_arrivals(rate, n_jobs, seed + 1)
    return [Request(float(t), templates[names[k]], iterations) for t, k in zip(times, kinds)]


# The served form of the bench line: every admitted job iterates on its own
# schedule on one of four streams; two jobs share the device at a time, four
# when at least four more are waiting.
SERVED = dict(streams=4, max_jobs=2, busy_jobs=4, busy_queue=4)


def bench_serving(args):
    """bench.py --workload serving: one JSON line.

    The served form (SERVED), the plain per-job form (one job at a time, each
    iteration its own loss_grad call) and the lockstep plan form run the same
    request trace on the wall clock; ``--seeds`` runs the served and per-job
    forms on further traces (other arrival seeds) as well.  Then the first
    quarter of the jobs arrives at once (saturation) for every form."""
    import json
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctx = Context(dev)
    t0 = time.perf_counter()
    templates = build_templates(ctx)
    setup_s = time.perf_counter() - t0
    n_jobs = getattr(args, "jobs", 200) or 200
    rate = getattr(args, "rate", 4.0) or 4.0
    seeds = [int(x) for x in str(getattr(args, "seeds", "5") or "5").split(",")]
    reqs = serving_requests(templates, n_jobs, rate, seed=seeds[0])
    # warm up every kernel the loop uses (and JIT-free first launches)
    warm = [Request(0.0, templates[k], 2) for k in sorted(templates)]
    log = lambda msg: print(f"[serving] {msg} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    log("templates ready")
    Server(ctx).run(warm, realtime=False)
    Server(ctx, **SERVED).run(warm, realtime=False)
    log("warm-up done")
    served = Server(ctx, **SERVED).run(reqs, realtime=True)
    log(f"served trace done: job p50/p99 {served['p50_job_ms']:.0f}/{served['p99_job_ms']:.0f} ms")
    per_job = Server(ctx, max_jobs=1, batched=False).run(reqs, realtime=True)
    log(f"per-job trace done: job p50/p99 {per_job['p50_job_ms']:.0f}/{per_job['p99_job_ms']:.0f} ms")
    lockstep = Server(ctx).run(reqs, realtime=True)
    log(f"lockstep-plan trace done: job p50/p99 {lockstep['p50_job_ms']:.0f}/{lockstep['p99_job_ms']:.0f} ms")
    keys = ("positions_per_s", "p50_iter_ms", "p99_iter_ms", "p50_wait_ms", "p99_wait_ms", "p50_job_ms",
            "p99_job_ms", "peak_jobs")
    pick = lambda st: {k: st[k] for k in keys}
    traces = [{"seed": seeds[0], "served": pick(served), "per_job": pick(per_job)}]
    for sd in seeds[1:]:
        r = serving_requests(templates, n_jobs, rate, seed=sd)
        a = Server(ctx, **SERVED).run(r, realtime=True)
        b = Server(ctx, max_jobs=1, batched=False).run(r, realtime=True)
        traces.append({"seed": sd, "served": pick(a), "per_job": pick(b)})
        log(f"trace seed {sd}: job p99 served {a['p99_job_ms']:.0f} ms, per-job {b['p99_job_ms']:.0f} ms")
    sat = [dataclasses.replace(r, arrival_s=0.0) for r in reqs[:max(8, n_jobs // 4)]]
    sat_served = Server(ctx, **SERVED).run(sat, realtime=False)
    log("saturated served done")
    sat_per_job = Server(ctx, max_jobs=1, batched=False).run(sat, realtime=False)
    log("saturated per-job done")
    sat_lockstep = Server(ctx).run(sat, realtime=False)
    log("saturated lockstep done")
    strip = lambda d: {k: v for k, v in d.items() if k != "records"}
    line = {
        "metric": "served multislice fwd+adjoint positions/s; p50/p99 per-iteration latency",
        "value": served["positions_per_s"], "unit": "positions/s", "n_gpus": 1, "steps": served["ticks"],
        "warmup": 1, "ms_per_step": served["wall_s"] * 1e3 / max(served["ticks"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n_jobs} jobs, Poisson arrivals {rate}/s, types uniform over 2D ptychography "
                               "(N=64, 128x128), 64-slice (N=128, 256x256x64), 128-slice (N=128, 512x512x128) "
                               "and tilt series (N=128, 256^3), "
                               "20 iterations each (minibatch or angle + Adam); jobs admitted by HBM footprint, "
                               "iterating concurrently on 4 streams, 2 at a time (4 with 4 or more waiting)"},
        "p50_iter_ms": served["p50_iter_ms"], "p99_iter_ms": served["p99_iter_ms"],
        "p50_job_ms": served["p50_job_ms"], "p99_job_ms": served["p99_job_ms"],
        "served": strip(served), "per_job_fifo": strip(per_job), "lockstep_plan": strip(lockstep),
        "traces": traces,
        "saturated": {"jobs": len(sat),
                      "served_positions_per_s": sat_served["positions_per_s"],
                      "per_job_positions_per_s": sat_per_job["positions_per_s"],
                      "lockstep_plan_positions_per_s": sat_lockstep["positions_per_s"],
                      "speedup_served": sat_served["positions_per_s"] / sat_per_job["positions_per_s"],
                      "speedup_lockstep_plan": sat_lockstep["positions_per_s"] / sat_per_job["positions_per_s"]},
        "setup_s": setup_s,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
