"""Benchmark: multislice forward + adjoint throughput on one MI355X.

Workload (default): 128x128 probe, 64 slices of delta/beta at 10 nm and
10 keV, a 256x256 object of random ellipsoids, 400 positions on a jittered
20x20 raster processed in minibatches of 50, Poisson loss on 1e4-photon
patterns, evaluated at delta = beta = 0 with the true probe and positions.
One step = one minibatch through the whole path: chunk gather, Fourier
shift, slice modulation, Fresnel propagation, far field, loss and the
reverse sweep with checkpoint re-anchoring and gradient scatter.

Prints ONE JSON line.  `value` = positions per second of the timed steps
(inputs already resident in HBM).  `roofline` prices the dominant kernel
(the fused multislice kernel) against HBM peak using algorithmic bytes per
position 24 N^2 S + 4 N^2 + 16 N^2 ceil(S/16); its duration comes from HIP
events recorded around each of its launches on its own stream.
`cpu_baseline` times the FP64 oracle on consecutive full minibatches of the same
workload on the host cores.

Measured data: Poisson(I_true) with I_true from this library's forward
model at the ground-truth object (synthetic data, not a parity claim).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3       # MI355X vector FP32, published


def algorithmic_bytes_per_position(n, s, c=16):
    return 24 * n * n * s + 4 * n * n + 16 * n * n * math.ceil(s / c)


def algorithmic_flops_per_position(n, s):
    return 6 * s * 5 * n * n * math.log2(n * n) + 60 * n * n * s


def kernel_source_hash():
    """Hash of the sources the measured kernel is compiled from (the tile
    engine, the kernel templates and its instantiation unit)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2012_12686_amd", "csrc")
    for f in ("context.hpp", "fastmath.hpp", "multislice_impl.hpp", "tile.hpp", "ms_n128_k4.hip"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counters, if they were
    taken on the kernel sources as they are now; else None."""
    path = os.path.join(ROOT, "profiles", "multislice_n128_s64_b50_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("csrc_sha256") != kernel_source_hash():
        return None
    return rec["read_bytes"] + rec["write_bytes"]


def measured_copy_gbs(reps=10):
    """Bandwidth of a plain 1 GiB device-to-device copy (read + write bytes
    over its event-timed duration): the practical HBM ceiling next to the
    published 8 TB/s.  Run after the timed region; the buffers are freed."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2 * src.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def with_copy_peak(line):
    """Add the measured copy ceiling to an HBM roofline record."""
    r = line.get("roofline")
    if r and r.get("unit") == "GB/s":
        c = measured_copy_gbs()
        r["measured_copy_GBps"] = c
        r["frac_of_measured_copy"] = r["achieved"] / c
    return line


def cpu_baseline(sc, mb, i_meas_np, min_seconds=10.0):
    """Time the FP64 oracle (fwd + loss + adjoint) on consecutive minibatches
    of the same scan, at the GPU's evaluation point, until at least
    ``min_seconds`` of work (one minibatch at least, every minibatch at most)."""
    from oracle import multislice as om
    geom = om.Geometry.from_scan(sc)
    z = np.zeros(sc.obj_shape)
    n_mb = len(sc.positions) // mb
    done, k, dt = 0, 0, 0.0
    while k < n_mb and (k == 0 or dt < min_seconds):
        sl = slice(k * mb, (k + 1) * mb)
        t0 = time.perf_counter()
        om.loss_grad(geom, z, z, sc.probe, sc.positions[sl], i_meas_np[sl].astype(np.float64))
        dt += time.perf_counter() - t0
        done += mb
        k += 1
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": done / dt, "unit": "positions/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} consecutive minibatch{'es' if k > 1 else ''} of {mb} positions (N=128, S=64), "
                      f"FP64 fwd+loss+adjoint, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--split", type=int, default=0,
                    help="workgroups per position (0 = the library's automatic choice)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM counters)")
    ap.add_argument("--workload", default="multislice", choices=["multislice", "batching", "serving", "sparse", "priors", "mdh", "differentiation"],
                    help="multislice: the 64-slice minibatch (default line); batching: 32 mixed scans, "
                         "batched vs per-job; serving: the request loop")
    ap.add_argument("--ckpt", type=int, default=16, help="slice checkpoint interval of the adjoint")
    ap.add_argument("--deterministic", action="store_true", help="FP64 ordered object-gradient sums")
    ap.add_argument("--modes", type=int, default=1, help="incoherent probe modes (Eq. multimode)")
    ap.add_argument("--defocus", type=float, default=0.0,
                    help="probe defocus in metres: data simulated at this defocus, evaluated 10%% away, "
                         "with the defocus gradient (single probe mode)")
    ap.add_argument("--jobs", type=int, default=200, help="serving: number of requests")
    ap.add_argument("--rate", type=float, default=4.0, help="serving: Poisson arrival rate (jobs/s)")
    ap.add_argument("--seeds", default="5",
                    help="serving: arrival seeds, comma-separated; the served and per-job forms run on each trace")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is a "
              f"design note, not built", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")    # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 4}))
        return

    if args.workload == "batching":
        return bench_batching(args)
    if args.workload == "serving":
        from paper_2012_12686_amd.serve import bench_serving
        return bench_serving(args)
    if args.workload == "sparse":
        return bench_sparse(args)
    if args.workload == "priors":
        return bench_priors(args)
    if args.workload == "mdh":
        return bench_mdh(args)
    if args.workload == "differentiation":
        return bench_differentiation(args)

    import synth
    from paper_2012_12686_amd import Context, Geometry, split_positions

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sc = synth.multislice_n128_s64()
    n, s = sc.n, sc.n_slices
    mb = sc.minibatch
    n_mb = len(sc.positions) // mb
    ctx = Context(dev)
    geom = Geometry.from_scan(sc, ckpt_every=args.ckpt, deterministic=args.deterministic)
    if args.split:
        ctx.set_split(n, args.split)

    to_t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    true_a, true_b = to_t(sc.obj_a, torch.float32), to_t(sc.obj_b, torch.float32)
    n_modes = args.modes
    probes = to_t(synth.probe_modes(sc.probe, n_modes, seed=11), torch.complex64)
    probe = probes[0]
    corner, shift = split_positions(to_t(sc.positions, torch.float64))
    # synthetic measurements: Poisson counts of the forward model at the truth
    # (summed over the probe modes)
    defocus = args.defocus if n_modes == 1 else 0.0

    def simulate(p, sl):
        if defocus:
            return ctx.forward_defocus(geom, true_a, true_b, p, corner[sl], shift[sl], defocus)
        return ctx.forward(geom, true_a, true_b, p, corner[sl], shift[sl])

    i_true = torch.cat([sum(simulate(p, slice(k * mb, (k + 1) * mb)) for p in probes) for k in range(n_mb)])
    rng = np.random.default_rng(2)
    i_meas_np = rng.poisson(i_true.cpu().numpy().astype(np.float64)).astype(np.float32)
    i_meas = to_t(i_meas_np, torch.float32)

    # evaluation point: delta = beta = 0
    a = torch.zeros_like(true_a)
    b = torch.zeros_like(true_b)
    if n_modes == 1:
        ws = ctx.workspace(geom, mb)
    else:
        ws = torch.empty(ctx.modes_workspace_size(geom, mb, n_modes), dtype=torch.uint8, device=dev)
    out = {"loss": torch.empty((), dtype=torch.float64, device=dev),
           "g_a": torch.empty_like(a), "g_b": torch.empty_like(b),
           "g_probe": torch.empty_like(probe if n_modes == 1 else probes),
           "g_shift": torch.empty((mb, 2), dtype=torch.float32, device=dev)}
    if defocus:
        out["g_defocus"] = torch.empty((), dtype=torch.float64, device=dev)

    def step(k):
        sl = slice((k % n_mb) * mb, (k % n_mb + 1) * mb)
        if defocus:
            ctx.loss_grad_defocus(geom, a, b, probe, corner[sl], shift[sl], 1.1 * defocus, i_meas[sl], out=out,
                                  workspace=ws)
        elif n_modes == 1:
            ctx.loss_grad(geom, a, b, probe, corner[sl], shift[sl], i_meas[sl], out=out, workspace=ws)
        else:
            ctx.loss_grad_modes(geom, a, b, probes, corner[sl], shift[sl], i_meas[sl], out=out, workspace=ws)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ctx.sync_error()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ctx.profile_start(args.steps * 2 * n_modes + 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record()
        step(k)
        ends[k].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, kern_n = ctx.profile_stop()
    ctx.sync_error()

    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / args.steps
    lat = sorted(st.elapsed_time(en) for st, en in zip(starts, ends))
    p50 = float(np.percentile(lat, 50))
    p99 = float(np.percentile(lat, 99))
    value = mb * args.steps / elapsed

    kern_avg_s = kern_ms / max(kern_n, 1) / 1e3
    bytes_launch = algorithmic_bytes_per_position(n, s, args.ckpt) * mb
    if n_modes > 1:
        # per mode a forward launch (object read, checkpoints and exit wave
        # written, intensity written) and a loss launch resuming from them
        # (exit wave and summed intensity read besides the one-launch bytes)
        per_mode = algorithmic_bytes_per_position(n, s, args.ckpt) + 24 * n * n
        bytes_launch = per_mode * mb / 2
    achieved_gbs = bytes_launch / kern_avg_s / 1e9
    flops_launch = algorithmic_flops_per_position(n, s) * mb
    achieved_tflops = flops_launch / kern_avg_s / 1e12

    traffic = measured_traffic() if n_modes == 1 else None
    step_gbs = value * bytes_launch * (1 if n_modes == 1 else 2 * n_modes) / mb / 1e9
    line = {
        "metric": "multislice fwd+adjoint positions/s, % HBM roofline; p50/p99 iter latency",
        "value": value,
        "unit": "positions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "multislice ptychography N=128 S=64 object 256x256x64 (10 nm, 10 keV), "
                               "minibatch 50 of 400 positions, Poisson 1e4 photons, fwd+loss+adjoint"
                               + (f", {n_modes} incoherent probe modes" if n_modes > 1 else "")
                               + (f", probe defocused (data at {defocus:g} m, evaluated at {1.1 * defocus:g} m) "
                                  f"with the defocus gradient" if defocus else ""),
                   "global_batch": mb, "seq_len": s, "parallelism": "none"},
        "p50_iter_ms": p50,
        "p99_iter_ms": p99,
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "multislice_kernel<N=128, delta/beta, Poisson, loss+adjoint>" if n_modes == 1 else
                               "multislice_kernel<N=128>: forward and loss+adjoint launches, averaged",
                     "kernel_avg_ms": kern_avg_s * 1e3, "kernel_launches": kern_n,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     # the measured HBM bytes of one launch over its duration
                     "traffic_GBps": traffic / kern_avg_s / 1e9 if traffic else None,
                     # whole step: positions/s x algorithmic bytes per position
                     "step_effective_GBps": step_gbs, "step_frac": step_gbs / HBM_PEAK_GBS,
                     "fp32_tflops": achieved_tflops, "fp32_frac": achieved_tflops / FP32_PEAK_TFLOPS},
    }
    if not args.no_cpu_baseline and n_modes == 1 and not defocus:
        line["cpu_baseline"] = cpu_baseline(sc, mb, i_meas_np)
    print(json.dumps(with_copy_peak(line)), flush=True)
    ctx.close()


def bench_sparse(args):
    """Sparse multislice (two layers 10 um apart, N = 128, 12 keV): loss and
    gradients including the gap gradient, one minibatch of 202 positions per
    step (adorym_loss_grad_gaps)."""
    import torch

    import synth
    from paper_2012_12686_amd import Context, Geometry, split_positions

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sc = synth.sparse_multislice()
    n, s, mb = sc.n, sc.n_slices, sc.minibatch
    n_mb = len(sc.positions) // mb
    ctx = Context(dev)
    geom = Geometry.from_scan(sc, ckpt_every=args.ckpt)
    to_t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    true_a, true_b = to_t(sc.obj_a, torch.float32), to_t(sc.obj_b, torch.float32)
    probe = to_t(sc.probe, torch.complex64)
    corner, shift = split_positions(to_t(sc.positions, torch.float64))
    gaps_true, gaps = to_t(sc.gaps, torch.float64), to_t(sc.eval_gaps, torch.float64)
    i_true = torch.cat([ctx.forward_gaps(geom, true_a, true_b, probe, corner[k * mb:(k + 1) * mb],
                                         shift[k * mb:(k + 1) * mb], gaps_true) for k in range(n_mb)])
    i_meas_np = np.random.default_rng(2).poisson(i_true.cpu().numpy().astype(np.float64)).astype(np.float32)
    i_meas = to_t(i_meas_np, torch.float32)
    a, b = torch.zeros_like(true_a), torch.zeros_like(true_b)
    ws = torch.empty(ctx.gaps_workspace_size(geom, mb), dtype=torch.uint8, device=dev)
    out = {"loss": torch.empty((), dtype=torch.float64, device=dev), "g_a": torch.empty_like(a),
           "g_b": torch.empty_like(b), "g_probe": torch.empty_like(probe),
           "g_shift": torch.empty((mb, 2), dtype=torch.float32, device=dev),
           "g_gaps": torch.empty((s - 1,), dtype=torch.float64, device=dev)}

    def step(k):
        sl = slice((k % n_mb) * mb, (k % n_mb + 1) * mb)
        ctx.loss_grad_gaps(geom, a, b, probe, corner[sl], shift[sl], gaps, i_meas[sl], out=out, workspace=ws)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ctx.sync_error()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ctx.profile_start(args.steps + 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record()
        step(k)
        ends[k].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, kern_n = ctx.profile_stop()
    ctx.sync_error()
    elapsed = t1 - t0
    lat = sorted(st.elapsed_time(en) for st, en in zip(starts, ends))
    kern_avg_s = kern_ms / max(kern_n, 1) / 1e3
    bytes_launch = algorithmic_bytes_per_position(n, s, args.ckpt) * mb
    achieved_gbs = bytes_launch / kern_avg_s / 1e9
    line = {
        "metric": "sparse multislice fwd+adjoint (with gap gradient) positions/s, % HBM roofline",
        "value": mb * args.steps / elapsed, "unit": "positions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "sparse multislice N=128, 2 layers 10 um apart, object 512x512x2 (7.3 nm, "
                               "12 keV), minibatch 202 of 1414 positions, Poisson 1e5 photons, "
                               "fwd+loss+adjoint+gap gradient", "global_batch": mb, "seq_len": s,
                   "parallelism": "none"},
        "p50_iter_ms": float(np.percentile(lat, 50)), "p99_iter_ms": float(np.percentile(lat, 99)),
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "multislice_kernel<N=128, delta/beta, Poisson, loss+adjoint, unequal gaps>",
                     "kernel_avg_ms": kern_avg_s * 1e3, "kernel_launches": kern_n,
                     "algorithmic_bytes_per_launch": bytes_launch},
    }
    if not args.no_cpu_baseline:
        from oracle import multislice as om
        sample = 16
        og = om.Geometry(n, s, sc.wavelength_m, sc.pixel_m, sc.slice_dz_m, sc.obj_repr, sc.loss, sc.eps,
                         gaps=sc.eval_gaps)
        z = np.zeros(sc.obj_a.shape)
        t = time.perf_counter()
        om.loss_grad_gaps(og, z, z, sc.probe, sc.positions[:sample], i_meas_np[:sample].astype(np.float64))
        dt = time.perf_counter() - t
        line["cpu_baseline"] = {"value": sample / dt, "unit": "positions/s", "cores": om._WORKERS, "kind": "oracle",
                                "sample": f"FP64 oracle loss_grad_gaps on {sample} positions of the first minibatch"}
    print(json.dumps(with_copy_peak(line)), flush=True)
    ctx.close()


def bench_differentiation(args):
    """The 128-slice differentiation workload: 512 x 512 x 128 object, 128
    probe, minibatches of 200 of 1024 positions, checkpoints every 16 slices,
    evaluated at half the true object, a perturbed probe and nominal
    positions (the true ones are shifted by up to 1 px)."""
    import torch

    import synth
    from paper_2012_12686_amd import Context, Geometry, split_positions

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sc = synth.multislice_n128_s128()
    n, s, mb = sc.n, sc.n_slices, sc.minibatch
    n_mb = len(sc.positions) // mb
    ctx = Context(dev)
    geom = Geometry.from_scan(sc, ckpt_every=args.ckpt, deterministic=args.deterministic)
    if args.split:
        ctx.set_split(n, args.split)
    to_t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    ta, tb = to_t(sc.obj_a, torch.float32), to_t(sc.obj_b, torch.float32)
    corner_t, shift_t = split_positions(to_t(sc.positions, torch.float64))
    probe_t = to_t(sc.probe, torch.complex64)
    i_meas = torch.cat([ctx.forward(geom, ta, tb, probe_t, corner_t[k * mb:(k + 1) * mb],
                                    shift_t[k * mb:(k + 1) * mb]) for k in range(n_mb)])
    del ta, tb
    a, b = to_t(sc.eval_obj_a, torch.float32), to_t(sc.eval_obj_b, torch.float32)
    probe = to_t(sc.eval_probe, torch.complex64)
    corner, shift = split_positions(to_t(sc.eval_positions, torch.float64))
    ws = ctx.workspace(geom, mb)
    out = {"loss": torch.empty((), dtype=torch.float64, device=dev), "g_a": torch.empty_like(a),
           "g_b": torch.empty_like(b), "g_probe": torch.empty_like(probe),
           "g_shift": torch.empty((mb, 2), dtype=torch.float32, device=dev)}

    def step(k):
        sl = slice((k % n_mb) * mb, (k % n_mb + 1) * mb)
        ctx.loss_grad(geom, a, b, probe, corner[sl], shift[sl], i_meas[sl], out=out, workspace=ws)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ctx.sync_error()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ctx.profile_start(args.steps + 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record()
        step(k)
        ends[k].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms, kern_n = ctx.profile_stop()
    ctx.sync_error()
    lat = sorted(st.elapsed_time(en) for st, en in zip(starts, ends))
    kern_avg_s = kern_ms / max(kern_n, 1) / 1e3
    bytes_launch = algorithmic_bytes_per_position(n, s, args.ckpt) * mb
    achieved = bytes_launch / kern_avg_s / 1e9
    flops = algorithmic_flops_per_position(n, s) * mb / kern_avg_s / 1e12

    # The same minibatches through the torch.autograd.Function front end
    # (default form: loss in forward, the reverse sweep from the kept
    # checkpoints when backward runs), timed apart from the line's value.
    from paper_2012_12686_amd import multislice_loss
    leaves = [t.clone().requires_grad_() for t in (a, b, probe)]
    pos_all = to_t(sc.eval_positions, torch.float64)

    def ag_step(k):
        sl = slice((k % n_mb) * mb, (k % n_mb + 1) * mb)
        pos = pos_all[sl].clone().requires_grad_()
        for t in leaves:
            t.grad = None
        multislice_loss(*leaves, pos, i_meas[sl], geom, ctx).backward()

    n_ag = min(args.steps, 12)
    for k in range(2):
        ag_step(k)
    torch.cuda.synchronize()
    t_ag = time.perf_counter()
    for k in range(n_ag):
        ag_step(k)
    torch.cuda.synchronize()
    ag_ms = 1e3 * (time.perf_counter() - t_ag) / n_ag
    ctx.sync_error()
    del leaves

    line = {
        "metric": "multislice fwd+adjoint positions/s, % HBM roofline (differentiation workload)",
        "value": mb * args.steps / elapsed, "unit": "positions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "multislice N=128 S=128 object 512x512x128 (10 nm, 10 keV), minibatch 200 of "
                               "1024 positions, Gaussian loss, checkpoints every 16 slices, gradients for "
                               "delta, beta, probe and shifts", "global_batch": mb, "seq_len": s,
                   "parallelism": "none"},
        "p50_iter_ms": float(np.percentile(lat, 50)), "p99_iter_ms": float(np.percentile(lat, 99)),
        "autograd": {"ms_per_step": ag_ms, "positions_per_s": mb / ag_ms * 1e3, "steps": n_ag,
                     "form": "multislice_loss(...).backward(): adorym_loss_fwd in forward, adorym_loss_bwd "
                             "in backward"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "multislice_kernel<N=128, delta/beta, Gaussian, loss+adjoint>",
                     "kernel_avg_ms": kern_avg_s * 1e3, "kernel_launches": kern_n,
                     "algorithmic_bytes_per_launch": bytes_launch, "fp32_tflops": flops,
                     "fp32_frac": flops / FP32_PEAK_TFLOPS},
    }
    if not args.no_cpu_baseline:
        from oracle import multislice as om
        sample = 8
        og = om.Geometry.from_scan(sc)
        im = i_meas[:sample].cpu().numpy().astype(np.float64)
        t = time.perf_counter()
        om.loss_grad(og, sc.eval_obj_a, sc.eval_obj_b, sc.eval_probe, np.asarray(sc.eval_positions)[:sample], im)
        dt = time.perf_counter() - t
        line["cpu_baseline"] = {"value": sample / dt, "unit": "positions/s", "cores": om._WORKERS, "kind": "oracle",
                                "sample": f"FP64 oracle loss_grad on {sample} positions of the first minibatch, "
                                          f"{dt:.1f} s"}
    print(json.dumps(with_copy_peak(line)), flush=True)
    ctx.close()


def bench_mdh(args):
    """Multi-distance holography as near-field tiles: 25 tiles x 4 distances
    of a 512 x 512 complex object per step (adorym_loss_grad_nearfield with
    the distance gradient)."""
    import torch

    import synth
    from paper_2012_12686_amd import Context, Geometry, split_positions

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sc, dists, idx = synth.mdh_tiles()
    n, s, b = sc.n, sc.n_slices, len(sc.positions)
    ctx = Context(dev)
    geom = Geometry.from_scan(sc, ckpt_every=args.ckpt)
    to_t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    probe = to_t(sc.probe, torch.complex64)
    corner, shift = split_positions(to_t(sc.positions, torch.float64))
    td, ti = to_t(dists, torch.float64), to_t(idx, torch.int32)
    i_true = ctx.forward_nearfield(geom, to_t(sc.obj_a, torch.float32), to_t(sc.obj_b, torch.float32), probe,
                                   corner, shift, td, ti)
    i_meas_np = np.random.default_rng(2).poisson(i_true.cpu().numpy().astype(np.float64)).astype(np.float32)
    i_meas = to_t(i_meas_np, torch.float32)
    a, b_ = to_t(sc.eval_obj_a, torch.float32), to_t(sc.eval_obj_b, torch.float32)
    ev = td * 1.02
    ws = torch.empty(ctx.nearfield_workspace_size(geom, b, len(dists)), dtype=torch.uint8, device=dev)
    out = {"loss": torch.empty((), dtype=torch.float64, device=dev), "g_a": torch.empty_like(a),
           "g_b": torch.empty_like(b_), "g_probe": torch.empty_like(probe),
           "g_shift": torch.empty((b, 2), dtype=torch.float32, device=dev),
           "g_dist": torch.empty((len(dists),), dtype=torch.float64, device=dev)}

    def step():
        ctx.loss_grad_nearfield(geom, a, b_, probe, corner, shift, ev, ti, i_meas, out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.sync_error()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ctx.profile_start(args.steps + 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record()
        step()
        ends[k].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms, kern_n = ctx.profile_stop()
    ctx.sync_error()
    lat = sorted(st.elapsed_time(en) for st, en in zip(starts, ends))
    kern_avg_s = kern_ms / max(kern_n, 1) / 1e3
    # per position: the far-field model's bytes plus the detector spectrum stashed and reread
    bytes_launch = (algorithmic_bytes_per_position(n, s, args.ckpt) + 16 * n * n) * b
    achieved = bytes_launch / kern_avg_s / 1e9
    line = {
        "metric": "near-field (multi-distance holography tiles) fwd+adjoint positions/s, % HBM roofline",
        "value": b * args.steps / elapsed, "unit": "positions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "multi-distance holography: 512x512 complex object, 1 um, 17.5 keV, 25 tiles of "
                               "128x128 at 4 distances (0.4-1.0 m), plane wave, Poisson, paraxial near field, "
                               "fwd+loss+adjoint+distance gradient", "global_batch": b, "seq_len": s,
                   "parallelism": "none"},
        "p50_iter_ms": float(np.percentile(lat, 50)), "p99_iter_ms": float(np.percentile(lat, 99)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "multislice_kernel<N=128, real/imag, Poisson, loss+adjoint, near field>",
                     "kernel_avg_ms": kern_avg_s * 1e3, "kernel_launches": kern_n,
                     "algorithmic_bytes_per_launch": bytes_launch},
    }
    if not args.no_cpu_baseline:
        from oracle import multislice as om
        og = om.Geometry.from_scan(sc)
        t = time.perf_counter()
        om.loss_grad_nearfield(og, sc.eval_obj_a, sc.eval_obj_b, sc.probe, sc.positions,
                               i_meas_np.astype(np.float64), dists * 1.02, idx)
        dt = time.perf_counter() - t
        line["cpu_baseline"] = {"value": b / dt, "unit": "positions/s", "cores": om._WORKERS, "kind": "oracle",
                                "sample": f"FP64 oracle loss_grad_nearfield on the whole 100-position step, {dt:.1f} s"}
    print(json.dumps(with_copy_peak(line)), flush=True)
    ctx.close()


def bench_priors(args):
    """Object priors (l1 + TV, value and gradient added onto a data gradient)
    on the 512 x 512 x 128 delta/beta object of the 128-slice workload."""
    import torch

    import synth
    from paper_2012_12686_amd import Context

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sc = synth.multislice_n128_s128()
    ctx = Context(dev)
    a = torch.as_tensor(sc.obj_a, dtype=torch.float32, device=dev).contiguous()
    b = torch.as_tensor(sc.obj_b, dtype=torch.float32, device=dev).contiguous()
    out = {"g_a": torch.zeros_like(a), "g_b": torch.zeros_like(b)}
    n_vox = a.numel()

    def step():
        ctx.prior_grad("delta_beta", a, b, l1_a=0.05, l1_b=0.5, tv=0.02, out=out, accumulate=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.sync_error()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(args.steps):
        step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    avg_s = sum(lat) / len(lat) / 1e3
    bytes_call = 24 * n_vox          # read delta, beta, g_a, g_b; write g_a, g_b
    achieved = bytes_call / avg_s / 1e9
    line = {
        "metric": "object prior (l1 + TV) value+gradient voxels/s, % HBM roofline",
        "value": n_vox * args.steps / elapsed, "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "l1 (delta, beta) + total variation on the 512x512x128 delta/beta object, "
                               "gradient added onto the data gradient", "voxels": n_vox},
        "p50_iter_ms": float(np.percentile(lat, 50)), "p99_iter_ms": float(np.percentile(lat, 99)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "prior_grad_kernel<delta/beta> + its FP64 partial sum",
                     "algorithmic_bytes_per_launch": bytes_call, "call_avg_ms": avg_s * 1e3},
    }
    if not args.no_cpu_baseline:
        from oracle import regularizers as orr
        sub = (16, 512, 512)
        aa, bb = sc.obj_a[:sub[0]], sc.obj_b[:sub[0]]
        t = time.perf_counter()
        orr.value(aa, bb, "delta_beta", 0.05, 0.5, 0.02)
        orr.grad(aa, bb, "delta_beta", 0.05, 0.5, 0.02)
        dt = time.perf_counter() - t
        line["cpu_baseline"] = {"value": aa.size / dt, "unit": "voxels/s", "cores": 1, "kind": "oracle",
                                "sample": f"FP64 NumPy oracle value + gradient on 16 of the 128 slices, {dt:.1f} s"}
    print(json.dumps(with_copy_peak(line)), flush=True)
    ctx.close()


def bench_batching(args):
    """32 independent scans (N in {64, 96, 128, 192}, S in 1..64, 50..500
    positions): one iteration = loss and gradients of every job and an Adam
    step on every object.  Times the plain per-job form, the batched plan
    (eager) and the whole iteration captured in one graph."""
    import torch

    import synth
    from paper_2012_12686_amd import Context
    from paper_2012_12686_amd.autotune import autotune
    from paper_2012_12686_amd.batch import BatchRunner, to_device_scan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctx = Context(dev)
    t0 = time.perf_counter()
    scans = [to_device_scan(ctx, sc, seed=i) for i, sc in enumerate(synth.mixed_scan_jobs())]
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    runner = BatchRunner(ctx, scans)
    npos = runner.positions()
    tune = autotune(ctx, runner.jobs, reps=1)
    runner.build_plan()
    runner.capture(adam=True)

    def timed(fn, reps):
        for _ in range(max(1, args.warmup // 2)):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record()
        for r in range(reps):
            fn()
            ev[r + 1].record()
        torch.cuda.synchronize()
        ctx.sync_error()
        lat = [ev[r].elapsed_time(ev[r + 1]) for r in range(reps)]
        return sum(lat) / reps, lat

    reps = max(2, min(args.steps, 8))
    # every form does the whole iteration: loss and gradients of every job,
    # then Adam on every object (inside the graph for the captured form)
    ms_job, _ = timed(lambda: runner.run_per_job(adam=True), reps)
    ms_plan, _ = timed(lambda: runner.step(adam=True), reps)
    ms_graph, lat = timed(lambda: runner.step_graph(), reps)
    line = {
        "metric": "batched multislice fwd+adjoint positions/s (32 mixed scans)",
        "value": npos / (ms_graph / 1e3), "unit": "positions/s", "n_gpus": 1, "steps": reps,
        "warmup": args.warmup, "ms_per_step": ms_graph, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "32 scans, N in {64,96,128,192}, S in 1..64, 50..500 positions each, "
                               "full-batch loss+gradient and Adam per iteration, one captured graph",
                   "positions": npos},
        "per_job_ms": ms_job, "plan_eager_ms": ms_plan, "plan_graph_ms": ms_graph,
        "speedup_vs_per_job": ms_job / ms_graph,
        "p50_iter_ms": float(np.percentile(lat, 50)), "p99_iter_ms": float(np.percentile(lat, 99)),
        "autotune": {str(k): v for k, v in tune.items()}, "prep_s": prep_s,
    }
    print(json.dumps(with_copy_peak(line)), flush=True)
    runner.close()
    ctx.close()


if __name__ == "__main__":
    main()
