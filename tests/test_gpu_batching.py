"""Batched plans: graph capture replays equal eager runs; autotuner picks a split."""
import numpy as np
import pytest

import synth
from tests.gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_12686_amd import Context
    c = Context()
    yield c
    c.close()


def _runner(ctx):
    from paper_2012_12686_amd.batch import BatchRunner, to_device_scan
    specs = [(64, 4, 90, 6, "poisson"), (96, 9, 120, 5, "gaussian"), (128, 6, 150, 4, "poisson"),
             (192, 3, 220, 3, "gaussian")]
    scans = [synth.small_case(seed=700 + i, n=n, n_slices=s, lateral=lat, n_pos=p, loss=loss, strength=30.0)
             for i, (n, s, lat, p, loss) in enumerate(specs)]
    return BatchRunner(ctx, [to_device_scan(ctx, sc, seed=i) for i, sc in enumerate(scans)])


def test_graph_replays_equal_eager_runs(ctx):
    import torch
    r = _runner(ctx)
    r.build_plan()
    r.plan.run()
    torch.cuda.synchronize()
    eager = [{k: v.detach().cpu().numpy().copy() for k, v in j.out.items()} for j in r.jobs]
    r.capture(adam=False)
    for rep in range(3):
        # unrelated eager work and a synchronisation between replays
        junk = torch.ones(1 << 20, device="cuda") * rep
        junk.sum().item()
        for j in r.jobs:
            for v in j.out.values():
                v.zero_()
        r.graph.replay()
        torch.cuda.synchronize()
        ctx.sync_error()
        for j, ref in zip(r.jobs, eager):
            got = {k: v.cpu().numpy() for k, v in j.out.items()}
            assert abs(float(got["loss"]) - float(ref["loss"])) <= 1e-12 * abs(float(ref["loss"]))
            for k in ("g_a", "g_b", "g_probe", "g_shift"):
                assert rel_l2(got[k], ref[k]) < 1e-5, (rep, k)
    r.close()


def test_whole_iteration_with_adam_in_one_graph_equals_eager_iterations(ctx):
    """The captured graph holds loss, gradients, the advance of the device
    iteration count and every Adam step: three replays give the same objects
    and moments, bit for bit, as three eager iterations of an identical
    runner (deterministic jobs, so both evaluate with the same split), and
    the count reads 3 on both."""
    import dataclasses
    import torch
    from paper_2012_12686_amd.batch import BatchRunner, to_device_scan
    specs = [(64, 4, 90, 6, "poisson"), (128, 6, 150, 4, "gaussian"), (192, 3, 220, 3, "poisson")]
    scans = [synth.small_case(seed=710 + i, n=n, n_slices=s, lateral=lat, n_pos=p, loss=loss, strength=30.0)
             for i, (n, s, lat, p, loss) in enumerate(specs)]

    def runner():
        ds = [to_device_scan(ctx, sc, seed=i) for i, sc in enumerate(scans)]
        ds = [dataclasses.replace(d, geom=dataclasses.replace(d.geom, deterministic=True)) for d in ds]
        return BatchRunner(ctx, ds, lr=1e-6)

    eager, graph = runner(), runner()
    eager.build_plan()
    graph.build_plan()
    graph.capture(adam=True)
    for _ in range(3):
        eager.step(adam=True)
        graph.step_graph()
    torch.cuda.synchronize()
    ctx.sync_error()
    assert int(eager.t_dev) == 3 and int(graph.t_dev) == 3
    moved = 0.0
    for se, sg, sc in zip(eager.scans, graph.scans, scans):
        for k in ("a", "b", "m_a", "v_a", "m_b", "v_b"):
            assert torch.equal(getattr(se, k), getattr(sg, k)), k
        moved += float((se.a - torch.as_tensor(sc.eval_obj_a, dtype=torch.float32, device=se.a.device))
                       .abs().max())
    assert moved > 0
    eager.close()
    graph.close()


def test_autotuner_sets_a_supported_split(ctx, tmp_path):
    from paper_2012_12686_amd.autotune import SPLITS, autotune
    r = _runner(ctx)
    res = autotune(ctx, r.jobs, reps=1, cache_path=str(tmp_path / "tune.json"))
    assert set(res) == {64, 96, 128, 192}
    for n, v in res.items():
        assert v["split"] in SPLITS[n] and not v["cached"]
    again = autotune(ctx, r.jobs, reps=1, cache_path=str(tmp_path / "tune.json"))
    assert all(v["cached"] for v in again.values())
    for n in res:
        ctx.set_split(n, 0)
    r.close()


# the smallest job of each probe size in the 32-scan mix (positions x slices x N^2)
COMPARED_JOBS = {64: 14, 96: 17, 128: 13, 192: 18}


def test_mixed_scan_plan_matches_oracle_on_one_job_per_probe_size(ctx):
    """The 32-scan mix in the launch configuration the benchmark times
    (autotuned split per probe size, one captured plan over every job's whole
    position list), at half the true object.  The smallest job of each probe
    size gets measured data from the oracle at its true object (Poisson for
    the Poisson-loss jobs), and its intensities, loss and every gradient are
    compared with the oracle (no input comes from the GPU).  The other jobs'
    data are seeded Poisson noise at the probe's mean level: they share the
    persistent launches but do not enter the compared jobs' outputs.  The
    outputs FP32_LIMITED['mix-half-object'] lists for each compared job are
    held to its guard; the others to the tolerance."""
    import torch
    from oracle import multislice as om
    from paper_2012_12686_amd.batch import BatchRunner, DeviceScan
    from paper_2012_12686_amd import Geometry
    from tests.gpu_helpers import FP32_LIMITED, TOL_I, assert_grads, f32, loss_tolerance, xfail_if
    scans = synth.mixed_scan_jobs()
    assert {scans[j].n: j for j in COMPARED_JOBS.values()} == {n: j for n, j in COMPARED_JOBS.items()}
    dev = ctx.device
    t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    rng = np.random.default_rng(4040)
    dscans, refs = [], {}
    for i, sc in enumerate(scans):
        geom = om.Geometry.from_scan(sc)
        a64, b64, p64 = f32(0.5 * sc.obj_a), f32(0.5 * sc.obj_b), f32(sc.probe)
        corner_np, shift_np = synth.split_positions(np.asarray(sc.positions, dtype=np.float64))
        shift_np = f32(shift_np)
        if i in COMPARED_JOBS.values():
            i_true = om.forward(geom, sc.obj_a, sc.obj_b, sc.probe, np.asarray(sc.positions, dtype=np.float64))
            if sc.loss == "poisson":
                i_true = np.random.default_rng(500 + i).poisson(i_true)
            im = f32(i_true)
            pos = corner_np + shift_np
            refs[i] = (om.forward(geom, a64, b64, p64, pos), om.loss_grad(geom, a64, b64, p64, pos, im), geom, im)
        else:
            level = float(np.sum(np.abs(sc.probe) ** 2)) / sc.n ** 2
            im = rng.poisson(level, size=(len(sc.positions), sc.n, sc.n))
        a, b = t(a64, torch.float32), t(b64, torch.float32)
        z = torch.zeros_like
        dscans.append(DeviceScan(Geometry.from_scan(sc), a, b, t(p64, torch.complex64), t(corner_np, torch.int32),
                                 t(shift_np, torch.float32), t(im, torch.float32), z(a), z(a), z(b), z(b)))
    r = BatchRunner(ctx, dscans)
    try:
        ctx.autotune(r.jobs, reps=1)
        for i in COMPARED_JOBS.values():
            sc = scans[i]
            r.jobs[i].out["intensity"] = torch.empty((len(sc.positions), sc.n, sc.n), dtype=torch.float32,
                                                     device=dev)
        r.build_plan()
        r.capture(adam=False)
        r.graph.replay()
        torch.cuda.synchronize()
        ctx.sync_error()
        msgs = []
        for n, i in COMPARED_JOBS.items():
            i_ref, (L, ga, gb, gp, gs), geom, im = refs[i]
            got = {k: v.cpu().numpy() for k, v in r.jobs[i].out.items()}
            e_i = rel_l2(got["intensity"], i_ref)
            print(f"job {i} (N={n}, S={scans[i].n_slices}, {len(scans[i].positions)} positions): "
                  f"intensity rel-L2 {e_i:.3e}")
            assert e_i <= TOL_I, (n, e_i)
            assert abs(float(got["loss"]) - L) <= loss_tolerance(geom, i_ref, im), (n, float(got["loss"]), L)
            assert np.linalg.norm(gs) > 0
            limited = FP32_LIMITED["mix-half-object"]["outputs"][i]
            pairs = [(f"N={n} {k}", got[k], ref) for k, ref in (("g_a", ga), ("g_b", gb), ("g_probe", gp),
                                                                 ("g_shift", gs))]
            assert_grads([q for q in pairs if q[0].split()[1] not in limited])
            msgs += assert_grads([q for q in pairs if q[0].split()[1] in limited], "mix-half-object", defer=True)
        xfail_if(msgs)
    finally:
        for n in (64, 96, 128, 192):
            ctx.set_split(n, 0)
        r.close()
