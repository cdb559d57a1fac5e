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
    r.capture()
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


def test_mixed_scan_plan_matches_oracle_on_sampled_positions(ctx):
    """The 32-scan mix in the launch configuration the benchmark times
    (autotuned split per probe size, one captured plan), at half the true
    object so that shift gradients do not vanish, with seeded Poisson data
    (no input comes from the GPU).  A position's shift gradient depends on
    that position alone: the oracle evaluates it on a one-position batch,
    whose loss is normalised by N^2 instead of B N^2, so the plan's value is
    that divided by B.  Sampled: first, middle and last position of the first
    job of each probe size."""
    import torch
    from oracle import multislice as om
    from paper_2012_12686_amd.batch import BatchRunner, DeviceScan
    from paper_2012_12686_amd import Geometry, split_positions
    from tests.fp32_model import loss_grad_fp32
    from tests.gpu_helpers import f32
    scans = synth.mixed_scan_jobs()
    dev = ctx.device
    t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    rng = np.random.default_rng(4040)
    dscans = []
    for sc in scans:
        level = float(np.sum(np.abs(sc.probe) ** 2)) / sc.n ** 2
        im = rng.poisson(level, size=(len(sc.positions), sc.n, sc.n)).astype(np.float32)
        corner, shift = split_positions(t(sc.positions, torch.float64))
        a = t(0.5 * sc.obj_a, torch.float32)
        b = t(0.5 * sc.obj_b, torch.float32)
        z = torch.zeros_like
        dscans.append(DeviceScan(Geometry.from_scan(sc), a, b, t(sc.probe, torch.complex64), corner, shift,
                                 t(im, torch.float32), z(a), z(a), z(b), z(b)))
    r = BatchRunner(ctx, dscans)
    ctx.autotune(r.jobs, reps=1)
    r.build_plan()
    r.capture()
    r.graph.replay()
    torch.cuda.synchronize()
    ctx.sync_error()
    seen = set()
    try:
        for sc, ds, job in zip(scans, dscans, r.jobs):
            if sc.n in seen:
                continue
            seen.add(sc.n)
            B = len(sc.positions)
            geom = om.Geometry.from_scan(sc)
            a64, b64, p64 = f32(0.5 * sc.obj_a), f32(0.5 * sc.obj_b), f32(sc.probe)
            got_all = job.out["g_shift"].cpu().numpy().astype(np.float64)
            corner = ds.corner.cpu().numpy().astype(np.float64)
            shift = ds.shift.cpu().numpy().astype(np.float64)
            im = ds.i_meas.cpu().numpy().astype(np.float64)
            got, ref, model = [], [], []
            for bidx in (0, B // 2, B - 1):
                pos = (corner[bidx] + shift[bidx])[None]
                g_ref = om.loss_grad(geom, a64, b64, p64, pos, im[bidx:bidx + 1])[4][0] / B
                g_mod = np.asarray(loss_grad_fp32(geom, a64, b64, p64, pos, im[bidx:bidx + 1])[4][0]) / B
                got.append(got_all[bidx]); ref.append(g_ref); model.append(g_mod)
            e_gpu, e_f32 = rel_l2(np.array(got), np.array(ref)), rel_l2(np.array(model), np.array(ref))
            print(f"{sc.name}: sampled shift gradients GPU rel-L2 {e_gpu:.3e}, float32-model floor {e_f32:.3e}")
            assert np.linalg.norm(np.array(ref)) > 0
            assert e_gpu <= max(1e-4, 3.0 * e_f32), (sc.name, e_gpu, e_f32)
        assert seen == {64, 96, 128, 192}
    finally:
        for n in (64, 96, 128, 192):
            ctx.set_split(n, 0)
        r.close()
