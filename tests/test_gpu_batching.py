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
