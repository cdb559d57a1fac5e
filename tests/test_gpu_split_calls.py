"""Loss now / gradients later (adorym_loss_fwd, adorym_loss_bwd), the
one-shot batched call and the library autotuner, through the C ABI."""
import numpy as np
import pytest

import synth
from tests.gpu_helpers import Case, rel_l2

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


@pytest.mark.parametrize("n,s,loss", [(64, 5, "poisson"), (128, 19, "gaussian"), (192, 3, "poisson")])
def test_loss_fwd_bwd_equal_the_fused_call(ctx, n, s, loss):
    import torch
    from paper_2012_12686_amd import Geometry
    sc = synth.small_case(seed=990 + n, n=n, n_slices=s, lateral=n + 30, n_pos=4, strength=30.0, loss=loss)
    case = Case(sc, poisson_seed=4 if loss == "poisson" else None)
    inp, i_meas = case.torch_inputs()
    g = Geometry.from_scan(sc, deterministic=True)
    fused = ctx.loss_grad(g, **inp, i_meas=i_meas, intensity=True)
    lval, ws, inten = ctx.loss_fwd(g, **inp, i_meas=i_meas, intensity=True)
    torch.cuda.synchronize()
    assert torch.equal(inten, fused["intensity"])
    assert float(lval) == pytest.approx(float(fused["loss"]), rel=1e-12)
    g1 = ctx.loss_bwd(g, **inp, i_meas=i_meas, workspace=ws)
    g2 = ctx.loss_bwd(g, **inp, i_meas=i_meas, workspace=ws, grad_scale=2.0)
    torch.cuda.synchronize()
    for k in ("g_a", "g_b", "g_probe", "g_shift"):
        assert torch.equal(g1[k], fused[k]), k            # same kernels resumed, same split
        assert torch.equal(g2[k], 2 * fused[k]), k        # the reverse sweep is linear in the seed
    base = {k: torch.randn_like(v) for k, v in g1.items()}
    acc = {k: v.clone() for k, v in base.items()}
    ctx.loss_bwd(Geometry.from_scan(sc, deterministic=True, accumulate=True), **inp, i_meas=i_meas, workspace=ws,
                 out=acc)
    torch.cuda.synchronize()
    for k in acc:
        assert rel_l2(acc[k].cpu().numpy(), (base[k] + g1[k]).cpu().numpy()) <= 1e-6, k


def test_lazy_autograd_matches_the_eager_one(ctx):
    import torch
    from paper_2012_12686_amd import Geometry, multislice_loss
    sc = synth.small_case(seed=995, n=128, n_slices=9, lateral=150, n_pos=3, strength=30.0)
    case = Case(sc)
    inp, i_meas = case.torch_inputs()
    g = Geometry.from_scan(sc)
    pos = inp["corner"].double() + inp["shift"].double()
    res = []
    for lazy in (False, True):
        a = inp["obj_a"].clone().requires_grad_(True)
        p = inp["probe"].clone().requires_grad_(True)
        loss = multislice_loss(a, inp["obj_b"], p, pos, i_meas, g, ctx, lazy=lazy)
        (3.0 * loss).backward()
        res.append((float(loss.detach()), a.grad.cpu().numpy(), p.grad.cpu().numpy()))
    # the eager call picks its own split (a different float32 rounding of the intensities)
    assert res[1][0] == pytest.approx(res[0][0], rel=1e-6)
    assert rel_l2(res[1][1], res[0][1]) <= 1e-5 and rel_l2(res[1][2], res[0][2]) <= 1e-5


def test_batched_one_shot_and_autotune(ctx):
    import torch
    from paper_2012_12686_amd import Geometry, Job
    jobs = []
    for i, (n, s) in enumerate(((64, 3), (128, 5), (64, 7))):
        sc = synth.small_case(seed=1000 + i, n=n, n_slices=s, lateral=n + 40, n_pos=5, strength=30.0)
        case = Case(sc)
        inp, i_meas = case.torch_inputs()
        jobs.append(Job(Geometry.from_scan(sc), inp["obj_a"], inp["obj_b"], inp["probe"], inp["corner"],
                        inp["shift"], i_meas))
    chosen = ctx.autotune(jobs, reps=1)
    assert chosen[64] in (1, 2, 4) and chosen[128] in (1, 2, 4, 8)
    plan = ctx.plan(jobs)
    plan.run()
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in j.out.items()} for j in jobs]
    plan.close()
    for j in jobs:
        for v in j.out.values():
            v.zero_()
    ctx.loss_grad_batched(jobs)
    ctx.set_split(64, 0)
    ctx.set_split(128, 0)
    for j, r in zip(jobs, ref):
        for k in ("loss", "g_a", "g_b", "g_probe", "g_shift"):
            assert torch.equal(j.out[k], r[k]), k
