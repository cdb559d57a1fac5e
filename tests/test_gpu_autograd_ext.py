"""The torch.autograd front ends of the probe-mode, unequal-spacing,
near-field and prior entry points give the direct calls' numbers bit for
bit, and the data loss and a prior combine by plain addition."""
import numpy as np
import pytest

import synth
from tests.gpu_helpers import Case

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


def _setup(seed, n=64, s=3, npos=4):
    import torch
    sc = synth.small_case(seed=seed, n=n, n_slices=s, lateral=n + 32, n_pos=npos, strength=30.0)
    case = Case(sc)
    inp, i_meas = case.torch_inputs()
    pos = (inp["corner"].double() + inp["shift"].double())
    return sc, case, inp, i_meas, pos


def test_modes_autograd_equals_direct_call(ctx):
    import torch
    from paper_2012_12686_amd import Geometry, multislice_loss_modes
    sc, case, inp, i_meas, pos = _setup(971)
    probes = torch.as_tensor(synth.probe_modes(case.p, 2, seed=3), dtype=torch.complex64, device="cuda")
    g = Geometry.from_scan(sc)
    direct = ctx.loss_grad_modes(g, inp["obj_a"], inp["obj_b"], probes, inp["corner"], inp["shift"], i_meas)
    a = inp["obj_a"].clone().requires_grad_(True)
    pr = probes.clone().requires_grad_(True)
    p = pos.clone().requires_grad_(True)
    loss = multislice_loss_modes(a, inp["obj_b"], pr, p, i_meas, g, ctx)
    loss.backward()
    torch.cuda.synchronize()
    assert float(loss.detach()) == float(direct["loss"])
    assert torch.equal(a.grad, direct["g_a"]) and torch.equal(pr.grad, direct["g_probe"])
    assert torch.equal(p.grad.float(), direct["g_shift"])


def test_gaps_autograd_equals_direct_call(ctx):
    import torch
    from paper_2012_12686_amd import Geometry, multislice_loss_gaps
    sc, case, inp, i_meas, pos = _setup(972)
    g = Geometry.from_scan(sc)
    gaps = torch.tensor([0.7e-6, 1.9e-6], dtype=torch.float64, device="cuda")
    direct = ctx.loss_grad_gaps(g, **inp, gaps=gaps, i_meas=i_meas)
    gp = gaps.clone().requires_grad_(True)
    b = inp["obj_b"].clone().requires_grad_(True)
    loss = multislice_loss_gaps(inp["obj_a"], b, inp["probe"], pos, gp, i_meas, g, ctx)
    loss.backward()
    torch.cuda.synchronize()
    assert float(loss.detach()) == float(direct["loss"])
    assert torch.equal(gp.grad, direct["g_gaps"]) and torch.equal(b.grad, direct["g_b"])


def test_nearfield_autograd_equals_direct_call(ctx):
    import torch
    from paper_2012_12686_amd import Geometry, multislice_loss_nearfield
    sc, case, inp, i_meas, pos = _setup(973)
    g = Geometry.from_scan(sc)
    dists = torch.tensor([1e-6, 3e-6], dtype=torch.float64, device="cuda")
    idx = torch.tensor([0, 1, 0, 1], dtype=torch.int32, device="cuda")
    direct = ctx.loss_grad_nearfield(g, **inp, dists=dists, dist_idx=idx, i_meas=i_meas, kind="sommerfeld")
    d = dists.clone().requires_grad_(True)
    a = inp["obj_a"].clone().requires_grad_(True)
    loss = multislice_loss_nearfield(a, inp["obj_b"], inp["probe"], pos, d, idx, i_meas, g, "sommerfeld", ctx)
    (2.0 * loss).backward()
    torch.cuda.synchronize()
    assert float(loss.detach()) == float(direct["loss"])
    assert torch.equal(d.grad, 2.0 * direct["g_dist"]) and torch.equal(a.grad, 2.0 * direct["g_a"])


def test_data_loss_plus_prior_gradients_add(ctx):
    import torch
    from paper_2012_12686_amd import Geometry, multislice_loss, object_prior
    sc, case, inp, i_meas, pos = _setup(974)
    g = Geometry.from_scan(sc)
    a = inp["obj_a"].clone().requires_grad_(True)
    b = inp["obj_b"].clone().requires_grad_(True)
    data = multislice_loss(a, b, inp["probe"], pos, i_meas, g, ctx)
    prior = object_prior(a, b, "delta_beta", l1_a=0.3, l1_b=0.1, tv=0.2, ctx=ctx)
    (data + prior).backward()
    direct = ctx.loss_grad(g, **inp, i_meas=i_meas)
    pr = ctx.prior_grad("delta_beta", inp["obj_a"], inp["obj_b"], l1_a=0.3, l1_b=0.1, tv=0.2, accumulate=False)
    torch.cuda.synchronize()
    assert float(prior.detach()) == float(pr["value"])
    assert torch.equal(a.grad, direct["g_a"] + pr["g_a"]) and torch.equal(b.grad, direct["g_b"] + pr["g_b"])
