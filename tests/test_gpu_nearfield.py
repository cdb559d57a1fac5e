"""GPU parity of the near-field detector model (Fresnel propagation to the
detector with the paraxial or Sommerfeld kernel, one distance per position)
against the FP64 oracle, through the C ABI.

Tolerances as in the far-field parity tests: intensity rel-L2 <= 1e-5; loss
within the intensity tolerance pushed through the loss; every gradient, the
distance gradient included, rel-L2 <= 1e-4 (tests/gpu_helpers.py).
"""
import dataclasses

import numpy as np
import pytest

import synth
from tests.gpu_helpers import TOL_I, Case, assert_grads, f32, rel_l2

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


def _t(x, dt):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def run_and_check(ctx, sc, dists_true, scale, kind, poisson_seed=None):
    import torch
    from oracle import multislice as om
    from paper_2012_12686_amd import Geometry
    case = Case(sc)
    geom = case.geom
    b = len(case.pos)
    idx = (np.arange(b) % len(dists_true)).astype(np.int32)
    i_true = om.forward_nearfield(geom, sc.obj_a, sc.obj_b, sc.probe, np.asarray(sc.positions), dists_true, idx, kind)
    if poisson_seed is not None:
        i_true = np.random.default_rng(poisson_seed).poisson(i_true).astype(np.float64)
    i_meas = f32(i_true)
    dists = np.asarray(dists_true, dtype=np.float64) * np.asarray(scale)
    inp, _ = case.torch_inputs()
    g = Geometry.from_scan(sc)
    td, ti = _t(dists, torch.float64), _t(idx, torch.int32)
    i_fwd = ctx.forward_nearfield(g, **inp, dists=td, dist_idx=ti, kind=kind)
    got = ctx.loss_grad_nearfield(g, **inp, dists=td, dist_idx=ti, i_meas=_t(i_meas, torch.float32), kind=kind,
                                  intensity=True)
    torch.cuda.synchronize()
    ctx.sync_error()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    i_ref = om.forward_nearfield(geom, case.a, case.b, case.p, case.pos, dists, idx, kind)
    e_f, e_l = rel_l2(i_fwd.cpu().numpy(), i_ref), rel_l2(got["intensity"], i_ref)
    print(f"{sc.name} {kind}: intensity rel-L2 forward {e_f:.3e} loss_grad {e_l:.3e}")
    assert e_f <= TOL_I and e_l <= TOL_I
    L, ga, gb, gp, gs, gd = om.loss_grad_nearfield(geom, case.a, case.b, case.p, case.pos, i_meas, dists, idx, kind)
    dldi = om.loss_dI(geom.loss, i_ref, i_meas, geom.eps, i_ref.size)
    assert abs(float(got["loss"]) - L) <= 2 * TOL_I * np.linalg.norm(i_ref) * np.linalg.norm(dldi)
    assert_grads([(name, got[name], r) for name, r in
                  zip(("g_a", "g_b", "g_probe", "g_shift", "g_dist"), (ga, gb, gp, gs, gd))])
    return got


@pytest.mark.parametrize("n,s,lat,npos,repr_,loss,kind", [
    (64, 3, 96, 5, "delta_beta", "gaussian", "paraxial"),
    (64, 1, 90, 4, "real_imag", "poisson", "sommerfeld"),
    (96, 4, 130, 3, "delta_beta", "poisson", "paraxial"),
    (128, 9, 150, 3, "delta_beta", "gaussian", "sommerfeld"),
    (128, 2, 150, 4, "real_imag", "gaussian", "paraxial"),
    (192, 3, 220, 2, "delta_beta", "poisson", "paraxial"),
])
def test_nearfield_matches_oracle(ctx, n, s, lat, npos, repr_, loss, kind):
    sc = synth.small_case(seed=900 + n + s, n=n, n_slices=s, lateral=lat, n_pos=npos, obj_repr=repr_, loss=loss,
                          strength=30.0)
    run_and_check(ctx, sc, [0.8e-6, 5e-6], [1.04, 0.97], kind, poisson_seed=5 if loss == "poisson" else None)


def test_sommerfeld_with_evanescent_frequencies(ctx):
    """Pixels of 0.05 nm at 10 keV: lambda |nu| reaches 1.24 at the Nyquist
    edge, so the kernel's evanescent cut is exercised."""
    sc = synth.small_case(seed=951, n=64, n_slices=2, lateral=90, n_pos=3, strength=30.0)
    sc = dataclasses.replace(sc, pixel_m=5e-11)
    run_and_check(ctx, sc, [2e-9, 7e-9], [1.05, 0.96], "sommerfeld")


def test_mdh_tiles_full_iteration_matches_oracle(ctx):
    """The benchmarked multi-distance holography workload at full size: 25
    overlapping 128 x 128 tiles of a 512 x 512 complex object at 4 distances
    (100 positions, one iteration), plane-wave illumination, against the
    oracle on every output."""
    sc, dists, idx = synth.mdh_tiles()
    import torch
    from oracle import multislice as om
    from paper_2012_12686_amd import Geometry
    case = Case(sc, use_eval=False)
    geom = case.geom
    i_meas = f32(np.random.default_rng(6).poisson(
        om.forward_nearfield(geom, sc.obj_a, sc.obj_b, sc.probe, np.asarray(sc.positions), dists, idx)))
    a, b = f32(sc.eval_obj_a), f32(sc.eval_obj_b)
    ev = dists * 1.02
    got = ctx.loss_grad_nearfield(Geometry.from_scan(sc), _t(a, torch.float32), _t(b, torch.float32),
                                  _t(case.p, torch.complex64), _t(case.corner, torch.int32),
                                  _t(case.shift, torch.float32), _t(ev, torch.float64), _t(idx, torch.int32),
                                  _t(i_meas, torch.float32), intensity=True)
    torch.cuda.synchronize()
    ctx.sync_error()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    i_ref = om.forward_nearfield(geom, a, b, case.p, case.pos, ev, idx)
    e_i = rel_l2(got["intensity"], i_ref)
    print(f"intensity rel-L2 {e_i:.3e}")
    assert e_i <= TOL_I
    L, ga, gb, gp, gs, gd = om.loss_grad_nearfield(geom, a, b, case.p, case.pos, i_meas, ev, idx)
    assert_grads([(name, got[name], r) for name, r in
                  zip(("g_a", "g_b", "g_probe", "g_shift", "g_dist"), (ga, gb, gp, gs, gd))])


def test_bad_distance_index_is_reported_and_skipped(ctx):
    import torch
    from paper_2012_12686_amd import Geometry
    from paper_2012_12686_amd._lib import AdorymError
    sc = synth.small_case(seed=961, n=64, n_slices=2, lateral=90, n_pos=3, strength=30.0)
    case = Case(sc)
    inp, i_meas = case.torch_inputs()
    idx = _t(np.array([0, 5, 1], np.int32), torch.int32)
    out = ctx.forward_nearfield(Geometry.from_scan(sc), **inp, dists=_t([1e-6, 2e-6], torch.float64), dist_idx=idx)
    with pytest.raises(AdorymError):
        ctx.sync_error()
    torch.cuda.synchronize()
    assert float(out[1].abs().max()) == 0.0 and float(out[0].abs().max()) > 0.0
