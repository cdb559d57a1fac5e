"""GPU parity of unequal slice spacing (sparse multislice) against the FP64
oracle, through the C ABI (adorym_forward_gaps / adorym_loss_grad_gaps).

Tolerances as in the uniform-spacing parity tests: intensity rel-L2 <= 1e-5;
loss within the intensity tolerance pushed through the loss; every gradient,
the gap gradient included, rel-L2 <= 1e-4 (tests/gpu_helpers.py).
"""
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


class GapsCase(Case):
    """A scan whose slices sit at unequal distances: measured at the true
    gaps, evaluated at perturbed ones."""

    def __init__(self, scan, true_gaps, eval_scale, poisson_seed=None):
        super().__init__(scan)
        from oracle import multislice as om
        g = self.geom
        truth = om.Geometry(g.n, g.n_slices, g.wavelength_m, g.pixel_m, g.slice_dz_m, g.obj_repr, g.loss, g.eps,
                            gaps=true_gaps)
        i_true = om.forward(truth, scan.obj_a, scan.obj_b, scan.probe, np.asarray(scan.positions))
        if poisson_seed is not None:
            i_true = np.random.default_rng(poisson_seed).poisson(i_true).astype(np.float64)
        self.i_meas = f32(i_true)
        self.gaps = np.asarray(true_gaps, dtype=np.float64) * np.asarray(eval_scale)
        self.geom = om.Geometry(g.n, g.n_slices, g.wavelength_m, g.pixel_m, g.slice_dz_m, g.obj_repr, g.loss, g.eps,
                                gaps=self.gaps)

    def torch_gaps(self):
        import torch
        return torch.as_tensor(self.gaps, dtype=torch.float64, device="cuda").contiguous()


def _geom(case, **kw):
    from paper_2012_12686_amd import Geometry
    return Geometry.from_scan(case.scan, **kw)


def _case(n, s, lat, npos, repr_, loss, gaps, seed):
    sc = synth.small_case(seed=seed, n=n, n_slices=s, lateral=lat, n_pos=npos, obj_repr=repr_, loss=loss,
                          strength=30.0)
    scale = 1.0 + 0.06 * np.cos(np.arange(len(gaps)) + seed)          # evaluation gaps off the truth
    return GapsCase(sc, gaps, scale, poisson_seed=11 if loss == "poisson" else None)


CASES = [
    # n, s, lat, npos, repr, loss, gaps (m)
    (64, 4, 96, 5, "delta_beta", "gaussian", [0.4e-6, 1.5e-6, 0.8e-6]),
    (64, 3, 90, 3, "real_imag", "poisson", [2.0e-6, 0.5e-6]),
    (96, 3, 130, 3, "delta_beta", "poisson", [3.0e-6, 1.0e-6]),
    (128, 2, 160, 3, "delta_beta", "gaussian", [10e-6]),
    (128, 5, 150, 2, "delta_beta", "poisson", [0.2e-6, 2.0e-6, 0.0, 1.0e-6]),
    (192, 3, 220, 2, "delta_beta", "gaussian", [1.2e-6, 0.6e-6]),
]


@pytest.mark.parametrize("n,s,lat,npos,repr_,loss,gaps", CASES)
def test_gaps_forward_and_gradients_match_oracle(ctx, n, s, lat, npos, repr_, loss, gaps):
    import torch
    from oracle import multislice as om
    case = _case(n, s, lat, npos, repr_, loss, gaps, seed=800 + n + s)
    inp, i_meas = case.torch_inputs()
    g = _geom(case)
    i_fwd = ctx.forward_gaps(g, **inp, gaps=case.torch_gaps())
    got = ctx.loss_grad_gaps(g, **inp, gaps=case.torch_gaps(), i_meas=i_meas, intensity=True)
    torch.cuda.synchronize()
    ctx.sync_error()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    i_ref = om.forward(case.geom, case.a, case.b, case.p, case.pos)
    e_f, e_l = rel_l2(i_fwd.cpu().numpy(), i_ref), rel_l2(got["intensity"], i_ref)
    print(f"intensity rel-L2 forward {e_f:.3e}  loss_grad {e_l:.3e}")
    assert e_f <= TOL_I and e_l <= TOL_I
    L, ga, gb, gp, gs, gg = om.loss_grad_gaps(case.geom, case.a, case.b, case.p, case.pos, case.i_meas)
    dldi = om.loss_dI(case.geom.loss, i_ref, case.i_meas, case.geom.eps, i_ref.size)
    tol_l = 2 * TOL_I * np.linalg.norm(i_ref) * np.linalg.norm(dldi)
    assert abs(float(got["loss"]) - L) <= tol_l, (float(got["loss"]), L, tol_l)
    print("g_gaps", got["g_gaps"], "oracle", gg)
    assert_grads([(name, got[name], r) for name, r in
                  zip(("g_a", "g_b", "g_probe", "g_shift", "g_gaps"), (ga, gb, gp, gs, gg))])


def test_equal_gaps_match_the_uniform_call(ctx):
    """Gaps all equal to slice_dz_m: the same model as the uniform kernels
    (same split), to float32 rounding of the rebuilt tables."""
    import torch
    sc = synth.small_case(seed=851, n=128, n_slices=9, lateral=150, n_pos=3, strength=30.0, loss="poisson")
    case = Case(sc, poisson_seed=2)
    inp, i_meas = case.torch_inputs()
    g = _geom(case, deterministic=True)
    gaps = torch.full((sc.n_slices - 1,), sc.slice_dz_m, dtype=torch.float64, device="cuda")
    uni = ctx.loss_grad(g, **inp, i_meas=i_meas, intensity=True)
    var = ctx.loss_grad_gaps(g, **inp, gaps=gaps, i_meas=i_meas, intensity=True)
    torch.cuda.synchronize()
    for k in ("intensity", "g_a", "g_b", "g_probe", "g_shift"):
        e = rel_l2(var[k].cpu().numpy(), uni[k].cpu().numpy())
        print(k, "bitwise" if torch.equal(var[k], uni[k]) else f"rel-L2 {e:.2e}")
        assert e <= 1e-6, k
    assert abs(float(var["loss"]) - float(uni["loss"])) <= 1e-6 * abs(float(uni["loss"]))


def test_gaps_single_slice_accumulate_and_reproducible(ctx):
    """S = 1 takes no gaps (NULL); ACCUMULATE adds onto what is passed; the
    gap gradient is the same bits on every call."""
    import torch
    sc = synth.small_case(seed=861, n=64, n_slices=1, lateral=90, n_pos=4, strength=30.0)
    case = Case(sc)
    inp, i_meas = case.torch_inputs()
    one = ctx.loss_grad_gaps(_geom(case), **inp, gaps=None, i_meas=i_meas)
    ref = ctx.loss_grad(_geom(case), **inp, i_meas=i_meas)
    torch.cuda.synchronize()
    assert one["g_gaps"].numel() == 0
    assert rel_l2(one["g_a"].cpu().numpy(), ref["g_a"].cpu().numpy()) <= 1e-6

    c4 = _case(64, 4, 96, 5, "delta_beta", "gaussian", [0.4e-6, 1.5e-6, 0.8e-6], seed=871)
    inp, i_meas = c4.torch_inputs()
    g = _geom(c4)
    r1 = ctx.loss_grad_gaps(g, **inp, gaps=c4.torch_gaps(), i_meas=i_meas)
    r2 = ctx.loss_grad_gaps(g, **inp, gaps=c4.torch_gaps(), i_meas=i_meas)
    base = {k: (torch.randn_like(v) if k != "loss" else torch.empty_like(v)) for k, v in r1.items()}
    acc = {k: v.clone() for k, v in base.items()}
    ctx.loss_grad_gaps(_geom(c4, accumulate=True), **inp, gaps=c4.torch_gaps(), i_meas=i_meas, out=acc)
    torch.cuda.synchronize()
    assert torch.equal(r1["g_gaps"], r2["g_gaps"])
    for k in ("g_a", "g_b", "g_probe", "g_shift", "g_gaps"):
        assert rel_l2(acc[k].cpu().numpy(), (base[k] + r1[k]).cpu().numpy()) <= 1e-6, k


def test_sparse_multislice_full_minibatch_matches_oracle(ctx):
    """The benchmarked sparse-multislice workload at full size (object
    512 x 512 x 2, 7.3 nm, 12 keV, layers 10 um apart), one whole minibatch
    of 202 positions in the launch configuration the benchmark times,
    against the oracle on every output."""
    import torch
    from oracle import multislice as om
    from paper_2012_12686_amd import Geometry
    sc = synth.sparse_multislice()
    mb = sc.minibatch
    og_true = om.Geometry(sc.n, sc.n_slices, sc.wavelength_m, sc.pixel_m, sc.slice_dz_m, sc.obj_repr, sc.loss,
                          sc.eps, gaps=sc.gaps)
    pos = np.asarray(sc.positions[:mb])
    i_meas = f32(np.random.default_rng(4).poisson(om.forward(og_true, sc.obj_a, sc.obj_b, sc.probe, pos)))
    # evaluation point: half the true object, gaps 5% long
    a, b, p = f32(0.5 * sc.obj_a), f32(0.5 * sc.obj_b), f32(sc.probe)
    corner, shift = synth.split_positions(pos)
    shift = f32(shift)
    pos32 = corner + shift
    og = om.Geometry(sc.n, sc.n_slices, sc.wavelength_m, sc.pixel_m, sc.slice_dz_m, sc.obj_repr, sc.loss, sc.eps,
                     gaps=sc.eval_gaps)
    t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    got = ctx.loss_grad_gaps(Geometry.from_scan(sc), t(a, torch.float32), t(b, torch.float32),
                             t(p, torch.complex64), t(corner, torch.int32), t(shift, torch.float32),
                             t(sc.eval_gaps, torch.float64), t(i_meas, torch.float32), intensity=True)
    torch.cuda.synchronize()
    ctx.sync_error()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    i_ref = om.forward(og, a, b, p, pos32)
    e_i = rel_l2(got["intensity"], i_ref)
    print(f"intensity rel-L2 {e_i:.3e}")
    assert e_i <= TOL_I
    L, ga, gb, gp, gs, gg = om.loss_grad_gaps(og, a, b, p, pos32, i_meas)
    dldi = om.loss_dI(og.loss, i_ref, i_meas, og.eps, i_ref.size)
    assert abs(float(got["loss"]) - L) <= 2 * TOL_I * np.linalg.norm(i_ref) * np.linalg.norm(dldi)
    assert_grads([(name, got[name], r) for name, r in
                  zip(("g_a", "g_b", "g_probe", "g_shift", "g_gaps"), (ga, gb, gp, gs, gg))])
