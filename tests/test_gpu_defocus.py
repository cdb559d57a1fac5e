"""GPU parity of probe defocus against the FP64 oracle, through the C ABI
(adorym_forward_defocus / adorym_loss_grad_defocus).

Tolerances as in the other parity tests: intensity rel-L2 <= 1e-5; loss
within the intensity tolerance pushed through the loss; every gradient, the
defocus gradient included, rel <= 1e-4 (tests/gpu_helpers.py).
"""
import numpy as np
import pytest

import synth
from tests.gpu_helpers import TOL_G, TOL_I, Case, assert_grads, f32, rel_l2

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


class DefocusCase(Case):
    """Measured at the true defocus, evaluated at another one."""

    def __init__(self, scan, true_defocus, eval_defocus, poisson_seed=None):
        super().__init__(scan)
        from oracle import multislice as om
        i_true = om.forward_defocus(self.geom, scan.obj_a, scan.obj_b, scan.probe, np.asarray(scan.positions),
                                    true_defocus)
        if poisson_seed is not None:
            i_true = np.random.default_rng(poisson_seed).poisson(i_true).astype(np.float64)
        self.i_meas = f32(i_true)
        self.defocus = float(eval_defocus)


def _geom(case, **kw):
    from paper_2012_12686_amd import Geometry
    return Geometry.from_scan(case.scan, **kw)


def run_and_check(ctx, case, **kw):
    import torch
    from oracle import multislice as om
    inp, i_meas = case.torch_inputs()
    geom = _geom(case, **kw)
    i_fwd = ctx.forward_defocus(geom, **inp, defocus_m=case.defocus)
    got = ctx.loss_grad_defocus(geom, **inp, defocus_m=case.defocus, i_meas=i_meas, intensity=True)
    torch.cuda.synchronize()
    ctx.sync_error()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    i_ref = om.forward_defocus(case.geom, case.a, case.b, case.p, case.pos, case.defocus)
    e_f, e_l = rel_l2(i_fwd.cpu().numpy(), i_ref), rel_l2(got["intensity"], i_ref)
    print(f"{case.scan.name} defocus {case.defocus:.2e}: intensity rel-L2 forward {e_f:.3e} loss_grad {e_l:.3e}")
    assert e_f <= TOL_I and e_l <= TOL_I
    ref = om.loss_grad_defocus(case.geom, case.a, case.b, case.p, case.pos, case.i_meas, case.defocus)
    dldi = om.loss_dI(case.geom.loss, i_ref, case.i_meas, case.geom.eps, i_ref.size)
    assert abs(float(got["loss"]) - ref[0]) <= 2 * TOL_I * np.linalg.norm(i_ref) * np.linalg.norm(dldi)
    e_gpu = abs(float(got["g_defocus"]) - ref[5]) / abs(ref[5])
    print(f"g_defocus: GPU {float(got['g_defocus']):.6e} oracle {ref[5]:.6e} rel {e_gpu:.3e}")
    assert e_gpu <= TOL_G
    assert_grads([(name, got[name], r) for name, r in zip(("g_a", "g_b", "g_probe", "g_shift"), ref[1:5])])
    return got


@pytest.mark.parametrize("n,s,lat,npos,repr_,loss,true_d,eval_d", [
    (64, 3, 96, 5, "delta_beta", "gaussian", 0.8e-6, 1.0e-6),
    (64, 1, 90, 4, "real_imag", "poisson", -0.5e-6, -0.3e-6),
    (96, 5, 130, 3, "delta_beta", "poisson", 1.2e-6, 1.0e-6),
    (128, 9, 150, 3, "delta_beta", "gaussian", 2.0e-6, 2.4e-6),
    (128, 18, 150, 4, "real_imag", "gaussian", 0.6e-6, 0.7e-6),
    (192, 4, 230, 2, "delta_beta", "poisson", 1.5e-6, 1.2e-6),
])
def test_defocus_matches_oracle(ctx, n, s, lat, npos, repr_, loss, true_d, eval_d):
    sc = synth.small_case(seed=1100 + n + s, n=n, n_slices=s, lateral=lat, n_pos=npos, obj_repr=repr_, loss=loss,
                          strength=30.0)
    run_and_check(ctx, DefocusCase(sc, true_d, eval_d, poisson_seed=9 if loss == "poisson" else None))


def test_defocus_with_fixed_split_and_deterministic_mode(ctx):
    """Every split of the 128-probe kernels and the deterministic mode (its
    outputs bitwise reproducible)."""
    import torch
    sc = synth.small_case(seed=1190, n=128, n_slices=7, lateral=160, n_pos=3, strength=30.0)
    case = DefocusCase(sc, 1.0e-6, 1.2e-6)
    for k in (1, 2, 4, 8):
        ctx.set_split(128, k)
        try:
            run_and_check(ctx, case)
        finally:
            ctx.set_split(128, 0)
    inp, i_meas = case.torch_inputs()
    geom = _geom(case, deterministic=True)
    r1 = ctx.loss_grad_defocus(geom, **inp, defocus_m=case.defocus, i_meas=i_meas)
    r2 = ctx.loss_grad_defocus(geom, **inp, defocus_m=case.defocus, i_meas=i_meas)
    torch.cuda.synchronize()
    for k in r1:
        assert torch.equal(r1[k], r2[k]), k


def test_zero_defocus_gives_the_plain_calls_bits(ctx):
    import torch
    sc = synth.small_case(seed=1191, n=64, n_slices=6, lateral=96, n_pos=4, strength=30.0)
    case = Case(sc)
    inp, i_meas = case.torch_inputs()
    geom = _geom(case)
    plain = ctx.loss_grad(geom, **inp, i_meas=i_meas, intensity=True)
    zero = ctx.loss_grad_defocus(geom, **inp, defocus_m=0.0, i_meas=i_meas, intensity=True)
    f_plain = ctx.forward(geom, **inp)
    f_zero = ctx.forward_defocus(geom, **inp, defocus_m=0.0)
    torch.cuda.synchronize()
    assert torch.equal(f_plain, f_zero)
    for k in ("loss", "g_a", "g_b", "g_probe", "g_shift", "intensity"):
        assert torch.equal(plain[k], zero[k]), k


def test_defocus_gradient_alone_accumulate_and_autograd(ctx):
    """g_defocus without g_probe; the accumulate flag adds; the autograd front
    end returns the direct call's values."""
    import torch
    from paper_2012_12686_amd import multislice_loss_defocus
    from paper_2012_12686_amd._lib import AdorymError, EINVAL
    sc = synth.small_case(seed=1192, n=96, n_slices=4, lateral=130, n_pos=3, strength=30.0)
    case = DefocusCase(sc, 1.0e-6, 1.3e-6)
    inp, i_meas = case.torch_inputs()
    geom = _geom(case)
    full = ctx.loss_grad_defocus(geom, **inp, defocus_m=case.defocus, i_meas=i_meas)
    only = ctx.loss_grad_defocus(geom, **inp, defocus_m=case.defocus, i_meas=i_meas, grads=False,
                                 out={"g_defocus": torch.empty((), dtype=torch.float64, device="cuda")})
    torch.cuda.synchronize()
    assert float(only["g_defocus"]) == float(full["g_defocus"])
    acc = {k: v.clone() for k, v in full.items() if k != "loss"}
    ctx.loss_grad_defocus(_geom(case, accumulate=True), **inp, defocus_m=case.defocus, i_meas=i_meas, out=acc)
    torch.cuda.synchronize()
    for k in ("g_a", "g_b", "g_probe", "g_shift", "g_defocus"):
        assert rel_l2(acc[k].cpu().numpy(), 2 * full[k].cpu().numpy()) < 1e-6, k
    a = inp["obj_a"].clone().requires_grad_(True)
    p = inp["probe"].clone().requires_grad_(True)
    d = torch.tensor(case.defocus, dtype=torch.float64, device="cuda", requires_grad=True)
    pos = (inp["corner"].double() + inp["shift"].double()).requires_grad_(True)
    loss = multislice_loss_defocus(a, inp["obj_b"], p, pos, d, i_meas, geom, ctx)
    (2.0 * loss).backward()
    assert float(loss.detach()) == float(full["loss"])
    assert torch.allclose(a.grad, 2 * full["g_a"], rtol=1e-6, atol=0)
    assert torch.allclose(p.grad, 2 * full["g_probe"], rtol=1e-6, atol=0)
    assert float(d.grad) == pytest.approx(2 * float(full["g_defocus"]), rel=1e-12)
    with pytest.raises(AdorymError) as ei:
        ctx.forward_defocus(geom, **inp, defocus_m=float("nan"))
    assert ei.value.status == EINVAL
