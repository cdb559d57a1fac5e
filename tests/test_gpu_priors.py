"""GPU parity of the object priors (Eq. tikhonov, Table tab:regularizers)
against the FP64 oracle, through the C ABI.

The priors are sums of |.| of FP32 quantities and their gradients are signs
times coefficients: the GPU and the oracle agree to FP32 rounding except
where a quantity or a neighbour difference is within rounding of zero and
its sign flips.  Tolerances: value rel 1e-6; gradients rel-L2 <= 1e-5
(bitwise-equal signs almost everywhere); the support projection bitwise.
"""
import numpy as np
import pytest

import synth
from oracle import regularizers as orr
from tests.gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

REPRS = ["delta_beta", "real_imag"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_12686_amd import Context
    c = Context()
    yield c
    c.close()


def _obj(repr_, shape, seed):
    rng = np.random.default_rng(seed)
    if repr_ == "delta_beta":
        a, b = rng.uniform(-1e-5, 1e-5, shape), rng.uniform(-1e-6, 1e-6, shape)
    else:
        mod = rng.uniform(0.6, 1.0, shape)
        ph = rng.uniform(-1.2, 1.2, shape)
        a, b = mod * np.cos(ph), mod * np.sin(ph)
    return a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)


def _t(x, dt=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt or torch.float32, device="cuda")


@pytest.mark.parametrize("repr_", REPRS)
@pytest.mark.parametrize("shape", [(1, 5, 7), (3, 67, 130), (7, 100, 150)])
def test_prior_value_and_gradient_match_oracle(ctx, repr_, shape):
    import torch
    a, b = _obj(repr_, shape, seed=sum(shape))
    coef = dict(a1=1.3, a2=0.7, gamma=0.9)
    base_a = np.random.default_rng(1).standard_normal(shape) * 1e-3
    base_b = np.random.default_rng(2).standard_normal(shape) * 1e-3
    out = {"g_a": _t(base_a), "g_b": _t(base_b)}
    got = ctx.prior_grad(repr_, _t(a), _t(b), l1_a=coef["a1"], l1_b=coef["a2"], tv=coef["gamma"], out=out)
    torch.cuda.synchronize()
    ctx.sync_error()
    v = orr.value(a, b, repr_, **coef)
    ga, gb = orr.grad(a, b, repr_, **coef)
    print(repr_, shape, "value", float(got["value"]), v)
    assert float(got["value"]) == pytest.approx(v, rel=1e-6)
    ea = rel_l2(got["g_a"].cpu().numpy() - base_a.astype(np.float32), ga)
    eb = rel_l2(got["g_b"].cpu().numpy() - base_b.astype(np.float32), gb)
    print(f"g_a rel-L2 {ea:.2e}  g_b rel-L2 {eb:.2e}")
    assert ea <= 1e-5 and eb <= 1e-5
    # overwrite mode gives the gradient alone
    got2 = ctx.prior_grad(repr_, _t(a), _t(b), l1_a=coef["a1"], l1_b=coef["a2"], tv=coef["gamma"],
                          accumulate=False, out={"g_a": _t(base_a), "g_b": _t(base_b)})
    torch.cuda.synchronize()
    assert rel_l2(got2["g_a"].cpu().numpy(), ga) <= 1e-5 and rel_l2(got2["g_b"].cpu().numpy(), gb) <= 1e-5


@pytest.mark.parametrize("repr_", REPRS)
def test_reweighted_l1_weights_and_gradient_match_oracle(ctx, repr_):
    import torch
    shape = (4, 60, 90)
    a, b = _obj(repr_, shape, seed=5)
    sa, sb = _obj(repr_, shape, seed=6)
    eps = 1e-7 if repr_ == "delta_beta" else 1e-3
    w_a, w_b = ctx.prior_weights(repr_, _t(sa), _t(sb), eps)
    torch.cuda.synchronize()
    ow1, ow2 = orr.reweight(sa, sb, repr_, eps)
    e1, e2 = rel_l2(w_a.cpu().numpy(), ow1), rel_l2(w_b.cpu().numpy(), ow2)
    # W = max|q| / (|q| + eps): a rounding error dq of q moves W by dq / (|q| + eps)
    # relative.  For complex objects q1 = |O| - mean|O| is a cancelling FP32
    # difference (dq ~ 2^-24 |O|), so near q1 = 0 the bound is 2^-24 max|O| / eps.
    tol1 = 1e-5 if repr_ == "delta_beta" else max(1e-5, 4 * 2.0 ** -24 * np.max(np.hypot(sa, sb)) / eps)
    print(f"weights rel-L2 {e1:.2e} {e2:.2e} (tolerance {tol1:.1e}, 1e-5)")
    assert e1 <= tol1 and e2 <= 1e-5
    # the gradient with the oracle's own weights (rounded to float32), so only the prior is compared
    w1, w2 = ow1.astype(np.float32).astype(np.float64), ow2.astype(np.float32).astype(np.float64)
    got = ctx.prior_grad(repr_, _t(a), _t(b), l1_a=0.8, l1_b=1.1, tv=0.0, weights=(_t(w1), _t(w2)),
                         accumulate=False)
    torch.cuda.synchronize()
    v = orr.value(a, b, repr_, a1=0.8, a2=1.1, w1=w1, w2=w2)
    ga, gb = orr.grad(a, b, repr_, a1=0.8, a2=1.1, w1=w1, w2=w2)
    assert float(got["value"]) == pytest.approx(v, rel=1e-6)
    assert rel_l2(got["g_a"].cpu().numpy(), ga) <= 1e-5 and rel_l2(got["g_b"].cpu().numpy(), gb) <= 1e-5


@pytest.mark.parametrize("repr_", REPRS)
def test_support_projection_matches_oracle_bitwise(ctx, repr_):
    import torch
    shape = (3, 50, 70)
    a, b = _obj(repr_, shape, seed=9)
    mask = (np.random.default_rng(3).random(shape) > 0.3).astype(np.uint8)
    ta, tb = _t(a), _t(b)
    ctx.support_project(repr_, _t(mask, torch.uint8), ta, tb)
    torch.cuda.synchronize()
    pa, pb = orr.support_project(a.astype(np.float32), b.astype(np.float32), repr_, mask)
    assert np.array_equal(ta.cpu().numpy(), pa.astype(np.float32))
    assert np.array_equal(tb.cpu().numpy(), pb.astype(np.float32))


def test_prior_on_the_full_128_slice_object(ctx):
    """The benchmarked size: the 512 x 512 x 128 delta/beta object of the
    128-slice workload, l1 + TV, added onto a data gradient; reproducible
    bit for bit."""
    import torch
    sc = synth.multislice_n128_s128()
    a = sc.obj_a.astype(np.float32).astype(np.float64)
    b = sc.obj_b.astype(np.float32).astype(np.float64)
    ta, tb = _t(a), _t(b)
    coef = dict(a1=0.05, a2=0.5, gamma=0.02)
    r1 = ctx.prior_grad("delta_beta", ta, tb, l1_a=coef["a1"], l1_b=coef["a2"], tv=coef["gamma"], accumulate=False)
    r2 = ctx.prior_grad("delta_beta", ta, tb, l1_a=coef["a1"], l1_b=coef["a2"], tv=coef["gamma"], accumulate=False)
    torch.cuda.synchronize()
    assert torch.equal(r1["g_a"], r2["g_a"]) and float(r1["value"]) == float(r2["value"])
    v = orr.value(a, b, "delta_beta", **coef)
    ga, gb = orr.grad(a, b, "delta_beta", **coef)
    assert float(r1["value"]) == pytest.approx(v, rel=1e-6)
    ea, eb = rel_l2(r1["g_a"].cpu().numpy(), ga), rel_l2(r1["g_b"].cpu().numpy(), gb)
    print(f"full object: value {float(r1['value']):.6e} vs {v:.6e}; g_a {ea:.2e} g_b {eb:.2e}")
    assert ea <= 1e-5 and eb <= 1e-5
