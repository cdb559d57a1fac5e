"""GPU parity of the tilt rotation (and its transpose) and of Adam."""
import math

import numpy as np
import pytest

from oracle import adam as oadam
from oracle import rotation as orot
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


@pytest.mark.parametrize("shape", [(17, 3, 17), (24, 5, 31), (64, 2, 64)])
@pytest.mark.parametrize("deg", [0.0, 2.0, 37.0, 90.0, 133.0, 178.0])
def test_rotation_and_transpose_match_oracle(ctx, shape, deg):
    import torch
    rng = np.random.default_rng(int(deg * 10) + shape[0])
    o = rng.standard_normal(shape).astype(np.float32)
    g = rng.standard_normal(shape).astype(np.float32)
    th = math.radians(deg)
    ot = torch.tensor(o, device="cuda")
    gt = torch.tensor(g, device="cuda")
    fwd = ctx.rotate(ot, th).cpu().numpy()
    adj = ctx.rotate(gt, th, transpose=True).cpu().numpy()
    ref_f = orot.rotate(o.astype(np.float64), th)
    ref_a = orot.rotate_transpose(g.astype(np.float64), th)
    assert rel_l2(fwd, ref_f) < 1e-6
    assert rel_l2(adj, ref_a) < 1e-6
    # the GPU pair is itself an exact transpose: <R o, g> = <o, R^T g>
    lhs = float(np.sum(fwd.astype(np.float64) * g))
    rhs = float(np.sum(o.astype(np.float64) * adj))
    assert abs(lhs - rhs) < 1e-5 * max(abs(lhs), 1.0) + 1e-4


def test_rotation_full_tilt_object(ctx):
    """256^3 tilt object at 2 degrees, sampled lines against the oracle."""
    import torch
    rng = np.random.default_rng(5)
    o = rng.standard_normal((256, 8, 256)).astype(np.float32)   # 8 y-rows keep the oracle fast
    ot = torch.tensor(o, device="cuda")
    for deg in (2.0, 88.0):
        got = ctx.rotate(ot, math.radians(deg)).cpu().numpy()
        ref = orot.rotate(o.astype(np.float64), math.radians(deg))
        assert rel_l2(got, ref) < 1e-6


def test_adam_matches_oracle_over_steps(ctx):
    import torch
    rng = np.random.default_rng(6)
    n = 10007
    x = rng.standard_normal(n).astype(np.float32)
    xt, mt, vt = (torch.tensor(a, device="cuda") for a in (x, np.zeros(n, np.float32), np.zeros(n, np.float32)))
    xr, mr, vr = x.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        ctx.adam(xt, torch.tensor(g, device="cuda"), mt, vt, t, lr=1e-3)
        xr, mr, vr = oadam.adam_step(xr, g.astype(np.float64), mr, vr, t, lr=1e-3)
    torch.cuda.synchronize()
    assert rel_l2(xt.cpu().numpy(), xr) < 1e-6
    assert rel_l2(mt.cpu().numpy(), mr) < 1e-6
    assert rel_l2(vt.cpu().numpy(), vr) < 1e-6


def test_adam_with_device_count_matches_oracle_and_refuses_zero(ctx):
    """adorym_adam_dev reads t from device memory when the kernel runs: the
    same steps as the oracle's with t advanced on the device, the same bits
    as adorym_adam, and a count of 0 leaves everything unchanged and is
    reported by sync_error."""
    import torch
    from paper_2012_12686_amd._lib import EINVAL, AdorymError
    rng = np.random.default_rng(16)
    n = 10007
    x = rng.standard_normal(n).astype(np.float32)
    xt, mt, vt = (torch.tensor(a, device="cuda") for a in (x, np.zeros(n, np.float32), np.zeros(n, np.float32)))
    xh, mh, vh = xt.clone(), mt.clone(), vt.clone()
    xr, mr, vr = x.astype(np.float64), np.zeros(n), np.zeros(n)
    t_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    for t in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        gt = torch.tensor(g, device="cuda")
        t_dev.add_(1)
        ctx.adam(xt, gt, mt, vt, t_dev, lr=1e-3)
        ctx.adam(xh, gt, mh, vh, t, lr=1e-3)
        xr, mr, vr = oadam.adam_step(xr, g.astype(np.float64), mr, vr, t, lr=1e-3)
    torch.cuda.synchronize()
    ctx.sync_error()
    assert rel_l2(xt.cpu().numpy(), xr) < 1e-6
    assert rel_l2(mt.cpu().numpy(), mr) < 1e-6
    assert rel_l2(vt.cpu().numpy(), vr) < 1e-6
    for a, b in ((xt, xh), (mt, mh), (vt, vh)):
        assert torch.equal(a, b)
    before = xt.clone()
    ctx.adam(xt, gt, mt, vt, torch.zeros(1, dtype=torch.int32, device="cuda"), lr=1e-3)
    with pytest.raises(AdorymError) as ei:
        ctx.sync_error()
    assert ei.value.status == EINVAL
    assert torch.equal(xt, before)


def test_adam_complex_probe(ctx):
    import torch
    rng = np.random.default_rng(7)
    p = (rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))).astype(np.complex64)
    g = (rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))).astype(np.complex64)
    pt = torch.tensor(p, device="cuda")
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    ctx.adam(pt, torch.tensor(g, device="cuda"), m, v, 1, lr=1e-2)
    ref_re, _, _ = oadam.adam_step(p.real.astype(np.float64), g.real.astype(np.float64), 0, 0, 1, 1e-2)
    ref_im, _, _ = oadam.adam_step(p.imag.astype(np.float64), g.imag.astype(np.float64), 0, 0, 1, 1e-2)
    got = pt.cpu().numpy()
    assert rel_l2(got.real, ref_re) < 1e-6 and rel_l2(got.imag, ref_im) < 1e-6
