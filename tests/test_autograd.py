"""The autograd front end: convention pin on the CPU, parity on the GPU."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_helpers import Case, rel_l2


def test_torch_complex_gradient_convention_is_dre_plus_i_dim():
    """The library returns dL/dRe + i dL/dIm; PyTorch uses the same for real losses."""
    z = torch.tensor([1.5 - 0.5j, -0.25 + 2.0j], dtype=torch.complex128, requires_grad=True)
    loss = (z.real ** 3 + 2.0 * z.imag ** 2 + z.real * z.imag).sum()
    loss.backward()
    x, y = z.detach().real, z.detach().imag
    expect = (3 * x ** 2 + y) + 1j * (4 * y + x)
    assert torch.allclose(z.grad, expect)


@pytest.mark.gpu
def test_autograd_function_matches_oracle_and_scales():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_12686_amd import Geometry, multislice_loss
    sc = synth.small_case(seed=41, n=64, n_slices=5, lateral=96, n_pos=4, strength=30.0)
    case = Case(sc)
    dev = torch.device("cuda")
    a = torch.tensor(case.a, dtype=torch.float32, device=dev, requires_grad=True)
    b = torch.tensor(case.b, dtype=torch.float32, device=dev, requires_grad=True)
    p = torch.tensor(case.p, dtype=torch.complex64, device=dev, requires_grad=True)
    pos = torch.tensor(case.pos, dtype=torch.float64, device=dev, requires_grad=True)
    im = torch.tensor(case.i_meas, dtype=torch.float32, device=dev)
    geom = Geometry.from_scan(sc)
    loss = multislice_loss(a, b, p, pos, im, geom)
    (3.0 * loss).backward()
    L, ga, gb, gp, gs = case.oracle_loss_grad()
    assert abs(float(loss.detach()) - L) < 1e-4 * abs(L)
    for got, ref in ((a.grad, ga), (b.grad, gb), (p.grad, gp), (pos.grad, gs)):
        assert rel_l2(got.detach().cpu().numpy(), 3.0 * ref) < 1e-4
