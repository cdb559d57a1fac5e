"""The allocation-free forward entry point, adorym_forward_static, through the
C ABI: the same intensities as adorym_forward (whose workspace the caller
allocates) on two calls in a row, the second with a smaller input, and a
refusal, before any device work, of a batch whose workspace exceeds the
static scratch."""
import numpy as np
import pytest

import synth
from tests.gpu_helpers import TOL_I, Case, rel_l2

pytestmark = pytest.mark.gpu


def test_static_forward_equals_the_workspace_forward_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_12686_amd import Context, Geometry
    from paper_2012_12686_amd._lib import ENOMEM, AdorymError
    ctx = Context()
    try:
        cases = (synth.small_case(seed=61, n=128, n_slices=9, lateral=200, n_pos=50, strength=30.0),
                 synth.small_case(seed=62, n=64, n_slices=5, lateral=96, n_pos=3, strength=30.0))
        for sc in cases:
            case = Case(sc)
            inp, _ = case.torch_inputs()
            g = Geometry.from_scan(sc)
            print(f"{sc.name}: forward workspace {ctx.workspace_size(g, len(case.pos), True)} bytes", flush=True)
            ref = ctx.forward(g, **inp)
            out = torch.full_like(ref, float("nan"))
            ctx.forward_static(g, **inp, out=out)
            torch.cuda.synchronize()
            ctx.sync_error()
            assert torch.equal(out, ref), sc.name
            e = rel_l2(out.cpu().numpy(), case.oracle_forward())
            print(f"{sc.name}: bitwise equal to adorym_forward, rel-L2 to the oracle {e:.3e}")
            assert e <= TOL_I
        # 200 positions at N = 128 need more than the 64 MiB scratch
        big = synth.small_case(seed=63, n=128, n_slices=2, lateral=160, n_pos=200, strength=30.0)
        inp, _ = Case(big).torch_inputs()
        g = Geometry.from_scan(big)
        assert ctx.workspace_size(g, 200, True) > 64 << 20
        out = torch.zeros((200, 128, 128), dtype=torch.float32, device="cuda")
        with pytest.raises(AdorymError) as ei:
            ctx.forward_static(g, **inp, out=out)
        assert ei.value.status == ENOMEM and "64 MiB" in str(ei.value)
        torch.cuda.synchronize()
        assert torch.count_nonzero(out) == 0
        ctx.sync_error()
    finally:
        ctx.close()
