"""The float32 reference model agrees with the FP64 oracle where the problem
is well conditioned, so it measures rounding, not a different model."""
import numpy as np

import synth
from oracle import multislice as om
from tests.fp32_model import loss_grad_fp32
from tests.gpu_helpers import Case, rel_l2


def test_fp32_model_tracks_oracle_on_gaussian_case():
    sc = synth.small_case(seed=5, n=16, n_slices=6, lateral=30, n_pos=3, strength=30.0)
    case = Case(sc)
    ref = case.oracle_loss_grad()
    got = loss_grad_fp32(case.geom, case.a, case.b, case.p, case.pos, case.i_meas)
    assert abs(got[0] - ref[0]) < 1e-5 * abs(ref[0])
    for g, r in zip(got[1:], ref[1:]):
        assert rel_l2(g, r) < 1e-4
