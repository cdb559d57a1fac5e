"""CPU pins of the float32 limits the GPU parity tests rely on.

Each entry of tests/gpu_helpers.FP32_LIMITED claims that at its evaluation
point float32 storage of the wave alone moves the gradient by several times
the tolerance: rounding each slice's wave to complex64 once, every other
operation exact (tests/fp32_limits.py), already does.  These tests check
that claim on the same inputs the GPU test uses, and check the rounding
model itself against the oracle on a well-conditioned case.
"""
import synth
import dataclasses
import math

import numpy as np
import pytest

from oracle import multislice as om
from oracle import rotation as orot
from tests.fp32_limits import loss_grad_fp32_ffts, loss_grad_stored_f32
from tests.gpu_helpers import FP32_LIMITED, TOL_G, Case, f32, rel_l2


def test_rounding_model_equals_the_oracle_up_to_float32_on_a_well_conditioned_case():
    sc = synth.small_case(seed=5, n=32, n_slices=5, lateral=48, n_pos=3, strength=30.0)
    case = Case(sc)
    ref = case.oracle_loss_grad()
    got = loss_grad_stored_f32(case.geom, case.a, case.b, case.p, case.pos, case.i_meas)
    assert abs(got[0] - ref[0]) <= 1e-6 * abs(ref[0])
    for g, r in zip(got[1:], ref[1:]):
        e = rel_l2(g, r)
        assert 0 < e < 1e-5, e          # rounding happened, and stays at float32 level here


def test_c2_vacuum_start_is_beyond_float32():
    """FP32_LIMITED['c2-vacuum-poisson']: the first 50-position minibatch of the
    64-slice workload at delta = beta = 0 with Poisson data (seed 2), as in
    test_gpu_parity.test_multislice_n128_s64_first_minibatch.  The shift
    gradients vanish there; their deviation is measured against their norm
    at half the true object, the scale that GPU test uses."""
    sc = synth.multislice_n128_s64()
    case = Case(sc, idx=slice(0, 50), poisson_seed=2)
    ref = case.oracle_loss_grad()
    got = loss_grad_stored_f32(case.geom, case.a, case.b, case.p, case.pos, case.i_meas)
    errs = [rel_l2(g, r) for g, r in zip(got[1:4], ref[1:4])]
    print("storage-rounding deviation of g_a, g_b, g_probe:", errs)
    assert min(errs) > 3 * TOL_G
    half = Case(dataclasses.replace(sc, eval_obj_a=0.5 * sc.obj_a, eval_obj_b=0.5 * sc.obj_b), idx=slice(0, 50),
                poisson_seed=2)
    scale = np.linalg.norm(half.oracle_loss_grad()[4])
    e_s = np.linalg.norm(got[4] - ref[4]) / scale
    print("storage-rounding deviation of the vanishing shift gradients, relative to their scale:", e_s)
    assert e_s > TOL_G



def test_c3_sampled_shift_gradients_are_beyond_float32():
    """FP32_LIMITED['c3-shift']: the 128-slice workload's positions 0, 101 and
    199 at its evaluation point (half the true object, perturbed probe,
    nominal positions; Gaussian loss), as in the two 128-slice GPU tests.
    Only the shift gradients are affected; the object and probe gradients
    stay two orders of magnitude inside TOL_G."""
    import numpy as np
    sc = synth.multislice_n128_s128()
    case = Case(sc, idx=np.array([0, 101, 199]))
    ref = case.oracle_loss_grad()
    got = loss_grad_stored_f32(case.geom, case.a, case.b, case.p, case.pos, case.i_meas)
    errs = [rel_l2(g, r) for g, r in zip(got[1:], ref[1:])]
    print("storage-rounding deviation of g_a, g_b, g_probe, g_shift:", errs)
    assert errs[3] > TOL_G
    assert max(errs[:3]) < TOL_G / 10


def test_tilt_angle_at_256_slices_is_beyond_float32():
    """FP32_LIMITED['tilt-256-poisson']: the tilt job's positions 0, 44 and 99
    at 34 degrees, half the true object, Poisson data (seed 55), as in
    test_gpu_tilt.test_tilt_angle_three_positions_every_output."""
    sc, _ = synth.tilt_job()
    geom = om.Geometry.from_scan(sc)
    theta, sample = math.radians(34.0), np.array([0, 44, 99])
    a, b, p = f32(0.5 * sc.obj_a), f32(0.5 * sc.obj_b), f32(sc.probe)
    corner, shift = synth.split_positions(np.asarray(sc.positions, dtype=np.float64))
    pos = (corner + f32(shift))[sample]
    ra, rb = orot.rotate(a, theta), orot.rotate(b, theta)
    ta, tb = orot.rotate(sc.obj_a, theta), orot.rotate(sc.obj_b, theta)
    i_s = f32(np.random.default_rng(55).poisson(om.forward(geom, ta, tb, sc.probe, pos)))
    ref = om.loss_grad(geom, ra, rb, p, pos, i_s)
    got = loss_grad_stored_f32(geom, ra, rb, p, pos, i_s)
    errs = [rel_l2(g, r) for g, r in zip(got[1:4], ref[1:4])]
    print("storage-rounding deviation of g_a, g_b, g_probe:", errs)
    assert min(errs) > TOL_G


@pytest.mark.parametrize("job", [14, 17, 13, 18])
def test_mixed_scan_compared_jobs_are_beyond_float32(job):
    """FP32_LIMITED['mix-half-object']: each job of the 32-scan mix that
    test_gpu_batching compares with the oracle (its smallest of each probe
    size) at half the true object and the true positions, with its data
    (Poisson seed 500 + job for the Poisson-loss jobs).  For the outputs the
    entry lists, a float32 evaluation with single-precision library FFTs
    misses TOL_G; for the others it meets TOL_G."""
    limited = FP32_LIMITED["mix-half-object"]["outputs"][job]
    sc = synth.mixed_scan_jobs()[job]
    geom = om.Geometry.from_scan(sc)
    a, b, p = f32(0.5 * sc.obj_a), f32(0.5 * sc.obj_b), f32(sc.probe)
    corner, shift = synth.split_positions(np.asarray(sc.positions, dtype=np.float64))
    pos = corner + f32(shift)
    i_true = om.forward(geom, sc.obj_a, sc.obj_b, sc.probe, np.asarray(sc.positions, dtype=np.float64))
    if sc.loss == "poisson":
        i_true = np.random.default_rng(500 + job).poisson(i_true)
    im = f32(i_true)
    ref = om.loss_grad(geom, a, b, p, pos, im)
    got = loss_grad_fp32_ffts(geom, a, b, p, pos, im)
    errs = {k: rel_l2(g, r) for k, g, r in zip(("g_a", "g_b", "g_probe", "g_shift"), got[1:], ref[1:])}
    print(f"job {job}: float32-pipeline deviation", errs)
    for k, e in errs.items():
        assert (e > TOL_G) == (k in limited), (k, e)
