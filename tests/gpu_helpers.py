"""Shared helpers for the GPU parity tests (imports torch lazily)."""
import numpy as np

from oracle import multislice as om
import synth


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
    b = np.asarray(b, dtype=np.complex128 if np.iscomplexobj(b) else np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def f32(x):
    """Round to what the GPU sees, back in float64 / complex128 for the oracle."""
    x = np.asarray(x)
    if np.iscomplexobj(x):
        return x.astype(np.complex64).astype(np.complex128)
    return x.astype(np.float32).astype(np.float64)


class Case:
    """A scan evaluated at one point, with inputs rounded once to float32."""

    def __init__(self, scan, idx=None, poisson_seed=None, use_eval=True):
        sl = slice(None) if idx is None else idx
        self.scan = scan
        self.geom = om.Geometry.from_scan(scan)
        a = scan.eval_obj_a if (use_eval and scan.eval_obj_a is not None) else scan.obj_a
        b = scan.eval_obj_b if (use_eval and scan.eval_obj_b is not None) else scan.obj_b
        p = scan.eval_probe if (use_eval and scan.eval_probe is not None) else scan.probe
        pos = scan.eval_positions if (use_eval and scan.eval_positions is not None) else scan.positions
        self.a, self.b, self.p = f32(a), f32(b), f32(p)
        pos = np.asarray(pos, dtype=np.float64)[sl]
        corner, shift = synth.split_positions(pos)
        self.corner = corner
        self.shift = f32(shift)
        self.pos = corner.astype(np.float64) + self.shift     # what the GPU evaluates
        # measured data: the oracle at the ground truth (true positions)
        true_pos = np.asarray(scan.positions, dtype=np.float64)[sl]
        i_true = om.forward(self.geom, scan.obj_a, scan.obj_b, scan.probe, true_pos)
        if poisson_seed is not None:
            i_true = np.random.default_rng(poisson_seed).poisson(i_true).astype(np.float64)
        self.i_meas = f32(i_true)

    def torch_inputs(self, device="cuda"):
        import torch
        t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=device)
        return dict(obj_a=t(self.a, torch.float32), obj_b=t(self.b, torch.float32),
                    probe=t(self.p, torch.complex64), corner=t(self.corner, torch.int32),
                    shift=t(self.shift, torch.float32)), t(self.i_meas, torch.float32)

    def oracle_forward(self):
        return om.forward(self.geom, self.a, self.b, self.p, self.pos)

    def oracle_loss_grad(self):
        return om.loss_grad(self.geom, self.a, self.b, self.p, self.pos, self.i_meas)


# ---------------------------------------------------------------------------
# Tolerances (float32 GPU path against the float64 oracle)
# ---------------------------------------------------------------------------
TOL_I = 1e-5      # intensities, relative L2
TOL_G = 1e-4      # gradients, relative L2

# Evaluation points at which float32 storage of the wave alone moves the
# gradient by several times TOL_G: rounding each slice's wave to complex64
# once, with every other operation exact, already does.  That premise is
# pinned on the CPU for each entry (tests/test_fp32_limits.py).  A test at
# such a point still asserts the regression guard below (a fixed bound, not
# a parity claim), and reports the TOL_G comparison as an expected failure
# with the measured error.
FP32_LIMITED = {
    "c2-vacuum-poisson": dict(
        guard=1.5e-3,
        reason=("64-slice minibatch at the delta = beta = 0 start, Poisson loss: the residual "
                "1 - I_meas/(I + eps) of far-field pixels the vacuum model barely lights amplifies the "
                "absolute float32 noise of the detector field; rounding each slice's wave to complex64 "
                "alone moves the object and probe gradients by 6.3e-4 and the vanishing shift "
                "gradients by 1.3e-4 of their scale")),
    "c3-shift": dict(
        guard=5e-4,
        reason=("shift gradients of the 128-slice workload's sampled positions (Gaussian loss, half the "
                "true object): each is a small real sum over the probe spectrum, and rounding each "
                "slice's wave to complex64 alone moves them by 1.7e-4")),
    "tilt-256-poisson": dict(
        guard=1e-3,
        reason=("256-slice tilt angle at half the true object, Poisson loss: rounding each of the 256 "
                "slices' waves to complex64 alone moves the object and probe gradients by 1.75e-4")),
    "mix-half-object": dict(
        guard=3e-3,
        outputs={14: ("g_shift",), 17: ("g_b", "g_probe"), 13: ("g_b", "g_probe"),
                 18: ("g_a", "g_b", "g_probe", "g_shift")},
        reason=("the 32-scan mix's smallest job of each probe size at half the true object: a float32 "
                "evaluation with single-precision library FFTs misses the tolerance on these outputs "
                "(1.4e-4 to 1.2e-3), the far-field residual of barely lit pixels amplifying the "
                "transforms' absolute rounding")),
}


def assert_grads(pairs, limited=None, vanishing=(), defer=False):
    """Relative L2 of each (name, got, ref) gradient against TOL_G, and for
    each (name, got, ref, scale) of ``vanishing`` the absolute error against
    TOL_G * scale (outputs whose exact value vanishes at the evaluation point:
    relative L2 is meaningless there, so the bound is TOL_G times the
    output's norm at a non-degenerate point of the same scan).

    ``limited``: a key of FP32_LIMITED; the outputs are then held to its
    regression guard and a miss of TOL_G is reported with pytest.xfail (at
    once, or, with ``defer``, returned as messages for xfail_if)."""
    over = []
    for name, got, ref in pairs:
        e = rel_l2(got, ref)
        print(f"{name}: GPU rel-L2 {e:.3e}")
        if limited is None:
            assert e <= TOL_G, (name, e)
        else:
            assert e <= FP32_LIMITED[limited]["guard"], (name, e, limited)
            if e > TOL_G:
                over.append(f"{name} {e:.2e}")
    for name, got, ref, scale in vanishing:
        err = float(np.linalg.norm(np.asarray(got, dtype=np.float64).ravel()
                                   - np.asarray(ref, dtype=np.float64).ravel()))
        print(f"{name}: |GPU - oracle| {err:.3e} = {err / scale:.3e} x the scale {scale:.3e} "
              f"(|oracle| {np.linalg.norm(ref):.3e})")
        assert scale > 0
        if limited is None:
            assert err <= TOL_G * scale, (name, err, scale)
        else:
            assert err <= FP32_LIMITED[limited]["guard"] * scale, (name, err, scale, limited)
            if err > TOL_G * scale:
                over.append(f"{name} {err / scale:.2e} of its scale")
    msgs = [f"{limited}: {', '.join(over)} > {TOL_G:g} ({FP32_LIMITED[limited]['reason']})"] if over else []
    if not defer:
        xfail_if(msgs)
    return msgs


def xfail_if(msgs):
    """Report FP32_LIMITED misses of TOL_G (collected with defer=True) as an
    expected failure, after every other assertion of the test has passed."""
    import pytest
    if msgs:
        pytest.xfail("; ".join(msgs))


def loss_tolerance(geom, i_ref, i_meas):
    """TOL_I * ||I|| * ||dL/dI|| (Cauchy-Schwarz), doubled for rounding."""
    dldi = om.loss_dI(geom.loss, i_ref, i_meas, geom.eps, i_ref.size)
    return 2 * TOL_I * np.linalg.norm(i_ref) * np.linalg.norm(dldi)
