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
