"""torch.autograd front end of the multislice loss.

``multislice_loss(obj_a, obj_b, probe, positions, i_meas, geom)`` returns the
data-mismatch loss L (a float64 scalar tensor) of the far-field multislice
model and is differentiable with respect to the object (delta/beta or
real/imag), the complex probe and the float scan positions.

The gradient is the library's hand-written adjoint, not autograd tracing:
the forward call runs the fused forward + loss + reverse-sweep kernel
(which rebuilds slice waves from checkpoints instead of storing every
slice) and keeps the gradients; backward multiplies them by the incoming
gradient.  Complex gradients follow dL/dRe + i dL/dIm, PyTorch's own
convention for real-valued losses of complex tensors.
"""
from __future__ import annotations

from typing import Optional

import torch

from .api import Context, Geometry, split_positions

_default_ctx: dict = {}


def _context(device: torch.device) -> Context:
    key = (device.type, device.index)
    if key not in _default_ctx:
        _default_ctx[key] = Context(device)
    return _default_ctx[key]


class MultisliceLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, obj_a, obj_b, probe, positions, i_meas, geom: Geometry, lib: Optional[Context]):
        lib = lib or _context(obj_a.device)
        corner, shift = split_positions(positions.detach())
        out = lib.loss_grad(geom, obj_a.detach().contiguous(), obj_b.detach().contiguous(),
                            probe.detach().contiguous(), corner, shift, i_meas.contiguous(), grads=True)
        fctx.save_for_backward(out["g_a"], out["g_b"], out["g_probe"], out["g_shift"])
        fctx.pos_dtype = positions.dtype
        return out["loss"]

    @staticmethod
    def backward(fctx, grad_out):
        g_a, g_b, g_p, g_s = fctx.saved_tensors
        s = grad_out.to(torch.float32)
        ga = g_a * s if fctx.needs_input_grad[0] else None
        gb = g_b * s if fctx.needs_input_grad[1] else None
        gp = g_p * s.to(g_p.dtype) if fctx.needs_input_grad[2] else None
        gs = (g_s * s).to(fctx.pos_dtype) if fctx.needs_input_grad[3] else None
        return ga, gb, gp, gs, None, None, None


def multislice_loss(obj_a: torch.Tensor, obj_b: torch.Tensor, probe: torch.Tensor, positions: torch.Tensor,
                    i_meas: torch.Tensor, geom: Geometry, ctx: Optional[Context] = None) -> torch.Tensor:
    """Differentiable loss of one minibatch; see the module docstring."""
    return MultisliceLoss.apply(obj_a, obj_b, probe, positions, i_meas, geom, ctx)
