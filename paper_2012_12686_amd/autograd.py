"""torch.autograd front end of the multislice loss.

``multislice_loss(obj_a, obj_b, probe, positions, i_meas, geom)`` returns the
data-mismatch loss L (a float64 scalar tensor) of the far-field multislice
model and is differentiable with respect to the object (delta/beta or
real/imag), the complex probe and the float scan positions.

The gradient is the library's hand-written adjoint, not autograd tracing.
By default forward calls adorym_loss_fwd (forward sweep and loss; it keeps
each position's slice checkpoints and exit wave in a workspace held by the
autograd context) and backward calls adorym_loss_bwd, which resumes the
reverse sweep from them -- rebuilding slice waves from the checkpoints
instead of storing every slice -- and scales the gradients by the incoming
gradient.  ``lazy=False`` instead runs the fused forward + loss + reverse
sweep (adorym_loss_grad) inside forward and keeps its gradients.  Complex
gradients follow dL/dRe + i dL/dIm, PyTorch's own convention for
real-valued losses of complex tensors.
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
    """Fused form: loss and every gradient in forward (adorym_loss_grad)."""

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


class MultisliceLossLazy(torch.autograd.Function):
    """Split form (the default): gradients only when backward runs.  Forward
    computes the loss and keeps the slice checkpoints and exit waves in a
    workspace (adorym_loss_fwd); backward resumes from them
    (adorym_loss_bwd)."""

    @staticmethod
    def forward(fctx, obj_a, obj_b, probe, positions, i_meas, geom: Geometry, lib: Optional[Context]):
        lib = lib or _context(obj_a.device)
        corner, shift = split_positions(positions.detach())
        args = (obj_a.detach().contiguous(), obj_b.detach().contiguous(), probe.detach().contiguous(), corner,
                shift, i_meas.contiguous())
        loss, ws = lib.loss_fwd(geom, *args)
        fctx.lib, fctx.geom, fctx.args, fctx.ws = lib, geom, args, ws
        fctx.pos_dtype = positions.dtype
        return loss

    @staticmethod
    def backward(fctx, grad_out):
        out = fctx.lib.loss_bwd(fctx.geom, *fctx.args, workspace=fctx.ws)
        fctx.ws = None
        s = grad_out.to(torch.float32)
        ga = out["g_a"] * s if fctx.needs_input_grad[0] else None
        gb = out["g_b"] * s if fctx.needs_input_grad[1] else None
        gp = out["g_probe"] * s.to(torch.complex64) if fctx.needs_input_grad[2] else None
        gs = (out["g_shift"] * s).to(fctx.pos_dtype) if fctx.needs_input_grad[3] else None
        return ga, gb, gp, gs, None, None, None


def multislice_loss(obj_a: torch.Tensor, obj_b: torch.Tensor, probe: torch.Tensor, positions: torch.Tensor,
                    i_meas: torch.Tensor, geom: Geometry, ctx: Optional[Context] = None,
                    lazy: bool = True) -> torch.Tensor:
    """Differentiable loss of one minibatch; see the module docstring.  With
    ``lazy`` (the default) the gradients are computed only if backward runs;
    ``lazy=False`` computes them in forward with the fused call."""
    if lazy:
        return MultisliceLossLazy.apply(obj_a, obj_b, probe, positions, i_meas, geom, ctx)
    return MultisliceLoss.apply(obj_a, obj_b, probe, positions, i_meas, geom, ctx)


def _scaled(fctx, grads, grad_out, needs):
    s = grad_out.to(torch.float64)
    out = []
    for g, need in zip(grads, needs):
        if g is None or not need:
            out.append(None)
        elif g.is_complex():
            out.append(g * s.to(torch.float32).to(g.dtype))
        else:
            out.append((g * s.to(g.dtype)) if g.dtype == torch.float64 else g * s.to(torch.float32))
    return out


class MultisliceLossModes(torch.autograd.Function):
    """Loss of several incoherent probe modes (Eq. multimode); gradients for
    the object, the modes [M][N][N] and the positions."""

    @staticmethod
    def forward(fctx, obj_a, obj_b, probes, positions, i_meas, geom: Geometry, lib: Optional[Context]):
        lib = lib or _context(obj_a.device)
        corner, shift = split_positions(positions.detach())
        out = lib.loss_grad_modes(geom, obj_a.detach().contiguous(), obj_b.detach().contiguous(),
                                  probes.detach().contiguous(), corner, shift, i_meas.contiguous())
        fctx.save_for_backward(out["g_a"], out["g_b"], out["g_probe"], out["g_shift"])
        fctx.pos_dtype = positions.dtype
        return out["loss"]

    @staticmethod
    def backward(fctx, grad_out):
        ga, gb, gp, gs = _scaled(fctx, fctx.saved_tensors, grad_out, fctx.needs_input_grad[:4])
        return ga, gb, gp, (gs.to(fctx.pos_dtype) if gs is not None else None), None, None, None


class MultisliceLossGaps(torch.autograd.Function):
    """Sparse multislice loss; also differentiable in the S-1 gaps (float64)."""

    @staticmethod
    def forward(fctx, obj_a, obj_b, probe, positions, gaps, i_meas, geom: Geometry, lib: Optional[Context]):
        lib = lib or _context(obj_a.device)
        corner, shift = split_positions(positions.detach())
        out = lib.loss_grad_gaps(geom, obj_a.detach().contiguous(), obj_b.detach().contiguous(),
                                 probe.detach().contiguous(), corner, shift,
                                 None if gaps is None else gaps.detach().contiguous(), i_meas.contiguous())
        fctx.save_for_backward(out["g_a"], out["g_b"], out["g_probe"], out["g_shift"], out["g_gaps"])
        fctx.pos_dtype = positions.dtype
        return out["loss"]

    @staticmethod
    def backward(fctx, grad_out):
        ga, gb, gp, gs, gg = _scaled(fctx, fctx.saved_tensors, grad_out, fctx.needs_input_grad[:5])
        return ga, gb, gp, (gs.to(fctx.pos_dtype) if gs is not None else None), gg, None, None, None


class MultisliceLossNearfield(torch.autograd.Function):
    """Near-field loss; also differentiable in the detector distances (float64)."""

    @staticmethod
    def forward(fctx, obj_a, obj_b, probe, positions, dists, dist_idx, i_meas, geom: Geometry, kind: str,
                lib: Optional[Context]):
        lib = lib or _context(obj_a.device)
        corner, shift = split_positions(positions.detach())
        out = lib.loss_grad_nearfield(geom, obj_a.detach().contiguous(), obj_b.detach().contiguous(),
                                      probe.detach().contiguous(), corner, shift, dists.detach().contiguous(),
                                      dist_idx.contiguous(), i_meas.contiguous(), kind=kind)
        fctx.save_for_backward(out["g_a"], out["g_b"], out["g_probe"], out["g_shift"], out["g_dist"])
        fctx.pos_dtype = positions.dtype
        return out["loss"]

    @staticmethod
    def backward(fctx, grad_out):
        ga, gb, gp, gs, gd = _scaled(fctx, fctx.saved_tensors, grad_out, fctx.needs_input_grad[:5])
        return ga, gb, gp, (gs.to(fctx.pos_dtype) if gs is not None else None), gd, None, None, None, None, None


class MultisliceLossDefocus(torch.autograd.Function):
    """Loss with the probe defocused first; also differentiable in the
    defocus distance (a float64 scalar tensor; its value is read on the host)."""

    @staticmethod
    def forward(fctx, obj_a, obj_b, probe, positions, defocus, i_meas, geom: Geometry, lib: Optional[Context]):
        lib = lib or _context(obj_a.device)
        corner, shift = split_positions(positions.detach())
        out = lib.loss_grad_defocus(geom, obj_a.detach().contiguous(), obj_b.detach().contiguous(),
                                    probe.detach().contiguous(), corner, shift, float(defocus.detach().item()),
                                    i_meas.contiguous())
        g_def = out["g_defocus"].to(defocus.device, defocus.dtype)
        fctx.save_for_backward(out["g_a"], out["g_b"], out["g_probe"], out["g_shift"], g_def)
        fctx.pos_dtype = positions.dtype
        return out["loss"]

    @staticmethod
    def backward(fctx, grad_out):
        ga, gb, gp, gs, gd = _scaled(fctx, fctx.saved_tensors, grad_out, fctx.needs_input_grad[:5])
        return ga, gb, gp, (gs.to(fctx.pos_dtype) if gs is not None else None), gd, None, None, None


class ObjectPrior(torch.autograd.Function):
    """l1 / reweighted l1 / total-variation prior of the object (Eq. tikhonov)."""

    @staticmethod
    def forward(fctx, obj_a, obj_b, obj_repr: str, l1_a: float, l1_b: float, tv: float, weights, lib):
        lib = lib or _context(obj_a.device)
        out = lib.prior_grad(obj_repr, obj_a.detach().contiguous(), obj_b.detach().contiguous(), l1_a=l1_a,
                             l1_b=l1_b, tv=tv, weights=weights, accumulate=False)
        fctx.save_for_backward(out["g_a"], out["g_b"])
        return out["value"]

    @staticmethod
    def backward(fctx, grad_out):
        ga, gb = _scaled(fctx, fctx.saved_tensors, grad_out, fctx.needs_input_grad[:2])
        return ga, gb, None, None, None, None, None, None


def multislice_loss_modes(obj_a, obj_b, probes, positions, i_meas, geom, ctx=None):
    return MultisliceLossModes.apply(obj_a, obj_b, probes, positions, i_meas, geom, ctx)


def multislice_loss_gaps(obj_a, obj_b, probe, positions, gaps, i_meas, geom, ctx=None):
    return MultisliceLossGaps.apply(obj_a, obj_b, probe, positions, gaps, i_meas, geom, ctx)


def multislice_loss_nearfield(obj_a, obj_b, probe, positions, dists, dist_idx, i_meas, geom, kind="paraxial",
                              ctx=None):
    return MultisliceLossNearfield.apply(obj_a, obj_b, probe, positions, dists, dist_idx, i_meas, geom, kind, ctx)


def multislice_loss_defocus(obj_a, obj_b, probe, positions, defocus, i_meas, geom, ctx=None):
    return MultisliceLossDefocus.apply(obj_a, obj_b, probe, positions, defocus, i_meas, geom, ctx)


def object_prior(obj_a, obj_b, obj_repr="delta_beta", l1_a=0.0, l1_b=0.0, tv=0.0, weights=None, ctx=None):
    return ObjectPrior.apply(obj_a, obj_b, obj_repr, l1_a, l1_b, tv, weights, ctx)
