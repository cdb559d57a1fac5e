"""Python front end of libadorym over torch device tensors.

PyTorch supplies device memory and the stream; the computation is the C ABI
(include/adorym.h).  All functions here only check shapes/dtypes, allocate
outputs and workspace, and pass raw device pointers.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Optional

import torch

from . import _lib
from ._lib import Geom, check, load

LOSSES = {"gaussian": _lib.LOSS_GAUSSIAN, "poisson": _lib.LOSS_POISSON}
REPRS = {"delta_beta": _lib.OBJ_DELTA_BETA, "real_imag": _lib.OBJ_REAL_IMAG}


@dataclasses.dataclass
class Geometry:
    """Scan geometry and options (mirrors ``adorym_geom``)."""

    n: int
    n_slices: int
    obj_ny: int
    obj_nx: int
    wavelength_m: float
    pixel_m: float
    slice_dz_m: float
    loss: str = "gaussian"
    obj_repr: str = "delta_beta"
    ckpt_every: int = 16
    eps: float = 1e-6
    accumulate: bool = False
    deterministic: bool = False   # bitwise-reproducible object gradients (FP64 ordered sum)

    def to_c(self) -> Geom:
        return Geom(self.n, self.n_slices, self.obj_ny, self.obj_nx, self.wavelength_m, self.pixel_m,
                    self.slice_dz_m, LOSSES[self.loss], REPRS[self.obj_repr], self.ckpt_every, self.eps,
                    (_lib.ACCUMULATE_GRADS if self.accumulate else 0)
                    | (_lib.DETERMINISTIC if self.deterministic else 0))

    @classmethod
    def from_scan(cls, scan, **kw):
        s, ly, lx = scan.obj_shape
        return cls(scan.n, s, ly, lx, scan.wavelength_m, scan.pixel_m, scan.slice_dz_m, scan.loss,
                   scan.obj_repr, eps=scan.eps, **kw)


def split_positions(pos: torch.Tensor):
    """Float (y, x) positions -> int32 corners floor(r + 0.5) and float32 shifts r - corner."""
    corner = torch.floor(pos.double() + 0.5)
    shift = (pos.double() - corner).float()
    return corner.to(torch.int32).contiguous(), shift.contiguous()


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Context:
    """One library context per device/stream."""

    def __init__(self, device: Optional[torch.device] = None):
        load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._ctx = ctypes.c_void_p(0)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        check(load().adorym_create(ctypes.byref(self._ctx), self.device.index or 0, ctypes.c_void_p(stream)))

    def _bind_stream(self):
        stream = torch.cuda.current_stream(self.device).cuda_stream
        check(load().adorym_set_stream(self._ctx, ctypes.c_void_p(stream)), self._ctx)

    def close(self):
        if self._ctx:
            load().adorym_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync_error(self):
        """Synchronise and raise on a deferred device error (e.g. a chunk out of range)."""
        check(load().adorym_sync_error(self._ctx), self._ctx)

    def set_split(self, n: int, k: int):
        """Workgroups per position for probe size n (0 = automatic)."""
        check(load().adorym_set_split(self._ctx, n, k), self._ctx)

    def profile_start(self, max_launches: int = 4096):
        """Time the main multislice kernel of each later call with HIP events."""
        check(load().adorym_profile_start(self._ctx, max_launches), self._ctx)

    def profile_stop(self):
        """(summed kernel milliseconds, number of timed launches)."""
        ms, cnt = ctypes.c_double(0), ctypes.c_int32(0)
        check(load().adorym_profile_stop(self._ctx, ctypes.byref(ms), ctypes.byref(cnt)), self._ctx)
        return ms.value, cnt.value

    # --------------------------------------------------------------- calls
    def workspace_size(self, geom: Geometry, batch: int, forward: bool = False) -> int:
        """Workspace bytes of a loss_grad call (forward=True: of a forward call)."""
        fn = load().adorym_forward_workspace_size if forward else load().adorym_workspace_size
        return int(fn(ctypes.byref(geom.to_c()), batch))

    def workspace(self, geom: Geometry, batch: int, forward: bool = False) -> torch.Tensor:
        return torch.empty(self.workspace_size(geom, batch, forward), dtype=torch.uint8, device=self.device)

    def _check_inputs(self, geom, obj_a, obj_b, probe, corner, shift):
        n, s, ly, lx = geom.n, geom.n_slices, geom.obj_ny, geom.obj_nx
        for t, shape, dt, name in ((obj_a, (s, ly, lx), torch.float32, "obj_a"),
                                   (obj_b, (s, ly, lx), torch.float32, "obj_b"),
                                   (probe, (n, n), torch.complex64, "probe")):
            if tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous() or t.device != self.device:
                raise ValueError(f"{name}: expected contiguous {dt} {shape} on {self.device}, got "
                                 f"{t.dtype} {tuple(t.shape)} on {t.device}")
        b = corner.shape[0]
        if corner.dtype != torch.int32 or tuple(corner.shape) != (b, 2) or not corner.is_contiguous():
            raise ValueError("corner: expected contiguous int32 [B][2]")
        if shift.dtype != torch.float32 or tuple(shift.shape) != (b, 2) or not shift.is_contiguous():
            raise ValueError("shift: expected contiguous float32 [B][2]")
        return b

    def forward(self, geom, obj_a, obj_b, probe, corner, shift, out=None, workspace=None):
        """Predicted intensities [B][N][N] (zero frequency at N/2)."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        out = out if out is not None else torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=self.device)
        ws = workspace if workspace is not None else self.workspace(geom, b, forward=True)
        st = load().adorym_forward(self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b),
                                   _ptr(torch.view_as_real(probe)), _ptr(corner), _ptr(shift), b, _ptr(out),
                                   _ptr(ws), ws.numel())
        check(st, self._ctx)
        return out

    def forward_static(self, geom, obj_a, obj_b, probe, corner, shift, out):
        """forward() with the library's static 64 MiB device scratch as its
        workspace (adorym_forward_static): no allocation by the library or
        here; ``out`` is the caller's float32 [B][N][N] tensor."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        if out.dtype != torch.float32 or tuple(out.shape) != (b, geom.n, geom.n) or not out.is_contiguous():
            raise ValueError("out: expected contiguous float32 [B][N][N]")
        st = load().adorym_forward_static(self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b),
                                          _ptr(torch.view_as_real(probe)), _ptr(corner), _ptr(shift), b, _ptr(out))
        check(st, self._ctx)
        return out

    def loss_grad(self, geom, obj_a, obj_b, probe, corner, shift, i_meas, grads=True, intensity=False,
                  out=None, workspace=None):
        """Loss (device float64 scalar) and gradients.

        Returns dict with ``loss`` and, if ``grads``, ``g_a``, ``g_b``, ``g_probe``
        (complex64), ``g_shift``; with ``intensity`` also the predicted ``intensity``.
        ``out`` may carry preallocated tensors under the same names.
        """
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        if tuple(i_meas.shape) != (b, geom.n, geom.n) or i_meas.dtype != torch.float32 or not i_meas.is_contiguous():
            raise ValueError("i_meas: expected contiguous float32 [B][N][N]")
        out = dict(out or {})
        dev = self.device
        if "loss" not in out:
            out["loss"] = torch.empty((), dtype=torch.float64, device=dev)
        if grads:
            for name, shape, dt in (("g_a", obj_a.shape, torch.float32), ("g_b", obj_b.shape, torch.float32),
                                    ("g_probe", probe.shape, torch.complex64), ("g_shift", (b, 2), torch.float32)):
                if name not in out:
                    out[name] = (torch.zeros if geom.accumulate else torch.empty)(shape, dtype=dt, device=dev)
        if intensity and "intensity" not in out:
            out["intensity"] = torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=dev)
        ws = workspace if workspace is not None else self.workspace(geom, b)
        gp = out.get("g_probe")
        st = load().adorym_loss_grad(
            self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b), _ptr(torch.view_as_real(probe)),
            _ptr(corner), _ptr(shift), b, _ptr(i_meas), _ptr(ws), ws.numel(), _ptr(out["loss"]),
            _ptr(out.get("g_a")), _ptr(out.get("g_b")), _ptr(torch.view_as_real(gp) if gp is not None else None),
            _ptr(out.get("g_shift")), _ptr(out.get("intensity")))
        check(st, self._ctx)
        return out

    # ------------------------------------------- probe defocus
    def forward_defocus(self, geom, obj_a, obj_b, probe, corner, shift, defocus_m: float, out=None, workspace=None):
        """Predicted intensities with the probe Fresnel-propagated by ``defocus_m`` metres first."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        out = out if out is not None else torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=self.device)
        ws = workspace if workspace is not None else self.workspace(geom, b, forward=True)
        st = load().adorym_forward_defocus(self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b),
                                           _ptr(torch.view_as_real(probe)), _ptr(corner), _ptr(shift), b,
                                           float(defocus_m), _ptr(out), _ptr(ws), ws.numel())
        check(st, self._ctx)
        return out

    def loss_grad_defocus(self, geom, obj_a, obj_b, probe, corner, shift, defocus_m: float, i_meas, grads=True,
                          intensity=False, out=None, workspace=None):
        """As :meth:`loss_grad` with the probe defocused by ``defocus_m``; with
        ``grads`` the outputs also hold ``g_defocus`` (float64 scalar, dL/d defocus in 1/m)
        and ``g_probe`` is the gradient with respect to the undefocused probe."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        if tuple(i_meas.shape) != (b, geom.n, geom.n) or i_meas.dtype != torch.float32 or not i_meas.is_contiguous():
            raise ValueError("i_meas: expected contiguous float32 [B][N][N]")
        out = dict(out or {})
        dev = self.device
        if "loss" not in out:
            out["loss"] = torch.empty((), dtype=torch.float64, device=dev)
        if grads:
            for name, shape, dt in (("g_a", obj_a.shape, torch.float32), ("g_b", obj_b.shape, torch.float32),
                                    ("g_probe", probe.shape, torch.complex64), ("g_shift", (b, 2), torch.float32),
                                    ("g_defocus", (), torch.float64)):
                if name not in out:
                    out[name] = (torch.zeros if geom.accumulate else torch.empty)(shape, dtype=dt, device=dev)
        if intensity and "intensity" not in out:
            out["intensity"] = torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=dev)
        ws = workspace if workspace is not None else self.workspace(geom, b)
        gp = out.get("g_probe")
        st = load().adorym_loss_grad_defocus(
            self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b), _ptr(torch.view_as_real(probe)),
            _ptr(corner), _ptr(shift), b, float(defocus_m), _ptr(i_meas), _ptr(ws), ws.numel(), _ptr(out["loss"]),
            _ptr(out.get("g_a")), _ptr(out.get("g_b")), _ptr(torch.view_as_real(gp) if gp is not None else None),
            _ptr(out.get("g_shift")), _ptr(out.get("g_defocus")), _ptr(out.get("intensity")))
        check(st, self._ctx)
        return out

    # ------------------------------------------- unequal slice spacing
    def _check_gaps(self, geom, gaps):
        if geom.n_slices == 1 and gaps is None:
            return None
        if (gaps is None or gaps.dtype != torch.float64 or tuple(gaps.shape) != (geom.n_slices - 1,)
                or not gaps.is_contiguous() or gaps.device != self.device):
            raise ValueError(f"gaps: expected contiguous float64 [{geom.n_slices - 1}] on {self.device}")
        return gaps

    def forward_gaps(self, geom, obj_a, obj_b, probe, corner, shift, gaps, out=None, workspace=None):
        """Predicted intensities with unequal slice spacing: ``gaps`` float64
        [S-1] (metres, device) are the distances from slice j to j+1."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        gaps = self._check_gaps(geom, gaps)
        out = out if out is not None else torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=self.device)
        ws = workspace if workspace is not None else self.workspace(geom, b, forward=True)
        st = load().adorym_forward_gaps(self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b),
                                        _ptr(torch.view_as_real(probe)), _ptr(corner), _ptr(shift), b, _ptr(gaps),
                                        _ptr(out), _ptr(ws), ws.numel())
        check(st, self._ctx)
        return out

    def gaps_workspace_size(self, geom: Geometry, batch: int) -> int:
        return int(load().adorym_gaps_workspace_size(ctypes.byref(geom.to_c()), batch))

    def loss_grad_gaps(self, geom, obj_a, obj_b, probe, corner, shift, gaps, i_meas, grads=True, intensity=False,
                       out=None, workspace=None):
        """As :meth:`loss_grad` with unequal slice spacing ``gaps``; with
        ``grads`` the outputs also hold ``g_gaps`` (float64 [S-1], dL/d gap in 1/m)."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        gaps = self._check_gaps(geom, gaps)
        if tuple(i_meas.shape) != (b, geom.n, geom.n) or i_meas.dtype != torch.float32 or not i_meas.is_contiguous():
            raise ValueError("i_meas: expected contiguous float32 [B][N][N]")
        out = dict(out or {})
        dev = self.device
        if "loss" not in out:
            out["loss"] = torch.empty((), dtype=torch.float64, device=dev)
        if grads:
            for name, shape, dt in (("g_a", obj_a.shape, torch.float32), ("g_b", obj_b.shape, torch.float32),
                                    ("g_probe", probe.shape, torch.complex64), ("g_shift", (b, 2), torch.float32),
                                    ("g_gaps", (max(geom.n_slices - 1, 0),), torch.float64)):
                if name not in out:
                    out[name] = (torch.zeros if geom.accumulate else torch.empty)(shape, dtype=dt, device=dev)
        if intensity and "intensity" not in out:
            out["intensity"] = torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=dev)
        ws = workspace if workspace is not None else torch.empty(self.gaps_workspace_size(geom, b),
                                                                 dtype=torch.uint8, device=dev)
        gp = out.get("g_probe")
        gg = out.get("g_gaps")
        st = load().adorym_loss_grad_gaps(
            self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b), _ptr(torch.view_as_real(probe)),
            _ptr(corner), _ptr(shift), b, _ptr(gaps), _ptr(i_meas), _ptr(ws), ws.numel(), _ptr(out["loss"]),
            _ptr(out.get("g_a")), _ptr(out.get("g_b")), _ptr(torch.view_as_real(gp) if gp is not None else None),
            _ptr(out.get("g_shift")), _ptr(gg if gg is not None and gg.numel() else None),
            _ptr(out.get("intensity")))
        check(st, self._ctx)
        return out

    # ------------------------------------------------- near field
    _KINDS = {"paraxial": _lib.PROP_PARAXIAL, "sommerfeld": _lib.PROP_SOMMERFELD}

    def _check_nf(self, b, dists, dist_idx):
        if dists.dtype != torch.float64 or dists.dim() != 1 or not dists.is_contiguous() or dists.device != self.device:
            raise ValueError("dists: expected contiguous float64 [n_dist] on the device")
        if dist_idx.dtype != torch.int32 or tuple(dist_idx.shape) != (b,) or not dist_idx.is_contiguous() \
                or dist_idx.device != self.device:
            raise ValueError("dist_idx: expected contiguous int32 [B] on the device")
        return dists.numel()

    def nearfield_workspace_size(self, geom: Geometry, batch: int, n_dist: int) -> int:
        return int(load().adorym_nearfield_workspace_size(ctypes.byref(geom.to_c()), batch, n_dist))

    def forward_nearfield(self, geom, obj_a, obj_b, probe, corner, shift, dists, dist_idx, kind="paraxial",
                          out=None, workspace=None):
        """Near-field detector intensities [B][N][N] (natural order): the exit
        wave Fresnel-propagated over dists[dist_idx[b]] (paraxial or Sommerfeld kernel)."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        nd = self._check_nf(b, dists, dist_idx)
        out = out if out is not None else torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=self.device)
        ws = workspace if workspace is not None else torch.empty(self.nearfield_workspace_size(geom, b, nd),
                                                                 dtype=torch.uint8, device=self.device)
        st = load().adorym_forward_nearfield(self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b),
                                             _ptr(torch.view_as_real(probe)), _ptr(corner), _ptr(shift), b,
                                             self._KINDS[kind], _ptr(dists), nd, _ptr(dist_idx), _ptr(out), _ptr(ws),
                                             ws.numel())
        check(st, self._ctx)
        return out

    def loss_grad_nearfield(self, geom, obj_a, obj_b, probe, corner, shift, dists, dist_idx, i_meas,
                            kind="paraxial", grads=True, intensity=False, out=None, workspace=None):
        """As :meth:`loss_grad` for the near-field detector; with ``grads`` also
        ``g_dist`` (float64 [n_dist], dL/d distance in 1/m)."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        nd = self._check_nf(b, dists, dist_idx)
        if tuple(i_meas.shape) != (b, geom.n, geom.n) or i_meas.dtype != torch.float32 or not i_meas.is_contiguous():
            raise ValueError("i_meas: expected contiguous float32 [B][N][N]")
        out = dict(out or {})
        dev = self.device
        if "loss" not in out:
            out["loss"] = torch.empty((), dtype=torch.float64, device=dev)
        if grads:
            for name, shape, dt in (("g_a", obj_a.shape, torch.float32), ("g_b", obj_b.shape, torch.float32),
                                    ("g_probe", probe.shape, torch.complex64), ("g_shift", (b, 2), torch.float32),
                                    ("g_dist", (nd,), torch.float64)):
                if name not in out:
                    out[name] = (torch.zeros if geom.accumulate else torch.empty)(shape, dtype=dt, device=dev)
        if intensity and "intensity" not in out:
            out["intensity"] = torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=dev)
        ws = workspace if workspace is not None else torch.empty(self.nearfield_workspace_size(geom, b, nd),
                                                                 dtype=torch.uint8, device=dev)
        gp = out.get("g_probe")
        st = load().adorym_loss_grad_nearfield(
            self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b), _ptr(torch.view_as_real(probe)),
            _ptr(corner), _ptr(shift), b, self._KINDS[kind], _ptr(dists), nd, _ptr(dist_idx), _ptr(i_meas), _ptr(ws),
            ws.numel(), _ptr(out["loss"]), _ptr(out.get("g_a")), _ptr(out.get("g_b")),
            _ptr(torch.view_as_real(gp) if gp is not None else None), _ptr(out.get("g_shift")),
            _ptr(out.get("g_dist")), _ptr(out.get("intensity")))
        check(st, self._ctx)
        return out

    # ------------------------------------------------- object priors
    def _check_obj(self, *ts):
        shape = tuple(ts[0].shape)
        for t in ts:
            if t is None:
                continue
            if t.dtype != torch.float32 or t.dim() != 3 or tuple(t.shape) != shape or not t.is_contiguous() \
                    or t.device != self.device:
                raise ValueError(f"expected contiguous float32 [S][Ly][Lx] tensors of one shape on {self.device}")
        return shape

    def prior_grad(self, obj_repr, obj_a, obj_b, l1_a=0.0, l1_b=0.0, tv=0.0, weights=None, out=None,
                   accumulate=True, workspace=None):
        """Object priors (Eq. tikhonov): l1 / reweighted l1 (``weights`` = (w_a, w_b)) and TV.
        Returns ``{"value", "g_a", "g_b"}``; with ``accumulate`` the gradients are added onto
        ``out["g_a"], out["g_b"]`` (e.g. the data gradient)."""
        self._bind_stream()
        w_a, w_b = weights if weights is not None else (None, None)
        s, ly, lx = self._check_obj(obj_a, obj_b, w_a, w_b)
        out = dict(out or {})
        dev = self.device
        out.setdefault("value", torch.empty((), dtype=torch.float64, device=dev))
        for k, ref in (("g_a", obj_a), ("g_b", obj_b)):
            if k not in out:
                out[k] = torch.zeros_like(ref)
        self._check_obj(obj_a, out["g_a"], out["g_b"])
        ws = workspace if workspace is not None else torch.empty(
            int(load().adorym_prior_workspace_size(s, ly, lx)), dtype=torch.uint8, device=dev)
        check(load().adorym_prior_grad(self._ctx, REPRS[obj_repr], _ptr(obj_a), _ptr(obj_b), s, ly, lx,
                                       float(l1_a), float(l1_b), float(tv), _ptr(w_a), _ptr(w_b), _ptr(ws),
                                       ws.numel(), _ptr(out["value"]), _ptr(out["g_a"]), _ptr(out["g_b"]),
                                       int(bool(accumulate))), self._ctx)
        return out

    def prior_weights(self, obj_repr, snap_a, snap_b, eps, workspace=None):
        """Reweighted-l1 weights W = max|q| / (|q| + eps) of a snapshot."""
        self._bind_stream()
        s, ly, lx = self._check_obj(snap_a, snap_b)
        w_a, w_b = torch.empty_like(snap_a), torch.empty_like(snap_b)
        ws = workspace if workspace is not None else torch.empty(
            int(load().adorym_prior_workspace_size(s, ly, lx)), dtype=torch.uint8, device=self.device)
        check(load().adorym_prior_weights(self._ctx, REPRS[obj_repr], _ptr(snap_a), _ptr(snap_b), s, ly, lx,
                                          float(eps), _ptr(ws), ws.numel(), _ptr(w_a), _ptr(w_b)), self._ctx)
        return w_a, w_b

    def support_project(self, obj_repr, mask, obj_a, obj_b):
        """Finite support, in place: voxels with mask == 0 become vacuum."""
        self._bind_stream()
        self._check_obj(obj_a, obj_b)
        if mask.dtype != torch.uint8 or mask.numel() != obj_a.numel() or not mask.is_contiguous() \
                or mask.device != self.device:
            raise ValueError("mask: expected contiguous uint8 of the object's size")
        check(load().adorym_support_project(self._ctx, REPRS[obj_repr], _ptr(mask), _ptr(obj_a), _ptr(obj_b),
                                            obj_a.numel()), self._ctx)
        return obj_a, obj_b

    # ------------------------------------------------- probe modes
    def modes_workspace_size(self, geom: Geometry, batch: int, n_modes: int) -> int:
        return int(load().adorym_modes_workspace_size(ctypes.byref(geom.to_c()), batch, n_modes))

    def loss_grad_modes(self, geom, obj_a, obj_b, probes, corner, shift, i_meas, grads=True, intensity=False,
                        out=None, workspace=None):
        """Loss and gradients for M incoherent probe modes ``probes`` complex64 [M][N][N]
        (Eq. multimode): the loss sees the intensity summed over the modes.

        Same outputs as :meth:`loss_grad`, with ``g_probe`` [M][N][N] and
        ``intensity`` the summed intensity.
        """
        self._bind_stream()
        if probes.dim() != 3 or probes.dtype != torch.complex64 or not probes.is_contiguous():
            raise ValueError("probes: expected contiguous complex64 [M][N][N]")
        m = probes.shape[0]
        b = self._check_inputs(geom, obj_a, obj_b, probes[0], corner, shift)
        if tuple(i_meas.shape) != (b, geom.n, geom.n) or i_meas.dtype != torch.float32 or not i_meas.is_contiguous():
            raise ValueError("i_meas: expected contiguous float32 [B][N][N]")
        out = dict(out or {})
        dev = self.device
        if "loss" not in out:
            out["loss"] = torch.empty((), dtype=torch.float64, device=dev)
        if grads:
            for name, shape, dt in (("g_a", obj_a.shape, torch.float32), ("g_b", obj_b.shape, torch.float32),
                                    ("g_probe", probes.shape, torch.complex64), ("g_shift", (b, 2), torch.float32)):
                if name not in out:
                    out[name] = (torch.zeros if geom.accumulate else torch.empty)(shape, dtype=dt, device=dev)
        if intensity and "intensity" not in out:
            out["intensity"] = torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=dev)
        ws = workspace if workspace is not None else torch.empty(self.modes_workspace_size(geom, b, m),
                                                                 dtype=torch.uint8, device=dev)
        gp = out.get("g_probe")
        st = load().adorym_loss_grad_modes(
            self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b), _ptr(torch.view_as_real(probes)), m,
            _ptr(corner), _ptr(shift), b, _ptr(i_meas), _ptr(ws), ws.numel(), _ptr(out["loss"]),
            _ptr(out.get("g_a")), _ptr(out.get("g_b")), _ptr(torch.view_as_real(gp) if gp is not None else None),
            _ptr(out.get("g_shift")), _ptr(out.get("intensity")))
        check(st, self._ctx)
        return out

    def rotate(self, obj: torch.Tensor, theta: float, transpose: bool = False, out=None) -> torch.Tensor:
        """Rotate a float32 [Z][Y][X] object about y by theta (radians); transpose=True is R^T."""
        self._bind_stream()
        if obj.dtype != torch.float32 or obj.dim() != 3 or not obj.is_contiguous():
            raise ValueError("obj: expected contiguous float32 [Z][Y][X]")
        out = out if out is not None else torch.empty_like(obj)
        lz, ly, lx = obj.shape
        check(load().adorym_rotate(self._ctx, _ptr(obj), _ptr(out), lz, ly, lx, float(theta), int(transpose)),
              self._ctx)
        return out

    def adam(self, x: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, t, lr: float,
             beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        """In-place Adam step on float32 (or complex64, as pairs of reals) tensors.
        ``t``: the 1-based iteration count, a Python int, or a device int32
        scalar tensor read when the kernel runs (adorym_adam_dev: graph
        capturable with a count that advances between replays)."""
        self._bind_stream()
        arrs = [torch.view_as_real(a) if a.is_complex() else a for a in (x, g, m, v)]
        n = arrs[0].numel()
        for a in arrs:
            if a.dtype != torch.float32 or a.numel() != n or not a.is_contiguous():
                raise ValueError("adam: expected contiguous float32/complex64 tensors of one size")
        if isinstance(t, torch.Tensor):
            if t.dtype != torch.int32 or t.numel() != 1 or t.device != self.device:
                raise ValueError("adam: t must be an int32 scalar tensor on the context's device")
            check(load().adorym_adam_dev(self._ctx, *[_ptr(a) for a in arrs], n, lr, beta1, beta2, eps, _ptr(t)),
                  self._ctx)
        else:
            check(load().adorym_adam(self._ctx, *[_ptr(a) for a in arrs], n, lr, beta1, beta2, eps, t), self._ctx)


    def plan(self, jobs) -> "Plan":
        """A batched plan over many jobs; see ``Plan``."""
        return Plan(self, jobs)

    def loss_grad_batched(self, jobs):
        """One-shot batched loss and gradients of ``jobs`` (outputs in each job's ``out``)."""
        self._bind_stream()
        jobs = list(jobs)
        cjobs = _job_structs(self, jobs)
        check(load().adorym_loss_grad_batched(self._ctx, cjobs, len(jobs)), self._ctx)
        return jobs

    def autotune(self, jobs, reps: int = 2):
        """Library autotuner: the fastest split per probe size among ``jobs``, set on this
        context.  Returns {N: split}."""
        self._bind_stream()
        jobs = list(jobs)
        cjobs = _job_structs(self, jobs)
        chosen = (ctypes.c_int32 * 4)()
        check(load().adorym_autotune(self._ctx, cjobs, len(jobs), reps, chosen), self._ctx)
        present = {j.geom.n for j in jobs if not j.geom.deterministic}
        return {n: int(k) for n, k in zip((64, 96, 128, 192), chosen) if n in present}

    # ------------------------------------------------- loss now, gradients later
    def loss_fwd_workspace_size(self, geom: Geometry, batch: int) -> int:
        return int(load().adorym_loss_fwd_workspace_size(ctypes.byref(geom.to_c()), batch))

    def loss_fwd(self, geom, obj_a, obj_b, probe, corner, shift, i_meas, workspace=None, intensity=False):
        """Loss only; the workspace keeps what :meth:`loss_bwd` needs.  Returns (loss, workspace[, intensity])."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        ws = workspace if workspace is not None else torch.empty(self.loss_fwd_workspace_size(geom, b),
                                                                 dtype=torch.uint8, device=self.device)
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        inten = torch.empty((b, geom.n, geom.n), dtype=torch.float32, device=self.device) if intensity else None
        check(load().adorym_loss_fwd(self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b),
                                     _ptr(torch.view_as_real(probe)), _ptr(corner), _ptr(shift), b, _ptr(i_meas),
                                     _ptr(ws), ws.numel(), _ptr(loss), _ptr(inten)), self._ctx)
        return (loss, ws, inten) if intensity else (loss, ws)

    def loss_bwd(self, geom, obj_a, obj_b, probe, corner, shift, i_meas, workspace, grad_scale=1.0, out=None):
        """Gradients of grad_scale * L from a :meth:`loss_fwd` workspace."""
        self._bind_stream()
        b = self._check_inputs(geom, obj_a, obj_b, probe, corner, shift)
        out = dict(out or {})
        dev = self.device
        for name, shape, dt in (("g_a", obj_a.shape, torch.float32), ("g_b", obj_b.shape, torch.float32),
                                ("g_probe", probe.shape, torch.complex64), ("g_shift", (b, 2), torch.float32)):
            if name not in out:
                out[name] = (torch.zeros if geom.accumulate else torch.empty)(shape, dtype=dt, device=dev)
        check(load().adorym_loss_bwd(self._ctx, ctypes.byref(geom.to_c()), _ptr(obj_a), _ptr(obj_b),
                                     _ptr(torch.view_as_real(probe)), _ptr(corner), _ptr(shift), b, _ptr(i_meas),
                                     _ptr(workspace), workspace.numel(), float(grad_scale), _ptr(out["g_a"]),
                                     _ptr(out["g_b"]), _ptr(torch.view_as_real(out["g_probe"])),
                                     _ptr(out["g_shift"])), self._ctx)
        return out


@dataclasses.dataclass
class Job:
    """One scan for a batched plan: inputs, outputs and workspace (all device tensors)."""

    geom: Geometry
    obj_a: torch.Tensor
    obj_b: torch.Tensor
    probe: torch.Tensor
    corner: torch.Tensor
    shift: torch.Tensor
    i_meas: torch.Tensor
    out: dict = dataclasses.field(default_factory=dict)
    workspace: Optional[torch.Tensor] = None


class Plan:
    """Loss and gradients of many jobs in one persistent launch per probe size.

    The plan keeps references to every tensor it names; ``run()`` only enqueues
    kernels (capturable in a graph).  Outputs are in each job's ``out`` dict
    (``loss``, ``g_a``, ``g_b``, ``g_probe``, ``g_shift``, and ``intensity``
    [B][N][N] float32 if the job's ``out`` held that tensor when the plan was
    made).
    """

    def __init__(self, ctx: "Context", jobs):
        self.ctx = ctx
        self.jobs = list(jobs)
        self._cjobs = _job_structs(ctx, self.jobs)
        self._plan = ctypes.c_void_p(0)
        check(load().adorym_plan_create(ctx._ctx, self._cjobs, len(self.jobs), ctypes.byref(self._plan)), ctx._ctx)

    def run(self):
        self.ctx._bind_stream()
        check(load().adorym_plan_run(self.ctx._ctx, self._plan), self.ctx._ctx)

    def close(self):
        if self._plan:
            load().adorym_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _job_structs(ctx: "Context", jobs):
    """C job table of ``jobs`` (allocating missing outputs and workspaces)."""
    dev = ctx.device
    cjobs = (_lib.Job * len(jobs))()
    for i, j in enumerate(jobs):
        b = ctx._check_inputs(j.geom, j.obj_a, j.obj_b, j.probe, j.corner, j.shift)
        o = j.out
        o.setdefault("loss", torch.empty((), dtype=torch.float64, device=dev))
        o.setdefault("g_a", torch.empty_like(j.obj_a))
        o.setdefault("g_b", torch.empty_like(j.obj_b))
        o.setdefault("g_probe", torch.empty_like(j.probe))
        o.setdefault("g_shift", torch.empty((b, 2), dtype=torch.float32, device=dev))
        if j.workspace is None:
            j.workspace = ctx.workspace(j.geom, b)
        cj = cjobs[i]
        cj.g = j.geom.to_c()
        cj.obj_a, cj.obj_b = j.obj_a.data_ptr(), j.obj_b.data_ptr()
        cj.probe = torch.view_as_real(j.probe).data_ptr()
        cj.corner, cj.shift, cj.batch = j.corner.data_ptr(), j.shift.data_ptr(), b
        cj.i_meas = j.i_meas.data_ptr()
        cj.loss, cj.g_a, cj.g_b = o["loss"].data_ptr(), o["g_a"].data_ptr(), o["g_b"].data_ptr()
        cj.g_probe = torch.view_as_real(o["g_probe"]).data_ptr()
        cj.g_shift = o["g_shift"].data_ptr()
        cj.workspace, cj.ws_bytes = j.workspace.data_ptr(), j.workspace.numel()
        if "intensity" in o:
            n = j.geom.n
            if (o["intensity"].dtype != torch.float32 or tuple(o["intensity"].shape) != (b, n, n)
                    or not o["intensity"].is_contiguous() or o["intensity"].device != dev):
                raise ValueError("out['intensity'] must be a contiguous float32 [B][N][N] tensor on the device")
            cj.intensity = o["intensity"].data_ptr()
    return cjobs


def supports_n(n: int) -> bool:
    return bool(load().adorym_supports_n(n))
