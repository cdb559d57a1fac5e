"""C ABI contract tests that need no GPU.

The library loads, exports every function include/adorym.h declares, the
ctypes struct mirrors the C struct byte for byte, and host-side argument
validation and workspace sizing behave as documented.
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2012_12686_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adorym.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adorym_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = _lib.load()
    names = declared_functions()
    assert names, "no declarations found"
    for n in names:
        assert hasattr(lib, n), f"{n} not exported"
    assert sorted(_lib.SIGNATURES) == names


def test_geom_struct_layout_matches_c(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "adorym.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(adorym_geom),'
                   ' offsetof(adorym_geom, wavelength_m), offsetof(adorym_geom, loss),'
                   ' offsetof(adorym_geom, eps), offsetof(adorym_geom, flags)); return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    G = _lib.Geom
    assert got == [ctypes.sizeof(G), G.wavelength_m.offset, G.loss.offset, G.eps.offset, G.flags.offset]


def test_job_struct_layout_matches_c(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "adorym.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(adorym_job),'
                   ' offsetof(adorym_job, obj_a), offsetof(adorym_job, batch),'
                   ' offsetof(adorym_job, i_meas), offsetof(adorym_job, ws_bytes),'
                   ' offsetof(adorym_job, intensity)); return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    J = _lib.Job
    assert got == [ctypes.sizeof(J), J.obj_a.offset, J.batch.offset, J.i_meas.offset, J.ws_bytes.offset,
                   J.intensity.offset]


def _geom(**kw):
    base = dict(n=128, n_slices=64, obj_ny=256, obj_nx=256, wavelength_m=1.24e-10, pixel_m=1e-8,
                slice_dz_m=1e-8, loss=0, obj_repr=0, ckpt_every=16, eps=1e-6, flags=0)
    base.update(kw)
    return _lib.Geom(**base)


def test_workspace_size_formula():
    lib = _lib.load()
    g = _geom()
    size = lib.adorym_workspace_size(ctypes.byref(g), 50)
    nn = 128 * 128 * 8                  # one complex64 field
    slots = 63 // 16 + 1 + 1            # slices 0, 16, 32, 48 and the last (63)
    # probe spectrum + its gradient sum, loss and shift partials for up to 8
    # workgroups per position, barrier counters and the 64 slices' absorption
    # bounds, XCD ids, probe-kernel counters, probe-gradient partials,
    # checkpoints, the 15 interior waves of one recomputed checkpoint segment,
    # two double-buffered exchange fields per position, and every position's
    # float32 object gradient of both planes
    small = 2 * nn + 50 * 8 * 8 + 50 * 8 * 2 * 8 + (50 + 64) * 4 + 50 * 8 * 4 + 64 * 4 + 50 * 4 * nn
    expect = small + 50 * nn + 50 * slots * nn + 50 * 15 * nn + 50 * 64 * 2 * 128 * 128 * 4
    assert expect <= size < expect + 12 * 256
    assert lib.adorym_workspace_size(ctypes.byref(_geom(n_slices=0)), 50) == 0
    assert lib.adorym_workspace_size(ctypes.byref(g), 0) == 0
    # a forward call needs no checkpoints, partials or staging
    fwd = lib.adorym_forward_workspace_size(ctypes.byref(g), 50)
    assert small <= fwd < small + 12 * 256
    # the deterministic flag does not change the workspace
    gd = _geom(flags=_lib.DETERMINISTIC)
    assert lib.adorym_workspace_size(ctypes.byref(gd), 50) == size


def test_supported_sizes():
    lib = _lib.load()
    assert all(lib.adorym_supports_n(n) == 1 for n in (64, 96, 128, 192))
    assert lib.adorym_supports_n(100) == 0 and lib.adorym_supports_n(0) == 0


def test_set_split_validation_without_device():
    lib = _lib.load()
    assert lib.adorym_set_split(None, 128, 4) == _lib.EINVAL


def test_null_context_rejected_without_touching_the_device():
    lib = _lib.load()
    g = _geom()
    st = lib.adorym_forward(None, ctypes.byref(g), None, None, None, None, None, 1, None, None, 0)
    assert st == _lib.EINVAL
    st = lib.adorym_loss_grad(None, ctypes.byref(g), None, None, None, None, None, 1, None, None, 0,
                              None, None, None, None, None, None)
    assert st == _lib.EINVAL
    assert lib.adorym_sync_error(None) == _lib.EINVAL
    assert lib.adorym_destroy(None) == _lib.EINVAL


def test_extension_workspace_sizes():
    """Unequal spacing, probe modes, near field and priors: the documented
    sizes on top of the loss-and-gradient workspace; 0 on bad input."""
    lib = _lib.load()
    g = _geom()
    base = lib.adorym_workspace_size(ctypes.byref(g), 50)
    nn8 = 128 * 128 * 8
    # gap-gradient partials: 50 positions x up to 8 parts x 63 gaps, FP64
    gaps = lib.adorym_gaps_workspace_size(ctypes.byref(g), 50)
    assert base + 50 * 8 * 63 * 8 <= gaps < base + 50 * 8 * 63 * 8 + 256
    # probe modes: two intensity planes, per mode the checkpoints and the exit wave
    slots = 63 // 16 + 1 + 1
    for m in (1, 3):
        got = lib.adorym_modes_workspace_size(ctypes.byref(g), 50, m)
        expect = base + 2 * 50 * 128 * 128 * 4 + m * (50 * slots * nn8 + 50 * nn8)
        assert expect <= got < expect + (2 + 2 * m) * 256
    assert lib.adorym_modes_workspace_size(ctypes.byref(g), 50, 0) == 0
    # near field: distance partials, detector spectra, one transfer function per distance, phase slope
    nf = lib.adorym_nearfield_workspace_size(ctypes.byref(g), 50, 4)
    expect = base + 50 * 8 * 8 + 50 * nn8 + 4 * nn8 + 128 * 128 * 4
    assert expect <= nf < expect + 4 * 256
    assert lib.adorym_nearfield_workspace_size(ctypes.byref(g), 50, 0) == 0
    # priors: a few scalars and one FP64 partial per (64 x 4 tile, 32-slice run), at least 2048
    assert lib.adorym_prior_workspace_size(128, 512, 512) == (8 + 8 * 128 * 4) * 8
    assert lib.adorym_prior_workspace_size(1, 5, 7) == (8 + 2048) * 8
    assert lib.adorym_prior_workspace_size(0, 5, 7) == 0


def test_extension_entry_points_reject_bad_arguments_without_a_device():
    lib = _lib.load()
    g = _geom()
    P = None
    assert lib.adorym_loss_grad_gaps(None, ctypes.byref(g), P, P, P, P, P, 1, P, P, P, 0, P, P, P, P, P, P,
                                     P) == _lib.EINVAL
    assert lib.adorym_forward_gaps(None, ctypes.byref(g), P, P, P, P, P, 1, P, P, P, 0) == _lib.EINVAL
    assert lib.adorym_loss_grad_modes(None, ctypes.byref(g), P, P, P, 2, P, P, 1, P, P, 0, P, P, P, P, P,
                                      P) == _lib.EINVAL
    assert lib.adorym_forward_nearfield(None, ctypes.byref(g), P, P, P, P, P, 1, 0, P, 1, P, P, P,
                                        0) == _lib.EINVAL
    assert lib.adorym_loss_grad_nearfield(None, ctypes.byref(g), P, P, P, P, P, 1, 0, P, 1, P, P, P, 0, P, P, P,
                                          P, P, P, P) == _lib.EINVAL
    assert lib.adorym_prior_grad(None, 0, P, P, 1, 1, 1, 0.0, 0.0, 0.0, P, P, P, 0, P, P, P, 1) == _lib.EINVAL
    assert lib.adorym_prior_weights(None, 0, P, P, 1, 1, 1, 1e-3, P, 0, P, P) == _lib.EINVAL
    assert lib.adorym_support_project(None, 0, P, P, P, 4) == _lib.EINVAL
    assert lib.adorym_forward_defocus(None, ctypes.byref(g), P, P, P, P, P, 1, 1e-6, P, P, 0) == _lib.EINVAL
    assert lib.adorym_loss_grad_defocus(None, ctypes.byref(g), P, P, P, P, P, 1, 1e-6, P, P, 0, P, P, P, P, P, P,
                                        P) == _lib.EINVAL
