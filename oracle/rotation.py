"""Object rotation for tilt series, FP64 (test infrastructure only).

Rotation of the object about the vertical (y) axis by resampling every
xz-plane (Sec. S1.D.2 "Object orientation", Eq. rotation_transform): each
output voxel (x_t, z_t) is mapped back to the unrotated object by

    x_0 = cos(t) (x_t - c) - sin(t) (z_t - c) + c
    z_0 = sin(t) (x_t - c) + cos(t) (z_t - c) + c

with c = (L - 1)/2 the plane centre, and the value is taken by bilinear
interpolation, zero outside the array.  The operation is linear, o_t = R o,
with at most four non-zeros per row of R; its adjoint is the exact transpose
R^T (a scatter with the same weights), which is what a gradient needs.

Object layout is slice-major [Z][Y][X] (Z along the beam).
"""
from __future__ import annotations

import numpy as np


def _taps(theta, lz, lx):
    """Source indices and weights of the four bilinear taps per output voxel."""
    cz, cx = (lz - 1) / 2.0, (lx - 1) / 2.0
    zt, xt = np.meshgrid(np.arange(lz, dtype=np.float64), np.arange(lx, dtype=np.float64), indexing="ij")
    c, s = np.cos(theta), np.sin(theta)
    x0 = c * (xt - cx) - s * (zt - cz) + cx
    z0 = s * (xt - cx) + c * (zt - cz) + cz
    xf, zf = np.floor(x0), np.floor(z0)
    wx, wz = x0 - xf, z0 - zf
    xf, zf = xf.astype(np.int64), zf.astype(np.int64)
    taps = []
    for dz, wzz in ((0, 1.0 - wz), (1, wz)):
        for dx, wxx in ((0, 1.0 - wx), (1, wx)):
            zi, xi = zf + dz, xf + dx
            ok = (zi >= 0) & (zi < lz) & (xi >= 0) & (xi < lx)
            taps.append((np.where(ok, zi, 0), np.where(ok, xi, 0), np.where(ok, wzz * wxx, 0.0)))
    return taps


def rotate(obj, theta):
    """R_theta obj for obj [Z][Y][X]: rotate every xz-plane by theta (radians)."""
    lz, ly, lx = obj.shape
    out = np.zeros(obj.shape, dtype=np.float64)
    for zi, xi, w in _taps(theta, lz, lx):
        # out[z_t, y, x_t] += w[z_t, x_t] * obj[zi, y, xi]
        out += w[:, None, :] * obj[zi[:, None, :], np.arange(ly)[None, :, None], xi[:, None, :]]
    return out


def rotate_transpose(g, theta):
    """R_theta^T g: scatter every output voxel back onto its four taps."""
    lz, ly, lx = g.shape
    out = np.zeros(g.shape, dtype=np.float64)
    yy = np.broadcast_to(np.arange(ly)[None, :, None], (lz, ly, lx))
    for zi, xi, w in _taps(theta, lz, lx):
        zz = np.broadcast_to(zi[:, None, :], (lz, ly, lx))
        xx = np.broadcast_to(xi[:, None, :], (lz, ly, lx))
        np.add.at(out, (zz, yy, xx), w[:, None, :] * g)
    return out
