"""How far float32 evaluation moves the gradient at a given point.

TEST INFRASTRUCTURE ONLY.  Two models of a float32 evaluation, each compared
with the FP64 oracle on the CPU to show that an evaluation point is beyond
what float32 can reach (tests/gpu_helpers.FP32_LIMITED):

* loss_grad_stored_f32: the oracle's forward model and reverse sweep in
  FP64 throughout, with one change: every wave a float32 implementation has
  to hold between two steps of the multislice recursion is rounded to
  complex64 when it is formed -- the placed probe p_b and the wave psi_{j+1}
  after each propagation (Alg. 1, MultislicePropagate).  Transforms,
  modulation, loss, residual and the reverse sweep stay exact.  Rounding to
  nearest is the smallest error such storage makes, so the deviation of this
  model estimates what storing the wave in float32 alone costs.
* loss_grad_fp32_ffts: the whole evaluation in complex64/float32 with
  SciPy's single-precision FFTs (pocketfft), every slice wave kept: what a
  float32 evaluation with library-quality transforms deviates where the
  transforms' rounding, not the storage, dominates.

Both are built from the oracle's steps and NumPy/SciPy; they share nothing
with the HIP library and are used by CPU tests only.
"""
import numpy as np
import scipy.fft as sfft

from oracle import multislice as om

C64 = np.complex64
F32 = np.float32


def _r64(x):
    return np.asarray(x).astype(np.complex64).astype(np.complex128)


def loss_grad_stored_f32(geom, obj_a, obj_b, probe, positions, i_meas):
    """(loss, g_a, g_b, g_probe, g_shift) as om.loss_grad, with the waves held
    between slices rounded to complex64."""
    corners, shifts = om.split_position(positions)
    n, s = geom.n, geom.n_slices
    kdz = geom.kdz
    ta = om.take_chunks(obj_a, corners, n)
    tb = om.take_chunks(obj_b, corners, n)
    t = om.transmission(ta, tb, geom.obj_repr, kdz)
    hs = geom.gap_kernels()
    psi = _r64(om.fourier_shift(probe, shifts))
    psis = np.empty((len(corners), s, n, n), dtype=np.complex128)
    phis = np.empty_like(psis)
    for j in range(s):
        psis[:, j] = psi
        phi = psi * t[:, j]
        phis[:, j] = phi
        if j < s - 1:
            psi = _r64(om.fresnel_propagate(phi, hs[j]))
    det = om.far_field(phi)
    i_pred = np.abs(det) ** 2
    value = om.loss_value(geom.loss, i_pred, i_meas, geom.eps)
    d_di = om.loss_dI(geom.loss, i_pred, i_meas, geom.eps, i_pred.size)
    lam = om.far_field_adjoint(2.0 * d_di * det)
    g_ta = np.empty_like(ta)
    g_tb = np.empty_like(tb)
    for j in range(s - 1, -1, -1):
        if geom.obj_repr == "delta_beta":
            z = np.conj(phis[:, j]) * lam
            g_ta[:, j] = kdz * np.imag(z)
            g_tb[:, j] = -kdz * np.real(z)
        else:
            z = np.conj(psis[:, j]) * lam
            g_ta[:, j] = np.real(z)
            g_tb[:, j] = np.imag(z)
        mu = np.conj(t[:, j]) * lam
        if j > 0:
            lam = om.fresnel_propagate_adjoint(mu, hs[j - 1])
    e = om.shift_ramp(n, shifts)
    big_g = om.fft2u(mu)
    big_p = om.fft2u(probe)
    g_probe = om.ifft2u(np.sum(big_g * np.conj(e), axis=0))
    f = np.fft.fftfreq(n)
    z = np.conj(big_g) * big_p[None] * e
    g_shift = np.stack([np.sum(np.real(z * (-2j * np.pi) * f[None, :, None]), axis=(1, 2)),
                        np.sum(np.real(z * (-2j * np.pi) * f[None, None, :]), axis=(1, 2))], axis=1)
    return (value, om.scatter_chunks(g_ta, corners, obj_a.shape), om.scatter_chunks(g_tb, corners, obj_b.shape),
            g_probe, g_shift)


def loss_grad_fp32_ffts(geom, a, b, p, pos, i_meas):
    """(loss, g_a, g_b, g_probe, g_shift) of the plain multislice model and its
    reverse sweep in complex64/float32 (single-precision FFTs; sums of the
    loss and of the shift gradient in FP64)."""
    n, s = geom.n, geom.n_slices
    corner, shifts = om.split_position(pos)
    shift = shifts.astype(F32)
    f = np.fft.fftfreq(n)
    nu2 = (f[:, None] ** 2 + f[None, :] ** 2) / geom.pixel_m ** 2
    hs = [np.exp(1j * np.pi * geom.wavelength_m * geom.gap(j) * nu2).astype(C64) for j in range(s - 1)]
    kdz = F32(geom.kdz)
    ta = om.take_chunks(a, corner, n).astype(F32)
    tb = om.take_chunks(b, corner, n).astype(F32)
    if geom.obj_repr == "delta_beta":
        t = (np.exp(-kdz * tb) * (np.cos(kdz * ta) + 1j * np.sin(kdz * ta))).astype(C64)
    else:
        t = (ta + 1j * tb).astype(C64)
    e = np.exp(-2j * np.pi * (shift[:, 0, None, None] * f[:, None] + shift[:, 1, None, None] * f[None, :])).astype(C64)
    pf = sfft.fft2(np.asarray(p).astype(C64), norm="ortho")
    psi = sfft.ifft2(pf[None] * e, norm="ortho")
    psis, phis = [], []
    for j in range(s):
        phi = psi * t[:, j]
        psis.append(psi)
        phis.append(phi)
        if j < s - 1:
            psi = sfft.ifft2(sfft.fft2(phi, norm="ortho") * hs[j], norm="ortho")
    det = np.fft.fftshift(sfft.ifft2(phi, norm="ortho"), axes=(-2, -1))
    ip = (det.real ** 2 + det.imag ** 2).astype(F32)
    im = np.asarray(i_meas).astype(F32)
    eps, nn = F32(geom.eps), F32(ip.size)
    if geom.loss == "gaussian":
        sp, sm = np.sqrt(ip + eps), np.sqrt(im + eps)
        value = float(np.sum(((sp - sm) ** 2).astype(np.float64))) / ip.size
        dldi = (F32(1) - sm / sp) / nn
    else:
        value = float(np.sum((ip - im * np.log(ip + eps)).astype(np.float64))) / ip.size
        dldi = (F32(1) - im / (ip + eps)) / nn
    lam = sfft.fft2(np.fft.ifftshift((F32(2) * dldi * det).astype(C64), axes=(-2, -1)), norm="ortho")
    g_ta = np.empty(ta.shape, F32)
    g_tb = np.empty(tb.shape, F32)
    for j in range(s - 1, -1, -1):
        if geom.obj_repr == "delta_beta":
            z = np.conj(phis[j]) * lam
            g_ta[:, j], g_tb[:, j] = kdz * z.imag, -kdz * z.real
        else:
            z = np.conj(psis[j]) * lam
            g_ta[:, j], g_tb[:, j] = z.real, z.imag
        mu = np.conj(t[:, j]) * lam
        if j > 0:
            lam = sfft.ifft2(sfft.fft2(mu, norm="ortho") * np.conj(hs[j - 1]), norm="ortho")
    big_g = sfft.fft2(mu, norm="ortho")
    g_probe = sfft.ifft2(np.sum(big_g * np.conj(e), axis=0), norm="ortho")
    z = (np.conj(big_g) * pf[None] * e).astype(np.complex128)
    g_shift = np.stack([2 * np.pi * np.sum(f[None, :, None] * z.imag, axis=(1, 2)),
                        2 * np.pi * np.sum(f[None, None, :] * z.imag, axis=(1, 2))], axis=1)
    return (value, om.scatter_chunks(g_ta.astype(np.float64), corner, a.shape),
            om.scatter_chunks(g_tb.astype(np.float64), corner, b.shape), g_probe, g_shift)
