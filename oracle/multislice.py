"""CPU FP64 oracle of the multislice ptychography forward model and its gradient.

TEST INFRASTRUCTURE ONLY.  This module is the independent reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
never does.  It shares no code with the HIP kernels (FFTs come from
``scipy.fft``/pocketfft, everything else is plain NumPy in float64).

Conventions (the paper leaves these open; the reading taken here is stated
once and used everywhere):

* ``F`` is the unitary 2D DFT with NumPy's sign, ``fft2(norm="ortho")``, and
  ``F^-1`` its inverse.  The paper's Fraunhofer transform has a positive
  exponent (Eq. fraunhofer, Sec. S1.C), so in the negative-phase convention it
  is NumPy's ``ifft2``; the detector image is ``fftshift``-ed so the zero
  frequency sits at index (N/2, N/2).
* Frequencies: ``f = fftfreq(N)`` in cycles/pixel for the Fourier shift,
  ``nu = fftfreq(N, dx)`` in 1/m for the Fresnel kernel.
* A position r (float, top-left chunk corner, (y, x), object pixels) splits
  into the integer corner ``c = floor(r + 0.5)`` and the residual shift
  ``s = r - c``; the probe is moved by s with the Fourier shift theorem
  (Eq. fourier_shift) so that ``p_s(x) = p(x - s)`` (circularly).
* S slices give S - 1 inter-slice Fresnel propagations (Eq. multislice
  product, Sec. S1.C): the wave is modulated by slice j, propagated to slice
  j+1, ..., and the exit wave after the last modulation goes to the far field.
* Loss normalisation: the mean over all B*N^2 pixels of a minibatch.  The
  small constant eps sits inside both square roots of the LSQ loss
  (Eq. lsq_loss) and inside the logarithm of the Poisson loss (Eq.
  poisson_loss).
* Complex gradients follow dL/dRe + i dL/dIm.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

# FFT worker threads: the CPU cores this process may run on
_WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


# ---------------------------------------------------------------------------
# Transforms (Sec. S1.C, Eq. fraunhofer and the sign-convention paragraph)
# ---------------------------------------------------------------------------

def fft2u(a):
    """Unitary forward 2D DFT over the last two axes (NumPy sign)."""
    return sfft.fft2(a, norm="ortho", workers=_WORKERS)


def ifft2u(a):
    """Unitary inverse 2D DFT over the last two axes."""
    return sfft.ifft2(a, norm="ortho", workers=_WORKERS)


def far_field(exit_wave):
    """Fraunhofer propagation to the detector, Eq. fraunhofer.

    The transform has a positive exponent in the negative-phase convention,
    i.e. the inverse DFT; the result is centred with ``fftshift``.
    """
    return np.fft.fftshift(ifft2u(exit_wave), axes=(-2, -1))


def far_field_adjoint(g_det):
    """Adjoint of ``far_field``: un-centre, then the forward unitary DFT."""
    return fft2u(np.fft.ifftshift(g_det, axes=(-2, -1)))


# ---------------------------------------------------------------------------
# Fresnel propagation (Eqs. fresnel_prop and paraxial_kernel)
# ---------------------------------------------------------------------------

def fresnel_kernel(n, wavelength_m, pixel_m, dist_m):
    """Paraxial transfer function H1(nu, d) = exp(i pi lambda d |nu|^2)."""
    nu = np.fft.fftfreq(n, d=pixel_m)
    nu2 = nu[:, None] ** 2 + nu[None, :] ** 2
    return np.exp(1j * np.pi * wavelength_m * dist_m * nu2)


def sommerfeld_kernel(n, wavelength_m, pixel_m, dist_m):
    """Sommerfeld-Rayleigh transfer function, Eq. sommerfeld_kernel:
    H2 = exp(-i k d sqrt(1 - lambda^2 |nu|^2)) where 1 - lambda^2 |nu|^2 > 0,
    0 elsewhere (evanescent).  Evaluated as the global phase exp(-i k d)
    times exp(-i k d (sqrt(1 - x) - 1)), x = lambda^2 |nu|^2, with
    sqrt(1 - x) - 1 = -x / (sqrt(1 - x) + 1): the same function, without
    the cancellation of a ~1e10 rad phase."""
    nu = np.fft.fftfreq(n, d=pixel_m)
    x = wavelength_m ** 2 * (nu[:, None] ** 2 + nu[None, :] ** 2)
    k = 2.0 * np.pi / wavelength_m
    inside = x < 1.0
    xs = np.where(inside, x, 0.0)
    rel = -xs / (np.sqrt(1.0 - xs) + 1.0)
    kd = k * dist_m
    glob = np.exp(-1j * np.fmod(kd, 2.0 * np.pi))
    return np.where(inside, glob * np.exp(-1j * kd * rel), 0.0)


def fresnel_propagate(psi, h):
    """Fresnel propagation F^-1{ F[psi] H }, Eq. fresnel_prop."""
    return ifft2u(fft2u(psi) * h)


def fresnel_propagate_adjoint(g, h):
    """Adjoint of ``fresnel_propagate``: F^-1{ F[g] conj(H) }."""
    return ifft2u(fft2u(g) * np.conj(h))


# ---------------------------------------------------------------------------
# Probe placement (Eq. fourier_shift; position split, Sec. S1.D)
# ---------------------------------------------------------------------------

def split_position(r):
    """Integer corner floor(r + 0.5) and subpixel residual r - corner."""
    r = np.asarray(r, dtype=np.float64)
    c = np.floor(r + 0.5)
    return c.astype(np.int64), r - c


def shift_ramp(n, shift):
    """exp(-2 pi i (s_y f_y + s_x f_x)) for shifts ``[..., 2]`` (cycles/px freq)."""
    f = np.fft.fftfreq(n)
    s = np.asarray(shift, dtype=np.float64)
    return np.exp(-2j * np.pi * (s[..., 0, None, None] * f[:, None] + s[..., 1, None, None] * f[None, :]))


def fourier_shift(probe, shift):
    """Shift the probe by ``shift`` pixels: F^-1{ F[p] exp(-2 pi i s.f) }."""
    return ifft2u(fft2u(probe) * shift_ramp(probe.shape[-1], shift))


# ---------------------------------------------------------------------------
# Object modulation (Eqs. complex_modulation and ri_modulation)
# ---------------------------------------------------------------------------

def k_dz(wavelength_m, dz_m):
    """k * dz with k = 2 pi / lambda (Eq. ri_modulation)."""
    return 2.0 * np.pi / wavelength_m * dz_m


def transmission(a, b, obj_repr, kdz):
    """Per-slice transmission t.

    ``delta_beta``: t = exp(-k beta dz) exp(i k delta dz)  (Eq. ri_modulation).
    ``real_imag``:  t = Re O + i Im O                    (Eq. complex_modulation).
    """
    if obj_repr == "delta_beta":
        return np.exp(1j * kdz * a - kdz * b)
    if obj_repr == "real_imag":
        return a + 1j * b
    raise ValueError(obj_repr)


def take_chunks(obj, corners, n):
    """Object chunks on each beam path (Alg. 1, TakeObjectChunk).

    ``obj`` is [S][Ly][Lx]; returns [B][S][N][N].  Raises if a chunk leaves
    the object (the paper pads the object instead; this library treats it as
    an error).
    """
    s, ly, lx = obj.shape
    out = np.empty((len(corners), s, n, n), dtype=obj.dtype)
    for b, (cy, cx) in enumerate(np.asarray(corners)):
        if cy < 0 or cx < 0 or cy + n > ly or cx + n > lx:
            raise IndexError(f"chunk {b} at ({cy},{cx}) leaves the {ly}x{lx} object")
        out[b] = obj[:, cy:cy + n, cx:cx + n]
    return out


def scatter_chunks(g_chunks, corners, obj_shape):
    """Transpose of ``take_chunks``: add chunk gradients into the object."""
    g = np.zeros(obj_shape, dtype=g_chunks.dtype)
    n = g_chunks.shape[-1]
    for b, (cy, cx) in enumerate(np.asarray(corners)):
        g[:, cy:cy + n, cx:cx + n] += g_chunks[b]
    return g


# ---------------------------------------------------------------------------
# Forward model (Alg. 1; multislice, Sec. S1.C)
# ---------------------------------------------------------------------------

class Geometry:
    """Physical parameters of one scan."""

    def __init__(self, n, n_slices, wavelength_m, pixel_m, slice_dz_m, obj_repr="delta_beta",
                 loss="gaussian", eps=1e-6, gaps=None):
        self.n = int(n)
        self.n_slices = int(n_slices)
        self.wavelength_m = float(wavelength_m)
        self.pixel_m = float(pixel_m)
        self.slice_dz_m = float(slice_dz_m)
        self.obj_repr = obj_repr
        self.loss = loss
        self.eps = float(eps)
        # Sparse multislice with unequal spacing (Sec. S1.C, the variable
        # variant): gaps[j] is the free-space distance from slice j to slice
        # j+1 in metres.  slice_dz_m stays the thickness in the transmission.
        # None: every gap equals slice_dz_m.
        self.gaps = None if gaps is None else np.asarray(gaps, dtype=np.float64).reshape(-1)
        if self.gaps is not None and self.gaps.size != max(self.n_slices - 1, 0):
            raise ValueError("gaps needs n_slices - 1 entries")

    def gap(self, j):
        """Distance from slice j to slice j+1 (metres)."""
        return self.slice_dz_m if self.gaps is None else float(self.gaps[j])

    def gap_kernels(self):
        """The S - 1 Fresnel transfer functions, one per gap."""
        if self.gaps is None:
            return [self.h] * (self.n_slices - 1)
        return [fresnel_kernel(self.n, self.wavelength_m, self.pixel_m, d) for d in self.gaps]

    @property
    def kdz(self):
        return k_dz(self.wavelength_m, self.slice_dz_m)

    @property
    def h(self):
        return fresnel_kernel(self.n, self.wavelength_m, self.pixel_m, self.slice_dz_m)

    @classmethod
    def from_scan(cls, scan):
        return cls(scan.n, scan.n_slices, scan.wavelength_m, scan.pixel_m, scan.slice_dz_m,
                   scan.obj_repr, scan.loss, scan.eps)


def exit_waves(geom, obj_a, obj_b, probe, positions, keep_slices=False):
    """Exit waves for every position of a batch (Alg. 1 up to MultislicePropagate).

    For position b: p_b = FourierShift(p, s_b); psi_0 = p_b; for each slice
    j: phi_j = psi_j * t_j, and for j < S-1 psi_{j+1} = Fresnel(phi_j).
    Returns phi_{S-1} [B][N][N]; with ``keep_slices`` also every psi_j and
    phi_j, each [B][S][N][N].
    """
    corners, shifts = split_position(positions)
    n, s = geom.n, geom.n_slices
    ta = take_chunks(obj_a, corners, n)
    tb = take_chunks(obj_b, corners, n)
    t = transmission(ta, tb, geom.obj_repr, geom.kdz)          # [B][S][N][N]
    psi = fourier_shift(probe, shifts)                          # [B][N][N]
    hs = geom.gap_kernels()
    if keep_slices:
        psis = np.empty((len(corners), s, n, n), dtype=np.complex128)
        phis = np.empty_like(psis)
    phi = None
    for j in range(s):
        phi = psi * t[:, j]
        if keep_slices:
            psis[:, j] = psi
            phis[:, j] = phi
        if j < s - 1:
            psi = fresnel_propagate(phi, hs[j])
    return (phi, psis, phis) if keep_slices else phi


def forward(geom, obj_a, obj_b, probe, positions):
    """Predicted far-field intensities I = |far_field(exit)|^2, [B][N][N]."""
    return np.abs(far_field(exit_waves(geom, obj_a, obj_b, probe, positions))) ** 2


def forward_pure_projection(geom, obj_a, obj_b, probe, positions):
    """Projection-approximation exit wave (Eqs. obj_complex_modulation, obj_ri_modulation).

    delta_beta: psi * exp(-k dz sum beta) * exp(i k dz sum delta);
    real_imag:  psi * prod_j O_j.
    """
    corners, shifts = split_position(positions)
    ta = take_chunks(obj_a, corners, geom.n)
    tb = take_chunks(obj_b, corners, geom.n)
    psi = fourier_shift(probe, shifts)
    if geom.obj_repr == "delta_beta":
        return psi * np.exp(-geom.kdz * tb.sum(axis=1)) * np.exp(1j * geom.kdz * ta.sum(axis=1))
    return psi * np.prod(ta + 1j * tb, axis=1)


# ---------------------------------------------------------------------------
# Loss (Eqs. lsq_loss, poisson_loss)
# ---------------------------------------------------------------------------

def loss_value(kind, i_pred, i_meas, eps, n_norm=None):
    """Data mismatch D averaged over all pixels of the batch."""
    n_norm = i_pred.size if n_norm is None else n_norm
    if kind == "gaussian":
        return float(np.sum((np.sqrt(i_pred + eps) - np.sqrt(i_meas + eps)) ** 2) / n_norm)
    if kind == "poisson":
        return float(np.sum(i_pred - i_meas * np.log(i_pred + eps)) / n_norm)
    raise ValueError(kind)


def loss_dI(kind, i_pred, i_meas, eps, n_norm):
    """dD/dI_pred elementwise."""
    if kind == "gaussian":
        return (1.0 - np.sqrt(i_meas + eps) / np.sqrt(i_pred + eps)) / n_norm
    if kind == "poisson":
        return (1.0 - i_meas / (i_pred + eps)) / n_norm
    raise ValueError(kind)


def loss(geom, obj_a, obj_b, probe, positions, i_meas):
    return loss_value(geom.loss, forward(geom, obj_a, obj_b, probe, positions), i_meas, geom.eps)


# ---------------------------------------------------------------------------
# Gradient (reverse sweep through the multislice product)
# ---------------------------------------------------------------------------

def loss_grad(geom, obj_a, obj_b, probe, positions, i_meas):
    """Loss and its gradient w.r.t. the object, the probe and the shifts.

    Differentiates D(I(x)) through the steps of ``exit_waves`` in reverse:
    the far-field residual g = 2 dD/dI * Psi is pulled back through the
    Fraunhofer transform, then through each slice (modulation and Fresnel
    propagation, whose adjoints are multiplication by conj(t) and
    propagation with conj(H)), the Fourier shift and the chunk gather.

    Returns (loss, g_a [S][Ly][Lx], g_b [S][Ly][Lx], g_probe [N][N] complex,
    g_shift [B][2]).  ``g_shift`` is dL/ds for the residual shift s of each
    position, which equals dL/dr for the float position r.
    """
    i_pred = forward(geom, obj_a, obj_b, probe, positions)
    n_norm = i_pred.size
    value = loss_value(geom.loss, i_pred, i_meas, geom.eps, n_norm)
    d_di = loss_dI(geom.loss, i_pred, i_meas, geom.eps, n_norm)
    return (value,) + reverse_sweep(geom, obj_a, obj_b, probe, positions, d_di)


def reverse_sweep(geom, obj_a, obj_b, probe, positions, d_di, want_gaps=False, lam_exit=None):
    """Gradient of a loss whose derivative with respect to the predicted
    intensity I = |Psi|^2 of this probe is d_di [B][N][N]: the far-field
    residual g = 2 d_di Psi is pulled back through the Fraunhofer transform,
    each slice, the Fourier shift and the chunk gather.  Returns (g_a, g_b,
    g_probe, g_shift) as in loss_grad; with ``want_gaps`` also g_gaps [S-1],
    the derivative with respect to each inter-slice distance.

    A gap d_j enters only through psi_{j+1} = F^-1[H_j F phi_j] with
    H_j = exp(i pi lambda d_j |nu|^2), so dpsi_{j+1}/dd_j =
    F^-1[i pi lambda |nu|^2 F psi_{j+1}], and with mu = dL/dpsi_{j+1}
    dL/dd_j = Re sum conj(F mu) (i pi lambda |nu|^2) F psi_{j+1}
    (the real inner product of a real parameter's derivative; F unitary).
    ``lam_exit``, if given, is dL/dphi_{S-1} (another detector model than
    the far field); d_di is then unused.
    """
    corners, shifts = split_position(positions)
    n, s = geom.n, geom.n_slices
    kdz = geom.kdz
    hs = geom.gap_kernels()
    nu = np.fft.fftfreq(n, d=geom.pixel_m)
    dh_dd = 1j * np.pi * geom.wavelength_m * (nu[:, None] ** 2 + nu[None, :] ** 2)
    g_gaps = np.zeros(max(s - 1, 0))
    ta = take_chunks(obj_a, corners, n)
    tb = take_chunks(obj_b, corners, n)
    t = transmission(ta, tb, geom.obj_repr, kdz)
    exit_phi, psis, phis = exit_waves(geom, obj_a, obj_b, probe, positions, keep_slices=True)
    if lam_exit is None:
        g_det = 2.0 * d_di * far_field(exit_phi)
        lam = far_field_adjoint(g_det)                   # dL/dphi_{S-1}
    else:
        lam = lam_exit
    g_ta = np.empty_like(ta)
    g_tb = np.empty_like(tb)
    for j in range(s - 1, -1, -1):
        if geom.obj_repr == "delta_beta":
            # phi = psi exp(i u - v), u = kdz delta, v = kdz beta:
            # dL/du = Im(conj(phi) lam), dL/dv = -Re(conj(phi) lam)
            z = np.conj(phis[:, j]) * lam
            g_ta[:, j] = kdz * np.imag(z)
            g_tb[:, j] = -kdz * np.real(z)
        else:
            # phi = psi O (complex-linear in O): dL/dO = conj(psi) lam
            z = np.conj(psis[:, j]) * lam
            g_ta[:, j] = np.real(z)
            g_tb[:, j] = np.imag(z)
        mu = np.conj(t[:, j]) * lam                      # dL/dpsi_j
        if j > 0:
            if want_gaps:
                g_gaps[j - 1] = np.sum(np.real(np.conj(fft2u(mu)) * dh_dd * fft2u(psis[:, j])))
            lam = fresnel_propagate_adjoint(mu, hs[j - 1])   # dL/dphi_{j-1}
    g_pb = mu                                            # dL/d(shifted probe)

    # Fourier shift: p_b = F^-1[ P e_b ],  P = F[p],  e_b = exp(-2 pi i s_b.f)
    e = shift_ramp(n, shifts)
    big_g = fft2u(g_pb)
    big_p = fft2u(probe)
    g_probe = ifft2u(np.sum(big_g * np.conj(e), axis=0))
    f = np.fft.fftfreq(n)
    z = np.conj(big_g) * big_p[None] * e
    g_shift = np.stack([np.sum(np.real(z * (-2j * np.pi) * f[None, :, None]), axis=(1, 2)),
                        np.sum(np.real(z * (-2j * np.pi) * f[None, None, :]), axis=(1, 2))], axis=1)

    g_a = scatter_chunks(g_ta, corners, obj_a.shape)
    g_b = scatter_chunks(g_tb, corners, obj_b.shape)
    if want_gaps:
        return g_a, g_b, g_probe, g_shift, g_gaps
    return g_a, g_b, g_probe, g_shift


def loss_grad_gaps(geom, obj_a, obj_b, probe, positions, i_meas):
    """loss_grad plus the gradient with respect to the inter-slice distances
    (slice-position refinement of sparse multislice, Sec. S1.C and the list
    of refinable parameters in Sec. S1.D).  Returns (loss, g_a, g_b, g_probe,
    g_shift, g_gaps [S-1])."""
    i_pred = forward(geom, obj_a, obj_b, probe, positions)
    n_norm = i_pred.size
    value = loss_value(geom.loss, i_pred, i_meas, geom.eps, n_norm)
    d_di = loss_dI(geom.loss, i_pred, i_meas, geom.eps, n_norm)
    return (value,) + reverse_sweep(geom, obj_a, obj_b, probe, positions, d_di, want_gaps=True)


# ---------------------------------------------------------------------------
# Near field (holography, near-field ptychography): Fresnel propagation to
# the detector instead of the Fraunhofer transform (Eq. fresnel_prop with
# the paraxial or the Sommerfeld kernel; Sec. S1.D, free propagation
# distance refinement)
# ---------------------------------------------------------------------------

def nearfield_kernels(geom, dists, kind):
    """Transfer functions to the detector for each distance (metres)."""
    make = {"paraxial": fresnel_kernel, "sommerfeld": sommerfeld_kernel}[kind]
    return [make(geom.n, geom.wavelength_m, geom.pixel_m, d) for d in np.asarray(dists, dtype=np.float64)]


def nearfield_kernel_ddist(geom, kind):
    """d log H / d d: i pi lambda |nu|^2 (paraxial), and for the Sommerfeld
    kernel -i k (sqrt(1 - lambda^2 |nu|^2) - 1) inside the propagating band
    (0 outside).  The Sommerfeld kernel's own derivative is
    -i k sqrt(1 - lambda^2 |nu|^2); the two differ by -i k, the derivative of
    the global phase exp(-i k d), whose term -k Im<g, psi_det> vanishes for
    any loss of the intensity (g = 2 dL/dI psi_det makes <g, psi_det> real).
    Leaving it out avoids a ~1e11 rad/m factor times a rounding residual."""
    nu = np.fft.fftfreq(geom.n, d=geom.pixel_m)
    nu2 = nu[:, None] ** 2 + nu[None, :] ** 2
    if kind == "paraxial":
        return 1j * np.pi * geom.wavelength_m * nu2
    x = geom.wavelength_m ** 2 * nu2
    k = 2.0 * np.pi / geom.wavelength_m
    xs = np.where(x < 1.0, x, 0.0)
    return np.where(x < 1.0, 1j * k * xs / (np.sqrt(1.0 - xs) + 1.0), 0.0)


def forward_nearfield(geom, obj_a, obj_b, probe, positions, dists, dist_idx, kind="paraxial"):
    """Detector intensities |F^-1[H_b F phi_exit]|^2 [B][N][N] (natural order),
    H_b the transfer function of position b's distance dists[dist_idx[b]]."""
    hs = nearfield_kernels(geom, dists, kind)
    exit_phi = exit_waves(geom, obj_a, obj_b, probe, positions)
    hb = np.stack([hs[i] for i in np.asarray(dist_idx)])
    return np.abs(fresnel_propagate(exit_phi, hb)) ** 2


def loss_nearfield(geom, obj_a, obj_b, probe, positions, i_meas, dists, dist_idx, kind="paraxial"):
    i_pred = forward_nearfield(geom, obj_a, obj_b, probe, positions, dists, dist_idx, kind)
    return loss_value(geom.loss, i_pred, i_meas, geom.eps)


def loss_grad_nearfield(geom, obj_a, obj_b, probe, positions, i_meas, dists, dist_idx, kind="paraxial"):
    """Loss and gradients of the near-field model: (loss, g_a, g_b, g_probe,
    g_shift, g_dist [n_dist]).  With g = 2 dL/dI psi_det the residual at the
    detector, the exit-wave gradient is F^-1[conj(H_b) F g] and
    dL/dd_b = Re sum conj(F g) (dH_b/dd) F phi_exit, summed over the
    positions that share a distance."""
    hs = nearfield_kernels(geom, dists, kind)
    dlog = nearfield_kernel_ddist(geom, kind)
    idx = np.asarray(dist_idx)
    hb = np.stack([hs[i] for i in idx])
    exit_phi = exit_waves(geom, obj_a, obj_b, probe, positions)
    exit_f = fft2u(exit_phi)
    psi_det = ifft2u(exit_f * hb)
    i_pred = np.abs(psi_det) ** 2
    n_norm = i_pred.size
    value = loss_value(geom.loss, i_pred, i_meas, geom.eps, n_norm)
    g_det = 2.0 * loss_dI(geom.loss, i_pred, i_meas, geom.eps, n_norm) * psi_det
    g_f = fft2u(g_det)
    per_pos = np.sum(np.real(np.conj(g_f) * dlog * hb * exit_f), axis=(1, 2))
    g_dist = np.zeros(len(np.atleast_1d(dists)))
    np.add.at(g_dist, idx, per_pos)
    lam_exit = ifft2u(g_f * np.conj(hb))
    return (value,) + reverse_sweep(geom, obj_a, obj_b, probe, positions, None, lam_exit=lam_exit) + (g_dist,)


# ---------------------------------------------------------------------------
# Probe defocus (a refinable experimental parameter, Sec. S1.D): the probe is
# Fresnel-propagated (Eqs. fresnel_prop, paraxial_kernel) by the defocus
# distance before it meets the object, and the distance gets a gradient.
# ---------------------------------------------------------------------------

def defocus_probe(geom, probe, dist_m):
    """The probe propagated by dist_m metres: F^-1[H(dist_m) F p]."""
    return fresnel_propagate(probe, fresnel_kernel(geom.n, geom.wavelength_m, geom.pixel_m, dist_m))


def forward_defocus(geom, obj_a, obj_b, probe, positions, dist_m):
    """Far-field intensities with the probe defocused by dist_m."""
    return forward(geom, obj_a, obj_b, defocus_probe(geom, probe, dist_m), positions)


def loss_grad_defocus(geom, obj_a, obj_b, probe, positions, i_meas, dist_m):
    """Loss and gradients with a defocused probe: (loss, g_a, g_b, g_probe,
    g_shift, g_defocus).  With p_d = F^-1[H F p] and g_d = dL/dp_d from
    ``loss_grad`` at p_d, the chain rule gives g_probe = F^-1[conj(H) F g_d]
    (the adjoint of the propagation) and
    dL/d(dist) = Re sum conj(F g_d) (i pi lambda |nu|^2) H F p."""
    h = fresnel_kernel(geom.n, geom.wavelength_m, geom.pixel_m, dist_m)
    p_d = fresnel_propagate(probe, h)
    value, g_a, g_b, g_pd, g_shift = loss_grad(geom, obj_a, obj_b, p_d, positions, i_meas)
    g_probe = fresnel_propagate_adjoint(g_pd, h)
    dlog = nearfield_kernel_ddist(geom, "paraxial")
    g_def = float(np.sum(np.real(np.conj(fft2u(g_pd)) * dlog * h * fft2u(probe))))
    return value, g_a, g_b, g_probe, g_shift, g_def


# ---------------------------------------------------------------------------
# Several mutually incoherent probe modes (Eq. multimode)
# ---------------------------------------------------------------------------

def forward_modes(geom, obj_a, obj_b, probes, positions):
    """Predicted intensity with probe modes probes [M][N][N]: each mode goes
    through the object on its own and the detector adds their intensities,
    I = sum_m |Psi_m|^2 (Eq. multimode)."""
    return sum(forward(geom, obj_a, obj_b, p, positions) for p in probes)


def loss_modes(geom, obj_a, obj_b, probes, positions, i_meas):
    return loss_value(geom.loss, forward_modes(geom, obj_a, obj_b, probes, positions), i_meas, geom.eps)


def loss_grad_modes(geom, obj_a, obj_b, probes, positions, i_meas):
    """Loss of the summed intensity and its gradient.

    dL/dI is taken at the summed intensity; each mode's reverse sweep starts
    from 2 dL/dI Psi_m.  Object and shift gradients add over the modes (every
    mode sees the same object and moves with the same position); the probe
    gradient is per mode, [M][N][N].
    """
    i_pred = forward_modes(geom, obj_a, obj_b, probes, positions)
    n_norm = i_pred.size
    value = loss_value(geom.loss, i_pred, i_meas, geom.eps, n_norm)
    d_di = loss_dI(geom.loss, i_pred, i_meas, geom.eps, n_norm)
    g_a = g_b = g_shift = 0.0
    g_probe = []
    for p in probes:
        ga, gb, gp, gs = reverse_sweep(geom, obj_a, obj_b, p, positions, d_di)
        g_a, g_b, g_shift = g_a + ga, g_b + gb, g_shift + gs
        g_probe.append(gp)
    return value, g_a, g_b, np.stack(g_probe), g_shift
