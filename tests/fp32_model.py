"""Float32 reference model: the conditioning floor of any FP32 implementation.

TEST INFRASTRUCTURE ONLY.  This is the plain multislice forward model and its
gradient written exactly like the FP64 oracle (every slice wave stored, no
checkpoints, no inversion), but evaluated in complex64/float32 with SciPy's
single-precision FFTs.  Its distance to the FP64 oracle measures how much a
faithful float32 evaluation of the *same mathematics* must deviate at a
given evaluation point.  Where that floor is above the gradient tolerance
(ill-conditioned points: Poisson residuals of far-field pixels the model
barely illuminates, or weak absorption gradients that are small real parts
of large complex products) the parity tests bound the GPU error by a small
multiple of this floor instead, and print both.

It shares no code with the HIP library and is never used by it.
"""
import numpy as np
import scipy.fft as sfft

C64 = np.complex64
F32 = np.float32


def _c64(x):
    return np.asarray(x).astype(C64)


def _forward(geom, a, b, p, pos):
    """Every slice's wave and the detector field of one probe, in float32."""
    n, s = geom.n, geom.n_slices
    corner = np.floor(pos + 0.5).astype(np.int64)
    shift = (pos - corner).astype(F32)
    f = np.fft.fftfreq(n)
    nu2 = (f[:, None] ** 2 + f[None, :] ** 2) / geom.pixel_m ** 2
    gaps = getattr(geom, "gaps", None)
    gaps = [geom.slice_dz_m] * (s - 1) if gaps is None else list(gaps)
    hs = [_c64(np.exp(1j * np.pi * geom.wavelength_m * d * nu2)) for d in gaps]
    kdz = F32(2 * np.pi / geom.wavelength_m * geom.slice_dz_m)
    nb = len(corner)
    ta = np.stack([a[:, cy:cy + n, cx:cx + n] for cy, cx in corner]).astype(F32)
    tb = np.stack([b[:, cy:cy + n, cx:cx + n] for cy, cx in corner]).astype(F32)
    if geom.obj_repr == "delta_beta":
        t = (np.exp(-kdz * tb) * (np.cos(kdz * ta) + 1j * np.sin(kdz * ta))).astype(C64)
    else:
        t = (ta + 1j * tb).astype(C64)
    e = _c64(np.exp(-2j * np.pi * (shift[:, 0, None, None] * f[:, None] + shift[:, 1, None, None] * f[None, :])))
    pf = sfft.fft2(_c64(p), norm="ortho")
    psi = sfft.ifft2(pf[None] * e, norm="ortho")
    psis = np.empty((nb, s, n, n), C64)
    phis = np.empty((nb, s, n, n), C64)
    for j in range(s):
        psis[:, j] = psi
        phi = psi * t[:, j]
        phis[:, j] = phi
        if j < s - 1:
            psi = sfft.ifft2(sfft.fft2(phi, norm="ortho") * hs[j], norm="ortho")
    det = np.fft.fftshift(sfft.ifft2(phi, norm="ortho"), axes=(-2, -1))
    dh = _c64(1j * np.pi * geom.wavelength_m * nu2)
    return dict(corner=corner, f=f, hs=hs, dh=dh, kdz=kdz, t=t, e=e, pf=pf, psis=psis, phis=phis, det=det)


def _loss(geom, ip, i_meas):
    im = i_meas.astype(F32)
    eps = F32(geom.eps)
    nn = F32(ip.size)
    if geom.loss == "gaussian":
        sp, sm = np.sqrt(ip + eps), np.sqrt(im + eps)
        value = float(np.sum(((sp - sm) ** 2).astype(np.float64))) / ip.size
        dldi = (F32(1) - sm / sp) / nn
    else:
        value = float(np.sum((ip - im * np.log(ip + eps)).astype(np.float64))) / ip.size
        dldi = (F32(1) - im / (ip + eps)) / nn
    return value, dldi


def _reverse(geom, st, a, b, dldi, lam0=None):
    n, s = geom.n, geom.n_slices
    corner, f, hs, kdz, t, e, pf = (st[k] for k in ("corner", "f", "hs", "kdz", "t", "e", "pf"))
    psis, phis, det = st["psis"], st["phis"], st["det"]
    if lam0 is None:
        lam = sfft.fft2(np.fft.ifftshift((F32(2) * dldi * det).astype(C64), axes=(-2, -1)), norm="ortho")
    else:
        lam = lam0
    ga = np.zeros(a.shape, F32)
    gb = np.zeros(b.shape, F32)
    for j in range(s - 1, -1, -1):
        if geom.obj_repr == "delta_beta":
            z = np.conj(phis[:, j]) * lam
            da, db = kdz * z.imag, -kdz * z.real
        else:
            z = np.conj(psis[:, j]) * lam
            da, db = z.real, z.imag
        for k, (cy, cx) in enumerate(corner):
            ga[j, cy:cy + n, cx:cx + n] += da[k]
            gb[j, cy:cy + n, cx:cx + n] += db[k]
        mu = np.conj(t[:, j]) * lam
        if j > 0:
            mu_f = sfft.fft2(mu, norm="ortho")
            st.setdefault("g_gaps", np.zeros(s - 1))[j - 1] = float(
                np.sum(np.real(np.conj(mu_f) * st["dh"] * sfft.fft2(psis[:, j], norm="ortho")).astype(np.float64)))
            lam = sfft.ifft2(mu_f * np.conj(hs[j - 1]), norm="ortho")
    big_g = sfft.fft2(mu, norm="ortho")
    gp = sfft.ifft2(np.sum(big_g * np.conj(e), axis=0), norm="ortho")
    z = np.conj(big_g) * pf[None] * e
    gs = np.stack([2 * np.pi * np.sum(f[None, :, None] * z.imag, axis=(1, 2)),
                   2 * np.pi * np.sum(f[None, None, :] * z.imag, axis=(1, 2))], axis=1)
    return ga, gb, gp, gs


def _intensity(det):
    return (det.real ** 2 + det.imag ** 2).astype(F32)


def loss_grad_fp32(geom, a, b, p, pos, i_meas):
    st = _forward(geom, a, b, p, pos)
    value, dldi = _loss(geom, _intensity(st["det"]), i_meas)
    return (value,) + _reverse(geom, st, a, b, dldi)


def loss_grad_fp32_gaps(geom, a, b, p, pos, i_meas):
    """As loss_grad_fp32 with the geometry's unequal gaps; adds g_gaps."""
    st = _forward(geom, a, b, p, pos)
    value, dldi = _loss(geom, _intensity(st["det"]), i_meas)
    out = _reverse(geom, st, a, b, dldi)
    return (value,) + out + (st.get("g_gaps", np.zeros(max(geom.n_slices - 1, 0))),)


def loss_grad_fp32_modes(geom, a, b, probes, pos, i_meas):
    """Several incoherent probe modes: the loss at the summed intensity,
    object and shift gradients summed over modes, one probe gradient each."""
    sts = [_forward(geom, a, b, p, pos) for p in probes]
    ip = sts[0]["det"].real * 0
    for st in sts:
        ip = ip + _intensity(st["det"])
    value, dldi = _loss(geom, ip.astype(F32), i_meas)
    ga = gb = gs = 0
    gps = []
    for st in sts:
        a_, b_, p_, s_ = _reverse(geom, st, a, b, dldi)
        ga, gb, gs = ga + a_, gb + b_, gs + s_
        gps.append(p_)
    return value, ga, gb, np.stack(gps), gs


def loss_grad_fp32_nearfield(geom, a, b, p, pos, i_meas, dists, dist_idx, kind, hs_det, dlog):
    """Near-field detector in float32: hs_det [n_dist] transfer functions
    and dlog = d log H / d d from the FP64 oracle, rounded to complex64."""
    st = _forward(geom, a, b, p, pos)
    hb = np.stack([_c64(hs_det[i]) for i in np.asarray(dist_idx)])
    exit_f = sfft.fft2(st["phis"][:, -1], norm="ortho")
    psi = sfft.ifft2(exit_f * hb, norm="ortho")
    value, dldi = _loss(geom, _intensity(psi), i_meas)
    g = (F32(2) * dldi * psi).astype(C64)
    g_f = sfft.fft2(g, norm="ortho")
    per = np.sum(np.real(np.conj(g_f) * _c64(dlog) * hb * exit_f).astype(np.float64), axis=(1, 2))
    g_dist = np.zeros(len(dists))
    np.add.at(g_dist, np.asarray(dist_idx), per)
    lam0 = sfft.ifft2(g_f * np.conj(hb), norm="ortho")
    return (value,) + _reverse(geom, st, a, b, dldi, lam0=lam0) + (g_dist,)
