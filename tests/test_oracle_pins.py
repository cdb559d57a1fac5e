"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks the oracle against mathematics or the paper, not against a
retyped copy of its own formula: closed-form optics, brute-force sums,
invariants, limits the paper states, adjoint dot products and finite
differences.  A plausible slip in the oracle (a dropped term, a wrong sign,
a transposed operand, a wrong FFT direction) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import adam as oadam
from oracle import multislice as om
from oracle import rotation as orot
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(1234)


def crand(*shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# ---------------------------------------------------------------- transforms

@pytest.mark.parametrize("n", [4, 8, 12, 16])
def test_fft_matches_bruteforce_dft(n):
    """fft2u/ifft2u equal the unitary DFT matrix written out by hand."""
    x = crand(n, n)
    j, k = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    w = np.exp(-2j * np.pi * j * k / n) / math.sqrt(n)
    ref = w @ x @ w.T
    assert rel(om.fft2u(x), ref) < 1e-13
    assert rel(om.ifft2u(x), np.conj(w) @ x @ np.conj(w).T) < 1e-13


def test_far_field_direction_negative_phase_convention():
    """Eq. fraunhofer has a +i exponent: a wave exp(-2 pi i k0 x / N) lands at +k0.

    With the zero frequency centred at N/2, the detector peak must be at
    column N/2 + k0 (a forward-sign FFT would put it at N/2 - k0).
    """
    n, k0y, k0x = 32, 3, 5
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    psi = np.exp(-2j * np.pi * (k0y * yy + k0x * xx) / n)
    det = np.abs(om.far_field(psi)) ** 2
    iy, ix = np.unravel_index(np.argmax(det), det.shape)
    assert (iy, ix) == (n // 2 + k0y, n // 2 + k0x)
    assert det[iy, ix] == pytest.approx(n * n, rel=1e-12)


# ---------------------------------------------------------------- Fresnel

def test_fresnel_gaussian_beam_closed_form():
    """Paraxial free-space propagation of a Gaussian beam (Eq. paraxial_kernel).

    psi_0 = exp(-r^2/w0^2) becomes (1/q) exp(-r^2/(w0^2 q)), q = 1 - i d/z_R,
    z_R = pi w0^2 / lambda, for the kernel exp(+i pi lambda d |nu|^2).
    """
    n, dx, lam = 256, 10e-9, 1.2398419843320002e-10
    w0 = 8 * dx
    zr = math.pi * w0 ** 2 / lam
    c = (np.arange(n) - n / 2) * dx
    r2 = c[:, None] ** 2 + c[None, :] ** 2
    psi0 = np.exp(-r2 / w0 ** 2)
    for d in (0.3 * zr, zr, 2.0 * zr):
        q = 1.0 - 1j * d / zr
        ref = np.exp(-r2 / (w0 ** 2 * q)) / q
        out = om.fresnel_propagate(psi0, om.fresnel_kernel(n, lam, dx, d))
        assert rel(out, ref) < 1e-12
        # the opposite kernel sign gives the conjugate beam: clearly different
        bad = om.fresnel_propagate(psi0, np.conj(om.fresnel_kernel(n, lam, dx, d)))
        assert rel(bad, ref) > 0.1


def test_fresnel_unitary_and_semigroup():
    n, dx, lam = 64, 10e-9, 1.24e-10
    psi = crand(n, n)
    h1 = om.fresnel_kernel(n, lam, dx, 3e-7)
    h2 = om.fresnel_kernel(n, lam, dx, 5e-7)
    h12 = om.fresnel_kernel(n, lam, dx, 8e-7)
    hm = om.fresnel_kernel(n, lam, dx, -3e-7)
    out = om.fresnel_propagate(psi, h1)
    assert np.linalg.norm(out) == pytest.approx(np.linalg.norm(psi), rel=1e-13)
    assert rel(om.fresnel_propagate(om.fresnel_propagate(psi, h1), h2), om.fresnel_propagate(psi, h12)) < 1e-13
    assert rel(om.fresnel_propagate(out, hm), psi) < 1e-13


# ---------------------------------------------------------------- Fourier shift

def test_fourier_shift_integer_is_roll_and_additive():
    """Eq. fourier_shift moves the probe to x + s: integer s is a circular roll."""
    n = 32
    p = crand(n, n)
    for sy, sx in [(1, 0), (0, 3), (-2, 5), (7, -4)]:
        assert rel(om.fourier_shift(p, np.array([sy, sx], float)), np.roll(p, (sy, sx), axis=(0, 1))) < 1e-13
    s1, s2 = np.array([0.3, -0.7]), np.array([-0.45, 0.2])
    assert rel(om.fourier_shift(om.fourier_shift(p, s1), s2), om.fourier_shift(p, s1 + s2)) < 1e-13
    assert rel(om.fourier_shift(p, np.zeros(2)), p) < 1e-14


def test_split_position_rule():
    c, s = om.split_position(np.array([[3.49, 3.5], [-0.2, 7.0]]))
    assert c.tolist() == [[3, 4], [0, 7]]
    assert np.allclose(s, [[0.49, -0.5], [-0.2, 0.0]])


# ---------------------------------------------------------------- modulation and multislice

def _geom(n, s, obj_repr="delta_beta", loss="gaussian", dz=10e-9):
    return om.Geometry(n, s, 1.2398419843320002e-10, 10e-9, dz, obj_repr, loss)


class _NoPropGeom(om.Geometry):
    """Geometry whose Fresnel kernel is the identity (projection limit)."""

    @property
    def h(self):
        return np.ones((self.n, self.n), complex)


def test_golden_unit_conversion():
    with open(os.path.join(GOLDEN, "constants.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        lam = synth.wavelength_from_energy(c["energy_ev"])
        assert lam == pytest.approx(c["wavelength_m"], rel=1e-9)
        assert om.k_dz(lam, c["dz_m"]) == pytest.approx(c["k_dz"], rel=1e-8)


def test_zero_object_is_unit_transmission():
    t = om.transmission(np.zeros((2, 4, 4)), np.zeros((2, 4, 4)), "delta_beta", 506.77)
    assert np.array_equal(t, np.ones((2, 4, 4), complex))
    t = om.transmission(np.ones((2, 4, 4)), np.zeros((2, 4, 4)), "real_imag", 506.77)
    assert np.array_equal(t, np.ones((2, 4, 4), complex))


def test_pure_projection_limit():
    """With H = 1 the multislice exit wave is the projection of Eq. obj_ri_modulation."""
    rng = np.random.default_rng(5)
    n, s, lat = 16, 5, 24
    for repr_ in ("delta_beta", "real_imag"):
        g = _NoPropGeom(n, s, 1.24e-10, 10e-9, 10e-9, repr_)
        if repr_ == "delta_beta":
            a, b = rng.uniform(0, 1e-3, (s, lat, lat)), rng.uniform(0, 1e-4, (s, lat, lat))
        else:
            a, b = rng.uniform(0.8, 1.0, (s, lat, lat)), rng.uniform(-0.2, 0.2, (s, lat, lat))
        p = crand(n, n, rng=rng)
        pos = np.array([[2.3, 4.6], [6.0, 1.2]])
        assert rel(om.exit_waves(g, a, b, p, pos), om.forward_pure_projection(g, a, b, p, pos)) < 1e-13


def test_single_slice_is_far_field_of_probe_times_transmission():
    """S = 1: I = |fftshift(ifft2(p_s * t, ortho))|^2 (written here with numpy.fft)."""
    rng = np.random.default_rng(6)
    n, lat = 16, 32
    g = _geom(n, 1)
    a, b = rng.uniform(0, 1e-3, (1, lat, lat)), rng.uniform(0, 1e-4, (1, lat, lat))
    p = crand(n, n, rng=rng)
    pos = np.array([[3.0, 9.0], [10.0, 2.0]])
    out = om.forward(g, a, b, p, pos)
    kdz = 2 * math.pi / g.wavelength_m * g.slice_dz_m
    for i, (cy, cx) in enumerate(pos.astype(int)):
        t = np.exp(-kdz * b[0, cy:cy + n, cx:cx + n]) * np.exp(1j * kdz * a[0, cy:cy + n, cx:cx + n])
        ref = np.abs(np.fft.fftshift(np.fft.ifft2(p * t, norm="ortho"))) ** 2
        assert rel(out[i], ref) < 1e-13


def test_vacuum_any_depth_gives_far_field_of_shifted_probe():
    rng = np.random.default_rng(7)
    n, lat = 16, 24
    p = crand(n, n, rng=rng)
    pos = np.array([[2.4, 3.7]])
    ref = np.abs(np.fft.fftshift(np.fft.ifft2(om.fourier_shift(p, pos - np.floor(pos + 0.5)),
                                              norm="ortho"))) ** 2
    for s in (1, 3, 8):
        z = np.zeros((s, lat, lat))
        assert rel(om.forward(_geom(n, s), z, z, p, pos)[0], ref[0]) < 1e-12


def test_energy_conservation_and_uniform_absorption():
    """Unitary propagation: sum I = |p|^2 exp(-2 k dz sum_j beta_j) for uniform beta."""
    rng = np.random.default_rng(8)
    n, s, lat = 16, 6, 24
    g = _geom(n, s)
    p = crand(n, n, rng=rng)
    a = rng.uniform(0, 1e-3, (s, lat, lat))
    pos = np.array([[1.0, 2.0], [5.5, 6.25]])
    i0 = om.forward(g, a, np.zeros_like(a), p, pos)
    assert np.allclose(i0.sum(axis=(1, 2)), np.sum(np.abs(p) ** 2), rtol=1e-12)
    beta = np.full_like(a, 3e-5)
    i1 = om.forward(g, a, beta, p, pos)
    expect = np.sum(np.abs(p) ** 2) * math.exp(-2 * g.kdz * 3e-5 * s)
    assert np.allclose(i1.sum(axis=(1, 2)), expect, rtol=1e-12)


def test_trailing_propagation_does_not_change_intensity():
    """S - 1 vs S propagations: an extra vacuum slice leaves I unchanged."""
    rng = np.random.default_rng(9)
    n, s, lat = 16, 4, 24
    a, b = rng.uniform(0, 1e-3, (s, lat, lat)), rng.uniform(0, 1e-4, (s, lat, lat))
    p = crand(n, n, rng=rng)
    pos = np.array([[3.2, 1.9]])
    i_s = om.forward(_geom(n, s), a, b, p, pos)
    a2 = np.concatenate([a, np.zeros((1, lat, lat))])
    b2 = np.concatenate([b, np.zeros((1, lat, lat))])
    assert rel(om.forward(_geom(n, s + 1), a2, b2, p, pos), i_s) < 1e-12


def test_chunk_out_of_bounds_raises():
    z = np.zeros((1, 20, 20))
    with pytest.raises(IndexError):
        om.forward(_geom(16, 1), z, z, crand(16, 16), np.array([[5.0, 0.0]]))


# ---------------------------------------------------------------- losses

def test_loss_closed_forms():
    i = np.array([[[4.0, 9.0], [0.0, 1.0]]])
    m = np.array([[[1.0, 9.0], [0.0, 4.0]]])
    # LSQ on amplitudes: ((2-1)^2 + 0 + 0 + (1-2)^2) / 4 with eps = 0
    assert om.loss_value("gaussian", i, m, 0.0) == pytest.approx(0.5)
    # Poisson: (4 - log 4 + 9 - 9 log 9 + 0 + 1 - 4 log 1) / 4 (eps=0, 0*log0 := 0)
    ip, mp = np.array([[[4.0, 9.0], [1.0, 1.0]]]), np.array([[[1.0, 9.0], [0.0, 4.0]]])
    ref = (4 - math.log(4) + 9 - 9 * math.log(9) + 1 + 1) / 4
    assert om.loss_value("poisson", ip, mp, 0.0) == pytest.approx(ref)
    # Residuals vanish at the data (Gaussian: I = I_m; Poisson: I + eps = I_m)
    x = RNG.uniform(1, 5, (3, 4))
    assert np.all(om.loss_dI("gaussian", x, x, 1e-6, 12) == 0)
    assert np.allclose(om.loss_dI("poisson", x - 1e-6, x, 1e-6, 12), 0, atol=1e-15)


# ---------------------------------------------------------------- adjoints

def _dot(a, b):
    return np.vdot(a, b)   # conj(a) . b


def test_adjoint_dot_products_linear_factors():
    """<A x, y> = <x, A^H y> for every linear factor of the model."""
    rng = np.random.default_rng(10)
    n = 16
    x, y = crand(3, n, n, rng=rng), crand(3, n, n, rng=rng)
    h = om.fresnel_kernel(n, 1.24e-10, 10e-9, 10e-9)
    pairs = [
        (om.fft2u, om.ifft2u),
        (om.far_field, om.far_field_adjoint),
        (lambda v: om.fresnel_propagate(v, h), lambda v: om.fresnel_propagate_adjoint(v, h)),
    ]
    t = crand(n, n, rng=rng)
    pairs.append((lambda v: v * t, lambda v: v * np.conj(t)))
    e = om.shift_ramp(n, np.array([0.3, -0.4]))
    pairs.append((lambda v: om.ifft2u(om.fft2u(v) * e), lambda v: om.ifft2u(om.fft2u(v) * np.conj(e))))
    for fwd, adj in pairs:
        lhs, rhs = _dot(fwd(x), y), _dot(x, adj(y))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gather_scatter_are_transposes():
    rng = np.random.default_rng(11)
    obj = rng.standard_normal((3, 30, 30))
    corners = np.array([[0, 0], [5, 7], [14, 14], [5, 7]])
    g = rng.standard_normal((4, 3, 16, 16))
    lhs = np.sum(om.take_chunks(obj, corners, 16) * g)
    rhs = np.sum(obj * om.scatter_chunks(g, corners, obj.shape))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def _exit_linear_in_probe(geom, a, b, pos, probe):
    return om.exit_waves(geom, a, b, probe, pos)


def test_probe_to_exit_map_adjoint():
    """For a fixed object the exit wave is complex-linear in the probe; its adjoint
    (what the gradient applies) passes the dot-product test."""
    rng = np.random.default_rng(12)
    n, s, lat = 16, 4, 24
    g = _geom(n, s)
    a, b = rng.uniform(0, 1e-2, (s, lat, lat)), rng.uniform(0, 1e-3, (s, lat, lat))
    pos = np.array([[3.3, 2.2]])
    p, y = crand(n, n, rng=rng), crand(1, n, n, rng=rng)
    c, sh = om.split_position(pos)
    t = om.transmission(om.take_chunks(a, c, n), om.take_chunks(b, c, n), "delta_beta", g.kdz)
    # adjoint by hand: reverse the slices
    lam = y.copy()
    for j in range(s - 1, -1, -1):
        mu = np.conj(t[:, j]) * lam
        if j > 0:
            lam = om.fresnel_propagate_adjoint(mu, g.h)
    gp = om.ifft2u(om.fft2u(mu) * np.conj(om.shift_ramp(n, sh)))[0]
    lhs = _dot(_exit_linear_in_probe(g, a, b, pos, p), y)
    rhs = _dot(p, gp)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ---------------------------------------------------------------- finite differences

def _fd_case(loss, obj_repr="delta_beta"):
    sc = synth.fd_subcase_n16_s4()
    geom = om.Geometry(sc.n, sc.n_slices, sc.wavelength_m, sc.pixel_m, sc.slice_dz_m, obj_repr, loss)
    if obj_repr == "delta_beta":
        a, b = sc.eval_obj_a, sc.eval_obj_b
        at, bt = sc.obj_a, sc.obj_b
    else:
        rng = np.random.default_rng(77)
        o_true = np.exp(1j * 50 * sc.obj_a - 50 * sc.obj_b) * (1 + 0.05 * rng.standard_normal(sc.obj_a.shape))
        at, bt = o_true.real, o_true.imag
        o_eval = 0.5 * (1 + o_true)
        a, b = o_eval.real.copy(), o_eval.imag.copy()
    i_true = om.forward(geom, at, bt, sc.probe, sc.positions)
    i_meas = i_true if loss == "gaussian" else np.random.default_rng(3).poisson(i_true).astype(float)
    return geom, a, b, sc.eval_probe, sc.eval_positions, i_meas


@pytest.mark.parametrize("loss", ["gaussian", "poisson"])
@pytest.mark.parametrize("obj_repr", ["delta_beta", "real_imag"])
def test_gradient_matches_central_finite_differences(loss, obj_repr):
    """FP64 central differences on the tiny sub-case, every input kind.

    Steps are taken in dimensionless units: 1e-3 rad of k dz delta (and of
    k dz beta), 1e-3 of the object modulus for real/imag objects, 1e-3 px
    for shifts and 1e-3 max|p| for the probe.
    """
    geom, a, b, p, pos, i_meas = _fd_case(loss, obj_repr)
    L, ga, gb, gp, gs = om.loss_grad(geom, a, b, p, pos, i_meas)
    assert L == pytest.approx(om.loss(geom, a, b, p, pos, i_meas), rel=1e-14)

    def f(a_=a, b_=b, p_=p, pos_=pos):
        return om.loss(geom, a_, b_, p_, pos_, i_meas)

    rng = np.random.default_rng(99)
    # delta/beta: 1e-3 in dimensionless units as the workload states; the
    # real/imag object is strongly nonlinear at that step, so 1e-4 there.
    hu = 1e-3 if obj_repr == "delta_beta" else 1e-4
    h_obj = hu / geom.kdz if obj_repr == "delta_beta" else hu
    checks = []
    corners, _ = om.split_position(pos)
    for arr, grad, which in ((a, ga, "a"), (b, gb, "b")):
        for _ in range(6):
            # pick a voxel inside some chunk
            k = rng.integers(len(corners))
            z = rng.integers(geom.n_slices)
            y = corners[k, 0] + rng.integers(geom.n)
            x = corners[k, 1] + rng.integers(geom.n)
            ap, am = arr.copy(), arr.copy()
            ap[z, y, x] += h_obj
            am[z, y, x] -= h_obj
            kw_p = {"a_": ap} if which == "a" else {"b_": ap}
            kw_m = {"a_": am} if which == "a" else {"b_": am}
            checks.append(((f(**kw_p) - f(**kw_m)) / (2 * h_obj), grad[z, y, x]))
    hp = hu * np.max(np.abs(p))
    for _ in range(4):
        iy, ix = rng.integers(geom.n, size=2)
        for unit, comp in ((1.0, np.real), (1j, np.imag)):
            pp, pm = p.copy(), p.copy()
            pp[iy, ix] += unit * hp
            pm[iy, ix] -= unit * hp
            checks.append(((f(p_=pp) - f(p_=pm)) / (2 * hp), comp(gp[iy, ix])))
    for k in range(len(pos)):
        for ax in range(2):
            pp, pm = pos.copy(), pos.copy()
            pp[k, ax] += hu
            pm[k, ax] -= hu
            checks.append(((f(pos_=pp) - f(pos_=pm)) / (2 * hu), gs[k, ax]))
    fd = np.array([c[0] for c in checks])
    an = np.array([c[1] for c in checks])
    scale = np.max(np.abs(an))
    assert np.max(np.abs(fd - an)) < 2e-5 * scale, (fd, an)


# ---------------------------------------------------------------- rotation

def test_rotation_identity_and_right_angles():
    rng = np.random.default_rng(13)
    o = rng.standard_normal((10, 3, 10))
    assert np.allclose(orot.rotate(o, 0.0), o, atol=1e-14)
    r90 = orot.rotate(o, math.pi / 2)
    # out[z, y, x] = o[x, y, L-1-z]  (every xz-plane rotated by 90 degrees)
    ref = np.stack([np.rot90(o[:, yy, :]) for yy in range(3)], axis=1)
    assert np.allclose(r90, ref, atol=1e-12)
    r180 = orot.rotate(o, math.pi)
    assert np.allclose(r180, o[::-1, :, ::-1], atol=1e-12)


def test_rotation_transpose_dot_product_and_half_pixel():
    rng = np.random.default_rng(14)
    o = rng.standard_normal((12, 2, 12))
    g = rng.standard_normal((12, 2, 12))
    for th in (0.3, 1.1, 2.9):
        lhs = np.sum(orot.rotate(o, th) * g)
        rhs = np.sum(o * orot.rotate_transpose(g, th))
        assert lhs == pytest.approx(rhs, rel=1e-12)
    # bilinear interpolation reproduces a linear ramp wherever all taps are inside
    zz, yy, xx = np.meshgrid(np.arange(12.0), np.arange(2.0), np.arange(12.0), indexing="ij")
    ramp = 2.0 * xx - 0.5 * zz
    th = 0.4
    out = orot.rotate(ramp, th)
    c = 5.5
    x0 = math.cos(th) * (xx - c) - math.sin(th) * (zz - c) + c
    z0 = math.sin(th) * (xx - c) + math.cos(th) * (zz - c) + c
    inside = (x0 >= 0) & (x0 <= 11) & (z0 >= 0) & (z0 <= 11)
    assert np.allclose(out[inside], (2.0 * x0 - 0.5 * z0)[inside], atol=1e-12)


# ---------------------------------------------------------------- Adam

def test_adam_first_step_closed_form():
    rng = np.random.default_rng(15)
    x, g = rng.standard_normal(50), rng.standard_normal(50)
    x1, m, v = oadam.adam_step(x, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(x1, x - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-15)
    # constant gradient: bias-corrected moments stay exactly g and g^2
    x2, m, v = oadam.adam_step(x1, g, m, v, 2, lr=1e-3)
    assert np.allclose(x2, x1 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- probe modes (Eq. multimode)

def _modes_case(loss="gaussian", n_modes=3):
    geom, a, b, p, pos, _ = _fd_case(loss, "delta_beta")
    rng = np.random.default_rng(7)
    probes = np.stack([p] + [0.4 * p * np.exp(1j * rng.uniform(-1, 1, p.shape)) for _ in range(n_modes - 1)])
    sc = synth.fd_subcase_n16_s4()
    i_true = om.forward_modes(geom, sc.obj_a, sc.obj_b, probes * 1.1, sc.positions)
    i_meas = i_true if loss == "gaussian" else rng.poisson(i_true).astype(float)
    return geom, a, b, probes, pos, i_meas


def test_one_mode_is_the_single_probe_model():
    geom, a, b, probes, pos, i_meas = _modes_case(n_modes=1)
    p = probes[0]
    assert np.array_equal(om.forward_modes(geom, a, b, probes, pos), om.forward(geom, a, b, p, pos))
    one = om.loss_grad(geom, a, b, p, pos, i_meas)
    many = om.loss_grad_modes(geom, a, b, probes, pos, i_meas)
    assert many[0] == one[0]
    for x, y in zip(many[1:], one[1:]):
        assert np.allclose(np.squeeze(x), y, rtol=0, atol=1e-15 * np.max(np.abs(y)))


def test_two_halves_of_one_probe_equal_that_probe():
    """p/sqrt2 twice carries the same power: I, L, object and shift gradients
    equal the single-probe ones; each mode's probe gradient is g_p / sqrt2."""
    for loss in ("gaussian", "poisson"):
        geom, a, b, probes, pos, i_meas = _modes_case(loss, n_modes=1)
        p = probes[0]
        half = np.stack([p, p]) / np.sqrt(2.0)
        L1, ga1, gb1, gp1, gs1 = om.loss_grad(geom, a, b, p, pos, i_meas)
        L2, ga2, gb2, gp2, gs2 = om.loss_grad_modes(geom, a, b, half, pos, i_meas)
        assert rel(om.forward_modes(geom, a, b, half, pos), om.forward(geom, a, b, p, pos)) < 1e-14
        assert L2 == pytest.approx(L1, rel=1e-13)
        for x, y in ((ga2, ga1), (gb2, gb1), (gs2, gs1), (gp2[0], gp1 / np.sqrt(2)), (gp2[1], gp1 / np.sqrt(2))):
            assert rel(x, y) < 1e-12


def test_intensity_is_invariant_under_unitary_mixing_of_modes():
    """The incoherent sum over modes depends only on the modes' span with its
    metric: p'_m = sum_k U_mk p_k with U unitary leaves I unchanged (a model
    that added amplitudes instead of intensities would not)."""
    geom, a, b, probes, pos, _ = _modes_case(n_modes=3)
    rng = np.random.default_rng(21)
    u, _ = np.linalg.qr(crand(3, 3, rng=rng))
    mixed = np.einsum("mk,kyx->myx", u, probes)
    assert rel(om.forward_modes(geom, a, b, mixed, pos), om.forward_modes(geom, a, b, probes, pos)) < 1e-13
    single = om.forward(geom, a, b, probes.sum(axis=0), pos)
    assert rel(single, om.forward_modes(geom, a, b, probes, pos)) > 1e-3


@pytest.mark.parametrize("loss", ["gaussian", "poisson"])
def test_mode_gradients_match_central_finite_differences(loss):
    geom, a, b, probes, pos, i_meas = _modes_case(loss, n_modes=3)
    L, ga, gb, gp, gs = om.loss_grad_modes(geom, a, b, probes, pos, i_meas)

    def f(a_=a, probes_=probes, pos_=pos):
        return om.loss_modes(geom, a_, b, probes_, pos_, i_meas)

    rng = np.random.default_rng(5)
    hu = 1e-3
    checks = []
    corners, _ = om.split_position(pos)
    for _ in range(6):
        k = rng.integers(len(corners))
        z, y, x = rng.integers(geom.n_slices), corners[k, 0] + rng.integers(geom.n), corners[k, 1] + rng.integers(geom.n)
        ap, am = a.copy(), a.copy()
        ap[z, y, x] += hu / geom.kdz
        am[z, y, x] -= hu / geom.kdz
        checks.append(((f(a_=ap) - f(a_=am)) / (2 * hu / geom.kdz), ga[z, y, x]))
    hp = hu * np.max(np.abs(probes))
    for m in range(len(probes)):
        iy, ix = rng.integers(geom.n, size=2)
        for unit, comp in ((1.0, np.real), (1j, np.imag)):
            pp, pm = probes.copy(), probes.copy()
            pp[m, iy, ix] += unit * hp
            pm[m, iy, ix] -= unit * hp
            checks.append(((f(probes_=pp) - f(probes_=pm)) / (2 * hp), comp(gp[m, iy, ix])))
    for k in range(len(pos)):
        for ax in range(2):
            pp, pm = pos.copy(), pos.copy()
            pp[k, ax] += hu
            pm[k, ax] -= hu
            checks.append(((f(pos_=pp) - f(pos_=pm)) / (2 * hu), gs[k, ax]))
    fd = np.array([c[0] for c in checks])
    an = np.array([c[1] for c in checks])
    assert np.max(np.abs(fd - an)) < 2e-5 * np.max(np.abs(an)), (fd, an)


# ---------------------------------------------------------------- unequal slice spacing (sparse multislice)

GAPS = np.array([0.4e-6, 1.5e-6, 0.8e-6])    # slice j -> j+1, metres (phase at Nyquist 0.4 - 1.5 rad)


def _gaps_geom(geom, gaps, loss=None):
    return om.Geometry(geom.n, geom.n_slices if gaps is None else len(gaps) + 1, geom.wavelength_m, geom.pixel_m,
                       geom.slice_dz_m, geom.obj_repr, loss or geom.loss, geom.eps, gaps=gaps)


def _gaps_case(loss="gaussian"):
    geom, a, b, p, pos, _ = _fd_case(loss)
    sc = synth.fd_subcase_n16_s4()
    truth = _gaps_geom(geom, GAPS)
    i_true = om.forward(truth, sc.obj_a, sc.obj_b, sc.probe, sc.positions)
    i_meas = i_true if loss == "gaussian" else np.random.default_rng(3).poisson(i_true).astype(float)
    return _gaps_geom(geom, GAPS * np.array([1.1, 0.9, 1.05])), a, b, p, pos, i_meas


def test_equal_gaps_are_the_uniform_model():
    geom, a, b, p, pos, i_meas = _fd_case("poisson")
    eq = _gaps_geom(geom, np.full(geom.n_slices - 1, geom.slice_dz_m))
    assert np.array_equal(om.forward(eq, a, b, p, pos), om.forward(geom, a, b, p, pos))
    one = om.loss_grad(geom, a, b, p, pos, i_meas)
    var = om.loss_grad_gaps(eq, a, b, p, pos, i_meas)
    assert var[0] == one[0]
    for x, y in zip(var[1:5], one[1:]):
        assert np.array_equal(x, y)


def test_vacuum_slice_between_two_gaps_is_one_gap():
    """Free space composes: H(d1) H(d2) = H(d1 + d2), so an empty slice
    (t = 1) between gaps d1 and d2 is the same as one gap d1 + d2."""
    geom, a, b, p, pos, _ = _fd_case("gaussian")
    a3, b3 = a[:3].copy(), b[:3].copy()
    a3[1] = 0.0
    b3[1] = 0.0
    three = _gaps_geom(geom, np.array([0.7e-6, 1.3e-6]))
    two = _gaps_geom(geom, np.array([2.0e-6]))
    i3 = om.forward(three, a3, b3, p, pos)
    i2 = om.forward(two, a3[[0, 2]], b3[[0, 2]], p, pos)
    assert rel(i3, i2) < 1e-13
    # and the distance matters: a different split of the same object differs
    assert rel(om.forward(_gaps_geom(geom, np.array([1.3e-6, 0.7e-6])), a3, b3, p, pos), i2) < 1e-13
    assert rel(om.forward(_gaps_geom(geom, np.array([1.0e-6])), a3[[0, 2]], b3[[0, 2]], p, pos), i2) > 1e-3


def test_zero_gaps_give_the_projection_approximation():
    """All gaps zero: the slices act as one thin object, the product of their
    transmissions (the projection approximation the paper states)."""
    geom, a, b, p, pos, _ = _fd_case("gaussian")
    zero = _gaps_geom(geom, np.zeros(geom.n_slices - 1))
    ref = np.abs(om.far_field(om.forward_pure_projection(geom, a, b, p, pos))) ** 2
    assert rel(om.forward(zero, a, b, p, pos), ref) < 1e-13


def test_gap_gradients_with_empty_middle_slices_are_the_two_slice_derivative():
    """Only the first and the last slice hold matter: every gap then only
    adds to the one distance D between them, so all gap gradients are equal,
    and equal dL/dD of the two-slice model (central differences).  With no
    object at all the far-field intensity does not depend on free-space
    distance, and the gap gradients vanish."""
    geom, a, b, p, pos, i_meas = _gaps_case("gaussian")
    a2, b2 = a.copy(), b.copy()
    a2[1:-1] = 0.0
    b2[1:-1] = 0.0
    g_gaps = om.loss_grad_gaps(geom, a2, b2, p, pos, i_meas)[5]
    assert np.max(np.abs(g_gaps - g_gaps[0])) <= 1e-9 * abs(g_gaps[0])
    total = float(np.sum(geom.gaps))
    h = 1e-9

    def f(d):
        return om.loss(_gaps_geom(geom, np.array([d])), a2[[0, -1]], b2[[0, -1]], p, pos, i_meas)

    fd = (f(total + h) - f(total - h)) / (2 * h)
    assert g_gaps[0] == pytest.approx(fd, rel=1e-6)
    z = np.zeros_like(a)
    g0 = om.loss_grad_gaps(geom, z, z, p, pos, i_meas)[5]
    assert np.max(np.abs(g0)) <= 1e-9 * abs(g_gaps[0])


@pytest.mark.parametrize("loss", ["gaussian", "poisson"])
def test_gap_gradients_match_central_finite_differences(loss):
    """dL/d(gap) by central differences, and the object gradient at unequal
    gaps (a propagator applied at the wrong gap in the reverse sweep fails
    these).  The gap step is 0.03 nm on gaps of ~1 um: the central
    difference error falls as h^2 (5e-5 relative at 1 nm, 5e-8 here) while
    rounding stays near 1e-8."""
    geom, a, b, p, pos, i_meas = _gaps_case(loss)
    L, ga, gb, gp, gs, gg = om.loss_grad_gaps(geom, a, b, p, pos, i_meas)
    assert L == pytest.approx(om.loss(geom, a, b, p, pos, i_meas), rel=1e-14)
    h = 3e-11
    for j in range(len(geom.gaps)):
        gpl, gmi = geom.gaps.copy(), geom.gaps.copy()
        gpl[j] += h
        gmi[j] -= h
        fd = (om.loss(_gaps_geom(geom, gpl), a, b, p, pos, i_meas)
              - om.loss(_gaps_geom(geom, gmi), a, b, p, pos, i_meas)) / (2 * h)
        assert gg[j] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.max(np.abs(gg))), j
    rng = np.random.default_rng(8)
    corners, _ = om.split_position(pos)
    hu = 1e-5 / geom.kdz      # 1e-5 rad of k dz delta: truncation ~1e-9 relative
    for _ in range(6):
        k = rng.integers(len(corners))
        zz, y, x = rng.integers(geom.n_slices), corners[k, 0] + rng.integers(geom.n), corners[k, 1] + rng.integers(geom.n)
        for arr, g in ((a, ga), (b, gb)):
            ap, am = arr.copy(), arr.copy()
            ap[zz, y, x] += hu
            am[zz, y, x] -= hu
            args_p = (ap, b) if arr is a else (a, ap)
            args_m = (am, b) if arr is a else (a, am)
            fd = (om.loss(geom, *args_p, p, pos, i_meas) - om.loss(geom, *args_m, p, pos, i_meas)) / (2 * hu)
            assert g[zz, y, x] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.max(np.abs(g)))


# ---------------------------------------------------------------- near field (Eqs. fresnel_prop, sommerfeld_kernel)

def test_sommerfeld_kernel_on_plane_waves():
    """A plane wave of grid frequency nu0 is an eigenfunction of free space:
    it picks up exp(-i k d sqrt(1 - lambda^2 |nu0|^2)) if it propagates and is
    removed if it is evanescent (lambda |nu0| > 1)."""
    n, dx, lam, d = 32, 1e-10, 1.5e-10, 2e-9           # lambda / (2 dx) = 0.75: some frequencies evanescent
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    k = 2 * np.pi / lam
    h = om.sommerfeld_kernel(n, lam, dx, d)
    for ky, kx in ((0, 0), (3, -2), (5, 7), (-9, 4), (12, 12), (16, 0)):
        psi = np.exp(2j * np.pi * (ky * yy + kx * xx) / n)
        nu2 = (ky ** 2 + kx ** 2) / (n * dx) ** 2
        out = om.fresnel_propagate(psi, h)
        if lam ** 2 * nu2 < 1:
            assert rel(out, psi * np.exp(-1j * k * d * np.sqrt(1 - lam ** 2 * nu2))) < 1e-12, (ky, kx)
        else:
            assert np.max(np.abs(out)) < 1e-13, (ky, kx)


def test_sommerfeld_reduces_to_paraxial_at_small_angles():
    """H2 exp(+i k d) - H1 = O(k d lambda^4 |nu|^4 / 8): at 1 um pixels and
    hard X-rays the two near-field models agree to that order, and they
    part where the angle is large."""
    sc = synth.fd_subcase_n16_s4()
    lam = sc.wavelength_m
    for dx, d, close in ((1e-6, 0.4, True), (2e-10, 3e-8, False)):
        geom = om.Geometry(sc.n, sc.n_slices, lam, dx, sc.slice_dz_m)
        i1 = om.forward_nearfield(geom, sc.obj_a, sc.obj_b, sc.probe, sc.positions, [d], np.zeros(9, int), "paraxial")
        i2 = om.forward_nearfield(geom, sc.obj_a, sc.obj_b, sc.probe, sc.positions, [d], np.zeros(9, int), "sommerfeld")
        bound = 2 * np.pi / lam * d * lam ** 4 * (0.5 / dx) ** 4 * 2 / 8 * 4
        if close:
            assert rel(i2, i1) < max(bound, 1e-12)
        else:
            assert rel(i2, i1) > 1e-3


def test_nearfield_of_a_gaussian_beam_through_vacuum():
    """Vacuum slices: the detector sees the Gaussian beam's closed form at the
    total distance (S-1) dz + d."""
    n, dx, lam, dz, s = 64, 10e-9, 1.2398419843320002e-10, 10e-9, 3
    w0 = 5 * dx
    zr = math.pi * w0 ** 2 / lam
    c = (np.arange(n) - n / 2) * dx
    r2 = c[:, None] ** 2 + c[None, :] ** 2
    probe = np.exp(-r2 / w0 ** 2)
    geom = om.Geometry(n, s, lam, dx, dz)
    z = np.zeros((s, n, n))
    for d in (0.5 * zr, 1.5 * zr):
        q = 1.0 - 1j * ((s - 1) * dz + d) / zr
        ref = np.abs(np.exp(-r2 / (w0 ** 2 * q)) / q) ** 2
        got = om.forward_nearfield(geom, z, z, probe, np.zeros((1, 2)), [d], [0], "paraxial")[0]
        assert rel(got, ref) < 1e-9      # the periodic window's aliasing of the tails is ~3e-11


def test_nearfield_distance_is_an_empty_last_slice():
    """Detector distance dz behind S slices = S + 1 slices (the last empty) at distance 0."""
    geom, a, b, p, pos, _ = _fd_case("gaussian")
    i_d = om.forward_nearfield(geom, a, b, p, pos, [geom.slice_dz_m], np.zeros(len(pos), int))
    a1 = np.concatenate([a, np.zeros_like(a[:1])])
    b1 = np.concatenate([b, np.zeros_like(b[:1])])
    g1 = om.Geometry(geom.n, geom.n_slices + 1, geom.wavelength_m, geom.pixel_m, geom.slice_dz_m)
    i_0 = om.forward_nearfield(g1, a1, b1, p, pos, [0.0], np.zeros(len(pos), int))
    assert rel(i_d, i_0) < 1e-13


def _nf_case(loss, kind):
    geom, a, b, p, pos, _ = _fd_case(loss)
    sc = synth.fd_subcase_n16_s4()
    dists = np.array([0.6e-6, 1.4e-6])
    idx = np.arange(len(pos)) % 2
    i_true = om.forward_nearfield(geom, sc.obj_a, sc.obj_b, sc.probe, sc.positions, dists, idx, kind)
    i_meas = i_true if loss == "gaussian" else np.random.default_rng(3).poisson(i_true).astype(float)
    return geom, a, b, p, pos, i_meas, dists * np.array([1.07, 0.95]), idx


@pytest.mark.parametrize("kind", ["paraxial", "sommerfeld"])
@pytest.mark.parametrize("loss", ["gaussian", "poisson"])
def test_nearfield_gradients_match_central_finite_differences(loss, kind):
    geom, a, b, p, pos, i_meas, dists, idx = _nf_case(loss, kind)
    L, ga, gb, gp, gs, gd = om.loss_grad_nearfield(geom, a, b, p, pos, i_meas, dists, idx, kind)

    def f(a_=a, p_=p, pos_=pos, d_=dists):
        return om.loss_nearfield(geom, a_, b, p_, pos_, i_meas, d_, idx, kind)

    assert L == pytest.approx(f(), rel=1e-14)
    h = 3e-11
    for j in range(len(dists)):
        dp, dm = dists.copy(), dists.copy()
        dp[j] += h
        dm[j] -= h
        assert gd[j] == pytest.approx((f(d_=dp) - f(d_=dm)) / (2 * h), rel=1e-6, abs=1e-9 * np.max(np.abs(gd))), j
    rng = np.random.default_rng(17)
    corners, _ = om.split_position(pos)
    hu = 1e-5 / geom.kdz
    for _ in range(4):
        k = rng.integers(len(corners))
        zz, y, x = rng.integers(geom.n_slices), corners[k, 0] + rng.integers(geom.n), corners[k, 1] + rng.integers(geom.n)
        ap, am = a.copy(), a.copy()
        ap[zz, y, x] += hu
        am[zz, y, x] -= hu
        assert ga[zz, y, x] == pytest.approx((f(a_=ap) - f(a_=am)) / (2 * hu), rel=1e-5, abs=1e-7 * np.max(np.abs(ga)))
    hp = 1e-6 * np.max(np.abs(p))
    for _ in range(3):
        iy, ix = rng.integers(geom.n, size=2)
        for unit, comp in ((1.0, np.real), (1j, np.imag)):
            pp, pm = p.copy(), p.copy()
            pp[iy, ix] += unit * hp
            pm[iy, ix] -= unit * hp
            assert comp(gp[iy, ix]) == pytest.approx((f(p_=pp) - f(p_=pm)) / (2 * hp), rel=1e-5,
                                                     abs=1e-7 * np.max(np.abs(gp)))
    for k in range(2):
        for c in range(2):
            pp, pm = pos.copy(), pos.copy()
            pp[k, c] += 1e-6
            pm[k, c] -= 1e-6
            assert gs[k, c] == pytest.approx((f(pos_=pp) - f(pos_=pm)) / 2e-6, rel=1e-5, abs=1e-7 * np.max(np.abs(gs)))


# ---------------------------------------------------------------- probe defocus

DEFOCUS = 0.9e-6        # metres; on the tiny sub-case the Nyquist phase is about 1 rad


def _defocus_case(loss="gaussian"):
    """Measured data at the true defocus, evaluated 10 % away from it."""
    geom, a, b, p, pos, _ = _fd_case(loss)
    sc = synth.fd_subcase_n16_s4()
    i_true = om.forward_defocus(geom, sc.obj_a, sc.obj_b, sc.probe, sc.positions, DEFOCUS)
    i_meas = i_true if loss == "gaussian" else np.random.default_rng(3).poisson(i_true).astype(float)
    return geom, a, b, p, pos, i_meas, 1.1 * DEFOCUS


def test_zero_defocus_is_the_plain_model():
    geom, a, b, p, pos, i_meas, _ = _defocus_case("poisson")
    assert rel(om.forward_defocus(geom, a, b, p, pos, 0.0), om.forward(geom, a, b, p, pos)) < 1e-14
    got = om.loss_grad_defocus(geom, a, b, p, pos, i_meas, 0.0)
    ref = om.loss_grad(geom, a, b, p, pos, i_meas)
    assert got[0] == pytest.approx(ref[0], rel=1e-13)
    for x, y in zip(got[1:5], ref[1:]):
        assert rel(x, y) < 1e-12


@pytest.mark.parametrize("loss", ["gaussian", "poisson"])
def test_defocus_is_an_empty_leading_slice(loss):
    """Defocusing the probe by d is free-space propagation before slice 0, so
    it equals the same object behind one extra empty slice at gap d (the
    unequal-spacing model, whose gap gradient comes from the reverse sweep,
    not from this chain rule).  Intensities, every gradient and dL/dd agree."""
    geom, a, b, p, pos, i_meas, d = _defocus_case(loss)
    z = np.zeros_like(a[:1])
    a1, b1 = np.concatenate([z, a]), np.concatenate([z, b])
    gaps = np.concatenate([[d], np.full(geom.n_slices - 1, geom.slice_dz_m)])
    g1 = _gaps_geom(geom, gaps)
    assert rel(om.forward_defocus(geom, a, b, p, pos, d), om.forward(g1, a1, b1, p, pos)) < 1e-13
    L, ga, gb, gp, gs, gd = om.loss_grad_defocus(geom, a, b, p, pos, i_meas, d)
    L1, ga1, gb1, gp1, gs1, gg1 = om.loss_grad_gaps(g1, a1, b1, p, pos, i_meas)
    assert L == pytest.approx(L1, rel=1e-13)
    assert rel(ga, ga1[1:]) < 1e-11 and rel(gb, gb1[1:]) < 1e-11
    assert rel(gp, gp1) < 1e-11 and rel(gs, gs1) < 1e-11
    assert gd == pytest.approx(gg1[0], rel=1e-9)
    assert abs(gd) > 0


@pytest.mark.parametrize("loss", ["gaussian", "poisson"])
def test_defocus_gradients_match_central_finite_differences(loss):
    """dL/dd and dL/dp (complex: dL/dRe + i dL/dIm) by central differences."""
    geom, a, b, p, pos, i_meas, d = _defocus_case(loss)
    L, ga, gb, gp, gs, gd = om.loss_grad_defocus(geom, a, b, p, pos, i_meas, d)

    def f(p_=p, d_=d):
        return loss_value_at(geom, a, b, p_, pos, i_meas, d_)

    h = 3e-11
    fd = (f(d_=d + h) - f(d_=d - h)) / (2 * h)
    assert gd == pytest.approx(fd, rel=1e-6)
    hp = 1e-6 * np.max(np.abs(p))
    for (y, x) in ((3, 4), (8, 8), (12, 1)):
        for unit in (1.0, 1j):
            pp, pm = p.copy(), p.copy()
            pp[y, x] += hp * unit
            pm[y, x] -= hp * unit
            fd = (f(p_=pp) - f(p_=pm)) / (2 * hp)
            comp = gp[y, x].real if unit == 1.0 else gp[y, x].imag
            assert comp == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.max(np.abs(gp)))


def loss_value_at(geom, a, b, p, pos, i_meas, d):
    return om.loss_value(geom.loss, om.forward_defocus(geom, a, b, p, pos, d), i_meas, geom.eps)


def test_defocus_composes_and_vanishes_in_vacuum():
    """Two defocus steps add (H(d1) H(d2) = H(d1 + d2)).  With no object the
    far-field intensity is |F p_s|^2 whatever the defocus (|H| = 1), so the
    defocus gradient vanishes."""
    geom, a, b, p, pos, i_meas, d = _defocus_case("gaussian")
    two = om.defocus_probe(geom, om.defocus_probe(geom, p, 0.3e-6), 0.5e-6)
    assert rel(two, om.defocus_probe(geom, p, 0.8e-6)) < 1e-13
    assert rel(om.defocus_probe(geom, p, 0.8e-6), p) > 1e-2
    zero = np.zeros_like(a)
    i0 = om.forward_defocus(geom, zero, zero, p, pos, 0.0)
    assert rel(om.forward_defocus(geom, zero, zero, p, pos, 2e-6), i0) < 1e-13
    gd_obj = om.loss_grad_defocus(geom, a, b, p, pos, i_meas, d)[5]
    gd_vac = om.loss_grad_defocus(geom, zero, zero, p, pos, i0 * 1.3, d)[5]
    assert abs(gd_vac) <= 1e-9 * abs(gd_obj)
