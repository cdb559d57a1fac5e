"""Seeded synthetic inputs for the multislice ptychography workloads.

This module is shared by the CPU oracle, the tests and the benchmark.  It
draws objects, probes and scan positions; it holds none of the forward
model's arithmetic (no propagation, no modulation, no FFT of a wavefield).
Measured intensities are *not* produced here: whoever needs them simulates
them with the model of their choice from the inputs drawn here.

Workload shapes follow the paper's experiments (far-field 2D ptychography,
Sec. 3 "fly-scan ptychography"; multislice ptychotomography, Sec. 3 and
Sec. S1.C "Module Propagate") scaled to synthetic stand-ins, since the
paper's datasets are not available.

Everything is FP64 NumPy driven by ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy.ndimage import gaussian_filter

# h*c in eV*m (CODATA 2018 exact-derived).  The paper gives beam energies in
# eV (user-interface parameter ``energy_ev``); the wavelength is hc/E.
HC_EV_M = 1.239841984332e-6


def wavelength_from_energy(energy_ev: float) -> float:
    """Photon wavelength in metres for an energy in eV (unit conversion)."""
    return HC_EV_M / float(energy_ev)


@dataclasses.dataclass
class Scan:
    """One synthetic ptychography workload.

    Arrays are slice-major: ``obj_a``/``obj_b`` have shape ``[S][Ly][Lx]``.
    For ``obj_repr == "delta_beta"`` they hold delta and beta (refractive
    index decrements); for ``"real_imag"`` the real and imaginary parts of
    the complex transmission.  ``positions`` are float (y, x) top-left chunk
    corners in object pixels, shape ``[P][2]``.
    """

    name: str
    n: int
    obj_a: np.ndarray
    obj_b: np.ndarray
    probe: np.ndarray            # complex128 [N][N]
    positions: np.ndarray        # float64 [P][2] (y, x)
    wavelength_m: float
    pixel_m: float
    slice_dz_m: float
    obj_repr: str                # "delta_beta" | "real_imag"
    loss: str                    # "gaussian" | "poisson"
    minibatch: int
    eps: float = 1e-6
    # Evaluation point (where a gradient is evaluated), if it differs from
    # the ground truth used to simulate data.
    eval_obj_a: Optional[np.ndarray] = None
    eval_obj_b: Optional[np.ndarray] = None
    eval_probe: Optional[np.ndarray] = None
    eval_positions: Optional[np.ndarray] = None
    photons: Optional[float] = None   # Poisson counting: expected photons / pattern
    # Unequal slice spacing: distance from slice j to j+1 (metres), [S-1];
    # None: every gap is slice_dz_m.  eval_gaps: where gradients are taken.
    gaps: Optional[np.ndarray] = None
    eval_gaps: Optional[np.ndarray] = None

    @property
    def n_slices(self) -> int:
        return int(self.obj_a.shape[0])

    @property
    def obj_shape(self):
        return tuple(int(v) for v in self.obj_a.shape)


# ---------------------------------------------------------------------------
# Building blocks
# ---------------------------------------------------------------------------

def smooth_random_field(rng, shape, sigma, lo, hi):
    """Uniform noise in [lo, hi) smoothed by a periodic Gaussian filter."""
    return gaussian_filter(rng.uniform(lo, hi, size=shape), sigma=sigma, mode="wrap")


def gaussian_probe(rng, n, sigma_px, phase_sigma_px, phase_std=1.0, total=1e4):
    """Gaussian-apodised probe with a random smooth phase.

    Amplitude exp(-r^2 / (2 sigma^2)) about the array centre; the phase is
    periodic-Gaussian-smoothed noise rescaled to ``phase_std`` radians;
    the probe is scaled so that sum |p|^2 = ``total`` (photons).
    """
    yy, xx = np.meshgrid(np.arange(n) - n / 2.0, np.arange(n) - n / 2.0, indexing="ij")
    amp = np.exp(-(yy ** 2 + xx ** 2) / (2.0 * sigma_px ** 2))
    ph = smooth_random_field(rng, (n, n), phase_sigma_px, -np.pi, np.pi)
    ph = (ph - ph.mean()) / ph.std() * phase_std
    p = amp * np.exp(1j * ph)
    p *= math.sqrt(total / np.sum(np.abs(p) ** 2))
    return p.astype(np.complex128)


def ellipsoid_volume(rng, shape, count, lat=(8.0, 48.0), ax=(4.0, 24.0),
                     delta_range=(2e-6, 1e-5), beta_ratio=(0.02, 0.1)):
    """Random axis-aligned ellipsoids; each voxel takes the max over covers.

    ``shape`` is (S, Ly, Lx).  Returns (delta, beta) FP64 arrays.
    """
    s, ly, lx = shape
    delta = np.zeros(shape)
    beta = np.zeros(shape)
    for _ in range(count):
        cz, cy, cx = rng.uniform(0, s), rng.uniform(0, ly), rng.uniform(0, lx)
        ry, rx = rng.uniform(*lat), rng.uniform(*lat)
        rz = rng.uniform(*ax)
        d = rng.uniform(*delta_range)
        b = d * rng.uniform(*beta_ratio)
        z0, z1 = max(0, int(cz - rz)), min(s, int(cz + rz) + 2)
        y0, y1 = max(0, int(cy - ry)), min(ly, int(cy + ry) + 2)
        x0, x1 = max(0, int(cx - rx)), min(lx, int(cx + rx) + 2)
        if z0 >= z1 or y0 >= y1 or x0 >= x1:
            continue
        zz, yy, xx = np.meshgrid(np.arange(z0, z1) + 0.5, np.arange(y0, y1) + 0.5,
                                 np.arange(x0, x1) + 0.5, indexing="ij")
        inside = ((zz - cz) / rz) ** 2 + ((yy - cy) / ry) ** 2 + ((xx - cx) / rx) ** 2 <= 1.0
        sub_d = delta[z0:z1, y0:y1, x0:x1]
        sub_b = beta[z0:z1, y0:y1, x0:x1]
        np.maximum(sub_d, np.where(inside, d, 0.0), out=sub_d)
        np.maximum(sub_b, np.where(inside, b, 0.0), out=sub_b)
    return delta, beta


def raster(side_y, side_x, origin, step, jitter=0.0, rng=None):
    """Raster of (y, x) corners, optionally jittered by U[-jitter, jitter]."""
    iy, ix = np.meshgrid(np.arange(side_y), np.arange(side_x), indexing="ij")
    pos = np.stack([origin + step * iy.ravel(), origin + step * ix.ravel()], axis=1).astype(np.float64)
    if jitter:
        pos += rng.uniform(-jitter, jitter, size=pos.shape)
    return pos


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def ptycho2d_n64(seed: int = 1) -> Scan:
    """Plain 2D ptychography, one thin slice, complex (real/imag) object.

    Object 128x128: amplitude U[0.9, 1], phase Gaussian-smoothed (sigma 3 px)
    U[-0.5, 0.5].  Probe 64x64, Gaussian apodisation sigma 12 px, smooth
    random phase.  8x8 raster, step 8 px (64 positions, integer).
    Evaluated at the vacuum object O = 1 with the true probe.
    """
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.9, 1.0, size=(128, 128))
    ph = smooth_random_field(rng, (128, 128), 3.0, -0.5, 0.5)
    obj = amp * np.exp(1j * ph)
    probe = gaussian_probe(rng, 64, 12.0, 4.0)
    pos = raster(8, 8, 4.0, 8.0)
    return Scan(name="ptycho2d_n64", n=64, obj_a=obj.real[None].copy(), obj_b=obj.imag[None].copy(),
                probe=probe, positions=pos, wavelength_m=wavelength_from_energy(8801.0),
                pixel_m=13.2e-9, slice_dz_m=13.2e-9, obj_repr="real_imag", loss="gaussian",
                minibatch=64,
                eval_obj_a=np.ones((1, 128, 128)), eval_obj_b=np.zeros((1, 128, 128)))


def multislice_n128_s64(seed: int = 2, n_slices: int = 64, lateral: int = 256) -> Scan:
    """Multislice ptychography at 10 keV, delta/beta volume 256x256x64, 10 nm.

    24 random ellipsoids; probe 128x128 (Gaussian sigma 24 px, smooth phase);
    400 positions on a 20x20 raster, origin 7 px, step 6 px, jitter
    U[-2, 2] px; Poisson data with 1e4 photons per pattern; minibatch 50.
    Evaluated at delta = beta = 0 with the true probe and positions.
    """
    rng = np.random.default_rng(seed)
    delta, beta = ellipsoid_volume(rng, (n_slices, lateral, lateral), 24)
    probe = gaussian_probe(rng, 128, 24.0, 8.0)
    pos = raster(20, 20, 7.0, 6.0, jitter=2.0, rng=rng)
    z = np.zeros_like(delta)
    return Scan(name="multislice_n128_s64", n=128, obj_a=delta, obj_b=beta, probe=probe,
                positions=pos, wavelength_m=wavelength_from_energy(10000.0), pixel_m=10e-9,
                slice_dz_m=10e-9, obj_repr="delta_beta", loss="poisson", minibatch=50,
                eval_obj_a=z, eval_obj_b=z, photons=1e4)


def multislice_n128_s128(seed: int = 3) -> Scan:
    """Differentiation workload: 512x512x128 delta/beta, 1024 positions.

    64 ellipsoids; probe as in config 2; 32x32 raster, origin 6, step 12;
    data simulated at nominal + true shifts U[-1, 1] px (Gaussian loss,
    noise-free).  Evaluated at 0.5 x truth, probe x (1 + 0.05 complex
    noise), shifts 0.  Minibatch 200, slice checkpoints every 16 slices.
    """
    rng = np.random.default_rng(seed)
    delta, beta = ellipsoid_volume(rng, (128, 512, 512), 64)
    probe = gaussian_probe(rng, 128, 24.0, 8.0)
    nominal = raster(32, 32, 6.0, 12.0)
    true_pos = nominal + rng.uniform(-1.0, 1.0, size=nominal.shape)
    noise = rng.standard_normal((128, 128)) + 1j * rng.standard_normal((128, 128))
    return Scan(name="multislice_n128_s128", n=128, obj_a=delta, obj_b=beta, probe=probe,
                positions=true_pos, wavelength_m=wavelength_from_energy(10000.0), pixel_m=10e-9,
                slice_dz_m=10e-9, obj_repr="delta_beta", loss="gaussian", minibatch=200,
                eval_obj_a=0.5 * delta, eval_obj_b=0.5 * beta,
                eval_probe=probe * (1.0 + 0.05 * noise), eval_positions=nominal)


def fd_subcase_n16_s4(seed: int = 3) -> Scan:
    """Tiny finite-difference sub-case: 32x32x4 delta/beta, probe 16x16.

    3x3 raster, origin 1, step 7, probe sigma 3 px; fractional positions kept
    away from the rounding boundary.
    """
    rng = np.random.default_rng(seed + 1000)
    delta, beta = ellipsoid_volume(rng, (4, 32, 32), 6, lat=(3.0, 10.0), ax=(1.0, 3.0),
                                   delta_range=(2e-4, 1e-3))
    probe = gaussian_probe(rng, 16, 3.0, 2.0, total=1e2)
    pos = raster(3, 3, 1.0, 7.0) + rng.uniform(-0.3, 0.3, size=(9, 2))
    return Scan(name="fd_subcase_n16_s4", n=16, obj_a=delta, obj_b=beta, probe=probe, positions=pos,
                wavelength_m=wavelength_from_energy(10000.0), pixel_m=10e-9, slice_dz_m=10e-9,
                obj_repr="delta_beta", loss="gaussian", minibatch=9,
                eval_obj_a=0.6 * delta, eval_obj_b=0.6 * beta,
                eval_probe=probe * (1.0 + 0.05 * (rng.standard_normal((16, 16))
                                                  + 1j * rng.standard_normal((16, 16)))),
                eval_positions=pos + rng.uniform(-0.1, 0.1, size=pos.shape))


def mixed_scan_jobs(seed: int = 4, n_jobs: int = 32):
    """Batching workload: independent scans of uneven probe size and depth.

    Per job: N ~ U{64, 96, 128, 192}, S ~ U{1..64}, P ~ U{50..500}; raster
    side ceil(sqrt(P)), step max(2, round(N/16)), jitter +-step/4; object
    side = N + (side-1) step + 2 ceil(step/4) + 4 rounded up to 16;
    8 + S/4 ellipsoids; probe sigma 0.1875 N; Poisson loss for even jobs,
    Gaussian for odd.  Returns a list of ``Scan``.
    """
    root = np.random.default_rng(seed)
    jobs = []
    for j, rng in enumerate(root.spawn(n_jobs)):
        n = int(rng.choice([64, 96, 128, 192]))
        s = int(rng.integers(1, 65))
        p = int(rng.integers(50, 501))
        side = int(math.ceil(math.sqrt(p)))
        step = max(2, int(round(n / 16)))
        jit = step / 4.0
        lat = n + (side - 1) * step + 2 * int(math.ceil(jit)) + 4
        lat = int(math.ceil(lat / 16.0) * 16)
        delta, beta = ellipsoid_volume(rng, (s, lat, lat), 8 + s // 4)
        probe = gaussian_probe(rng, n, 0.1875 * n, n / 16.0)
        pos = raster(side, side, 2.0 + math.ceil(jit), step, jitter=jit, rng=rng)[:p]
        jobs.append(Scan(name=f"mixed_job{j}_n{n}_s{s}_p{p}", n=n, obj_a=delta, obj_b=beta, probe=probe,
                         positions=pos, wavelength_m=wavelength_from_energy(10000.0), pixel_m=10e-9,
                         slice_dz_m=10e-9, obj_repr="delta_beta",
                         loss="poisson" if j % 2 == 0 else "gaussian", minibatch=p, photons=1e4,
                         eval_obj_a=np.zeros_like(delta), eval_obj_b=np.zeros_like(beta)))
    return jobs


def tilt_job(seed: int = 5, side: int = 256, n_angles: int = 90):
    """Tilt-series ptychotomography job: cubic delta/beta object, 10 nm.

    Angles 0, 2, ..., 178 degrees about the y axis; 10x10 positions per
    angle (origin 5, step 13), probe 128x128, Poisson data 1e4 photons.
    Returns (Scan at angle 0, angles in radians).
    """
    rng = np.random.default_rng(seed)
    delta, beta = ellipsoid_volume(rng, (side, side, side), 48)
    probe = gaussian_probe(rng, 128, 24.0, 8.0)
    pos = raster(10, 10, 5.0, 13.0)
    angles = np.deg2rad(2.0 * np.arange(n_angles))
    scan = Scan(name=f"tilt_n128_s{side}", n=128, obj_a=delta, obj_b=beta, probe=probe, positions=pos,
                wavelength_m=wavelength_from_energy(10000.0), pixel_m=10e-9, slice_dz_m=10e-9,
                obj_repr="delta_beta", loss="poisson", minibatch=100, photons=1e4,
                eval_obj_a=np.zeros_like(delta), eval_obj_b=np.zeros_like(beta))
    return scan, angles


def sparse_multislice(seed: int = 6, n_pos: int = 1414) -> Scan:
    """Sparse multislice ptychography: two thin layers 10 um apart.

    The shape of the paper's sparse-multislice experiment (Sec. 3, two
    layers of nanoflakes on either side of a window): 12 keV, 7.3 nm pixels,
    N = 128, object 512 x 512 x 2 (the 501 x 500 x 2 field padded to a
    multiple of 128), 1414 positions on a jittered 38 x 38 raster (step 9.9
    px), Poisson data at 1e5 photons per pattern, minibatch 202 (7 per
    epoch).  Each layer holds 40 random flakes (ellipses, 5-40 px, delta
    1e-5..5e-5, beta 0.05-0.15 delta) of thickness slice_dz_m = 100 nm.
    Evaluated at delta = beta = 0 and at gaps 5% longer than the truth.
    """
    rng = np.random.default_rng(seed)
    side = 512
    layers = [ellipsoid_volume(rng, (1, side, side), 40, lat=(5.0, 40.0), ax=(2.0, 2.0),
                               delta_range=(1e-5, 5e-5), beta_ratio=(0.05, 0.15)) for _ in range(2)]
    delta = np.concatenate([d for d, _ in layers])
    beta = np.concatenate([b for _, b in layers])
    probe = gaussian_probe(rng, 128, 16.0, 6.0, phase_std=2.0, total=1e5)
    pos = raster(38, 38, 8.0, 9.9, jitter=2.0, rng=rng)[:n_pos]
    z = np.zeros_like(delta)
    gaps = np.array([10e-6])
    return Scan(name="sparse_multislice_n128_s2", n=128, obj_a=delta, obj_b=beta, probe=probe, positions=pos,
                wavelength_m=wavelength_from_energy(12000.0), pixel_m=7.3e-9, slice_dz_m=100e-9,
                obj_repr="delta_beta", loss="poisson", minibatch=202, photons=1e5,
                eval_obj_a=z, eval_obj_b=z, gaps=gaps, eval_gaps=gaps * 1.05)


def mdh_tiles(seed: int = 7, side: int = 512, n: int = 128, step: int = 96):
    """Multi-distance holography as tiles: a 512 x 512 complex object, 1 um
    pixels, 17.5 keV, holograms at 40, 60, 80 and 100 cm (the paper's
    simulated MDH case, Sec. 3), cut into 25 overlapping 128 x 128 tiles
    (step 96) under plane-wave illumination, each tile at every distance:
    100 (tile, distance) positions per iteration.  Magnitude 0.6 - 1.0 and
    phase -0.5 - 0.5 rad are independent smooth random fields (they stand in
    for the paper's two test images); Poisson data at 100 photons per pixel.
    Evaluated at the mean of the truth and a vacuum object.
    Returns (scan, dists [4] metres, dist_idx [100] int32)."""
    rng = np.random.default_rng(seed)
    mag = smooth_random_field(rng, (1, side, side), 4.0, 0.0, 1.0)
    mag = 0.6 + 0.4 * (mag - mag.min()) / (mag.max() - mag.min())
    ph = smooth_random_field(rng, (1, side, side), 4.0, 0.0, 1.0)
    ph = -0.5 + (ph - ph.min()) / (ph.max() - ph.min())
    o = mag * np.exp(1j * ph)
    dists = np.array([0.4, 0.6, 0.8, 1.0])
    corners = raster(5, 5, 0.0, float(step))
    pos = np.repeat(corners, len(dists), axis=0)
    idx = np.tile(np.arange(len(dists), dtype=np.int32), len(corners))
    probe = np.full((n, n), 10.0 + 0j)
    ev = 0.5 * (o + 1.0)
    sc = Scan(name="mdh_tiles_n128", n=n, obj_a=o.real.copy(), obj_b=o.imag.copy(), probe=probe, positions=pos,
              wavelength_m=wavelength_from_energy(17500.0), pixel_m=1e-6, slice_dz_m=1e-6, obj_repr="real_imag",
              loss="poisson", minibatch=len(pos), photons=100.0 * n * n,
              eval_obj_a=ev.real.copy(), eval_obj_b=ev.imag.copy())
    return sc, dists, idx


def split_positions(pos: np.ndarray):
    """Integer corner floor(r + 0.5) and the residual subpixel shift r - c."""
    corner = np.floor(pos + 0.5)
    return corner.astype(np.int32), (pos - corner)


def small_case(seed: int, n: int, n_slices: int, lateral: int, n_pos: int,
               obj_repr: str = "delta_beta", loss: str = "gaussian", strength: float = 1.0,
               photons: float = 1e4) -> Scan:
    """Small random scan for parity tests: random ellipsoids, random positions."""
    rng = np.random.default_rng(seed)
    if obj_repr == "delta_beta":
        a, b = ellipsoid_volume(rng, (n_slices, lateral, lateral), max(4, n_slices // 2),
                                lat=(n / 16.0, n / 3.0), ax=(1.0, max(1.5, n_slices / 3.0)),
                                delta_range=(2e-6 * strength, 1e-5 * strength))
        # Evaluate away from the truth so residuals do not vanish.
        ea, eb = 0.5 * a + 1e-6 * strength * rng.random(a.shape), 0.5 * b
    else:
        amp = rng.uniform(0.9, 1.0, size=(n_slices, lateral, lateral))
        ph = smooth_random_field(rng, (n_slices, lateral, lateral), 2.0, -0.5, 0.5)
        o = amp * np.exp(1j * ph)
        a, b = o.real.copy(), o.imag.copy()
        e = 1.0 + 0.02 * (rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape))
        ea, eb = e.real.copy(), e.imag.copy()
    probe = gaussian_probe(rng, n, 0.1875 * n, max(1.0, n / 16.0), total=photons)
    pos = rng.uniform(1.0, lateral - n - 1.0, size=(n_pos, 2))
    eprobe = probe * (1.0 + 0.03 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))))
    epos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    return Scan(name=f"small_n{n}_s{n_slices}_l{lateral}_p{n_pos}_{obj_repr}_{loss}", n=n,
                obj_a=a, obj_b=b, probe=probe, positions=pos,
                wavelength_m=wavelength_from_energy(10000.0), pixel_m=10e-9, slice_dz_m=10e-9,
                obj_repr=obj_repr, loss=loss, minibatch=n_pos, photons=photons,
                eval_obj_a=ea, eval_obj_b=eb, eval_probe=eprobe, eval_positions=epos)


def probe_modes(probe: np.ndarray, n_modes: int, seed: int, weight: float = 0.4) -> np.ndarray:
    """[M][N][N] probe modes: the given probe first, then weaker copies of it
    with a smooth random phase each (partial coherence; random inputs only)."""
    rng = np.random.default_rng(seed)
    n = probe.shape[0]
    modes = [np.asarray(probe, dtype=np.complex128)]
    for _ in range(n_modes - 1):
        ph = smooth_random_field(rng, (1, n, n), 2.0, -4 * np.pi, 4 * np.pi)[0]
        modes.append(weight * modes[0] * np.exp(1j * ph))
    return np.stack(modes)
