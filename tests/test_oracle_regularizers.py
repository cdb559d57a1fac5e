"""Pins of the object-prior oracle (Eq. tikhonov, Table tab:regularizers)
against closed forms, invariances and central finite differences."""
import numpy as np
import pytest

from oracle import regularizers as orr

RNG = np.random.default_rng(99)
REPRS = ["delta_beta", "real_imag"]


def _obj(repr_, shape=(3, 5, 6), rng=RNG):
    if repr_ == "delta_beta":
        return rng.uniform(-1e-5, 1e-5, shape), rng.uniform(-1e-6, 1e-6, shape)
    mod = rng.uniform(0.6, 1.0, shape)
    ph = rng.uniform(-1.2, 1.2, shape)
    return mod * np.cos(ph), mod * np.sin(ph)


def test_l1_of_a_constant_object_is_its_magnitude():
    a = np.full((2, 3, 4), -3e-6)
    b = np.full((2, 3, 4), 5e-7)
    assert orr.l1_value(a, b, "delta_beta", 2.0, 7.0) == pytest.approx(2.0 * 3e-6 + 7.0 * 5e-7, rel=1e-14)


def test_l1_of_a_pure_phase_object_is_the_mean_phase_magnitude():
    """|O| = 1 everywhere: the modulus term vanishes, the phase term is the mean |arg O|."""
    ph = RNG.uniform(-3, 3, (2, 4, 5))
    v = orr.l1_value(np.cos(ph), np.sin(ph), "real_imag", 5.0, 0.5)
    assert v == pytest.approx(0.5 * np.mean(np.abs(ph)), rel=1e-12)


def test_tv_of_a_ramp_is_slope_times_pair_count():
    s, ly, lx = 4, 5, 7
    z, y, x = np.meshgrid(np.arange(s), np.arange(ly), np.arange(lx), indexing="ij")
    a = 2e-6 * x - 3e-6 * y + 1e-6 * z
    b = np.zeros_like(a)
    n_o = a.size
    pairs = 2e-6 * (lx - 1) * ly * s + 3e-6 * lx * (ly - 1) * s + 1e-6 * lx * ly * (s - 1)
    assert orr.tv_value(a, b, "delta_beta", 3.0) == pytest.approx(3.0 * pairs / n_o, rel=1e-12)


def test_tv_is_shift_invariant_and_l1_positively_homogeneous():
    a, b = _obj("delta_beta")
    assert orr.tv_value(a + 1.0, b - 2.0, "delta_beta", 1.0) == pytest.approx(
        orr.tv_value(a, b, "delta_beta", 1.0), rel=1e-9)
    assert orr.l1_value(3 * a, 3 * b, "delta_beta", 1.0, 2.0) == pytest.approx(
        3 * orr.l1_value(a, b, "delta_beta", 1.0, 2.0), rel=1e-13)


def test_reweighting_with_its_own_snapshot_counts_the_support():
    """W = max|C|/(|C| + eps) from the object itself: W|C| -> max|C| on
    every nonzero voxel as eps -> 0, so the weighted l1 counts them."""
    a = np.zeros((2, 4, 4))
    a[0, 1, 2], a[1, 3, 3], a[1, 0, 0] = 4e-6, -1e-6, 2e-6
    b = np.zeros_like(a)
    w1, w2 = orr.reweight(a, b, "delta_beta", 1e-18)
    v = orr.l1_value(a, b, "delta_beta", 1.0, 1.0, w1, w2)
    assert v == pytest.approx(4e-6 * 3 / a.size, rel=1e-9)


def test_support_projection_is_idempotent_and_keeps_the_inside():
    for repr_ in REPRS:
        a, b = _obj(repr_)
        mask = RNG.random(a.shape) > 0.4
        pa, pb = orr.support_project(a, b, repr_, mask)
        assert np.array_equal(pa[mask], a[mask]) and np.array_equal(pb[mask], b[mask])
        vac = (0.0, 0.0) if repr_ == "delta_beta" else (1.0, 0.0)
        assert np.all(pa[~mask] == vac[0]) and np.all(pb[~mask] == vac[1])
        qa, qb = orr.support_project(pa, pb, repr_, mask)
        assert np.array_equal(qa, pa) and np.array_equal(qb, pb)


@pytest.mark.parametrize("repr_", REPRS)
@pytest.mark.parametrize("weighted", [False, True])
def test_gradients_match_central_finite_differences(repr_, weighted):
    """Every voxel's derivative, l1 (or reweighted l1) and TV together, by
    central differences; the random object keeps every |.| argument away
    from its kink by far more than the step."""
    a, b = _obj(repr_)
    coef = dict(a1=1.3, a2=0.7, gamma=0.9)
    if weighted:
        sa, sb = _obj(repr_, rng=np.random.default_rng(5))
        coef["w1"], coef["w2"] = orr.reweight(sa, sb, repr_, 1e-3 if repr_ == "real_imag" else 1e-7)
    ga, gb = orr.grad(a, b, repr_, **coef)
    h = 1e-11 if repr_ == "delta_beta" else 1e-7
    fa = np.empty_like(a)
    fb = np.empty_like(b)
    for arr, out in ((a, fa), (b, fb)):
        for idx in np.ndindex(arr.shape):
            old = arr[idx]
            arr[idx] = old + h
            vp = orr.value(a, b, repr_, **coef)
            arr[idx] = old - h
            vm = orr.value(a, b, repr_, **coef)
            arr[idx] = old
            out[idx] = (vp - vm) / (2 * h)
    scale = max(np.max(np.abs(ga)), np.max(np.abs(gb)))
    assert np.max(np.abs(fa - ga)) <= 1e-6 * scale
    assert np.max(np.abs(fb - gb)) <= 1e-6 * scale


def test_mean_modulus_term_is_differentiated_through_the_mean():
    """The modulus l1 term is 1-homogeneous under O -> c O (|cO| - mean|cO| =
    c (|O| - mean|O|)), so its derivative along O itself equals R (Euler).
    Dropping the mean's own derivative, a plausible slip, adds
    mean|O| * sum sign(.) / N_o and fails this."""
    a, b = _obj("real_imag")
    ga, gb = orr.grad(a, b, "real_imag", a1=1.0)
    directional = np.sum(ga * a + gb * b)
    assert directional == pytest.approx(orr.value(a, b, "real_imag", a1=1.0), rel=1e-12)
