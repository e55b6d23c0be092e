"""Pins of the FP64 force oracle against facts fixed outside it: the textbook
spline density it comes from, Newton's law, the Bessel-series field of an
infinite periodic line of point masses, the line-mass limit, the truncation
rate of the image sum, conservation laws and symmetries of the pair sum, and
the qualitative statement about the cylindrical force law (Sect. 2.1, the
comparison with R3 next to eq. ForceCylindrical)."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
import synth


# ---------------------------------------------------------------- spline law
def _spline_density(r, h):
    """Monaghan & Lattanzio (1985) cubic spline density of unit mass with
    support radius h (smoothing length h/2), textbook form."""
    q = r / h
    c = 8.0 / (math.pi * h ** 3)
    if q < 0.5:
        return c * (1.0 - 6.0 * q * q + 6.0 * q ** 3)
    if q < 1.0:
        return c * 2.0 * (1.0 - q) ** 3
    return 0.0


@pytest.mark.parametrize("h", [0.03, 0.5, 2.0])
def test_spline_force_is_enclosed_mass_over_r2(h):
    # the softened force is G M(<r)/r^2 of the spline density: pins both
    # polynomial branches and the single-minus reading of the middle one
    for u in [0.05, 0.2, 0.37, 0.49, 0.5, 0.51, 0.7, 0.93, 0.999, 1.0, 1.3, 4.0]:
        r = u * h
        m_enc, _ = integrate.quad(lambda s: 4 * math.pi * s * s * _spline_density(s, h), 0.0, min(r, h),
                                  points=[0.5 * h] if r > 0.5 * h else None, epsabs=0, epsrel=1e-13)
        assert oracle.spline_force(r, h) == pytest.approx(m_enc / r ** 2, rel=1e-11)


def test_spline_total_mass_and_newton_outside():
    h = 0.7
    m, _ = integrate.quad(lambda s: 4 * math.pi * s * s * _spline_density(s, h), 0, h,
                          points=[0.5 * h], epsrel=1e-13)
    assert m == pytest.approx(1.0, rel=1e-12)
    for r in [h, 1.01 * h, 3 * h, 100.0]:
        assert oracle.spline_force(r, h) == pytest.approx(1.0 / r ** 2, rel=1e-15)
        assert oracle.spline_potential(r, h) == pytest.approx(-1.0 / r, rel=1e-15)


def test_spline_continuity_and_core_limit():
    h = 1.3
    for u in [0.5, 1.0]:
        lo, hi = (u - 1e-12) * h, (u + 1e-12) * h
        assert oracle.spline_force(lo, h) == pytest.approx(oracle.spline_force(hi, h), rel=1e-9)
        assert oracle.spline_potential(lo, h) == pytest.approx(oracle.spline_potential(hi, h), rel=1e-9)
    r = 1e-6 * h
    assert oracle.spline_force(r, h) == pytest.approx(32.0 * r / (3.0 * h ** 3), rel=1e-5)
    assert oracle.spline_potential(0.0, h) == pytest.approx(-2.8 / h, rel=1e-15)


@pytest.mark.parametrize("h", [0.05, 1.0])
def test_potential_derivative_is_force(h):
    # dP/dr = F by central differences, on both sides of the branch points
    for u in [0.1, 0.3, 0.45, 0.55, 0.8, 0.95, 1.5]:
        r, dr = u * h, 1e-6 * h
        dP = (oracle.spline_potential(r + dr, h) - oracle.spline_potential(r - dr, h)) / (2 * dr)
        assert dP == pytest.approx(oracle.spline_force(r, h), rel=1e-7)


def test_potential_is_minus_integral_of_force():
    h = 0.4
    for u in [0.0, 0.2, 0.6, 0.9]:
        r = u * h
        tail, _ = integrate.quad(lambda s: oracle.spline_force(s, h), r, h, points=[0.5 * h], epsrel=1e-13)
        assert oracle.spline_potential(r, h) == pytest.approx(-1.0 / h - tail, rel=1e-11)


# ---------------------------------------------------------------- Newton
def test_two_body_newton_and_third_law():
    pos = np.array([[0.1, -0.7], [0.2, 0.4], [0.25, 0.30]])
    m = np.array([2.0, 3.0])
    eps = np.array([0.01, 0.02])
    a, p = oracle.forces(pos, m, eps, L=1000.0, n_img=0)
    s = pos[:, 0] - pos[:, 1]
    r = np.linalg.norm(s)
    np.testing.assert_allclose(a[:, 0], -m[1] * s / r ** 3, rtol=1e-14)
    np.testing.assert_allclose(a[:, 1], m[0] * s / r ** 3, rtol=1e-14)
    np.testing.assert_allclose(p, [-m[1] / r, -m[0] / r], rtol=1e-14)


def test_coincident_pair_and_self_exclusion():
    pos = np.array([[0.3, 0.3], [0.1, 0.1], [0.2, 0.2]])
    m = np.array([1.0, 2.0])
    eps = np.array([0.05, 0.15])
    a, p = oracle.forces(pos, m, eps, L=1000.0, n_img=0)
    assert np.all(a == 0.0)
    np.testing.assert_allclose(p, [-2.8 * 2.0 / 0.2, -2.8 * 1.0 / 0.2], rtol=1e-14)
    # a single particle feels nothing, images of itself included
    a1, p1 = oracle.forces(pos[:, :1], m[:1], eps[:1], L=1.0, n_img=5)
    assert np.all(a1 == 0.0) and p1[0] == 0.0


# ---------------------------------------------------------------- image sums
def _bessel_line(d, rho, L, mmax=None):
    """Field of an infinite periodic line of unit point masses (period L) at
    axial offset d and radius rho: Fourier (K0/K1) series, G = 1."""
    if mmax is None:
        mmax = int(60 * L / (2 * math.pi * rho)) + 10
    m = np.arange(1, mmax + 1)
    k = 2 * math.pi * m / L
    fr = -2.0 / (L * rho) - (4.0 / L) * np.sum(k * special.k1(k * rho) * np.cos(k * d))
    fz = -(4.0 / L) * np.sum(k * special.k0(k * rho) * np.sin(k * d))
    return fz, fr


def _rod_tail(d, rho, S):
    """Images beyond |n| > K replaced by uniform rods from S = K + 1/2 outward
    (midpoint rule), closed form; unit line density, L = 1."""
    fz = 1.0 / math.hypot(S - d, rho) - 1.0 / math.hypot(S + d, rho)
    fr = -(1.0 / rho) * (2.0 - (S - d) / math.hypot(S - d, rho) - (S + d) / math.hypot(S + d, rho))
    return fz, fr


@pytest.mark.parametrize("d,rho", [(0.2, 0.3), (-0.45, 0.05), (0.01, 1.7), (0.33, 6.0)])
def test_image_band_matches_bessel_series(d, rho):
    K = 4000
    fz, fr, _ = oracle.image_band([d], [rho], 1.0, 0, K)
    tz, tr = _rod_tail(d, rho, K + 0.5)
    bz, br = _bessel_line(d, rho, 1.0)
    assert fz[0] + tz == pytest.approx(bz, rel=1e-9, abs=1e-12)
    assert fr[0] + tr == pytest.approx(br, rel=1e-9)


def test_pair_sum_matches_bessel_series():
    # the N-body oracle on a two-particle set reproduces the line field too
    d, rho = 0.27, 0.41
    pos = np.array([[rho, 0.0], [0.0, 0.0], [0.5 + d, 0.5]])
    m = np.array([1.0, 1.0])
    eps = np.array([1e-3, 1e-3])
    K = 3000
    a, _ = oracle.forces(pos, m, eps, L=1.0, n_img=K)
    tz, tr = _rod_tail(d, rho, K + 0.5)
    bz, br = _bessel_line(d, rho, 1.0)
    assert a[0, 0] + tr == pytest.approx(br, rel=1e-9)
    assert a[2, 0] + tz == pytest.approx(bz, rel=1e-9)
    assert abs(a[1, 0]) < 1e-15


def test_truncation_converges_as_inverse_square():
    d, rho = 0.1, 0.5
    bz, br = _bessel_line(d, rho, 1.0)
    errs = []
    for K in [16, 32, 64, 128]:
        _, fr, _ = oracle.image_band([d], [rho], 1.0, 0, K)
        errs.append(abs(fr[0] - br))
        # leading term of the missing tail: rho / (L Z^2), Z = (K + 1/2) L
        assert errs[-1] == pytest.approx(rho / (K + 0.5) ** 2, rel=2e-2)
    Ks = np.array([16, 32, 64, 128]) + 0.5
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    np.testing.assert_allclose(ratios, (Ks[1:] / Ks[:-1]) ** 2, rtol=1e-2)


@pytest.mark.parametrize("rho", [6.0, 12.0])
def test_line_mass_limit(rho):
    # at rho >> L the truncated image sum is the field of a finite rod of
    # half-height Z = (K + 1/2) L: -(2 G m / (L rho)) Z / sqrt(Z^2 + rho^2)
    K = 1024
    Z = K + 0.5
    fz, fr, _ = oracle.image_band([0.3], [rho], 1.0, 0, K)
    assert fr[0] == pytest.approx(-(2.0 / rho) * Z / math.hypot(Z, rho), rel=1e-9)
    # the axial field of the infinite line vanishes (K0 terms ~ e^-2 pi rho);
    # what remains is the end asymmetry of the truncated rod
    tz, _ = _rod_tail(0.3, rho, Z)
    assert abs(fz[0] + tz) < 1e-12
    # and the infinite line gives 2 G m / (L rho) exactly (K1 terms vanish)
    _, br = _bessel_line(0.3, rho, 1.0)
    assert br == pytest.approx(-2.0 / rho, rel=1e-12)


def test_cylindrical_force_radially_stronger_axially_weaker():
    # single source: S1xR2 radial force exceeds the R3 one, axial is weaker
    rng = np.random.default_rng(3)
    for _ in range(50):
        d = rng.uniform(-0.49, 0.49)
        rho = rng.uniform(0.02, 3.0)
        fz, fr, _ = oracle.image_band([d], [rho], 1.0, 0, 8)
        r3 = (rho * rho + d * d) ** 1.5
        assert abs(fr[0]) > rho / r3
        assert abs(fz[0]) < abs(d) / r3


def test_min_image_window_equals_half_integer_cutoff():
    # window 0 with n_img = K keeps exactly the images with |d - nL| < (K+1/2) L
    pos = np.array([[0.0, 0.3], [0.0, 0.1], [0.05, 0.81]])
    m = np.array([1.0, 1.0])
    eps = np.array([0.01, 0.01])
    a0, _ = oracle.forces(pos, m, eps, 1.0, 3, window=0)
    d = oracle.min_image(0.05 - 0.81, 1.0)
    rho = math.hypot(0.3, 0.1)
    fz, fr, _ = oracle.image_band([d], [rho], 1.0, 0, 3)
    assert a0[2, 0] == pytest.approx(fz[0], rel=1e-14)
    # literal N_cut window: 2 N_cut images on the unwrapped separation
    a1, _ = oracle.forces(pos, m, eps, 1.0, 3, window=1)
    rz = 0.05 - 0.81
    kept = [n for n in range(-3, 4) if abs(rz - n) < 3]
    assert len(kept) == 6
    expect = sum(-(rz - n) / (rho * rho + (rz - n) ** 2) ** 1.5 for n in kept)
    assert a1[2, 0] == pytest.approx(expect, rel=1e-13)


def test_wrap_and_min_image_definitions():
    assert oracle.wrap_position(1.25, 1.0) == 0.25
    assert oracle.wrap_position(-0.25, 1.0) == 0.75
    assert oracle.wrap_position(-1e-20, 1.0) == 0.0
    assert oracle.min_image(0.7, 1.0) == pytest.approx(-0.3)
    assert oracle.min_image(-0.7, 1.0) == pytest.approx(0.3)
    assert oracle.min_image(0.5, 1.0) == -0.5


# ---------------------------------------------------------------- invariants
@pytest.fixture(scope="module")
def small_load():
    return synth.cylinder_load(512, seed=11)


@pytest.fixture(scope="module")
def small_forces(small_load):
    p = small_load
    return oracle.forces(p.pos, p.mass, p.eps, p.L, 8)


def test_momentum_and_axial_angular_momentum_conserved(small_load, small_forces):
    p = small_load
    a, _ = small_forces
    scale = np.sum(p.mass * np.linalg.norm(a, axis=0))
    mom = (p.mass[None, :] * a).sum(axis=1)
    assert np.all(np.abs(mom) < 1e-13 * scale)
    x, y = p.pos[0], p.pos[1]
    lz = np.sum(p.mass * (x * a[1] - y * a[0]))
    assert abs(lz) < 1e-13 * np.sum(p.mass * np.hypot(x, y) * np.linalg.norm(a, axis=0))


def test_z_translation_invariance(small_load, small_forces):
    p = small_load
    a, pot = small_forces
    pos = p.pos.copy()
    pos[2] = pos[2] + 0.3719  # unwrapped on purpose: the oracle wraps
    a2, pot2 = oracle.forces(pos, p.mass, p.eps, p.L, 8)
    np.testing.assert_allclose(a2, a, rtol=1e-9, atol=1e-12 * np.abs(a).max())
    np.testing.assert_allclose(pot2, pot, rtol=1e-12)


def test_rotation_about_axis(small_load, small_forces):
    p = small_load
    a, pot = small_forces
    th = 0.813
    c, s = math.cos(th), math.sin(th)
    pos = p.pos.copy()
    pos[0], pos[1] = c * p.pos[0] - s * p.pos[1], s * p.pos[0] + c * p.pos[1]
    a2, pot2 = oracle.forces(pos, p.mass, p.eps, p.L, 8)
    rot = np.stack([c * a[0] - s * a[1], s * a[0] + c * a[1], a[2]])
    np.testing.assert_allclose(a2, rot, rtol=1e-9, atol=1e-12 * np.abs(a).max())
    np.testing.assert_allclose(pot2, pot, rtol=1e-12)


def test_z_reflection(small_load, small_forces):
    p = small_load
    a, pot = small_forces
    pos = p.pos.copy()
    pos[2] = (1.0 - pos[2]) % 1.0
    a2, pot2 = oracle.forces(pos, p.mass, p.eps, p.L, 8)
    np.testing.assert_allclose(a2[:2], a[:2], rtol=1e-9, atol=1e-12 * np.abs(a).max())
    np.testing.assert_allclose(a2[2], -a[2], rtol=1e-9, atol=1e-12 * np.abs(a).max())


def test_target_subset_equals_full(small_load, small_forces):
    p = small_load
    a, pot = small_forces
    t = synth.target_sample(p.N, 37, seed=2)
    a2, pot2 = oracle.forces(p.pos, p.mass, p.eps, p.L, 8, targets=t)
    np.testing.assert_array_equal(a2, a[:, t])
    np.testing.assert_array_equal(pot2, pot[t])


def test_homogeneous_load_feels_only_the_cylinder_pull():
    # the mass density of the load is flat, so the mean radial pair force in
    # an annulus is the pull of a uniform cylinder of half-height
    # (n_img + 1/2) L, which for R3-dominated inner radii is close to
    # -2 pi G rho0 rho; checked loosely here, precisely in the compensation
    # tests
    p = synth.cylinder_load(4096, seed=0)
    a, _ = oracle.forces(p.pos, p.mass, p.eps, p.L, 64)
    rho = np.hypot(p.pos[0], p.pos[1])
    ar = (a[0] * p.pos[0] + a[1] * p.pos[1]) / rho
    rmax = synth.r_max()
    rho0 = 1.0 / (math.pi * rmax ** 2 * p.L)
    sel = (rho > 0.3) & (rho < 1.5)
    ratio = np.mean(ar[sel] / rho[sel]) / (-2 * math.pi * rho0)
    assert 0.85 < ratio < 1.15
