"""Pins of the background oracle: the cylinder compensation against a
brute-force volume integral and its printed infinite-height limit, the
Friedmann solution against the closed form of flat LCDM and the CPL closed
form, and the leapfrog step against time reversal and conservation."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from oracle import background as bg


# ---------------------------------------------------------------- F_h
def _brute_field(rho, R, Z, rho0, n=600):
    """Radial field of the uniform cylinder at (rho, 0, 0) from the solid-angle
    form F = G rho0 int Omega l(Omega) dOmega (x component), l = chord length
    of the ray from the point along Omega inside the body: each cone of
    directions pulls toward its mass, and r^2 dr cancels the 1/r^2 (no use of
    the line-element derivation)."""
    mu, wmu = np.polynomial.legendre.leggauss(n)          # cos(theta) in [-1, 1]
    ph, wph = np.polynomial.legendre.leggauss(n)
    ph = math.pi * (ph + 1.0)                              # phi in [0, 2 pi)
    wph = math.pi * wph
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    W = np.outer(wmu, wph)
    s = np.sqrt(1.0 - MU * MU)
    dx, dy, dz = s * np.cos(PH), s * np.sin(PH), MU
    # ray x = (rho,0,0) + t (dx,dy,dz) against x^2 + y^2 = R^2
    a = dx * dx + dy * dy
    b = 2.0 * rho * dx
    c = rho * rho - R * R
    disc = b * b - 4 * a * c
    ok = (disc > 0) & (a > 0)
    sq = np.sqrt(np.where(ok, disc, 0.0))
    t1 = np.where(ok, (-b - sq) / (2 * np.where(a > 0, a, 1)), 0.0)
    t2 = np.where(ok, (-b + sq) / (2 * np.where(a > 0, a, 1)), 0.0)
    tcap = np.where(np.abs(dz) > 0, Z / np.maximum(np.abs(dz), 1e-300), np.inf)
    lo = np.maximum(t1, 0.0)
    hi = np.minimum(t2, tcap)
    ell = np.where(ok, np.maximum(hi - lo, 0.0), 0.0)
    return rho0 * np.sum(W * dx * ell)


@pytest.mark.parametrize("rho,Z", [(0.7, 8.5), (2.9, 8.5), (1.5, 2.0), (0.3, 1024.5)])
def test_cylinder_field_matches_volume_integral(rho, Z):
    R, rho0 = 3.157, 0.0319
    f = bg.cylinder_field(rho, R, Z, rho0)
    fb = _brute_field(rho, R, Z, rho0, n=1400)
    assert f == pytest.approx(fb, rel=2e-5)


def _outside_field(rho, R, Z, rho0, n=(80, 160, 400)):
    """Radial field at an exterior point from a Gauss-Legendre product rule over
    the cylinder volume (r', phi', z'); the integrand is smooth there."""
    r, wr = np.polynomial.legendre.leggauss(n[0])
    r, wr = 0.5 * R * (r + 1), 0.5 * R * wr
    ph, wph = np.polynomial.legendre.leggauss(n[1])
    ph, wph = math.pi * (ph + 1), math.pi * wph
    z, wz = np.polynomial.legendre.leggauss(n[2])
    z, wz = Z * z, Z * wz
    Rr, P, Zz = np.meshgrid(r, ph, z, indexing="ij")
    W = wr[:, None, None] * wph[None, :, None] * wz[None, None, :] * Rr
    sx = Rr * np.cos(P) - rho
    sy = Rr * np.sin(P)
    d3 = (sx * sx + sy * sy + Zz * Zz) ** 1.5
    return rho0 * np.sum(W * sx / d3)


@pytest.mark.parametrize("rho,Z", [(4.5, 8.5), (3.6, 2.0)])
def test_cylinder_field_outside_matches_volume_integral(rho, Z):
    R, rho0 = 3.157, 0.0319
    assert bg.cylinder_field(rho, R, Z, rho0) == pytest.approx(_outside_field(rho, R, Z, rho0), rel=1e-7)


@pytest.mark.parametrize("rho", [0.2, 1.0, 2.5, 3.0])
def test_cylinder_field_infinite_limit_inside(rho):
    R, rho0 = 3.157, 0.0319
    f = bg.cylinder_field(rho, R, 1e7, rho0)
    assert f == pytest.approx(-2 * math.pi * rho0 * rho, rel=1e-9)


def test_cylinder_field_infinite_limit_outside():
    R, rho0, rho = 1.0, 0.5, 2.5
    assert bg.cylinder_field(rho, R, 1e7, rho0) == pytest.approx(-2 * math.pi * rho0 * R * R / rho,
                                                                 rel=1e-9)


@pytest.mark.parametrize("rho", [0.2, 2.5, 3.157, 4.0])
def test_cylinder_field_of_infinite_cylinder_is_gauss_law(rho):
    # eq. F_horiz_infty inside; Gauss's law for an infinite line of mass outside
    R, rho0 = 3.157, 0.0319
    f = bg.cylinder_field(rho, R, math.inf, rho0)
    ref = -2 * math.pi * rho0 * (rho if rho <= R else R * R / rho)
    assert f == pytest.approx(ref, rel=1e-10)


def test_printed_formula_has_wrong_limit():
    # the finite-height expression as printed tends to +pi G rho0 rho: the
    # reading documented in the oracle (opposite sign, half the B term)
    R, rho0, rho = 3.0, 0.1, 1.2
    assert bg.cylinder_field_printed(rho, R, 1e7, rho0) == pytest.approx(math.pi * rho0 * rho,
                                                                         rel=1e-6)


def test_homogeneous_load_mean_radial_force_is_cylinder_pull():
    # the pair sum of the flat-density load with |n| <= 8 pulls every annulus
    # like a uniform cylinder of half-height 8.5 L (up to discreteness noise)
    p = synth.cylinder_load(4096, seed=0)
    a, _ = oracle.forces(p.pos, p.mass, p.eps, p.L, 8, potential=False)
    rho = np.hypot(p.pos[0], p.pos[1])
    ar = (a[0] * p.pos[0] + a[1] * p.pos[1]) / rho
    R = synth.r_max()
    rho0 = 1.0 / (math.pi * R * R * p.L)
    for lo, hi in [(0.4, 0.8), (0.8, 1.4), (1.4, 2.2)]:
        sel = (rho > lo) & (rho < hi)
        mid = np.median(rho[sel])
        expect = np.mean([bg.cylinder_field(r, R, 8.5, rho0) for r in rho[sel]])
        got = np.mean(ar[sel])
        assert got == pytest.approx(expect, rel=0.08), (lo, hi, mid)


# ---------------------------------------------------------------- Friedmann
def lcdm():
    return bg.Cosmology(H0=0.944, Om=0.3, OL=0.7)


def test_hubble_today_and_time_closed_form():
    c = lcdm()
    assert bg.hubble(1.0, c) == pytest.approx(c.H0, rel=1e-15)
    for a in [0.02, 0.1, 0.5, 1.0]:
        t = bg.cosmic_time(a, c)
        assert bg.lcdm_scale_factor(t, c) == pytest.approx(a, rel=1e-11)


def test_cpl_dark_energy_closed_form():
    c = bg.Cosmology(H0=1.0, Om=0.3, OL=0.7, w0=-0.9, wa=0.3)
    for a in [0.1, 0.6, 1.0, 1.3]:
        expect = 0.7 * a ** (-3 * (1 + c.w0 + c.wa)) * math.exp(3 * c.wa * (a - 1))
        assert bg.omega_de(a, c) == pytest.approx(expect, rel=1e-12)


def test_kdk_factors_are_the_time_integrals():
    c = lcdm()
    a0, a1 = 0.1, 0.12
    K1, D, K2 = bg.kdk_factors(a0, a1, c)
    t0, t1 = bg.cosmic_time(a0, c), bg.cosmic_time(a1, c)
    tm = 0.5 * (t0 + t1)
    f = lambda t, p: bg.lcdm_scale_factor(t, c) ** (-p)
    assert K1 == pytest.approx(integrate.quad(f, t0, tm, args=(1,), epsrel=1e-13)[0], rel=1e-10)
    assert K2 == pytest.approx(integrate.quad(f, tm, t1, args=(1,), epsrel=1e-13)[0], rel=1e-10)
    assert D == pytest.approx(integrate.quad(f, t0, t1, args=(2,), epsrel=1e-13)[0], rel=1e-10)
    # reversing the step reverses every factor
    K1r, Dr, K2r = bg.kdk_factors(a1, a0, c)
    assert K1r == pytest.approx(-K2, rel=1e-9) and K2r == pytest.approx(-K1, rel=1e-9)
    assert Dr == pytest.approx(-D, rel=1e-9)


# ---------------------------------------------------------------- KDK
def test_kdk_is_time_reversible_and_conserves_momentum():
    p = synth.displaced_load(256, seed=3)
    c = lcdm()
    R = synth.r_max()
    rho0 = 1.0 / (math.pi * R * R)
    mom0 = np.zeros_like(p.pos)
    x1, m1, _ = bg.kdk_step(p.pos, mom0, p.mass, p.eps, 1.0, 8, 0.05, 0.06, c, R, rho0, 8.5)
    # z-momentum: the pair sum is antisymmetric and F_h has no z part
    pz = np.sum(p.mass * m1[2])
    assert abs(pz) < 1e-13 * np.sum(p.mass * np.abs(m1[2]))
    x2, m2, _ = bg.kdk_step(x1, m1, p.mass, p.eps, 1.0, 8, 0.06, 0.05, c, R, rho0, 8.5)
    np.testing.assert_allclose(m2, mom0, atol=1e-12 * np.abs(m1).max())
    dz = (x2 - p.pos)
    dz[2] -= np.round(dz[2])
    assert np.abs(dz).max() < 1e-12


# ---------------------------------------------------------------- tabulated history
def test_history_interpolation_orders_are_exact_on_polynomials():
    t = np.linspace(0.0, 2.0, 9)
    for order in (1, 2, 3):
        a = 1.0 + 0.3 * t + (0.2 * t ** 2 if order >= 2 else 0) + (0.05 * t ** 3 if order >= 3 else 0)
        for x in [0.0, 0.13, 0.77, 1.5, 1.99, 2.0]:
            expect = 1.0 + 0.3 * x + (0.2 * x ** 2 if order >= 2 else 0) + (0.05 * x ** 3 if order >= 3 else 0)
            assert bg.history_interp(t, a, order, x) == pytest.approx(expect, rel=1e-13)


def test_history_factors_converge_to_closed_form():
    # sampled from the flat-LCDM closed form; errors fall as h^(order+1)
    c = lcdm()
    ref = np.array(bg.kdk_factors(0.1, 0.11, c))
    errs = {}
    for n in (200, 400):
        tt = np.linspace(bg.cosmic_time(0.05, c), bg.cosmic_time(0.5, c), n)
        aa = np.array([bg.lcdm_scale_factor(x, c) for x in tt])
        for order in (1, 2, 3):
            got = np.array(bg.history_factors(tt, aa, order, 0.1, 0.11))
            errs[(n, order)] = np.abs(got / ref - 1).max()
    for order in (1, 2, 3):
        assert errs[(200, order)] < 2e-4
        ratio = errs[(200, order)] / errs[(400, order)]
        # at least the pointwise order h^(order+1); integration can add one more
        assert ratio > 0.7 * 2 ** (order + 1), (order, ratio)
