"""Pins of the Ewald oracle and of the complete image sum: the modified
Bessel series of a periodic line (library K0/K1) against the direct sum with
its rod tail, the Ewald split with the incomplete-Bessel kernel against the
series for several splitting parameters, the large-alpha limit of the kernel,
the symmetry zeros of the band, the accuracy of the rod tail, and the alpha
dependence of the printed kernel (Sect. 2.2, eqs. EwaldRealSum, EwaldRecSum,
Bkernel)."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import ewald as ew
from oracle import table as tb

POINTS = [(0.2, 0.3), (0.45, 0.05), (0.1, 1.5), (0.3, 5.0), (0.05, 0.8), (0.0, 2.0), (0.5, 6.3)]


def near(d, r):
    """Newtonian force of the images n = -1, 0, 1 (L = 1)."""
    fz = fr = 0.0
    for n in (-1, 0, 1):
        u = d - n
        q = math.hypot(u, r)
        fz -= u / q ** 3
        fr -= r / q ** 3
    return fz, fr


def series_band(d, r):
    fz, fr = ew.line_series(d, r)
    nz, nr = near(d, r)
    return fz - nz, fr - nr


@pytest.mark.parametrize("d,r", POINTS)
def test_bessel_series_matches_direct_sum_with_tail(d, r):
    sz, sr = series_band(d, r)
    bz, br = ew.band_direct(np.array([d]), np.array([r]), 8192)
    scale = math.hypot(*ew.line_series(d, r))
    assert abs(bz[0] - sz) <= 1e-13 * scale and abs(br[0] - sr) <= 1e-13 * scale


@pytest.mark.parametrize("alpha", [1.5, 2.0, 3.0, 4.0])
@pytest.mark.parametrize("d,r", POINTS)
def test_ewald_with_incomplete_bessel_kernel_is_exact_for_any_alpha(alpha, d, r):
    fz, fr = ew.ewald(d, r, alpha, 6, 16)
    sz, sr = ew.line_series(d, r)
    scale = math.hypot(sz, sr)
    assert abs(fz - sz) <= 2e-13 * scale and abs(fr - sr) <= 2e-13 * scale
    bz, br = ew.band_ewald(d, r, alpha, 6, 16)
    tz, tr = series_band(d, r)
    assert abs(bz - tz) <= 2e-13 * scale and abs(br - tr) <= 2e-13 * scale


@pytest.mark.parametrize("k,rho", [(2 * math.pi, 0.3), (4 * math.pi, 1.0), (6 * math.pi, 0.05)])
def test_kernel_tends_to_K0_for_large_alpha(k, rho):
    # the omitted part of the integral, t < 1/(4 alpha^2), is below exp(-(alpha rho)^2)
    B, dB = ew.bessel_incomplete(k, rho, 7.0 / rho)
    assert B == pytest.approx(special.k0(k * rho), rel=1e-11)
    assert dB == pytest.approx(-k * special.k1(k * rho), rel=1e-11)


def test_band_symmetry_zeros():
    # T_rho vanishes on the axis, T_z on the plane d = 0; the complete sum
    # (not the band, whose three nearest images are not symmetric there) has
    # no axial component at d = L/2
    for r in (0.0, 0.7, 3.0):
        assert ew.band_ewald(0.0, r, 2.0, 5, 12)[0] == pytest.approx(0.0, abs=1e-15)
    for r in (0.7, 3.0):
        assert ew.ewald(0.5, r, 2.0, 5, 12)[0] == pytest.approx(0.0, abs=1e-14)
    for d in (0.0, 0.13, 0.5):
        assert ew.band_ewald(d, 0.0, 2.0, 5, 12)[1] == 0.0
    # band of the complete sum at the origin: both components vanish
    assert np.abs(ew.band_ewald(0.0, 0.0, 2.0, 5, 12)).max() < 1e-15


def test_rod_tail_accuracy():
    # the tail after 512 images matches the direct sum to 65536 plus its tail
    D = np.array([0.0, 0.13, 0.37, 0.5, 0.25])
    R = np.array([0.0, 0.4, 2.0, 6.0, 19.0])
    a = ew.band_direct(D, R, 512)
    b = ew.band_direct(D, R, 65536)
    np.testing.assert_allclose(a[0], b[0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(a[1], b[1], rtol=0, atol=1e-14)
    # and the tail itself is not negligible at that level
    tz, tr = ew.rod_tail(D, R, 512)
    assert np.abs(tr).max() > 1e-6


def test_printed_kernel_depends_on_alpha():
    # the kernel as printed gives the complete sum only where its Fourier
    # part is negligible (small alpha); at alpha = 2 it is off by percents
    d, r = 0.2, 0.3
    sz, sr = ew.line_series(d, r)
    scale = math.hypot(sz, sr)
    small = ew.ewald(d, r, 0.7, 5, 12, "printed")
    large = ew.ewald(d, r, 2.0, 5, 12, "printed")
    assert math.hypot(small[0] - sz, small[1] - sr) < 1e-7 * scale
    assert math.hypot(large[0] - sz, large[1] - sr) > 1e-2 * scale


def test_ewald_table_matches_long_band_table():
    T = tb.Table.ewald(6, 5, 4.0, 2.0, 5, 12)
    B = tb.Table(6, 5, 4.0, n_far=65536)
    # the band to 65536 images misses about r / 65536^2 of the radial tail
    assert np.abs(T.Tz - B.Tz).max() < 1e-9
    assert np.abs(T.Tr - B.Tr).max() < 2e-9
    D, R = T.grid()
    ref = np.array([series_band(d, abs(r)) if r != 0 else (0.0, 0.0) for d, r in zip(D.ravel(), R.ravel())])
    ok = R.ravel() != 0
    np.testing.assert_allclose(T.Tz.ravel()[ok], ref[ok, 0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.abs(T.Tr.ravel()[ok]), np.abs(ref[ok, 1]), rtol=0, atol=1e-12)


def test_complete_forces_of_a_pair_follow_the_series():
    # two particles far enough apart that no softening applies
    L = 2.0
    pos = np.array([[0.3, -0.5], [0.1, 0.4], [0.2, 1.7]])
    m = np.array([0.25, 0.75])
    h = np.array([0.01, 0.01])
    acc = ew.forces_complete(pos, m, h, L)
    dx, dy, dz = pos[:, 0] - pos[:, 1]
    dz -= L * math.floor(dz / L + 0.5)
    rho = math.hypot(dx, dy)
    fz, fr = ew.line_series(dz / L, rho / L)
    ref = m[1] / L ** 2 * np.array([fr * dx / rho, fr * dy / rho, fz])
    np.testing.assert_allclose(acc[:, 0], ref, rtol=1e-12)
    # Newton's third law, image by image
    np.testing.assert_allclose(m[0] * acc[:, 0], -m[1] * acc[:, 1], rtol=1e-12)


def test_complete_table_forces_follow_the_complete_sum():
    import synth
    p = synth.cylinder_load(48, seed=21)
    T = tb.Table.ewald(24, 16, 4.0, 2.0, 5, 12)
    ref = ew.forces_complete(p.pos, p.mass, p.eps, p.L)
    for order, tol in ((1, 3e-3), (2, 3e-3)):
        a = tb.forces_table(p.pos, p.mass, p.eps, p.L, T, order)
        e = np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert e.max() < tol, (order, e.max())
    # pairs beyond r_max (4 L) exist in this load and take the complete band
    r = np.hypot(p.pos[0][:, None] - p.pos[0][None], p.pos[1][:, None] - p.pos[1][None])
    assert (r > 4.0).any()
