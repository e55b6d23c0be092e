"""Pins of the tabulated correction oracle: the nodes are the image band,
CIC returns node values at nodes and both schemes reproduce linear data
exactly (TSC's bias on curvature is h^2 f''/8, checked on a quadratic), the
fold keeps pair forces antisymmetric, and the error against the exact band
falls with the grid spacing as h^2."""
import numpy as np
import pytest

import oracle
import synth
from oracle import table as ot


@pytest.fixture(scope="module")
def tab():
    return ot.Table(32, 36, 6.4)


def test_nodes_are_the_image_band(tab):
    rng = np.random.default_rng(0)
    for _ in range(10):
        i = rng.integers(-1, tab.n_d + 2)
        j = rng.integers(-1, tab.n_r + 2)
        fz, fr, _ = oracle.image_band([i * tab.h_d], [j * tab.h_r], 1.0, 2, tab.n_far)
        assert tab.Tz[j + 1, i + 1] == fz[0] and tab.Tr[j + 1, i + 1] == fr[0]


def test_cic_hits_nodes(tab):
    i, j = 7, 11
    z, r = ot.interpolate(tab, [i * tab.h_d], [j * tab.h_r], 1)
    assert z[0] == pytest.approx(tab.Tz[j + 1, i + 1], rel=1e-15)
    assert r[0] == pytest.approx(tab.Tr[j + 1, i + 1], rel=1e-15)


@pytest.mark.parametrize("order", [1, 2])
def test_linear_data_is_reproduced(order):
    t = ot.Table(8, 8, 4.0)
    di = np.arange(-1, t.n_d + 2) * t.h_d
    rj = np.arange(-1, t.n_r + 2) * t.h_r
    D, R = np.meshgrid(di, rj)
    t.Tz = 3.0 * D - 0.5 * R + 1.25
    t.Tr = -2.0 * D + 0.75 * R
    rng = np.random.default_rng(1)
    d = rng.uniform(0, 0.5, 200)
    r = rng.uniform(0, 4.0, 200)
    z, rr = ot.interpolate(t, d, r, order)
    np.testing.assert_allclose(z, 3.0 * d - 0.5 * r + 1.25, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(rr, -2.0 * d + 0.75 * r, rtol=1e-13, atol=1e-13)


def test_tsc_bias_on_a_quadratic():
    t = ot.Table(8, 8, 4.0)
    di = np.arange(-1, t.n_d + 2) * t.h_d
    rj = np.arange(-1, t.n_r + 2) * t.h_r
    D, R = np.meshgrid(di, rj)
    t.Tz = D * D
    t.Tr = R * R
    d = np.array([0.1234, 0.3])
    r = np.array([1.7, 2.25])
    z, rr = ot.interpolate(t, d, r, 2)
    np.testing.assert_allclose(z, d * d + t.h_d ** 2 / 4, rtol=1e-12)
    np.testing.assert_allclose(rr, r * r + t.h_r ** 2 / 4, rtol=1e-12)


@pytest.mark.parametrize("order", [1, 2])
def test_error_falls_as_h_squared(order):
    X = synth.remainder_inputs(3000, seed=2, rho_min=0.01, rho_max=6.0)
    fz, fr, _ = oracle.image_band(X[0], X[1], 1.0, 2, 1024)
    errs = []
    for n in (16, 32):
        t = ot.Table(n, int(n * 1.125), 6.4)
        z, r = ot.interpolate(t, X[0], X[1], order)
        errs.append(np.sqrt(np.mean((z - fz) ** 2 + (r - fr) ** 2)))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_table_pair_forces_are_antisymmetric():
    p = synth.cylinder_load(80, seed=3)
    t = ot.Table(16, 18, 6.4)
    for order in (1, 2):
        a = ot.forces_table(p.pos, p.mass, p.eps, p.L, t, order)
        mom = (p.mass[None, :] * a).sum(axis=1)
        scale = np.sum(p.mass * np.linalg.norm(a, axis=0))
        assert np.abs(mom).max() < 1e-13 * scale
