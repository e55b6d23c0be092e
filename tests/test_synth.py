"""The seeded generators produce loads with the structure the recipe states:
a flat mass density out to r_max (the stereographic load of the paper's
cylindrical initial conditions), the softening law, Plummer clumps of the
stated size, displacement rms, and byte-identical repeats for one seed."""
import math

import numpy as np
import pytest

import synth


def test_load_is_deterministic_and_normalised():
    a = synth.cylinder_load(5000, seed=3)
    b = synth.cylinder_load(5000, seed=3)
    assert a.pos.tobytes() == b.pos.tobytes() and a.mass.tobytes() == b.mass.tobytes()
    assert a.mass.sum() == pytest.approx(1.0, rel=1e-14)
    assert np.all((a.pos[2] >= 0) & (a.pos[2] < 1.0))


def test_radius_limit_and_softening_law():
    p = synth.cylinder_load(20000, seed=0)
    r = np.hypot(p.pos[0], p.pos[1])
    assert r.max() < synth.r_max() and r.max() > 0.98 * synth.r_max()
    assert synth.r_max() == pytest.approx(0.5 * math.tan(0.45 * math.pi))
    np.testing.assert_allclose(p.eps, 0.01 * np.cbrt(p.mass / p.mass.min()), rtol=1e-14)
    assert p.eps.min() == pytest.approx(0.01)


def test_mass_density_is_flat():
    # surface number density falls as (1 + r^2/R0^2)^-2 while masses grow as
    # its inverse, so the mass per unit area is the same at every radius
    p = synth.cylinder_load(200000, seed=1)
    r = np.hypot(p.pos[0], p.pos[1])
    edges = np.linspace(0.0, 3.0, 13)
    dens = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (r >= lo) & (r < hi)
        dens.append(p.mass[sel].sum() / (math.pi * (hi * hi - lo * lo)))
    dens = np.array(dens)
    mean = 1.0 / (math.pi * synth.r_max() ** 2)
    assert np.all(np.abs(dens / mean - 1.0) < 0.06)


def test_clustered_load_has_the_stated_clumps():
    N = 262144
    p = synth.clustered_load(N, seed=0)
    assert p.N == N
    per = round(0.005 * N)
    assert per == 1311
    clumps = p.pos[:, N - 64 * per:].reshape(3, 64, per)
    c = clumps.mean(axis=2, keepdims=True)
    d = clumps - c
    d[2] -= np.round(d[2])
    rr = np.sqrt((d ** 2).sum(axis=0))
    # Plummer with b = 0.005: the half-mass radius is b / sqrt(2^(2/3) - 1)
    med = np.median(rr)
    assert med == pytest.approx(0.005 / math.sqrt(2 ** (2 / 3) - 1), rel=0.1)
    assert p.mass.sum() == pytest.approx(1.0, rel=1e-14)


def test_displacements_have_the_stated_rms():
    N = 1 << 16
    base = synth.cylinder_load(N, seed=0)
    p = synth.displaced_load(N, seed=0)
    d = p.pos - base.pos
    d[2] -= np.round(d[2])
    spacing = (math.pi * synth.r_max() ** 2 / N) ** (1 / 3)
    rms3 = math.sqrt(np.mean((d ** 2).sum(axis=0)))
    assert rms3 == pytest.approx(0.5 * spacing, rel=0.02)


def test_remainder_inputs_cover_the_network_domain():
    X = synth.remainder_inputs(20000, seed=0)
    assert X.shape == (2, 20000)
    assert X[0].min() >= 0 and X[0].max() <= 0.5
    assert X[1].min() >= 0.05 and X[1].max() <= 20.0
    assert np.mean(X[1] > 5.0) > 0.05 and np.mean(X[1] < 0.2) > 0.05


def test_targets_are_distinct_and_sorted():
    t = synth.target_sample(1000, 300, seed=4)
    assert len(np.unique(t)) == 300 and np.all(np.diff(t) > 0) and t.max() < 1000


def test_core_load_is_flat_with_constant_core_masses():
    # constant-resolution core (Sect. 3.1): equal masses inside rho_c, the
    # outer mass law outside, and the mass density flat across the boundary
    omega_c = 1.2
    N = 200000
    p = synth.cylinder_load(N, seed=2, omega_c=omega_c)
    r = np.hypot(p.pos[0], p.pos[1])
    rho_c = 0.5 * math.tan(0.5 * omega_c)
    core = r < rho_c
    np.testing.assert_array_equal(p.mass[core], p.mass[core][0])
    assert p.mass[~core].min() >= p.mass[core][0] * (1 - 1e-12)
    assert abs(p.mass.sum() - 1.0) < 1e-12 and r.max() <= synth.r_max()
    edges = np.concatenate([np.linspace(0.0, rho_c, 5), np.linspace(rho_c, 3.0, 9)[1:]])
    mean = 1.0 / (math.pi * synth.r_max() ** 2)
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (r >= lo) & (r < hi)
        dens = p.mass[sel].sum() / (math.pi * (hi * hi - lo * lo))
        assert abs(dens / mean - 1.0) < 0.06, (lo, hi, dens / mean)
    # omega_c = 0 is the plain load, draw for draw
    q = synth.cylinder_load(1000, seed=3, omega_c=0.0)
    q0 = synth.cylinder_load(1000, seed=3)
    np.testing.assert_array_equal(q.pos, q0.pos)
