"""Pins of the octree oracle: with theta = 0 it is the direct tabulated force
(any shift and rotation of the domain); the cells partition the particles,
carry the mass and centre of mass of their content, respect the leaf size
and the depth-first skip structure; Morton keys interleave the cell
coordinates; the error grows with the opening angle and is bounded for small
angles; a group walk is at least as accurate as the per-particle walk; the
radial calibration removes the mean radial bias it measures (Sect. 2.4,
"Octree")."""
import math

import numpy as np
import pytest

import synth
from oracle import octree as oc
from oracle import table as ot

R = synth.r_max()


@pytest.fixture(scope="module")
def load():
    return synth.cylinder_load(700, seed=17)


@pytest.fixture(scope="module")
def tab():
    return ot.Table(24, 16, 6.5)


@pytest.fixture(scope="module")
def direct(load, tab):
    return ot.forces_table(load.pos, load.mass, load.eps, load.L, tab, 1)


def rel(a, ref):
    return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.mark.parametrize("shift,angle", [(0.0, 0.0), (0.37, 2.1), (0.99, -0.4)])
def test_zero_opening_angle_is_the_direct_force(load, tab, direct, shift, angle):
    a = oc.tree_forces(load.pos, load.mass, load.eps, load.L, R, tab, 1, 0.0, shift, angle,
                       leaf_size=8, group=32)
    assert rel(a, direct).max() < 1e-12


def test_morton_key_interleaves_cell_coordinates():
    lo, side = oc.root_cube(1.0, R)
    rng = np.random.default_rng(3)
    q = rng.integers(0, 1 << 21, size=(3, 50))
    pos = lo[:, None] + (q + 0.5) * (side / (1 << 21))
    key = oc.morton_keys(pos, lo, side)
    for k in range(50):
        back = [0, 0, 0]
        for b in range(21):
            back[0] |= ((int(key[k]) >> (3 * b + 2)) & 1) << b
            back[1] |= ((int(key[k]) >> (3 * b + 1)) & 1) << b
            back[2] |= ((int(key[k]) >> (3 * b)) & 1) << b
        assert back == [int(q[0, k]), int(q[1, k]), int(q[2, k])]


def test_cells_form_a_valid_tree(load):
    T = oc.Tree(load.pos, load.mass, load.eps, load.L, R, 0.2, 0.7, leaf_size=6)
    n = len(T.cells)
    # leaves partition the particles in key order
    leaves = [(T.start[k], T.end[k]) for k in range(n) if T.leaf[k]]
    assert leaves[0][0] == 0 and leaves[-1][1] == load.N
    assert all(a[1] == b[0] for a, b in zip(leaves[:-1], leaves[1:]))
    for k in range(n):
        cnt = T.end[k] - T.start[k]
        assert cnt >= 1
        if T.leaf[k]:
            assert cnt <= 6 or T.level[k] == oc.KEY_LEVELS
            assert T.skip[k] == k + 1
        else:
            # children follow directly, cover the parent's range, one level down
            kids = []
            c = k + 1
            while c < T.skip[k]:
                kids.append(c)
                c = T.skip[c]
            assert c == T.skip[k]
            assert all(T.level[c] == T.level[k] + 1 for c in kids)
            assert T.start[kids[0]] == T.start[k] and T.end[kids[-1]] == T.end[k]
            assert T.mass[k] == pytest.approx(sum(T.mass[c] for c in kids), rel=1e-13)
        s = slice(T.start[k], T.end[k])
        assert T.mass[k] == pytest.approx(T.sm[s].sum(), rel=1e-13)
        np.testing.assert_allclose(T.com[:, k], (T.sp[:, s] * T.sm[s]).sum(axis=1) / T.sm[s].sum(),
                                   rtol=1e-12, atol=1e-14)
        # the centre of mass lies in the cell's cube
        corner = T.lo + oc.Tree._cell_corner(T.skey[T.start[k]], int(T.level[k])) * T.size(k)
        assert np.all(T.com[:, k] >= corner - 1e-12) and np.all(T.com[:, k] <= corner + T.size(k) + 1e-12)
        assert T.hmax[k] == T.sh[s].max()
    # particles sit in key order
    assert np.all(np.diff(T.skey) >= 0)


def test_error_grows_with_opening_angle(load, tab, direct):
    means = []
    for theta in (0.25, 0.5, 0.8):
        a = oc.tree_forces(load.pos, load.mass, load.eps, load.L, R, tab, 1, theta, 0.1, 0.3,
                           leaf_size=8, group=16)
        means.append(rel(a, direct).mean())
    assert means[0] < means[1] < means[2]
    assert means[0] < 2e-3


def test_group_walk_is_at_least_as_accurate(load, tab, direct):
    g = oc.tree_forces(load.pos, load.mass, load.eps, load.L, R, tab, 1, 0.7, 0.5, 1.0,
                       leaf_size=8, group=32)
    s = oc.tree_forces(load.pos, load.mass, load.eps, load.L, R, tab, 1, 0.7, 0.5, 1.0,
                       leaf_size=8, group=1)
    assert rel(g, direct).mean() <= rel(s, direct).mean()


def test_radial_calibration_removes_the_mean_radial_bias(load, tab, direct):
    theta, nb = 0.9, 8
    rng = np.random.default_rng(5)
    shifts = rng.random(3) * load.L
    angles = rng.random(3) * 2 * math.pi
    corr = oc.calibrate(load.pos, load.mass, load.eps, load.L, R, tab, 1, theta, shifts, angles, nb,
                        leaf_size=8, group=16)
    assert np.abs(corr).max() > 0
    # on a realisation used for the calibration the corrected bias is smaller
    a = oc.tree_forces(load.pos, load.mass, load.eps, load.L, R, tab, 1, theta, shifts[0], angles[0],
                       leaf_size=8, group=16)
    ac = oc.apply_correction(load.pos, a, corr, R)
    s0, c0 = oc.radial_bins(load.pos, a - direct, R, nb)
    s1, c1 = oc.radial_bins(load.pos, ac - direct, R, nb)
    ok = c0 > 0
    assert np.abs(s1[ok] / c1[ok]).mean() < np.abs(s0[ok] / c0[ok]).mean()
    # theta = 0 has nothing to correct
    z = oc.calibrate(load.pos, load.mass, load.eps, load.L, R, tab, 1, 0.0, shifts[:1], angles[:1], nb,
                     leaf_size=8, group=16)
    assert np.abs(z).max() < 1e-12


@pytest.mark.parametrize("G,leaf", [(64, 16), (8, 16), (1, 4)])
def test_groups_partition_the_particles_into_compact_runs(load, G, leaf):
    T = oc.Tree(load.pos, load.mass, load.eps, load.L, R, 0.1, 0.2, leaf_size=leaf)
    gs = sorted(oc.groups(T, G))
    assert gs[0][0] == 0 and sum(n for _, n in gs) == load.N
    assert all(a[0] + a[1] == b[0] for a, b in zip(gs[:-1], gs[1:]))
    assert all(1 <= n <= G for _, n in gs)
    # each group is a run of whole children of one cell holding more than G
    # particles (or a run of a leaf holding more than G)
    cnt = T.end - T.start
    for s, n in gs:
        inside = [k for k in range(len(T.cells))
                  if T.start[k] <= s and s + n <= T.end[k] and cnt[k] > G]
        owner = max(inside, key=lambda k: T.level[k])
        if T.leaf[owner]:
            assert (s - T.start[owner]) % G == 0
            continue
        kids, c = [], owner + 1
        while c < T.skip[owner]:
            kids.append(c)
            c = T.skip[c]
        starts = {int(T.start[c]) for c in kids if cnt[c] <= G}
        ends = {int(T.end[c]) for c in kids if cnt[c] <= G}
        assert s in starts and s + n in ends


def test_target_subset_walks_the_same_groups(load, tab):
    tg = np.array([0, 5, 77, 311, 699])
    full = oc.tree_forces(load.pos, load.mass, load.eps, load.L, R, tab, 1, 0.5, 0.25, 1.7,
                          leaf_size=8, group=16)
    sub = oc.tree_forces(load.pos, load.mass, load.eps, load.L, R, tab, 1, 0.5, 0.25, 1.7,
                         leaf_size=8, group=16, targets=tg)
    np.testing.assert_array_equal(sub, full[:, tg])


def test_quadrupole_moments_converge_at_third_order():
    # a compact cluster seen from afar: the monopole error falls as the
    # cluster size squared, monopole + quadrupole as its cube
    L = 1000.0
    rng = np.random.default_rng(71)
    Y = rng.normal(size=(3, 20))
    m = rng.random(20)
    x = np.array([0.6, -0.3, 0.5])
    errs = []
    for scale in (0.04, 0.02, 0.01):
        pos = Y * scale + np.array([[0.0], [0.0], [L / 2]])
        T = oc.Tree(pos, m, np.full(20, 1e-6), L, 2.0, quadrupole=True)
        com, q = T.com[:, 0], T.quad[:, 0]
        s = x + np.array([0.0, 0.0, L / 2]) - pos.T
        exact = -(m[:, None] * s / (np.linalg.norm(s, axis=1) ** 3)[:, None]).sum(axis=0)
        sc_ = x + np.array([0.0, 0.0, L / 2]) - com
        r = np.linalg.norm(sc_)
        mono = -m.sum() * sc_ / r ** 3
        Q = np.array([[q[0], q[3], q[4]], [q[3], q[1], q[5]], [q[4], q[5], q[2]]])
        quad = mono + Q @ sc_ / r ** 5 - 2.5 * (sc_ @ Q @ sc_) * sc_ / r ** 7
        errs.append((np.linalg.norm(mono - exact), np.linalg.norm(quad - exact)))
    for (m0, q0), (m1, q1) in zip(errs[:-1], errs[1:]):
        assert 3.5 < m0 / m1 < 4.5
        assert 7.0 < q0 / q1 < 9.0


def test_quadrupole_walk_is_more_accurate(load, tab, direct):
    a = oc.tree_forces(load.pos, load.mass, load.eps, load.L, R, tab, 1, 0.4, 0.2, 0.4, leaf_size=8, group=16)
    b = oc.tree_forces(load.pos, load.mass, load.eps, load.L, R, tab, 1, 0.4, 0.2, 0.4, leaf_size=8, group=16,
                       quadrupole=True)
    assert rel(b, direct).mean() < 0.5 * rel(a, direct).mean()
