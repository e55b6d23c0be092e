"""GPU parity of the Barnes-Hut octree (Sect. 2.4) against its FP64 oracle.

Bars: the tree's integer structure (depth-first cells: level, particle
range, skip link, leaf flag; the particles' key order) and the interaction
counts are bit-exact (both sides take the cell and acceptance decisions in
FP64 with the same operations); cell masses and centres of mass to FP64
summation-order round-off; forces to 2e-5 relative (FP32 pair arithmetic
and FP32 table nodes, as for the tabulated scheme); theta = 0 reproduces
the direct tabulated kernel to FP32 summation-order round-off (2e-5: the
same pairs summed in another order) and the oracle's FP64 tabulated scheme
to the tabulated path's own bar against it (2e-5); the radial
correction to 1e-5 of the mean force (it is a mean of differences of FP32
forces).
"""
import math

import numpy as np
import pytest

import synth
from oracle import octree as oc
from oracle import table as ot

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = synth.r_max()


@pytest.fixture(scope="module")
def sc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_20787_amd as m
    return m


def to_dev(p):
    d = torch.device("cuda:0")
    return (torch.from_numpy(p.pos).to(d), torch.from_numpy(p.mass).to(d),
            torch.from_numpy(p.eps).to(d))


def rel(a, ref):
    return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.mark.parametrize("N,leaf,shift,angle", [(3000, 16, 0.3, 1.2), (777, 1, 0.0, 0.0), (40, 64, 0.9, -2.0)])
def test_tree_structure_matches_oracle(sc, N, leaf, shift, angle):
    p = synth.cylinder_load(N, seed=31)
    t = sc.Octree(leaf)
    tab = sc.CorrectionTable(16, 12, 6.5, 1024)
    sc.steps_cyl_tree_forces(t, *to_dev(p), p.L, R, tab, 1, 0.5, shift, angle)
    torch.cuda.synchronize()
    g = sc.steps_cyl_tree_cells(t, N)
    T = oc.Tree(p.pos, p.mass, p.eps, p.L, R, shift, angle, leaf)
    print(f"N={N} leaf={leaf}: {len(T.cells)} cells, depth {T.level.max()}")
    np.testing.assert_array_equal(g["order"], T.order)
    np.testing.assert_array_equal(g["level"], T.level)
    np.testing.assert_array_equal(g["start"], T.start)
    np.testing.assert_array_equal(g["count"], T.end - T.start)
    np.testing.assert_array_equal(g["skip"], T.skip)
    np.testing.assert_array_equal(g["leaf"].astype(bool), T.leaf)
    np.testing.assert_allclose(g["mass"], T.mass, rtol=1e-13)
    np.testing.assert_allclose(g["com"], T.com, rtol=1e-12, atol=1e-13)
    t.close()
    tab.close()


def test_zero_opening_angle_is_the_direct_kernel(sc):
    p = synth.cylinder_load(4000, seed=32)
    t = sc.Octree(16)
    tab = sc.CorrectionTable(32, 40, 6.5, 1024)
    pos, m, e = to_dev(p)
    a = sc.steps_cyl_tree_forces(t, pos, m, e, p.L, R, tab, 1, 0.0, 0.4, 0.8)
    d, _ = sc.steps_cyl_forces_table(pos, m, e, p.L, tab, order=1, potential=False)
    torch.cuda.synchronize()
    a_np = a.double().cpu().numpy()
    err = rel(a_np, d.double().cpu().numpy())
    # the same pairs summed in another order
    print(f"theta=0 vs direct kernel: max {err.max():.2e}")
    assert err.max() <= 2e-5, err.max()
    # and the oracle's FP64 tabulated scheme on sampled targets, at the
    # tabulated path's own bar against it
    tg = synth.target_sample(p.N, 64, seed=3)
    ref = ot.forces_table(p.pos, p.mass, p.eps, p.L, ot.Table(32, 40, 6.5), 1, targets=tg)
    e_ref = rel(a_np[:, tg], ref)
    print(f"theta=0 vs oracle tabulated scheme: max {e_ref.max():.2e}")
    assert e_ref.max() <= 2e-5, e_ref.max()
    n_cells, n_c, n_p = sc.steps_cyl_tree_info(t)
    assert n_c == 0 and n_p == p.N * p.N
    t.close()
    tab.close()


@pytest.mark.parametrize("theta,order,quad", [(0.3, 1, False), (0.6, 1, False), (1.0, 1, False),
                                              (0.6, 2, False), (0.6, 1, True), (1.0, 2, True)])
def test_tree_forces_match_oracle(sc, theta, order, quad):
    p = synth.clustered_load(2000, n_clumps=4, clump_frac=0.05, seed=33)
    t = sc.Octree(16, quadrupole=quad)
    tab = sc.CorrectionTable(24, 16, 6.5, 1024)
    a = sc.steps_cyl_tree_forces(t, *to_dev(p), p.L, R, tab, order, theta, 0.6, 2.5)
    torch.cuda.synchronize()
    st = {}
    ref = oc.tree_forces(p.pos, p.mass, p.eps, p.L, R, ot.Table(24, 16, 6.5), order, theta, 0.6, 2.5,
                         leaf_size=16, group=64, stats=st, quadrupole=quad)
    n_cells, n_c, n_p = sc.steps_cyl_tree_info(t)
    err = rel(a.double().cpu().numpy(), ref)
    print(f"theta={theta} order={order} quad={quad}: cells {n_cells}, cell/particle interactions {n_c}/{n_p}, "
          f"max rel err {err.max():.2e}")
    assert (n_cells, n_c, n_p) == (st["cells"], st["cell_interactions"], st["particle_interactions"])
    assert err.max() <= 2e-5
    t.close()
    tab.close()


def test_radial_calibration_matches_oracle(sc):
    p = synth.cylinder_load(1500, seed=34)
    t = sc.Octree(8)
    tab = sc.CorrectionTable(24, 16, 6.5, 1024)
    otab = ot.Table(24, 16, 6.5)
    theta, nb = 0.9, 8
    rng = np.random.default_rng(35)
    shifts = rng.random(3) * p.L
    angles = rng.random(3) * 2 * math.pi
    pos, m, e = to_dev(p)
    corr = sc.steps_cyl_tree_calibrate(t, pos, m, e, p.L, R, tab, 1, theta, shifts, angles, nb)
    ref = oc.calibrate(p.pos, p.mass, p.eps, p.L, R, otab, 1, theta, shifts, angles, nb,
                       leaf_size=8, group=64)
    direct = ot.forces_table(p.pos, p.mass, p.eps, p.L, otab, 1)
    scale = np.linalg.norm(direct, axis=0).mean()
    print("correction", corr, "oracle", ref)
    np.testing.assert_allclose(corr, ref, rtol=0, atol=1e-5 * scale)
    # the corrected walk subtracts it
    a = sc.steps_cyl_tree_forces(t, pos, m, e, p.L, R, tab, 1, theta, 0.2, 0.5, correct=True)
    torch.cuda.synchronize()
    b = oc.apply_correction(p.pos, oc.tree_forces(p.pos, p.mass, p.eps, p.L, R, otab, 1, theta, 0.2, 0.5,
                                                  leaf_size=8, group=64), ref, R)
    assert rel(a.double().cpu().numpy(), b).max() <= 2e-5
    sc.steps_cyl_tree_set_correction(t, None, R)
    with pytest.raises(sc.StepsError):
        sc.steps_cyl_tree_forces(t, pos, m, e, p.L, R, tab, 1, theta, correct=True)
    t.close()
    tab.close()


def test_force_error_statistics_follow_the_opening_angle(sc):
    # Fig. 3's measures on a 2^15-particle load: mean relative error, mean
    # radial and tangential ratio against the direct forces, with and
    # without the radial correction
    p = synth.cylinder_load(1 << 15, seed=36)
    pos, m, e = to_dev(p)
    tab = sc.CorrectionTable(128, 144, 6.4, 1024)
    d, _ = sc.steps_cyl_forces_table(pos, m, e, p.L, tab, order=1, potential=False)
    d = d.double().cpu().numpy()
    x, y = p.pos[0], p.pos[1]
    rho = np.hypot(x, y)
    ur = np.stack([x / rho, y / rho])
    ut = np.stack([-y / rho, x / rho])
    rng = np.random.default_rng(37)
    rows = []
    for theta in (0.3, 0.5, 0.7, 0.9):
        t = sc.Octree(16)
        sc.steps_cyl_tree_calibrate(t, pos, m, e, p.L, R, tab, 1, theta, rng.random(4) * p.L,
                                    rng.random(4) * 2 * math.pi, 32)
        s, a = rng.random() * p.L, rng.random() * 2 * math.pi
        raw = sc.steps_cyl_tree_forces(t, pos, m, e, p.L, R, tab, 1, theta, s, a).double().cpu().numpy()
        cor = sc.steps_cyl_tree_forces(t, pos, m, e, p.L, R, tab, 1, theta, s, a,
                                       correct=True).double().cpu().numpy()
        _, n_c, n_p = sc.steps_cyl_tree_info(t)
        t.close()
        out = [theta, (n_c + n_p) / p.N]
        for f in (raw, cor):
            out += [rel(f, d).mean(), np.mean((f[:2] * ur).sum(0) / (d[:2] * ur).sum(0)),
                    np.median((f[:2] * ut).sum(0) / (d[:2] * ut).sum(0))]
        rows.append(out)
        print("theta {:.1f}: {:.0f} interactions/particle; raw mean err {:.2e} radial ratio {:.5f} "
              "tangential {:.4f}; corrected {:.2e} {:.5f} {:.4f}".format(*out))
    err = [r[2] for r in rows]
    assert all(a < b for a, b in zip(err[:-1], err[1:]))
    assert err[1] < 1e-2
    # the correction, calibrated on 4 other random frames, removes the
    # systematic radial bias: where the raw bias stands above the spread of a
    # single frame's mean radial ratio (about 3e-4 on this load) it brings the
    # ratio closer to one, and elsewhere it leaves it within that spread
    for r in rows:
        assert abs(r[6] - 1) <= max(abs(r[3] - 1), 3e-4)
    assert abs(rows[2][6] - 1) < 0.6 * abs(rows[2][3] - 1)  # theta = 0.7: a clear bias, clearly reduced
    tab.close()


def test_kdk_step_with_octree_composes_its_parts(sc):
    # one step with octree forces over a complete table and the step's random
    # frame: the force at the drifted positions is the tree force there (the
    # build and walk are deterministic), and the momenta are the two kicks
    # with the infinite cylinder's pull.  The parts are each checked against
    # the oracle elsewhere; comparing the drifted state with the oracle would
    # let FP32-level position differences move particles across cell faces.
    p = synth.displaced_load(900, seed=38)
    rho0 = 1.0 / (math.pi * R * R * p.L)
    H0 = math.sqrt(8 * math.pi * rho0 / 0.9)
    t = sc.Octree(16)
    tab = sc.CorrectionTable.ewald(24, 16, 4.0, 2.0, 5, 12)
    theta, s0, a0, s1, a1 = 0.6, 0.1, 0.4, 0.7, 2.9
    pos, m, e = to_dev(p)
    pos0 = pos.clone()
    acc0 = sc.steps_cyl_tree_forces(t, pos, m, e, p.L, R, tab, 1, theta, s0, a0)
    acc = acc0.clone()
    mom = torch.zeros_like(pos)
    par = sc.kdk_params(0.05, 0.06, H0, 0.3, 0.7, R_cyl=R, rho0=rho0, table=tab, table_order=1,
                        tree=t, theta=theta, tree_shift=s1, tree_angle=a1)
    sc.steps_cyl_kdk_step(pos, mom, m, e, p.L, par, acc)
    acc1 = sc.steps_cyl_tree_forces(t, pos, m, e, p.L, R, tab, 1, theta, s1, a1)
    torch.cuda.synchronize()
    assert torch.equal(acc, acc1)
    K1, D, K2 = sc.steps_cyl_kdk_factors(par)
    c0 = sc.steps_cyl_compensation(pos0, R, math.inf, rho0)
    c1 = sc.steps_cyl_compensation(pos, R, math.inf, rho0)
    mid = K1 * (acc0.double() - c0)
    expect = mid + K2 * (acc1.double() - c1)
    torch.testing.assert_close(mom, expect, rtol=1e-12, atol=1e-15)
    dx = pos - pos0 - D * mid
    dx[2] -= torch.round(dx[2] / p.L) * p.L
    assert float(dx.abs().max()) < 1e-12
    t.close()
    tab.close()


def test_full_size_sampled_matches_oracle(sc):
    # the benchmark's size: N = 2^20, theta = 0.5, 144 x 128 band table; the
    # oracle walks only the groups holding the sampled targets
    N = 1 << 20
    p = synth.cylinder_load(N, seed=0)
    t = sc.Octree(16)
    tab = sc.CorrectionTable(128, 144, 6.4, 1024)
    a = sc.steps_cyl_tree_forces(t, *to_dev(p), p.L, R, tab, 1, 0.5, 0.25, 1.7)
    torch.cuda.synchronize()
    tg = synth.target_sample(N, 12, seed=51)
    ref = oc.tree_forces(p.pos, p.mass, p.eps, p.L, R, ot.Table(128, 144, 6.4), 1, 0.5, 0.25, 1.7,
                         targets=tg)
    err = rel(a[:, torch.from_numpy(tg).cuda()].double().cpu().numpy(), ref)
    print(f"N=2^20 theta=0.5: max rel err vs oracle {err.max():.2e} on {tg.size} targets")
    assert err.max() <= 2e-5
    t.close()
    tab.close()


@pytest.mark.parametrize("case", ["one", "two", "coincident", "outside"])
def test_edge_cases_match_oracle(sc, case):
    rng = np.random.default_rng(61)
    if case == "one":
        p = synth.cylinder_load(1, seed=62)
    elif case == "two":
        p = synth.cylinder_load(2, seed=63)
    else:
        base = synth.cylinder_load(300, seed=64)
        pos = base.pos.copy()
        if case == "coincident":
            pos[:, :100] = pos[:, [7]]          # 100 particles on one point: a level-21 leaf
        else:
            pos[0, :5] = 2.0 * R * (1 + rng.random(5))   # beyond the root cube: clamped cells
        p = synth.Particles(pos, base.mass, base.eps, base.L)
    t = sc.Octree(4)
    tab = sc.CorrectionTable(24, 16, 20.0, 1024)
    a = sc.steps_cyl_tree_forces(t, *to_dev(p), p.L, R, tab, 1, 0.6, 0.3, 0.9)
    torch.cuda.synchronize()
    st = {}
    ref = oc.tree_forces(p.pos, p.mass, p.eps, p.L, R, ot.Table(24, 16, 20.0), 1, 0.6, 0.3, 0.9,
                         leaf_size=4, group=64, stats=st)
    n_cells, n_c, n_p = sc.steps_cyl_tree_info(t)
    assert (n_cells, n_c, n_p) == (st["cells"], st["cell_interactions"], st["particle_interactions"])
    a = a.double().cpu().numpy()
    if case == "one":
        assert np.all(a == 0.0) and np.all(ref == 0.0)
    else:
        scale = np.linalg.norm(ref, axis=0).max()
        err = np.linalg.norm(a - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-3 * scale)
        print(f"{case}: cells {n_cells}, max rel err {err.max():.2e}")
        assert err.max() <= 2e-5
    t.close()
    tab.close()


def test_quadrupoles_cut_the_error_at_equal_cost(sc):
    # same acceptance decisions (same interaction counts), smaller error
    p = synth.cylinder_load(1 << 15, seed=39)
    pos, m, e = to_dev(p)
    tab = sc.CorrectionTable(128, 144, 6.4, 1024)
    d, _ = sc.steps_cyl_forces_table(pos, m, e, p.L, tab, order=1, potential=False)
    d = d.double().cpu().numpy()
    for theta in (0.3, 0.5):
        out = {}
        for quad in (False, True):
            t = sc.Octree(16, quadrupole=quad)
            a = sc.steps_cyl_tree_forces(t, pos, m, e, p.L, R, tab, 1, theta, 0.3, 0.7)
            out[quad] = (rel(a.double().cpu().numpy(), d).mean(), sc.steps_cyl_tree_info(t))
            t.close()
        print(f"theta={theta}: mean error monopole {out[False][0]:.2e}, quadrupole {out[True][0]:.2e}")
        assert out[False][1] == out[True][1]
        assert out[True][0] < 0.5 * out[False][0]
    tab.close()
