"""GPU parity of the pairwise exact path (STEPS_SUM_PAIRWISE: every unordered
pair evaluated once, the reaction of each pair added to its source) against
the FP64 oracle.

Bar: the exact path's 1e-5 on the largest relative acceleration error and on
the potential.  The pair term is evaluated once and applied with opposite
signs, so total momentum is conserved to the rounding of the sums: the
residual sum_i m_i a_i must stay below 1e-6 of sum_i m_i |a_i|.
"""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def sc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_20787_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def pairwise(sc, pos, mass, eps, L, n_img, potential=True):
    print(f"[case] pairwise N={mass.shape[0]} n_img={n_img} potential={potential}", flush=True)
    acc, pot = sc.steps_cyl_forces_ex(dev(pos), dev(mass), dev(eps), L, n_img, mode=sc.STEPS_SUM_PAIRWISE,
                                      potential=potential)
    torch.cuda.synchronize()
    return acc.cpu().numpy().astype(np.float64), (pot.cpu().numpy().astype(np.float64) if potential else None)


def rel(a, ref):
    return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)


def check(a, p, a_ref, p_ref):
    e = rel(a, a_ref)
    print(f"max {e.max():.3e} rms {math.sqrt(np.mean(e ** 2)):.3e}")
    assert e.max() <= TOL
    if p is not None:
        assert (np.abs(p - p_ref) / np.abs(p_ref)).max() <= TOL


def test_config1_all_targets(sc):
    p = synth.cylinder_load(4096, seed=0)
    a, pot = pairwise(sc, p.pos, p.mass, p.eps, p.L, 8)
    a_ref, p_ref = oracle.forces(p.pos, p.mass, p.eps, p.L, 8)
    check(a, pot, a_ref, p_ref)


# one group (N <= 1024), group edges, odd and even group counts, ragged tails
@pytest.mark.parametrize("N", [2, 3, 1023, 1024, 1025, 2048, 2049, 3000, 5000])
def test_ragged_sizes_and_group_counts(sc, N):
    p = synth.cylinder_load(N, seed=N)
    a, pot = pairwise(sc, p.pos, p.mass, p.eps, p.L, 8)
    a_ref, p_ref = oracle.forces(p.pos, p.mass, p.eps, p.L, 8)
    check(a, pot, a_ref, p_ref)


def test_single_particle_feels_nothing(sc):
    p = synth.cylinder_load(1, seed=1)
    a, pot = pairwise(sc, p.pos, p.mass, p.eps, p.L, 8)
    assert np.all(a == 0) and np.all(pot == 0)


@pytest.mark.parametrize("n_img", [0, 1, 3, 8])
def test_image_counts_without_potential(sc, n_img):
    # compile-time counts (0, 1, 8) and the run-time loop (3)
    p = synth.cylinder_load(2500, seed=7)
    a, _ = pairwise(sc, p.pos, p.mass, p.eps, p.L, n_img, potential=False)
    a_ref, _ = oracle.forces(p.pos, p.mass, p.eps, p.L, n_img, potential=False)
    check(a, None, a_ref, None)


def test_far_image_count_of_the_learned_comparison(sc):
    # |n| <= 1024 (the sum the far-image corrections are measured against) on
    # the run-time image loop, three groups with a ragged one, with the
    # potential; 256 sampled targets against the oracle
    p = synth.cylinder_load(2100, seed=5)
    a, pot = pairwise(sc, p.pos, p.mass, p.eps, p.L, 1024)
    t = synth.target_sample(2100, 256, seed=1)
    a_ref, p_ref = oracle.forces(p.pos, p.mass, p.eps, p.L, 1024, targets=t)
    check(a[:, t], pot[t], a_ref, p_ref)


def test_clustered_load_takes_the_spline_on_both_sides(sc):
    # 64 Plummer clumps: many pairs inside their softening length, across groups
    p = synth.clustered_load(6000, n_clumps=8, clump_frac=0.05, seed=3)
    a, pot = pairwise(sc, p.pos, p.mass, p.eps, p.L, 8)
    a_ref, p_ref = oracle.forces(p.pos, p.mass, p.eps, p.L, 8)
    check(a, pot, a_ref, p_ref)


def test_axial_separation_of_half_a_period(sc):
    # pairs at |z_i - z_j| = L/2 exactly take the same minimum image -L/2 on
    # both sides; the reaction must then keep the sign of F_z
    p = synth.cylinder_load(3000, seed=11)
    pos = p.pos.copy()
    for k in range(0, 40, 2):
        pos[2, k + 1] = pos[2, k] + 0.5 if pos[2, k] < 0.5 else pos[2, k] - 0.5
    pos[2, 100] = 0.125
    pos[2, 2999] = 0.625
    a, pot = pairwise(sc, pos, p.mass, p.eps, p.L, 8)
    a_ref, p_ref = oracle.forces(pos, p.mass, p.eps, p.L, 8)
    check(a, pot, a_ref, p_ref)


def test_matches_the_one_sided_kernel_and_conserves_momentum(sc):
    # every target of a 2^16 load: both paths against the FP64 GPU reference
    # (itself pinned to the oracle in test_gpu_forces) at the exact path's
    # bar, and against each other within the sum of their errors
    p = synth.cylinder_load(1 << 16, seed=4)
    pos, m, e = dev(p.pos), dev(p.mass), dev(p.eps)
    a1, p1 = sc.steps_cyl_forces_ex(pos, m, e, p.L, 8)
    a2, p2 = sc.steps_cyl_forces_ex(pos, m, e, p.L, 8, mode=sc.STEPS_SUM_PAIRWISE)
    ref, ref_pot = sc.steps_cyl_forces_f64(pos, m, e, p.L, 8)
    torch.cuda.synchronize()
    a1, a2, r = a1.double().cpu().numpy(), a2.double().cpu().numpy(), ref.cpu().numpy()
    e1, e2 = rel(a1, r), rel(a2, r)
    print(f"vs FP64 on all targets: one-sided max {e1.max():.2e}, pairwise max {e2.max():.2e}")
    assert e1.max() <= TOL and e2.max() <= TOL
    assert rel(a2, a1).max() <= e1.max() + e2.max()
    for pt in (p1, p2):
        assert (torch.abs(pt.double() - ref_pot) / torch.abs(ref_pot)).max().item() <= TOL
    mom = np.abs((p.mass[None, :] * a2).sum(axis=1)) / (p.mass[None, :] * np.abs(a2)).sum(axis=1)
    mom1 = np.abs((p.mass[None, :] * a1).sum(axis=1)) / (p.mass[None, :] * np.abs(a1)).sum(axis=1)
    print("momentum residual pairwise", mom, "one-sided", mom1)
    assert mom.max() <= 1e-6


def test_rejects_a_target_list(sc):
    p = synth.cylinder_load(100, seed=2)
    t = torch.arange(10, dtype=torch.int64, device="cuda:0")
    with pytest.raises(sc.StepsError):
        sc.steps_cyl_forces_ex(dev(p.pos), dev(p.mass), dev(p.eps), p.L, 8, targets=t,
                               mode=sc.STEPS_SUM_PAIRWISE)


def test_above_two_million_groups_hold_eight_parts(sc):
    # above 2^21 particles a group holds 8 parts instead of 16 (an odd number
    # of groups here, and a ragged last part): sampled targets against the
    # FP64 GPU reference and the oracle, total momentum as above
    N = (1 << 21) + 37
    p = synth.cylinder_load(N, seed=21)
    pos, m, e = dev(p.pos), dev(p.mass), dev(p.eps)
    a, pot = sc.steps_cyl_forces(pos, m, e, p.L, 8)
    tg = synth.target_sample(N, 512, seed=5)
    t = torch.from_numpy(tg).to(pos.device)
    ref, ref_pot = sc.steps_cyl_forces_f64(pos, m, e, p.L, 8, targets=t)
    torch.cuda.synchronize()
    a_s, r = a[:, t].double().cpu().numpy(), ref.cpu().numpy()
    check(a_s, pot[t].double().cpu().numpy(), r, ref_pot.cpu().numpy())
    a_o, p_o = oracle.forces(p.pos, p.mass, p.eps, p.L, 8, targets=tg[:32])
    check(a_s[:, :32], pot[t[:32]].double().cpu().numpy(), a_o, p_o)
    a_all = a.double().cpu().numpy()
    mom = np.abs((p.mass[None, :] * a_all).sum(axis=1)) / (p.mass[None, :] * np.abs(a_all)).sum(axis=1)
    print("momentum residual", mom)
    assert mom.max() <= 1e-6
