"""GPU parity of the learned-correction force kernel against the FP64 oracle
of the same scheme (exact |n| <= 1 + network correction on the images
2 <= |n| <= 1024, exact band outside the network's domain), with the
network's BF16 roundings emulated.

Bar: max relative acceleration error 2e-5.  Derivation: per pair the only
differences are FP32 rounding of the near terms (~1e-7 relative, as in the
exact kernel) and rare BF16 flips in the network (about 2 % of pairs move
their correction by ~1e-3 of s(r) <= 0.02 m_j/L^2, with random signs); over
2048 sources that adds ~1e-7 absolute against |a| >= 2e-3, i.e. ~5e-6.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp as om

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 2e-5


@pytest.fixture(scope="module")
def sc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_20787_amd as m
    return m


@pytest.fixture(scope="module")
def net(sc):
    n = sc.Mlp.create(synth.mlp_init(seed=21, out_gain=1.0))
    yield n
    n.close()


def to_dev(p):
    d = torch.device("cuda:0")
    return (torch.from_numpy(p.pos).to(d), torch.from_numpy(p.mass).to(d),
            torch.from_numpy(p.eps).to(d))


def load_with_axis_line(N, seed):
    # the stereographic load plus a few particles on and near the axis, so
    # that pairs with rho/L < 0.05 (outside the network's domain), a pair at
    # rho = 0 and coincident particles occur
    p = synth.cylinder_load(N, seed=seed)
    pos = p.pos.copy()
    pos[0, :12] = 0.01 * np.arange(12) / 12
    pos[1, :12] = 0.0
    pos[2, :12] = np.linspace(0.05, 0.95, 12)
    pos[:, 12] = pos[:, 13]
    return synth.Particles(pos, p.mass, p.eps, p.L)


def rel_err(a_gpu, a_ref):
    a = a_gpu.detach().cpu().numpy().astype(np.float64)
    return np.linalg.norm(a - a_ref, axis=0) / np.linalg.norm(a_ref, axis=0)


def test_learned_matches_oracle(sc, net):
    p = load_with_axis_line(2048, seed=31)
    pos, m, e = to_dev(p)
    print("[case] learned N=2048", flush=True)
    acc, pot = sc.steps_cyl_forces_learned(pos, m, e, p.L, net)
    torch.cuda.synchronize()
    t = np.unique(np.concatenate([np.arange(16), synth.target_sample(p.N, 80, seed=1)]))
    ref = om.forces_learned(p.pos, p.mass, p.eps, p.L, net.params().astype(np.float64), targets=t)
    err = rel_err(acc[:, torch.from_numpy(t).cuda()], ref)
    print(f"learned vs oracle scheme: max {err.max():.2e} median {np.median(err):.2e}")
    assert err.max() <= TOL
    # potential: the near images only
    _, pref = oracle.forces(p.pos, p.mass, p.eps, p.L, 1, targets=t)
    perr = np.abs(pot.cpu().numpy()[t] - pref) / np.abs(pref)
    assert perr.max() <= 1e-5


def test_learned_momentum_and_subset(sc, net):
    p = synth.cylinder_load(3000, seed=32)
    pos, m, e = to_dev(p)
    acc, pot = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net)  # per target, all targets
    tt = torch.tensor([0, 2999, 77, 77, 1500], dtype=torch.int64, device=pos.device)
    acc2, pot2 = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=tt)
    torch.cuda.synchronize()
    assert torch.equal(acc2, acc[:, tt]) and torch.equal(pot2, pot[tt])
    for a_t in (acc, sc.steps_cyl_forces_learned(pos, m, e, p.L, net)[0]):
        a = a_t.double().cpu().numpy()
        mom = np.abs((p.mass[None, :] * a).sum(axis=1))
        scale = np.sum(p.mass * np.linalg.norm(a, axis=0))
        print(f"|sum m a| / sum m|a| = {mom.max() / scale:.2e}")
        assert mom.max() <= 1e-5 * scale


@pytest.mark.parametrize("N", [2, 129, 1000, 5000])
def test_pairwise_learned_matches_per_target_and_oracle(sc, net, N):
    # steps_cyl_forces_learned evaluates every unordered pair once (groups of
    # 1024 in sub-groups of 128: one group with ragged sub-groups, and an odd
    # group count); the per-target kernel and the oracle of the learned scheme
    # are the references
    p = load_with_axis_line(N, seed=70 + N) if N >= 20 else synth.cylinder_load(N, seed=70)
    pos, m, e = to_dev(p)
    print(f"[case] pairwise learned N={N}", flush=True)
    full, fpot = sc.steps_cyl_forces_learned(pos, m, e, p.L, net)
    one, opot = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net)
    torch.cuda.synchronize()
    f = full.double().cpu().numpy()
    assert rel_err(full, one.double().cpu().numpy()).max() <= 1e-5
    assert (torch.abs(fpot.double() - opot.double()) / torch.abs(opot.double())).max().item() <= 1e-5
    t = np.arange(N) if N <= 200 else np.unique(np.concatenate([np.arange(16), synth.target_sample(N, 60, seed=3)]))
    ref = om.forces_learned(p.pos, p.mass, p.eps, p.L, net.params().astype(np.float64), targets=t)
    assert rel_err(full[:, torch.from_numpy(t).cuda()], ref).max() <= TOL
    # momentum: cross-group pairs cancel to rounding; pairs inside a group are
    # evaluated from both ends, like the per-target kernel (the exact band of
    # off-domain pairs sums its images in a sign-dependent order)
    mom = np.abs((p.mass[None, :] * f).sum(axis=1)) / (p.mass[None, :] * np.abs(f)).sum(axis=1)
    assert mom.max() <= 1e-5


def test_pairwise_learned_many_groups_sampled(sc, net):
    # 65 groups of 1024 after the spatial sort (an odd count, the last of 37
    # particles: one ragged sub-group), 2080 meetings; the near-axis particles
    # and 20 sampled targets against the oracle of the learned scheme
    N = (1 << 16) + 37
    p = load_with_axis_line(N, seed=123)
    pos, m, e = to_dev(p)
    print(f"[case] pairwise learned N={N}", flush=True)
    full, _ = sc.steps_cyl_forces_learned(pos, m, e, p.L, net, potential=False)
    torch.cuda.synchronize()
    t = np.unique(np.concatenate([np.arange(4), synth.target_sample(N, 20, seed=4)]))
    ref = om.forces_learned(p.pos, p.mass, p.eps, p.L, net.params().astype(np.float64), targets=t)
    err = rel_err(full[:, torch.from_numpy(t).cuda()], ref)
    print(f"max {err.max():.2e} over {t.size} targets")
    assert err.max() <= TOL


@pytest.mark.parametrize("N", [5000, 9000])
def test_pairwise_learned_is_deterministic(sc, net, N):
    # a fixed tournament of groups (even and odd group counts), no atomics:
    # repeated calls are bitwise equal (a race in the reactions' LDS sums or
    # in the read-modify-writes of the sums would show up here)
    p = load_with_axis_line(N, seed=90 + N)
    pos, m, e = to_dev(p)
    print(f"[case] pairwise learned determinism N={N}", flush=True)
    a1, p1 = sc.steps_cyl_forces_learned(pos, m, e, p.L, net)
    a2, p2 = sc.steps_cyl_forces_learned(pos, m, e, p.L, net)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(p1, p2)


def test_short_lists_split_the_sources_into_chunks(sc, net):
    # 300 targets of 20,000 sources: 3 target blocks, so the sources are
    # split into 5 chunks whose totals are added in order
    p = load_with_axis_line(20000, seed=95)
    pos, m, e = to_dev(p)
    tg = np.unique(np.concatenate([np.arange(16), synth.target_sample(p.N, 284, seed=96)]))
    t = torch.from_numpy(tg).cuda()
    print("[case] chunked learned per-target", flush=True)
    acc, _ = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=t, potential=False)
    torch.cuda.synchronize()
    sub = tg[:40]
    ref = om.forces_learned(p.pos, p.mass, p.eps, p.L, net.params().astype(np.float64), targets=sub)
    assert rel_err(acc[:, :40], ref).max() <= TOL


def test_learned_ragged_and_plain(sc, net):
    p = load_with_axis_line(333, seed=33)
    pos, m, e = to_dev(p)
    acc_c, _ = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, potential=False)
    acc_p, _ = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, mode=sc.STEPS_SUM_PLAIN,
                                              potential=False)
    torch.cuda.synchronize()
    ref = om.forces_learned(p.pos, p.mass, p.eps, p.L, net.params().astype(np.float64))
    assert rel_err(acc_c, ref).max() <= TOL
    assert rel_err(acc_p, ref).max() <= TOL


def test_all_targets_in_spatial_order_are_bitwise_the_subset_results(sc, net):
    p = synth.cylinder_load(9000, seed=48)
    pos, m, e = (torch.from_numpy(x).cuda() for x in (p.pos, p.mass, p.eps))
    full, fpot = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net)  # per target, all targets
    tg = torch.from_numpy(synth.target_sample(p.N, 400, seed=49)).cuda()
    sub, spot = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=tg)
    torch.cuda.synchronize()
    assert torch.equal(full[:, tg], sub)
    assert torch.equal(fpot[tg], spot)


def test_long_target_lists_in_spatial_order_are_bitwise_exact(sc, net):
    p = synth.cylinder_load(9000, seed=55)
    pos, m, e = (torch.from_numpy(x).cuda() for x in (p.pos, p.mass, p.eps))
    full, fpot = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net)  # per target, all targets
    rng = np.random.default_rng(56)
    tg = torch.from_numpy(rng.integers(0, p.N, 5000)).cuda()
    sub, spot = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=tg)
    torch.cuda.synchronize()
    assert torch.equal(full[:, tg], sub)
    assert torch.equal(fpot[tg], spot)


def test_near_axis_pairs_take_the_band_series(sc, net):
    # every pair closer than 0.05 L to the axis of the other: no pair is in the
    # network's domain, and the kernels evaluate the band 2 <= |n| <= 1024 of
    # each from its series in rho^2 (exact to FP32 rounding); the oracle sums
    # the 2046 images directly.  The band is 5-20 % of these forces, so a
    # missing series term (1e-5 of the band) or a wrong coefficient would
    # exceed the 1e-6 bar, FP32 rounding (~1e-7) would not.
    rng = np.random.default_rng(7)
    N = 256
    rr = 0.02 * np.sqrt(rng.random(N))
    phi = 2.0 * math.pi * rng.random(N)
    pos = np.stack([rr * np.cos(phi), rr * np.sin(phi), rng.random(N)])
    mass = np.full(N, 1.0 / N)
    eps = np.full(N, 1e-4)
    p = synth.Particles(pos, mass, eps, 1.0)
    d_pos, d_m, d_e = to_dev(p)
    print("[case] near-axis learned N=256", flush=True)
    acc, _ = sc.steps_cyl_forces_learned(d_pos, d_m, d_e, p.L, net, potential=False)
    t = torch.arange(0, N, 3, dtype=torch.int64, device=d_pos.device)
    acc_t, _ = sc.steps_cyl_forces_learned_ex(d_pos, d_m, d_e, p.L, net, targets=t, potential=False)
    torch.cuda.synchronize()
    ref = om.forces_learned(p.pos, p.mass, p.eps, p.L, net.params().astype(np.float64))
    err = rel_err(acc, ref)
    err_t = rel_err(acc_t, ref[:, t.cpu().numpy()])
    print(f"near-axis band: pairwise max {err.max():.2e}, per-target max {err_t.max():.2e}")
    assert err.max() <= 1e-6 and err_t.max() <= 1e-6
