"""Pins of the learned-correction oracle: BF16 rounding against the library
conversion, forward pass against a library network, gradients against
finite differences, the analytic baseline against quadrature and the exact
remainder, the symmetry of the folded model, Adam's first step, and the
antisymmetry of learned pair forces."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from oracle import mlp

torch = pytest.importorskip("torch")


def test_param_layout_matches_generator():
    assert mlp.n_params() == 12802 == synth.mlp_param_count()
    assert [s for _, s in mlp.param_shapes()] == [s for _, s in synth.mlp_param_shapes()]


def test_bf16_round_is_round_to_nearest_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [1.0, -2.5, 1.00390625, 1.01171875, 3.0e-39]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)


class _Silu2(torch.nn.Module):
    """SiLU(u ln 2) / ln 2 from the library SiLU."""

    def forward(self, u):
        return torch.nn.functional.silu(u * math.log(2.0)) / math.log(2.0)


def _torch_net(params):
    layers = mlp.unpack(params)
    mods = []
    for k, (W, b) in enumerate(layers):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        lin.weight.data = torch.from_numpy(W)
        lin.bias.data = torch.from_numpy(b)
        mods.append(lin)
        if k < len(layers) - 1:
            mods.append(_Silu2())
    return torch.nn.Sequential(*mods)


def test_activation_is_rescaled_silu():
    u = np.linspace(-30, 30, 601)
    ref = torch.nn.functional.silu(torch.from_numpy(u) * math.log(2.0)).numpy() / math.log(2.0)
    np.testing.assert_allclose(mlp.silu(u), ref, rtol=1e-14, atol=1e-300)
    h = 1e-6
    fd = (mlp.silu(u + h) - mlp.silu(u - h)) / (2 * h)
    np.testing.assert_allclose(mlp.silu_grad(u), fd, rtol=1e-7, atol=1e-9)


def test_forward_matches_library_network():
    p = synth.mlp_init(seed=3).astype(np.float64)
    F = np.random.default_rng(1).uniform(-1, 1, (2, 257))
    out, _ = mlp.forward(p, F)
    ref = _torch_net(p)(torch.from_numpy(F.T)).detach().numpy().T
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-14)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = synth.mlp_init(seed=4, out_gain=1.0).astype(np.float64)
    F = rng.uniform(-1, 1, (2, 64))
    T = rng.standard_normal((2, 64)) * 0.3
    _, g = mlp.loss_and_grad(p, F, T)
    idx = np.concatenate([rng.choice(p.size, 40, replace=False), [0, 191, 192, 12671, 12801]])
    for i in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, F, T)[0] - mlp.loss_and_grad(pm, F, T)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-10)


def test_gradient_matches_library_autograd():
    rng = np.random.default_rng(5)
    p = synth.mlp_init(seed=6, out_gain=1.0).astype(np.float64)
    F = rng.uniform(-1, 1, (2, 100))
    T = rng.standard_normal((2, 100))
    loss, g = mlp.loss_and_grad(p, F, T)
    net = _torch_net(p)
    out = net(torch.from_numpy(F.T))
    lt = ((out - torch.from_numpy(T.T)) ** 2).mean()
    lt.backward()
    ref = np.concatenate([t.grad.numpy().ravel() for t in net.parameters()])
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-14)


def _bf16_torch(x):
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def test_bf16_forward_straight_through_gradient_matches_library_autograd():
    # the BF16 forward with every rounding passed straight through in the
    # backward pass (round_dz=False): library autograd on the rounded
    # weights, with x + (bf16(x) - x).detach() for the rounded activations
    rng = np.random.default_rng(8)
    p = synth.mlp_init(seed=9, out_gain=1.0).astype(np.float64)
    F = rng.uniform(-1, 1, (2, 96))
    T = rng.standard_normal((2, 96)) * 0.4
    loss, g = mlp.loss_and_grad(p, F, T, bf16=True, round_dz=False)
    leaves = []
    for W, b in mlp.unpack(p):
        Wt = torch.from_numpy(W).requires_grad_(True)
        bt = torch.from_numpy(b).requires_grad_(True)
        leaves.append((Wt, bt))
    h = torch.from_numpy(F).to(torch.float32).to(torch.float64)
    for k, (Wt, bt) in enumerate(leaves):
        Wq = Wt + (_bf16_torch(Wt) - Wt).detach()
        bq = bt + (bt.to(torch.float32).to(torch.float64) - bt).detach()
        x = h + (_bf16_torch(h) - h).detach() if 1 <= k <= mlp.DEPTH - 1 else h
        z = Wq @ x + bq[:, None]
        h = torch.nn.functional.silu(z * math.log(2.0)) / math.log(2.0) if k < mlp.DEPTH else z
    lt = ((h - torch.from_numpy(T)) ** 2).mean()
    lt.backward()
    ref = np.concatenate([np.concatenate([Wt.grad.numpy().ravel(), bt.grad.numpy().ravel()])
                          for Wt, bt in leaves])
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-14)


def test_bf16_gradient_rounding_within_its_derived_bound(monkeypatch):
    # the deployed backward rounds dz of layers 2-4 to BF16; it may differ
    # from the plain backward of the same forward only by what that rounding
    # can cause (tests/mlp_bound.py), and the bound must be met closely
    from mlp_bound import grad_rounding_bound
    rng = np.random.default_rng(12)
    p = synth.mlp_init(seed=13, out_gain=1.0).astype(np.float64)
    F = rng.uniform(-1, 1, (2, 512))
    T = rng.standard_normal((2, 512)) * 0.4
    _, g_r = mlp.loss_and_grad(p, F, T, bf16=True)
    _, g_e = mlp.loss_and_grad(p, F, T, bf16=True, round_dz=False)
    bound = grad_rounding_bound(p, F, T)
    diff = np.abs(g_r - g_e)
    slack = 1e-13 * np.abs(g_e).max()
    assert np.all(diff <= bound * (1 + 1e-9) + slack)
    # per layer: the rounding shows wherever it can act, and nowhere else
    # (layer 5 and the layer-4 bias see no rounded quantity); on the layer
    # rounded last (W4) the worst case is met to within two orders, below it
    # the bound compounds absolute values over the units and samples
    off = 0
    for name, shape in mlp.param_shapes():
        n = int(np.prod(shape))
        d, b = diff[off:off + n], bound[off:off + n]
        if name in ("b4", "W5", "b5"):
            assert np.all(d == 0.0) and np.all(b == 0.0), name
        else:
            assert d.max() > 0.0, name
        off += n
    # one sample: the layer-4 weight gradient is a single product, and its
    # bound u |dz| |x| is met to within a factor 2; a rounding to 6
    # significant bits instead of 8 breaks it
    F1, T1 = F[:, :1], T[:, :1]
    b1 = grad_rounding_bound(p, F1, T1)
    _, g1 = mlp.loss_and_grad(p, F1, T1, bf16=True)
    _, g1e = mlp.loss_and_grad(p, F1, T1, bf16=True, round_dz=False)
    sizes = [int(np.prod(sh)) for _, sh in mlp.param_shapes()]
    w4 = [name for name, _ in mlp.param_shapes()].index("W4")
    sl = slice(sum(sizes[:w4]), sum(sizes[:w4 + 1]))
    r = np.abs(g1 - g1e)[sl] / np.maximum(b1[sl], 1e-300)
    assert r.max() <= 1 + 1e-9 and r.max() >= 0.5

    def coarse(x):
        f = np.asarray(x, dtype=np.float32)
        u = f.view(np.uint32).astype(np.uint64)
        u = (u + 0x1FFFF + ((u >> 18) & 1)) & 0xFFFC0000
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    monkeypatch.setattr(mlp, "bf16_round", coarse)
    _, g_c = mlp.loss_and_grad(p, F1, T1, bf16=True)
    _, g_ce = mlp.loss_and_grad(p, F1, T1, bf16=True, round_dz=False)
    monkeypatch.undo()
    assert np.any(np.abs(g_c - g_ce) > b1 * (1 + 1e-9) + 1e-13 * np.abs(g1e).max())


def test_rod_part_of_baseline_matches_quadrature():
    # remove the end corrections: the remaining rod integrals checked by quad
    for d, r in [(0.0, 0.05), (0.31, 0.7), (0.5, 3.0), (0.12, 19.0)]:
        def gz(s):
            u = s - d
            return u / (u * u + r * r) ** 1.5

        def gr(s):
            u = s - d
            return -r / (u * u + r * r) ** 1.5
        S1, S2 = 1.5, 1024.5
        qz = sum(integrate.quad(gz, a, b, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
                 for a, b in [(S1, S2), (-S2, -S1)])
        qr = sum(integrate.quad(gr, a, b, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
                 for a, b in [(S1, S2), (-S2, -S1)])
        bz, br = mlp.baseline(d, r)
        # end corrections (closed form derivatives at +-1.5) added back by hand
        cz = cr = 0.0
        for side in (1.0, -1.0):
            u = side * 1.5 - d
            q = (u * u + r * r) ** -2.5
            cz += side * (r * r - 2 * u * u) * q / 24
            cr += side * 3 * r * u * q / 24
        assert float(bz) - cz == pytest.approx(qz, rel=1e-9, abs=1e-13)
        assert float(br) - cr == pytest.approx(qr, rel=1e-9, abs=1e-13)


def test_baseline_approximates_the_exact_remainder():
    X = synth.remainder_inputs(4096, seed=7)
    Rz, Rr = mlp.exact_remainder(X[0], X[1])
    bz, br = mlp.baseline(X[0], X[1])
    mag = np.hypot(Rz, Rr)
    res = np.hypot(Rz - bz, Rr - br) / mag
    assert res.max() < 0.05
    # the end correction beats the bare rods almost everywhere
    S1 = 1.5
    bare_z = bz.copy()
    bare_r = br.copy()
    for side in (1.0, -1.0):
        u = side * S1 - X[0]
        q = (u * u + X[1] ** 2) ** -2.5
        bare_z -= side * (X[1] ** 2 - 2 * u * u) * q / 24
        bare_r -= side * 3 * X[1] * u * q / 24
    bare = np.hypot(Rz - bare_z, Rr - bare_r) / mag
    assert np.median(res) < 0.5 * np.median(bare)
    # far from the axis the images are smooth on the period and the
    # midpoint rule with its first correction is accurate
    far = X[1] > 8
    assert res[far].max() < 1e-4


def test_targets_are_order_one():
    X = synth.remainder_inputs(2048, seed=8)
    T = mlp.training_targets(X[0], X[1])
    assert np.all(np.isfinite(T)) and np.abs(T).max() < 2.0 and np.abs(T).std() > 0.01


def test_folded_model_symmetry():
    p = synth.mlp_init(seed=9)
    d = np.array([0.13, 0.4, 0.02])
    r = np.array([0.3, 2.0, 11.0])
    zp, rp = mlp.remainder_model(p, d, r)
    zm, rm = mlp.remainder_model(p, -d, r)
    np.testing.assert_array_equal(zp, -zm)
    np.testing.assert_array_equal(rp, rm)


def test_adam_first_step_moves_by_learning_rate():
    rng = np.random.default_rng(10)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # bias-corrected m/sqrt(v) = g/|g| on the first step
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_learned_pair_forces_are_antisymmetric():
    p = synth.cylinder_load(96, seed=11)
    w = synth.mlp_init(seed=12)
    a = mlp.forces_learned(p.pos, p.mass, p.eps, p.L, w)
    mom = (p.mass[None, :] * a).sum(axis=1)
    scale = np.sum(p.mass * np.linalg.norm(a, axis=0))
    assert np.abs(mom).max() < 1e-13 * scale


def test_learned_scheme_with_zero_network_is_near_plus_baseline():
    p = synth.cylinder_load(64, seed=13)
    w = np.zeros(mlp.n_params())
    a = mlp.forces_learned(p.pos, p.mass, p.eps, p.L, w, bf16=False)
    ref, _ = oracle.forces(p.pos, p.mass, p.eps, p.L, 1024, potential=False)
    near, _ = oracle.forces(p.pos, p.mass, p.eps, p.L, 1, potential=False)
    e_learn = np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)
    e_near = np.linalg.norm(near - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.median(e_learn) < 0.2 * np.median(e_near)
