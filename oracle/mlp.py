"""FP64 oracle of the learned far-image correction.

TEST INFRASTRUCTURE (see the package docstring).

What the correction computes.  For a pair with minimum-image axial offset d
(|d| <= L/2) and cylindrical separation rho, the images 2 <= |n| <= 1024 of
eq. (ForceCylindrical), summed exactly, give a force per unit G m_j / L^2

    R_z(d, rho)   = sum -(d - nL) / r_n^3 * L^2   (odd in d)
    R_rho(d, rho) = sum -rho / r_n^3 * L^2        (even in d),

(``oracle.image_band``).  The learned model replaces this sum by

    R_z   ~ sign(d) [ b_z(|d|, rho)   + s(rho) o_z ]
    R_rho ~           b_rho(|d|, rho) + s(rho) o_rho

where (o_z, o_rho) = MLP(f1, f2) and, with delta = |d|/L, r = rho/L:

  * features: f1 = 4 delta - 1,  f2 = 2 ln(r / 0.05) / ln 400 - 1
    (both in [-1, 1] over delta in [0, 1/2], r in [0.05, 20]);
  * output scale: s(r) = 0.02 / (1 + r^2);
  * fixed analytic baseline b: the images on each side replaced by a uniform
    rod from 1.5 L to 1024.5 L (midpoint rule; closed form), plus the first
    midpoint-rule correction term (1/24) g'(1.5 L) at the inner rod ends,
    with g the field of one image as a function of its axial position.
  * network: 2 -> 64 -> 64 -> 64 -> 64 -> 2 with the activation
    s(u) = u / (1 + 2^-u) after every hidden layer and a linear output;
    s(u) = SiLU(u ln 2) / ln 2, so this is a SiLU network whose first-layer
    weights and hidden biases carry a factor ln 2 and whose last-layer
    weights carry 1 / ln 2 (exp2 then needs no pre-scaling on the GPU).
    Parameters are stored in the order of ``synth.mlp_param_shapes``
    (weights (fan_out, fan_in) row-major).
  * precision of the deployed network: weights rounded to BF16, activations
    entering layers 2-4 rounded to BF16 (round-to-nearest-even), everything
    else FP32 (``bf16=True`` reproduces those roundings; features and FP64
    arithmetic otherwise).

Pairs with r < 0.05 or r > 20 are outside the network's domain: the
learned force path evaluates their far images exactly instead.

The fit target for one sample is T = (R - b) / s (FP64), trained with the
loss mean((o - T)^2) over both outputs and all samples.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

N_FAR = 1024          # outermost image of the replaced band
RHO_MIN = 0.05        # network domain in rho / L
RHO_MAX = 20.0
ROD_INNER = 1.5       # rods start half a period beyond the last exact image
WIDTH = 64
DEPTH = 4


def param_shapes():
    shapes = [("W1", (WIDTH, 2)), ("b1", (WIDTH,))]
    for k in range(2, DEPTH + 1):
        shapes += [(f"W{k}", (WIDTH, WIDTH)), (f"b{k}", (WIDTH,))]
    shapes += [(f"W{DEPTH + 1}", (2, WIDTH)), (f"b{DEPTH + 1}", (2,))]
    return shapes


def n_params():
    return int(sum(np.prod(s) for _, s in param_shapes()))


def unpack(params):
    """Flat vector -> list of (W, b) per layer (FP64 copies)."""
    params = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    shapes = param_shapes()
    for k in range(0, len(shapes), 2):
        (_, ws), (_, bs) = shapes[k], shapes[k + 1]
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        W = params[off:off + nw].reshape(ws)
        off += nw
        b = params[off:off + nb].reshape(bs)
        off += nb
        out.append((W.copy(), b.copy()))
    assert off == params.size
    return out


def bf16_round(x):
    """Round to BF16 (round-to-nearest-even) through FP32, returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


LN2 = math.log(2.0)


def silu(z):
    """Activation s(u) = u / (1 + 2^-u)."""
    return z / (1.0 + np.exp2(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp2(-z))
    return s * (1.0 + z * LN2 * (1.0 - s))


# ---------------------------------------------------------------- model parts
def features(d_abs, rho, L=1.0):
    f1 = 4.0 * np.asarray(d_abs) / L - 1.0
    f2 = 2.0 * np.log(np.asarray(rho) / (L * RHO_MIN)) / math.log(RHO_MAX / RHO_MIN) - 1.0
    return np.stack([f1, f2])


def out_scale(rho, L=1.0):
    r = np.asarray(rho) / L
    return 0.02 / (1.0 + r * r)


def baseline(d_abs, rho, L=1.0):
    """Rod baseline with the first midpoint-rule end correction, per unit
    G m / L^2; returns (b_z, b_rho) at d = +|d|."""
    d = np.asarray(d_abs, dtype=np.float64) / L
    r = np.asarray(rho, dtype=np.float64) / L
    S1, S2 = ROD_INNER, N_FAR + 0.5

    def inv(u):
        return 1.0 / np.sqrt(u * u + r * r)

    # rods on the + side (axial positions s in [S1, S2]) and - side ([-S2, -S1]):
    # int of g_z = (s - d)/|.|^3 and g_rho = -r/|.|^3 over s
    bz = inv(S1 - d) - inv(S2 - d) - inv(S1 + d) + inv(S2 + d)
    br = -(1.0 / r) * ((S2 - d) * inv(S2 - d) - (S1 - d) * inv(S1 - d)
                       + (S2 + d) * inv(S2 + d) - (S1 + d) * inv(S1 + d))
    # midpoint rule: sum_{n>=2} g(n) = int_{S1} g - (1/24)(g'(S2) - g'(S1)) + ...
    # only the inner ends are kept; g'(s) with u = s - d:
    #   d g_z / ds = (r^2 - 2 u^2)/|.|^5,   d g_rho / ds = 3 r u /|.|^5
    for side in (1.0, -1.0):
        u = side * S1 - d
        q5 = inv(u) ** 5
        # + side: + g'(S1)/24 ; - side (lower end of a rod ending at -S1): - g'(-S1)/24
        bz = bz + side * (r * r - 2.0 * u * u) * q5 / 24.0
        br = br + side * 3.0 * r * u * q5 / 24.0
    return bz, br


def exact_remainder(d, rho, L=1.0):
    """Exact 2 <= |n| <= 1024 image sum per unit G m / L^2: (R_z, R_rho)."""
    fz, fr, _ = oracle.image_band(np.asarray(d) / L, np.asarray(rho) / L, 1.0, 2, N_FAR)
    return fz, fr


def training_targets(d_abs, rho, L=1.0):
    """T = (R - b) / s for samples at d = +|d| (shape (2, n))."""
    Rz, Rr = exact_remainder(d_abs, rho, L)
    bz, br = baseline(d_abs, rho, L)
    s = out_scale(rho, L)
    return np.stack([(Rz - bz) / s, (Rr - br) / s])


# ---------------------------------------------------------------- network
def forward(params, F, bf16=False):
    """Network outputs (2, n) for features F (2, n); also returns the cache
    needed by :func:`loss_and_grad`."""
    layers = unpack(params)
    h = np.asarray(F, dtype=np.float64)
    if bf16:
        h = np.asarray(h, dtype=np.float32).astype(np.float64)
    cache = []
    for k, (W, b) in enumerate(layers):
        Wq = bf16_round(W) if bf16 else W
        bq = np.asarray(b, dtype=np.float32).astype(np.float64) if bf16 else b
        x_in = bf16_round(h) if (bf16 and 1 <= k <= DEPTH - 1) else h
        z = Wq @ x_in + bq[:, None]
        cache.append((x_in, Wq, z))
        h = silu(z) if k < DEPTH else z
    return h, cache


def loss_and_grad(params, F, T, bf16=False, round_dz=None):
    """Loss mean((o - T)^2) over both outputs and all samples, and its
    gradient with respect to the flat parameter vector.  With ``bf16`` the
    forward pass uses the rounded weights and activations and the backward
    pass treats each rounding as the identity (straight-through).
    ``round_dz`` (default: ``bf16``) also rounds the pre-activation gradients
    of layers 2-4 to BF16 before their matrix products, as BF16 matrix units
    do (dW = bf16(dz) x^T and the propagated gradient W^T bf16(dz)), while
    bias gradients and layers 1 and 5 use the unrounded values; with
    ``round_dz=False`` the backward pass is the plain FP64 one (the gradient
    the rounded variant approximates)."""
    if round_dz is None:
        round_dz = bf16
    out, cache = forward(params, F, bf16)
    T = np.asarray(T, dtype=np.float64)
    diff = out - T
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / diff.size            # d loss / d out
    grads = []
    for k in range(DEPTH, -1, -1):
        x_in, Wq, z = cache[k]
        dz = g if k == DEPTH else g * silu_grad(z)
        dzq = bf16_round(dz) if (round_dz and 1 <= k <= DEPTH - 1) else dz
        dW = dzq @ x_in.T
        db = dz.sum(axis=1)
        grads.append((dW, db))
        g = Wq.T @ dzq
    grads.reverse()
    flat = np.concatenate([np.concatenate([dW.ravel(), db.ravel()]) for dW, db in grads])
    return loss, flat


def remainder_model(params, d, rho, L=1.0, bf16=True):
    """Learned (R_z, R_rho) per unit G m / L^2 at signed offset d."""
    d = np.asarray(d, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    da = np.abs(d)
    o, _ = forward(params, features(da, rho, L), bf16)
    bz, br = baseline(da, rho, L)
    s = out_scale(rho, L)
    return np.sign(d) * (bz + s * o[0]), br + s * o[1]


# ---------------------------------------------------------------- Adam
def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) at step t >= 1; returns new copies."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- N-body
def forces_learned(pos, mass, eps, L, params, targets=None, bf16=True, n_near=1):
    """FP64 accelerations of the learned scheme: exact images |n| <= n_near
    (spline-softened, ``oracle.forces``), plus the learned remainder for
    pairs inside the network's domain and the exact 2..1024 band outside it.
    Pure NumPy over all pairs: small N only."""
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[1]
    tg = np.arange(N) if targets is None else np.asarray(targets)
    near, _ = oracle.forces(pos, mass, eps, L, n_near, targets=tg, potential=False)
    z = pos[2] - L * np.floor(pos[2] / L)
    z[z >= L] = 0.0
    acc = near.copy()
    for k, i in enumerate(tg):
        j = np.arange(N) != i
        dx = pos[0, i] - pos[0, j]
        dy = pos[1, i] - pos[1, j]
        t = z[i] - z[j]
        d = t - L * np.floor(t / L + 0.5)
        rho = np.hypot(dx, dy)
        r = rho / L
        inside = (r >= RHO_MIN) & (r <= RHO_MAX)
        Fz = np.zeros_like(d)
        Fr = np.zeros_like(d)
        if inside.any():
            Fz[inside], Fr[inside] = remainder_model(params, d[inside], rho[inside], L, bf16)
        out = ~inside
        if out.any():
            Fz[out], Fr[out] = exact_remainder(d[out], rho[out], L)
        m = mass[j] / (L * L)
        with np.errstate(invalid="ignore", divide="ignore"):
            ux = np.where(rho > 0, dx / rho, 0.0)
            uy = np.where(rho > 0, dy / rho, 0.0)
        acc[0, k] += np.sum(m * Fr * ux)
        acc[1, k] += np.sum(m * Fr * uy)
        acc[2, k] += np.sum(m * Fz)
    return acc
