"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module draws random numbers and lays out arrays; it holds none of the
force, background or network arithmetic of the method.  Every array is FP64
(positions, masses, softenings) or FP32 (network parameters) in NumPy, made by
``numpy.random.default_rng(seed)`` (PCG64) in a fixed draw order, so two calls
with the same arguments return identical bytes.

Particle loads follow the paper's cylindrical initial-load construction
(Sect. 3.1, inverse stereographic projection of the radial coordinate):
uniform in z and azimuth, the compact radial coordinate drawn so that the
surface number density falls as (1+r^2/R0^2)^-2, and masses growing as
(1+r^2/R0^2)^2 so that the mass density is flat out to the edge.  Softening
lengths scale with the cube root of the mass.
"""
from __future__ import annotations

import math

import numpy as np

R0_DEFAULT = 0.5
CHI_MAX_DEFAULT = 0.9 * math.pi


class Particles:
    """SoA particle set: ``pos`` is (3, N) FP64 (rows x, y, z), ``mass`` and
    ``eps`` are (N,) FP64, ``L`` the period along z."""

    def __init__(self, pos, mass, eps, L):
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.mass = np.ascontiguousarray(mass, dtype=np.float64)
        self.eps = np.ascontiguousarray(eps, dtype=np.float64)
        self.L = float(L)

    @property
    def N(self):
        return self.mass.shape[0]


def _radius_from_u(u, R0, chi_max):
    # chi has density proportional to sin(chi) on [0, chi_max): inverse CDF
    chi = np.arccos(1.0 - u * (1.0 - math.cos(chi_max)))
    return R0 * np.tan(0.5 * chi)


def _mass_law(r, R0):
    return (1.0 + (r / R0) ** 2) ** 2


def _softening(mass):
    return 0.01 * np.cbrt(mass / mass.min())


def cylinder_load(N, seed=0, L=1.0, R0=R0_DEFAULT, chi_max=CHI_MAX_DEFAULT, omega_c=0.0):
    """Stereographic cylinder load of ``N`` particles (total mass 1).

    ``omega_c`` > 0 adds the constant-resolution core of the paper's load
    (Sect. 3.1): inside the compact radius omega_c (physical radius
    rho_c = R0 tan(omega_c/2)) particles are uniform in area with the mass the
    outer law takes at rho_c; outside, the compact coordinate follows the
    sin(chi) law on [omega_c, chi_max).  The core holds the share of particles
    that keeps the number density continuous at rho_c,
        N_core / N_out = sin^2(omega_c) / (2 (cos omega_c - cos chi_max)),
    so the mass density stays flat across the core boundary.

    Draw order from ``default_rng(seed)``: z (N), azimuth (N), radial variate
    (N; the first N_core of them place the core particles).
    """
    rng = np.random.default_rng(seed)
    z = rng.random(N) * L
    phi = rng.random(N) * (2.0 * math.pi)
    u = rng.random(N)
    if omega_c > 0.0:
        if not omega_c < chi_max:
            raise ValueError("omega_c must lie below chi_max")
        ratio = math.sin(omega_c) ** 2 / (2.0 * (math.cos(omega_c) - math.cos(chi_max)))
        n_core = int(round(N * ratio / (1.0 + ratio)))
        rho_c = R0 * math.tan(0.5 * omega_c)
        r = np.empty(N)
        r[:n_core] = rho_c * np.sqrt(u[:n_core])
        cc = math.cos(omega_c)
        chi = np.arccos(cc - u[n_core:] * (cc - math.cos(chi_max)))
        r[n_core:] = R0 * np.tan(0.5 * chi)
        m = _mass_law(np.maximum(r, rho_c), R0)
    else:
        r = _radius_from_u(u, R0, chi_max)
        m = _mass_law(r, R0)
    pos = np.stack([r * np.cos(phi), r * np.sin(phi), z])
    m /= m.sum()
    return Particles(pos, m, _softening(m), L)


def r_max(R0=R0_DEFAULT, chi_max=CHI_MAX_DEFAULT):
    """Outer radius of the load, R0 tan(chi_max/2)."""
    return R0 * math.tan(0.5 * chi_max)


def clustered_load(N, n_clumps=64, clump_frac=0.005, scale=0.005, seed=0, L=1.0,
                   R0=R0_DEFAULT, chi_max=CHI_MAX_DEFAULT, u_max=0.999):
    """Cylinder load with ``n_clumps`` Plummer spheres of ``round(clump_frac*N)``
    particles each; the rest follow :func:`cylinder_load`.

    Clump centres are drawn from the same stereographic distribution.  Plummer
    radii come from inverting the cumulative mass profile, r = b / sqrt(u^(-2/3)-1),
    with u redrawn until u <= ``u_max`` (truncation).  Every particle takes the
    mass law at its own cylindrical radius; masses are then normalised to 1 and
    softenings recomputed.  z is wrapped into [0, L).
    """
    rng = np.random.default_rng(seed)
    per = int(round(clump_frac * N))
    n_cl = n_clumps * per
    n_bg = N - n_cl
    if n_bg < 0:
        raise ValueError("clumps hold more than N particles")
    # background
    zb = rng.random(n_bg) * L
    phib = rng.random(n_bg) * (2.0 * math.pi)
    rb = _radius_from_u(rng.random(n_bg), R0, chi_max)
    # clump centres
    zc = rng.random(n_clumps) * L
    phic = rng.random(n_clumps) * (2.0 * math.pi)
    rc = _radius_from_u(rng.random(n_clumps), R0, chi_max)
    cx, cy = rc * np.cos(phic), rc * np.sin(phic)
    # Plummer radii with truncation by redraw
    u = rng.random(n_cl)
    bad = u > u_max
    while bad.any():
        u[bad] = rng.random(int(bad.sum()))
        bad = u > u_max
    rp = scale / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    # isotropic directions
    cth = 2.0 * rng.random(n_cl) - 1.0
    ph = rng.random(n_cl) * (2.0 * math.pi)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    k = np.repeat(np.arange(n_clumps), per)
    xc = cx[k] + rp * sth * np.cos(ph)
    yc = cy[k] + rp * sth * np.sin(ph)
    zcl = np.mod(zc[k] + rp * cth, L)
    zcl[zcl >= L] = 0.0
    x = np.concatenate([rb * np.cos(phib), xc])
    y = np.concatenate([rb * np.sin(phib), yc])
    z = np.concatenate([zb, zcl])
    r = np.hypot(x, y)
    m = _mass_law(r, R0)
    m /= m.sum()
    return Particles(np.stack([x, y, z]), m, _softening(m), L)


def displaced_load(N, sigma=None, seed=0, L=1.0, R0=R0_DEFAULT, chi_max=CHI_MAX_DEFAULT):
    """:func:`cylinder_load` plus isotropic Gaussian displacements.

    ``sigma`` is the per-axis standard deviation; by default the 3D rms is half
    the global mean inter-particle spacing (pi r_max^2 L / N)^(1/3).  The
    displacement draws come from ``default_rng(seed + 1)`` after the load.
    z is wrapped into [0, L).
    """
    p = cylinder_load(N, seed=seed, L=L, R0=R0, chi_max=chi_max)
    if sigma is None:
        spacing = (math.pi * r_max(R0, chi_max) ** 2 * L / N) ** (1.0 / 3.0)
        sigma = 0.5 * spacing / math.sqrt(3.0)
    rng = np.random.default_rng(seed + 1)
    pos = p.pos + sigma * rng.standard_normal((3, N))
    pos[2] = np.mod(pos[2], L)
    pos[2][pos[2] >= L] = 0.0
    return Particles(pos, p.mass, p.eps, L)


def target_sample(N, k, seed=0):
    """``k`` distinct target indices in [0, N), sorted, as int64."""
    rng = np.random.default_rng(seed)
    k = min(k, N)
    return np.sort(rng.choice(N, size=k, replace=False)).astype(np.int64)


def tiny_load(N, seed=0, L=1.0, box=1.0):
    """Small random set for brute-force checks: x, y ~ U(-box, box), z ~ U[0, L),
    masses ~ U(0.5, 1.5), softenings ~ U(0.02, 0.08)."""
    rng = np.random.default_rng(seed)
    x = (2.0 * rng.random(N) - 1.0) * box
    y = (2.0 * rng.random(N) - 1.0) * box
    z = rng.random(N) * L
    m = 0.5 + rng.random(N)
    eps = 0.02 + 0.06 * rng.random(N)
    return Particles(np.stack([x, y, z]), m, eps, L)


# --------------------------------------------------------------------------
# network-side random draws (initial parameters, training inputs)
# --------------------------------------------------------------------------

MLP_WIDTH = 64
MLP_DEPTH = 4   # hidden layers
MLP_IN = 2
MLP_OUT = 2


def mlp_param_shapes(width=MLP_WIDTH, depth=MLP_DEPTH):
    """(name, shape) of every parameter tensor in storage order.  Weight
    matrices are (fan_out, fan_in), row-major."""
    shapes = [("W1", (width, MLP_IN)), ("b1", (width,))]
    for k in range(2, depth + 1):
        shapes += [(f"W{k}", (width, width)), (f"b{k}", (width,))]
    shapes += [(f"W{depth + 1}", (MLP_OUT, width)), (f"b{depth + 1}", (MLP_OUT,))]
    return shapes


def mlp_param_count(width=MLP_WIDTH, depth=MLP_DEPTH):
    return int(sum(np.prod(s) for _, s in mlp_param_shapes(width, depth)))


def mlp_init(seed=0, width=MLP_WIDTH, depth=MLP_DEPTH, out_gain=0.1):
    """Flat FP32 parameter vector: weights ~ U(-a, a) with a = sqrt(6/fan_in)
    for hidden layers and ``out_gain*sqrt(3/fan_in)`` for the output layer;
    biases ~ U(-0.1, 0.1) for hidden layers, zero for the output layer."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in mlp_param_shapes(width, depth):
        last = name.endswith(str(depth + 1))
        if name.startswith("W"):
            a = math.sqrt(6.0 / shape[1])
            if last:
                a = out_gain * math.sqrt(3.0 / shape[1])
            parts.append(rng.uniform(-a, a, size=shape).ravel())
        else:
            if last:
                parts.append(np.zeros(shape))
            else:
                parts.append(rng.uniform(-0.1, 0.1, size=shape))
    return np.concatenate(parts).astype(np.float32)


def remainder_inputs(n, seed=0, rho_min=0.05, rho_max=20.0, pair_load=None):
    """Training/validation inputs (|d|/L, rho/L), shape (2, n) FP64.

    Half are uniform in |d|/L on [0, 0.5] and log-uniform in rho/L on
    [rho_min, rho_max]; the other half are separations of random pairs of
    ``pair_load`` (a :class:`Particles`, default the 4096-particle cylinder
    load), min-imaged along z, with rho outside [rho_min, rho_max] redrawn.
    """
    rng = np.random.default_rng(seed)
    n1 = n // 2
    n2 = n - n1
    d1 = 0.5 * rng.random(n1)
    r1 = np.exp(math.log(rho_min) + (math.log(rho_max) - math.log(rho_min)) * rng.random(n1))
    if pair_load is None:
        pair_load = cylinder_load(4096, seed=0)
    P = pair_load
    d2 = np.empty(n2)
    r2 = np.empty(n2)
    filled = 0
    while filled < n2:
        want = n2 - filled
        i = rng.integers(0, P.N, size=2 * want)
        j = rng.integers(0, P.N, size=2 * want)
        dx = P.pos[0, i] - P.pos[0, j]
        dy = P.pos[1, i] - P.pos[1, j]
        t = (P.pos[2, i] - P.pos[2, j]) / P.L
        dz = np.abs(t - np.floor(t + 0.5))
        rr = np.hypot(dx, dy) / P.L
        ok = (rr >= rho_min) & (rr <= rho_max) & (i != j)
        take = np.flatnonzero(ok)[:want]
        d2[filled:filled + take.size] = dz[take]
        r2[filled:filled + take.size] = rr[take]
        filled += take.size
    d = np.concatenate([d1, d2])
    r = np.concatenate([r1, r2])
    perm = rng.permutation(n)
    return np.ascontiguousarray(np.stack([d[perm], r[perm]]))
