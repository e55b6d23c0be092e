"""FP64 oracle of the comoving background terms and the leapfrog step.

TEST INFRASTRUCTURE (see the package docstring).

* ``cylinder_field``: radial field F_h of a homogeneous cylinder of radius R,
  half-height Z and density rho0 in its mid-plane, the pull that the
  truncated image sum adds and the equations of motion subtract (Sect. 2.1,
  eqs. F_horiz and F_horiz_infty).  Written from the direct integration of
  vertical line elements over chords of the disk:

      F_h(rho) = 2 G rho0 [ 2 A - B ],
      A = int_0^R ln( (sqrt(Z^2 + w+) + Z) / (sqrt(Z^2 + w-) + Z) ) dY,
      B = int_0^R ln( w+ / w- ) dY,
      w+- = R^2 + rho^2 +- 2 rho sqrt(R^2 - Y^2).

  As Z -> infinity, A -> 0 and F_h -> -2 pi G rho0 rho inside (the printed
  limit).  The printed finite-Z form carries the opposite overall sign and
  half of the B term (it writes ln(sqrt(w+)/sqrt(w-))); it tends to
  +pi G rho0 rho, so it cannot be the field it describes.  It is kept as
  ``cylinder_field_printed`` to document that reading.
* ``hubble`` / ``omega_de``: the Friedmann equation with CPL dark energy
  (Sect. 2.3, eqs. Friedmann, DEdensity, CPLw0wa), the dark-energy integral
  evaluated by quadrature as printed.
* ``kdk_factors``: cosmic-time kick and drift integrals for one leapfrog step
  from a_begin to a_end: the step length dt = t(a_end) - t(a_begin), then the
  Friedmann equation da/dt = a H(a) advanced with fourth-order Runge-Kutta
  (the scheme of Sect. 2.3) together with int dt/a and int dt/a^2, in
  ``n_sub`` sub-steps per half step.
* ``kdk_step``: one kick-drift-kick step (Sect. 2.1, end) of
      dp/dt = (g(x) - F_h(x)) / a,   dx/dt = p / a^2,
  with p = a^2 dx/dt; g is the pair-sum acceleration at unit scale factor
  and F_h the compensation, both scaled by a^-3 in the equation of motion
  of x (the compensation must cancel the homogeneous pull at every epoch).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

import oracle


# ---------------------------------------------------------------- F_h
def _w(rho, R, Y):
    # w- = R^2 + rho^2 - 2 rho c written without cancellation:
    # (R - rho)^2 + 2 rho (R - c), with R - c = Y^2 / (R + c)
    c = math.sqrt(max(R * R - Y * Y, 0.0))
    return R * R + rho * rho + 2.0 * rho * c, (R - rho) ** 2 + 2.0 * rho * Y * Y / (R + c)


def cylinder_field(rho, R, Z, rho0, G=1.0):
    """Radial field (negative = inward) at cylindrical radius ``rho`` in the
    mid-plane of a homogeneous cylinder (radius R, half-height Z, density rho0)."""
    rho = float(rho)
    if rho == 0.0:
        return 0.0

    def fa(Y):
        wp, wm = _w(rho, R, Y)
        return math.log((math.sqrt(Z * Z + wp) + Z) / (math.sqrt(Z * Z + wm) + Z))

    def fb(Y):
        wp, wm = _w(rho, R, Y)
        return math.log(wp / wm)

    # the end-cap term vanishes for an infinite cylinder (Z -> inf)
    A = 0.0 if math.isinf(Z) else integrate.quad(fa, 0.0, R, epsabs=1e-15, epsrel=1e-12, limit=400)[0]
    if rho == R:
        # on the mantle w- = Y^2 2R / (R + c): take the log singularity out,
        # int_0^R -2 ln Y dY = -2 (R ln R - R)
        def fs(Y):
            c = math.sqrt(max(R * R - Y * Y, 0.0))
            return math.log((R * R + rho * rho + 2.0 * rho * c) * (R + c) / (2.0 * R))

        B = integrate.quad(fs, 0.0, R, epsabs=1e-15, epsrel=1e-12, limit=400)[0] - 2.0 * (R * math.log(R) - R)
    else:
        B = integrate.quad(fb, 0.0, R, epsabs=1e-15, epsrel=1e-12, limit=400)[0]
    return 2.0 * G * rho0 * (2.0 * A - B)


def cylinder_field_printed(rho, R, Z, rho0, G=1.0):
    """The finite-height formula exactly as printed (see module docstring)."""
    def f1(Y):
        c = math.sqrt(max(R * R - Y * Y, 0.0))
        return math.log((math.sqrt(Z * Z + R * R + rho * rho + 2 * rho * c) + Z)
                        / (math.sqrt(Z * Z + R * R + rho * rho - 2 * rho * c) + Z))

    def f2(Y):
        c = math.sqrt(max(R * R - Y * Y, 0.0))
        return math.log(math.sqrt(R * R + rho * rho + 2 * rho * c)
                        / math.sqrt(R * R + rho * rho - 2 * rho * c))

    I1, _ = integrate.quad(f1, 0.0, R, epsrel=1e-13, limit=400)
    I2, _ = integrate.quad(f2, 0.0, R, epsrel=1e-13, limit=400)
    return 2.0 * G * rho0 * (-2.0 * I1 + I2)


def compensation(pos, R, Z, rho0, G=1.0):
    """F_h as a vector field at the particle positions (3, N): radial in x, y,
    zero along z."""
    x, y = pos[0], pos[1]
    rho = np.hypot(x, y)
    fr = np.array([cylinder_field(r, R, Z, rho0, G) for r in rho])
    out = np.zeros_like(pos)
    nz = rho > 0
    out[0, nz] = fr[nz] * x[nz] / rho[nz]
    out[1, nz] = fr[nz] * y[nz] / rho[nz]
    return out


# ---------------------------------------------------------------- Friedmann
class Cosmology:
    """H0 and density parameters; CPL dark energy w(a) = w0 + wa (1 - a)."""

    def __init__(self, H0, Om, OL, Or=0.0, Ok=0.0, w0=-1.0, wa=0.0):
        self.H0, self.Om, self.OL, self.Or, self.Ok = H0, Om, OL, Or, Ok
        self.w0, self.wa = w0, wa


def omega_de(a, c):
    """Omega_DE(a) = Omega_DE,0 exp(-3 int_1^a (1 + w(a'))/a' da')."""
    if c.w0 == -1.0 and c.wa == 0.0:
        return c.OL
    val, _ = integrate.quad(lambda x: (1.0 + c.w0 + c.wa * (1.0 - x)) / x, 1.0, a,
                            epsabs=1e-16, epsrel=1e-13)
    return c.OL * math.exp(-3.0 * val)


def hubble(a, c):
    return c.H0 * math.sqrt(c.Or * a ** -4 + c.Om * a ** -3 + c.Ok * a ** -2 + omega_de(a, c))


def cosmic_time(a, c):
    """t(a) = int_0^a da' / (a' H(a'))."""
    val, _ = integrate.quad(lambda x: 1.0 / (x * hubble(x, c)), 0.0, a, epsabs=1e-16,
                            epsrel=1e-13, limit=200)
    return val


def kdk_factors(a_begin, a_end, c, n_sub=64):
    """(K1, D, K2): int dt/a over the first half step, int dt/a^2 over the
    whole step and int dt/a over the second half, cosmic time."""
    dt = cosmic_time(a_end, c) - cosmic_time(a_begin, c)

    def rhs(y):
        a = y[0]
        return np.array([a * hubble(a, c), 1.0 / a, 1.0 / (a * a)])

    def advance(a0, span):
        y = np.array([a0, 0.0, 0.0])
        h = span / n_sub
        for _ in range(n_sub):
            k1 = rhs(y)
            k2 = rhs(y + 0.5 * h * k1)
            k3 = rhs(y + 0.5 * h * k2)
            k4 = rhs(y + h * k3)
            y = y + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        return y

    y1 = advance(a_begin, 0.5 * dt)
    y2 = advance(y1[0], 0.5 * dt)
    return y1[1], y1[2] + y2[2], y2[1]


def lcdm_scale_factor(t, c):
    """Closed form of flat LCDM (Or = Ok = 0, w = -1)."""
    return (c.Om / c.OL) ** (1.0 / 3.0) * math.sinh(1.5 * math.sqrt(c.OL) * c.H0 * t) ** (2.0 / 3.0)


# ---------------------------------------------------------------- leapfrog
def kdk_step(pos, mom, mass, eps, L, n_img, a_begin, a_end, c, R, rho0, Z, acc=None,
             compensate=True, factors=None):
    """One KDK step in FP64.  ``pos`` and ``mom`` are (3, N); ``acc`` the pair
    acceleration at ``pos`` (computed when None); ``factors`` (K1, D, K2)
    replaces the Friedmann solution (e.g. from ``history_factors``).  Returns
    (pos, mom, acc_new)."""
    K1, D, K2 = kdk_factors(a_begin, a_end, c) if factors is None else factors
    if acc is None:
        acc, _ = oracle.forces(pos, mass, eps, L, n_img, potential=False)
    comp = compensation(pos, R, Z, rho0) if compensate else 0.0
    mom = mom + K1 * (acc - comp)
    pos = pos + D * mom
    z = pos[2] - L * np.floor(pos[2] / L)
    z[z >= L] = 0.0
    pos = np.stack([pos[0], pos[1], z])
    acc_new, _ = oracle.forces(pos, mass, eps, L, n_img, potential=False)
    comp = compensation(pos, R, Z, rho0) if compensate else 0.0
    mom = mom + K2 * (acc_new - comp)
    return pos, mom, acc_new


# ---------------------------------------------------------------- tabulated history
def history_interp(t_nodes, a_nodes, order, t):
    """a(t) from a tabulated expansion history (Sect. 2.3: histories loaded from
    a table and interpolated linearly, quadratically or cubically).  On the
    interval [t_k, t_k+1] the interpolant is the Lagrange polynomial through
    nodes k..k+1 (order 1), k..k+2 (order 2) or k-1..k+2 (order 3), the
    stencil shifted inwards at the ends of the table."""
    tn = np.asarray(t_nodes, dtype=np.float64)
    an = np.asarray(a_nodes, dtype=np.float64)
    n = tn.size
    k = int(np.clip(np.searchsorted(tn, t, side="right") - 1, 0, n - 2))
    first = {1: k, 2: k, 3: k - 1}[order]
    first = int(np.clip(first, 0, n - 1 - order))
    idx = range(first, first + order + 1)
    val = 0.0
    for p in idx:
        w = 1.0
        for q in idx:
            if q != p:
                w *= (t - tn[q]) / (tn[p] - tn[q])
        val += w * an[p]
    return val


def history_factors(t_nodes, a_nodes, order, a_begin, a_end):
    """(K1, D, K2) of one KDK step from a_begin to a_end on a tabulated history:
    t(a) by root finding on the interpolant, then int dt/a and int dt/a^2 by
    adaptive quadrature of the interpolant."""
    from scipy import optimize
    tn = np.asarray(t_nodes, dtype=np.float64)

    def t_of(a):
        return optimize.brentq(lambda t: history_interp(tn, a_nodes, order, t) - a, tn[0], tn[-1],
                               xtol=1e-15, rtol=1e-15)

    t0, t1 = t_of(a_begin), t_of(a_end)
    tm = 0.5 * (t0 + t1)
    pts = [x for x in tn if min(t0, t1) < x < max(t0, t1)]

    def integ(lo, hi, p):
        f = lambda t: history_interp(tn, a_nodes, order, t) ** (-p)
        inner = [x for x in pts if min(lo, hi) < x < max(lo, hi)]
        val, _ = integrate.quad(f, lo, hi, points=inner or None, epsabs=1e-15, epsrel=1e-13, limit=400)
        return val

    return integ(t0, tm, 1), integ(t0, t1, 2), integ(tm, t1, 1)
