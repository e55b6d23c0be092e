"""FP64 oracle of the S1 x R2 Ewald summation and of the complete image sum.

TEST INFRASTRUCTURE (see the package docstring).

The force of a unit point mass and all its periodic images along z (period
L, G = 1) at axial offset d and radial distance rho is split (Sect. 2.2, eq.
cylindricalEwaldSplit) into

  * a real-space part over the images n = -n_max..n_max (eq. EwaldRealSum):
        F = sum_n -s_n / |s_n|^3 * Q(3/2, alpha^2 |s_n|^2),   s_n = (rho, d - n L),
    where Q(3/2, x^2) = erfc(x) + 2 x exp(-x^2) / sqrt(pi) is the regularised
    upper incomplete gamma function;
  * a Fourier part over k_m = 2 pi m / L, m = 1..m_max (eq. EwaldRecSum);
  * the m = 0 mode, F_rho = -2 (1 - exp(-alpha^2 rho^2)) / (L rho).

Fourier kernel.  Poisson summation of the smooth part erf(alpha r)/r over the
images gives, per mode, the potential -(2/L) cos(k_m d) B(k_m, rho) with the
incomplete Bessel function

    B(k, rho) = int_{1/(4 alpha^2)}^inf exp(-k^2 t - rho^2 / (4 t)) dt / (2 t),

which tends to K0(k rho) as alpha -> inf; the two modes +-m give the force
(4/L) grad[cos(k_m d) B(k_m, rho)].  This is the "corrected" kernel.  The
kernel printed in eq. Bkernel,
    B_p = exp(k rho) erfc(k/(2 alpha) + alpha rho) + exp(-k rho) erfc(k/(2 alpha) - alpha rho),
with the printed prefactor -(2/L) grad[cos(k_m d) B_p], is the Fourier
kernel of a different geometry (one periodic plane pair, not a periodic
line); the sum built on it depends on alpha.  It is kept as the option
kernel="printed" so that the alpha scan of Fig. 2 can be reproduced; the
complete sum uses the corrected kernel.

The complete sum has the closed form of a periodic line of masses (the
modified Bessel series)
    F_rho = -2/(L rho) - (4/L) sum_m k_m K1(k_m rho) cos(k_m d),
    F_z   = -(4/L) sum_m k_m K0(k_m rho) sin(k_m d),
implemented here with the library Bessel functions as an independent check.

The "band" is the complete sum minus the three nearest images n = -1, 0, 1
(Newtonian, about the given d): the quantity a table of the complete
correction stores (eq. S1R2EwaldCorrectionTable with the images |n| <= 1
computed exactly).  Lengths are in units of L below (L = 1).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special

import oracle


# ---------------------------------------------------------------- closed form
def line_series(d, rho, m_max=None):
    """(F_z, F_rho) of the complete periodic line by the Bessel series; rho > 0.
    ``m_max`` defaults to the number of modes that bring k_m rho past 40."""
    if m_max is None:
        m_max = max(8, int(math.ceil(40.0 / (2.0 * math.pi * rho))) + 4)
    k = 2.0 * math.pi * np.arange(1, m_max + 1)
    fr = -2.0 / rho - 4.0 * np.sum(k * special.k1(k * rho) * np.cos(k * d))
    fz = -4.0 * np.sum(k * special.k0(k * rho) * np.sin(k * d))
    return float(fz), float(fr)


# ---------------------------------------------------------------- Ewald parts
def real_part(d, rho, alpha, n_max, skip_near=False):
    """Real-space sum over n = -n_max..n_max.  With ``skip_near`` the images
    |n| <= 1 enter as (Ewald term - Newtonian term), i.e. the real-space
    part of the band."""
    fz = fr = 0.0
    for n in range(-n_max, n_max + 1):
        u = d - n
        r2 = u * u + rho * rho
        if r2 == 0.0:
            continue  # the s_n -> 0 limit of the (subtracted) term is zero
        r = math.sqrt(r2)
        w = special.gammaincc(1.5, alpha * alpha * r2)
        if skip_near and abs(n) <= 1:
            w = -special.gammainc(1.5, alpha * alpha * r2)  # Q - 1 = -P
        fz += -u / (r2 * r) * w
        fr += -rho / (r2 * r) * w
    return fz, fr


def bessel_incomplete(k, rho, alpha):
    """(B, dB/drho) of the corrected kernel by adaptive quadrature, written in
    s = ln(4 alpha^2 t): B = 1/2 int_0^inf exp(-c e^s - b e^-s) ds with
    c = k^2/(4 alpha^2), b = alpha^2 rho^2."""
    c = k * k / (4.0 * alpha * alpha)
    b = alpha * alpha * rho * rho
    # the integrand is negligible once c e^s exceeds 800
    s_end = max(math.log(800.0 / c), 1.0)

    def f(s):
        return math.exp(-c * math.exp(s) - b * math.exp(-s))

    def g(s):
        return math.exp(-c * math.exp(s) - b * math.exp(-s) - s)
    pts = [x for x in (0.5 * math.log(b / c) if b > 0 else None,) if x is not None and 0 < x < s_end]
    kw = dict(epsabs=0.0, epsrel=1e-13, limit=400, points=pts or None)
    B = 0.5 * integrate.quad(f, 0.0, s_end, **kw)[0]
    dB = -alpha * alpha * rho * integrate.quad(g, 0.0, s_end, **kw)[0]
    return B, dB


def printed_kernel(k, rho, alpha):
    """(B_p, dB_p/drho) of the printed kernel, written overflow-free with the
    scaled complementary error function: exp(k rho) erfc(a+) =
    exp(-k^2/(4 alpha^2) - alpha^2 rho^2) erfcx(a+), a+- = k/(2 alpha) +- alpha rho."""
    ap = k / (2.0 * alpha) + alpha * rho
    am = k / (2.0 * alpha) - alpha * rho
    t1 = math.exp(-k * k / (4.0 * alpha * alpha) - alpha * alpha * rho * rho) * special.erfcx(ap)
    t2 = math.exp(-k * rho) * special.erfc(am)
    # the Gaussian terms of the two derivatives cancel
    return t1 + t2, k * (t1 - t2)


def fourier_part(d, rho, alpha, m_max, kernel="corrected"):
    fz = fr = 0.0
    for m in range(1, m_max + 1):
        k = 2.0 * math.pi * m
        if kernel == "corrected":
            B, dB = bessel_incomplete(k, rho, alpha)
            pre = 4.0
        elif kernel == "printed":
            B, dB = printed_kernel(k, rho, alpha)
            pre = -2.0
        else:
            raise ValueError("kernel: 'corrected' or 'printed'")
        fz += pre * (-k * math.sin(k * d)) * B
        fr += pre * math.cos(k * d) * dB
    return fz, fr


def zero_mode(rho, alpha):
    if rho == 0.0:
        return 0.0
    return 2.0 * math.expm1(-alpha * alpha * rho * rho) / rho


def ewald(d, rho, alpha, n_max, m_max, kernel="corrected"):
    """(F_z, F_rho) of the complete sum by the Ewald split."""
    rz, rr = real_part(d, rho, alpha, n_max)
    fz, fr = fourier_part(d, rho, alpha, m_max, kernel)
    return rz + fz, rr + fr + zero_mode(rho, alpha)


def band_ewald(delta, r, alpha, n_max, m_max, kernel="corrected"):
    """Complete sum minus the images |n| <= 1, by the Ewald split (r >= 0)."""
    rz, rr = real_part(delta, r, alpha, n_max, skip_near=True)
    fz, fr = fourier_part(delta, r, alpha, m_max, kernel)
    return rz + fz, rr + fr + zero_mode(r, alpha)


# ---------------------------------------------------------------- direct sum
def rod_tail(delta, r, n_far):
    """Images |n| > n_far as two rods from n_far + 1/2 outwards (midpoint rule)
    with the first Euler-Maclaurin end correction f'(n_far + 1/2)/24.

    Per side (sign sgn, rod end at s = sgn S, u = delta - sgn S,
    q = sqrt(u^2 + r^2)): the rod integrals are F_z = sgn/q and
    F_rho = -r/(q (q + |u|)) (the cancellation-free form of -(1 - |u|/q)/r),
    and the end corrections sgn (r^2 - 2u^2)/(24 q^5) and -sgn 3 r u/(24 q^5)."""
    delta = np.asarray(delta, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    S = n_far + 0.5
    fz = np.zeros(np.broadcast(delta, r).shape)
    fr = np.zeros_like(fz)
    for sgn in (1.0, -1.0):
        u = delta - sgn * S
        q = np.sqrt(u * u + r * r)
        q5 = q ** -5
        fz += sgn / q + sgn * (r * r - 2.0 * u * u) * q5 / 24.0
        fr += -r / (q * (q + np.abs(u))) - sgn * 3.0 * r * u * q5 / 24.0
    return fz, fr


def band_direct(delta, r, n_far=65536):
    """Complete sum minus the images |n| <= 1 as the direct sum over
    2 <= |n| <= n_far plus the rod tail (FP64)."""
    fz, fr, _ = oracle.image_band(delta, r, 1.0, 2, n_far)
    tz, tr = rod_tail(delta, r, n_far)
    return fz + tz, fr + tr


def forces_complete(pos, mass, eps, L, targets=None, n_far=65536):
    """FP64 accelerations of the complete image sum (N_cut -> inf): the
    spline-softened images |n| <= 1 of ``oracle.forces`` plus, per pair, the
    complete band of ``band_direct`` (every image is Newtonian beyond the
    nearest three when h_ij <= L/2)."""
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[1]
    tg = np.arange(N) if targets is None else np.asarray(targets)
    acc, _ = oracle.forces(pos, mass, eps, L, 1, targets=tg, potential=False)
    z = pos[2] - L * np.floor(pos[2] / L)
    z[z >= L] = 0.0
    for k, i in enumerate(tg):
        j = np.arange(N) != i
        dx = pos[0, i] - pos[0, j]
        dy = pos[1, i] - pos[1, j]
        t = z[i] - z[j]
        d = t - L * np.floor(t / L + 0.5)
        rho = np.hypot(dx, dy)
        Fz, Fr = band_direct(d / L, rho / L, n_far)
        m = mass[j] / (L * L)
        with np.errstate(invalid="ignore", divide="ignore"):
            ux = np.where(rho > 0, dx / rho, 0.0)
            uy = np.where(rho > 0, dy / rho, 0.0)
        acc[0, k] += np.sum(m * Fr * ux)
        acc[1, k] += np.sum(m * Fr * uy)
        acc[2, k] += np.sum(m * Fz)
    return acc
