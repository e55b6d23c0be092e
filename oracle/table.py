"""FP64 oracle of the tabulated far-image correction.

TEST INFRASTRUCTURE (see the package docstring).

The paper adds the contribution of distant periodic images to the
nearest-image forces through a correction vector D(rho, z) tabulated on an
equally spaced grid in the cylindrical coordinates and interpolated with the
cloud-in-cell (CIC) or triangular-shaped-cloud (TSC) scheme (Sect. 2.2, eq.
S1R2EwaldCorrectionTable).  Here the tabulated quantity is the image band
2 <= |n| <= n_far of eq. ForceCylindrical for one unit mass, as a function of
delta = |d|/L in [0, 1/2] and r = rho/L in [0, r_max] (per unit G m / L^2):

    T_z(delta, r)   = sum -(delta - n) / r_n^3,   T_rho = sum -r / r_n^3,

with R_z = sign(d) T_z(|d|/L, rho/L) and R_rho = T_rho (the band is odd in d
for z and even for rho).  Nodes sit at delta_i = i * h_d (i = -1..n_d + 1,
h_d = 0.5 / n_d) and r_j = j * h_r (j = -1..n_r + 1, h_r = r_max / n_r);
the nodes outside the domain are the band evaluated there (the formula holds
for any delta and signed r), so TSC needs no special edge rule.

CIC: bilinear weights of the cell containing the point.
TSC: the nearest node k and its neighbours with weights
    w_{k-1} = (1/2 - f)^2 / 2,  w_k = 3/4 - f^2,  w_{k+1} = (1/2 + f)^2 / 2,
    f = x - k in [-1/2, 1/2], per axis, product over the two axes.
Pairs with r > r_max use the exact band.

A table of the complete correction (every image |n| >= 2, N_cut -> inf) is
built from the Ewald split of ``oracle.ewald`` (``Table.ewald``); its pairs
beyond r_max take the complete band from ``oracle.ewald.band_direct``.
"""
from __future__ import annotations

import numpy as np

import oracle

N_FAR = 1024


class Table:
    def __init__(self, n_d, n_r, r_max, n_far=N_FAR, _nodes=None):
        self.n_d, self.n_r, self.r_max, self.n_far = int(n_d), int(n_r), float(r_max), int(n_far)
        self.h_d = 0.5 / self.n_d
        self.h_r = self.r_max / self.n_r
        self.complete = _nodes is not None
        D, R = self.grid()
        if _nodes is None:
            fz, fr, _ = oracle.image_band(D.ravel(), R.ravel(), 1.0, 2, self.n_far)
        else:
            fz, fr = _nodes(D.ravel(), R.ravel())
        self.Tz = fz.reshape(D.shape)           # index [j + 1][i + 1]
        self.Tr = fr.reshape(D.shape)

    def grid(self):
        """Node coordinates (delta, r), each [n_r + 3][n_d + 3]."""
        di = np.arange(-1, self.n_d + 2) * self.h_d
        rj = np.arange(-1, self.n_r + 2) * self.h_r
        return np.meshgrid(di, rj)

    @classmethod
    def ewald(cls, n_d, n_r, r_max, alpha, n_max, m_max, kernel="corrected"):
        """Table of the complete band (|n| >= 2) by the Ewald split; nodes at
        negative r take the odd/even continuation (T_rho odd, T_z even)."""
        from oracle import ewald as ew

        def nodes(D, R):
            fz = np.empty(D.size)
            fr = np.empty(D.size)
            for q, (d, r) in enumerate(zip(D, R)):
                z, p = ew.band_ewald(d, abs(r), alpha, n_max, m_max, kernel)
                fz[q] = z
                fr[q] = p if r >= 0 else -p
            return fz, fr
        return cls(n_d, n_r, r_max, 0, _nodes=nodes)


def _node(T, j, i):
    return T[j + 1, i + 1]


def interpolate(tab, delta, r, order):
    """(T_z, T_rho) at arrays delta in [0, 1/2], r in [0, r_max]."""
    delta = np.asarray(delta, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    x = delta / tab.h_d
    y = r / tab.h_r
    out_z = np.zeros_like(x)
    out_r = np.zeros_like(x)
    if order == 1:
        i0 = np.minimum(np.floor(x).astype(int), tab.n_d - 1)
        j0 = np.minimum(np.floor(y).astype(int), tab.n_r - 1)
        fx, fy = x - i0, y - j0
        for di, wx in ((0, 1.0 - fx), (1, fx)):
            for dj, wy in ((0, 1.0 - fy), (1, fy)):
                w = wx * wy
                out_z += w * _node(tab.Tz, j0 + dj, i0 + di)
                out_r += w * _node(tab.Tr, j0 + dj, i0 + di)
    elif order == 2:
        i0 = np.rint(x).astype(int)
        j0 = np.rint(y).astype(int)
        fx, fy = x - i0, y - j0

        def weights(f):
            return ((-1, 0.5 * (0.5 - f) ** 2), (0, 0.75 - f * f), (1, 0.5 * (0.5 + f) ** 2))
        for di, wx in weights(fx):
            for dj, wy in weights(fy):
                w = wx * wy
                out_z += w * _node(tab.Tz, j0 + dj, i0 + di)
                out_r += w * _node(tab.Tr, j0 + dj, i0 + di)
    else:
        raise ValueError("order must be 1 (CIC) or 2 (TSC)")
    return out_z, out_r


def band_pairs(dx, dy, d, L, tab, order):
    """Band acceleration per unit source mass for pair separations (dx, dy)
    and minimum-image axial offsets d (arrays): the interpolated table where
    rho/L <= r_max, the exact band beyond (the complete band for a complete
    table).  Returns (ax, ay, az) per unit G m."""
    dx = np.asarray(dx, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    rho = np.hypot(dx, dy)
    r = rho / L
    inside = r <= tab.r_max
    Fz = np.zeros_like(d)
    Fr = np.zeros_like(d)
    if inside.any():
        tz, tr = interpolate(tab, np.abs(d[inside]) / L, r[inside], order)
        Fz[inside] = np.sign(d[inside]) * tz
        Fr[inside] = tr
    out = ~inside
    if out.any():
        if tab.complete:
            from oracle import ewald as ew
            Fz[out], Fr[out] = ew.band_direct(d[out] / L, r[out])
        else:
            Fz[out], Fr[out], _ = oracle.image_band(d[out] / L, r[out], 1.0, 2, tab.n_far)
    with np.errstate(invalid="ignore", divide="ignore"):
        ux = np.where(rho > 0, dx / rho, 0.0)
        uy = np.where(rho > 0, dy / rho, 0.0)
    s = 1.0 / (L * L)
    return s * Fr * ux, s * Fr * uy, s * Fz


def forces_table(pos, mass, eps, L, tab, order, targets=None):
    """FP64 accelerations of the tabulated scheme: exact images |n| <= 1
    (spline-softened) plus the interpolated band for pairs with
    rho/L <= r_max and the exact band otherwise.  NumPy over all pairs."""
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[1]
    tg = np.arange(N) if targets is None else np.asarray(targets)
    near, _ = oracle.forces(pos, mass, eps, L, 1, targets=tg, potential=False)
    z = pos[2] - L * np.floor(pos[2] / L)
    z[z >= L] = 0.0
    acc = near.copy()
    for k, i in enumerate(tg):
        j = np.arange(N) != i
        t = z[i] - z[j]
        d = t - L * np.floor(t / L + 0.5)
        bx, by, bz = band_pairs(pos[0, i] - pos[0, j], pos[1, i] - pos[1, j], d, L, tab, order)
        acc[0, k] += np.sum(mass[j] * bx)
        acc[1, k] += np.sum(mass[j] * by)
        acc[2, k] += np.sum(mass[j] * bz)
    return acc
