"""FP64 CPU oracle for the cylindrical direct-sum gravity, its far-image
remainder, the homogeneous-cylinder compensation, the background cosmology, the
leapfrog step and the correction network.

TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check and the CPU-baseline leg
of the benchmark may import or run anything in this package.  It shares no
code with the GPU library (``paper_2602_20787_amd``) and never imports it.

The pair sums live in ``forces_oracle.c`` (plain C, FP64, OpenMP over
targets only), loaded here through ctypes; the rest is NumPy/SciPy in FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "forces_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Plain build: no fast-math, no FMA contraction, so every operation rounds as
# written.
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared"]


def build(force=False):
    """Compile ``forces_oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_forces.argtypes = [dp, dp, dp, dp, dp, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, lp, ctypes.c_int64, dp, dp]
        lib.oracle_forces.restype = ctypes.c_int
        lib.oracle_image_band.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_int, ctypes.c_int, dp, dp, dp]
        lib.oracle_image_band.restype = ctypes.c_int
        lib.oracle_pairs.argtypes = [dp, dp, dp, dp, lp, ctypes.c_int64, dp, dp, dp, dp, dp, lp,
                                     ctypes.c_int64, ctypes.c_double, ctypes.c_int, dp]
        lib.oracle_pairs.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        for name in ("oracle_spline_force", "oracle_spline_potential"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_double, ctypes.c_double]
            f.restype = ctypes.c_double
        for name in ("oracle_wrap_position", "oracle_min_image"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_double, ctypes.c_double]
            f.restype = ctypes.c_double
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads():
    """Threads the oracle's parallel loops use."""
    return int(_load().oracle_num_threads())


def spline_force(r, h):
    """F(r, h) of the cubic-spline softening, per unit G m (Sect. 2.1)."""
    lib = _load()
    return float(lib.oracle_spline_force(float(r), float(h)))


def spline_potential(r, h):
    """P(r, h) with dP/dr = F and P(inf) = 0, per unit G m."""
    lib = _load()
    return float(lib.oracle_spline_potential(float(r), float(h)))


def wrap_position(z, L):
    return float(_load().oracle_wrap_position(float(z), float(L)))


def min_image(t, L):
    return float(_load().oracle_min_image(float(t), float(L)))


def forces(pos, mass, eps, L, n_img, targets=None, window=0, potential=True):
    """FP64 accelerations (3, T) and potentials (T,) of the targets (all
    particles when ``targets`` is None), G = 1.

    ``pos`` is (3, N) FP64 SoA; ``eps`` are the per-particle softening lengths
    h_i (pair softening h_i + h_j).  ``window`` 0 is |n| <= n_img about the
    minimum image, 1 the literal N_cut condition with N_cut = n_img.
    """
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    N = mass.shape[0]
    if targets is None:
        T = N
        tp = None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        T = targets.shape[0]
        tp = targets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    acc = np.zeros(3 * T)
    pot = np.zeros(T) if potential else None
    x, y, z = (np.ascontiguousarray(pos[k]) for k in range(3))
    rc = lib.oracle_forces(_dptr(x), _dptr(y), _dptr(z), _dptr(mass), _dptr(eps),
                           N, float(L), int(n_img), int(window), tp, T, _dptr(acc),
                           _dptr(pot) if pot is not None else None)
    if rc != 0:
        raise ValueError("oracle_forces rejected its arguments")
    return acc.reshape(3, T), pot


def pairs(tpos, th, tid, spos, sm, sh, sid, L, n_img, acc=None):
    """Accelerations (3, T) of targets ``tpos`` (3, T) with softening ``th``
    and ids ``tid`` from sources ``spos`` (3, S), masses ``sm``, softening
    ``sh`` and ids ``sid``: spline-softened images |n| <= n_img about the
    minimum image, pairs with equal ids skipped; added into ``acc`` if given."""
    lib = _load()
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)
    tx, ty, tz = (f64(tpos[k]) for k in range(3))
    sx, sy, sz = (f64(spos[k]) for k in range(3))
    th, sm, sh, tid, sid = f64(th), f64(sm), f64(sh), i64(tid), i64(sid)
    T, S = tx.shape[0], sx.shape[0]
    out = np.zeros(3 * T) if acc is None else np.ascontiguousarray(acc, dtype=np.float64).reshape(-1).copy()
    lp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = lib.oracle_pairs(_dptr(tx), _dptr(ty), _dptr(tz), _dptr(th), lp(tid), T,
                          _dptr(sx), _dptr(sy), _dptr(sz), _dptr(sm), _dptr(sh), lp(sid), S,
                          float(L), int(n_img), _dptr(out))
    if rc != 0:
        raise ValueError("oracle_pairs rejected its arguments")
    return out.reshape(3, T)


def image_band(d, rho, L, n_lo, n_hi):
    """Unit-mass image sum over n_lo <= |n| <= n_hi at axial offset d and
    radial distance rho: returns (Fz, Frho, Pot), each FP64 of d's shape."""
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64).ravel()
    rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
    n = d.shape[0]
    Fz, Fr, P = np.zeros(n), np.zeros(n), np.zeros(n)
    rc = lib.oracle_image_band(_dptr(d), _dptr(rho), n, float(L), int(n_lo), int(n_hi),
                               _dptr(Fz), _dptr(Fr), _dptr(P))
    if rc != 0:
        raise ValueError("oracle_image_band rejected its arguments")
    return Fz, Fr, P
