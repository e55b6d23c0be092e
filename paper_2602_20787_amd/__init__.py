"""Python binding of ``libsteps_cyl.so``: direct-sum gravity in the S1 x R2
(periodic-along-z) topology of cylindrical StePS, on MI355X (gfx950).

The functions here carry the C names of ``include/steps_cyl.h`` and only
marshal arguments: torch tensors supply device memory and the HIP stream, and
every step of the computation runs in the library's HIP kernels.  There is no
CPU fallback; if the library is not built, every call raises.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "StepsError", "lib", "library_path",
    "steps_cyl_forces", "steps_cyl_forces_ex", "steps_cyl_forces_f64",
    "steps_cyl_last_error", "steps_cyl_version",
    "STEPS_SUM_COMPENSATED", "STEPS_SUM_PLAIN", "STEPS_MAX_NIMG",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_PKG, "libsteps_cyl.so")

STEPS_OK = 0
STEPS_EINVAL = -1
STEPS_EDOMAIN = -2
STEPS_ENODEV = -3
STEPS_EHIP = -4
STEPS_ENOMEM = -5
STEPS_EIO = -6
STATUS_NAMES = {0: "STEPS_OK", -1: "STEPS_EINVAL", -2: "STEPS_EDOMAIN", -3: "STEPS_ENODEV",
                -4: "STEPS_EHIP", -5: "STEPS_ENOMEM", -6: "STEPS_EIO"}
STEPS_SUM_COMPENSATED = 0
STEPS_SUM_PLAIN = 1
STEPS_MAX_NIMG = 4096


class StepsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int
_F64 = ctypes.c_double

_SIGNATURES = {
    "steps_cyl_forces": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _VP, _VP],
    "steps_cyl_forces_ex": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _I64, _I32, _VP, _VP, _VP],
    "steps_cyl_forces_f64": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _I64, _VP, _VP, _VP],
}


def lib():
    """The loaded ``libsteps_cyl.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError(f"{library_path} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(library_path)
        for name, args in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.steps_cyl_last_error.restype = ctypes.c_char_p
        L.steps_cyl_last_error.argtypes = []
        L.steps_cyl_version.restype = ctypes.c_char_p
        L.steps_cyl_version.argtypes = []
        _lib = L
    return _lib


def steps_cyl_last_error():
    return lib().steps_cyl_last_error().decode()


def steps_cyl_version():
    return lib().steps_cyl_version().decode()


def _check(rc):
    if rc != STEPS_OK:
        raise StepsError(rc, steps_cyl_last_error())


def _dev(t, dtype, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t.data_ptr()


def _stream(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _sources(pos, mass, eps):
    import torch
    N = mass.numel()
    return (N, _dev(pos, torch.float64, "pos", 3 * N), _dev(mass, torch.float64, "mass"),
            _dev(eps, torch.float64, "eps", N))


def steps_cyl_forces(pos, mass, eps, L, n_img, out_acc=None, out_pot=None, potential=True,
                     stream=None):
    """Exact image-sum accelerations (3, N) FP32 and potentials (N,) FP32 of
    all particles (``out_pot`` is None when ``potential`` is False).
    ``pos`` is a (3, N) FP64 device tensor, ``mass``/``eps`` (N,) FP64."""
    import torch
    N, p_pos, p_m, p_e = _sources(pos, mass, eps)
    if out_acc is None:
        out_acc = torch.empty((3, N), dtype=torch.float32, device=pos.device)
    if potential and out_pot is None:
        out_pot = torch.empty((N,), dtype=torch.float32, device=pos.device)
    p_acc = _dev(out_acc, torch.float32, "out_acc", 3 * N)
    p_pot = _dev(out_pot, torch.float32, "out_pot", N) if potential else None
    _check(lib().steps_cyl_forces(p_pos, p_m, p_e, N, float(L), int(n_img), p_acc, p_pot,
                                  _stream(stream, pos.device)))
    return out_acc, (out_pot if potential else None)


def steps_cyl_forces_ex(pos, mass, eps, L, n_img, targets=None, mode=STEPS_SUM_COMPENSATED,
                        out_acc=None, out_pot=None, potential=True, stream=None):
    """As :func:`steps_cyl_forces` for the targets listed in ``targets`` (an
    int64 device tensor, or None for all) with summation ``mode``."""
    import torch
    N, p_pos, p_m, p_e = _sources(pos, mass, eps)
    T = N if targets is None else targets.numel()
    p_t = None if targets is None else _dev(targets, torch.int64, "targets")
    if out_acc is None:
        out_acc = torch.empty((3, T), dtype=torch.float32, device=pos.device)
    if potential and out_pot is None:
        out_pot = torch.empty((T,), dtype=torch.float32, device=pos.device)
    p_acc = _dev(out_acc, torch.float32, "out_acc", 3 * T)
    p_pot = _dev(out_pot, torch.float32, "out_pot", T) if potential else None
    _check(lib().steps_cyl_forces_ex(p_pos, p_m, p_e, N, float(L), int(n_img), p_t, T, int(mode),
                                     p_acc, p_pot, _stream(stream, pos.device)))
    return out_acc, (out_pot if potential else None)


def steps_cyl_forces_f64(pos, mass, eps, L, n_img, targets=None, out_acc=None, out_pot=None,
                         potential=True, stream=None):
    """FP64 GPU evaluation of the same sum (precision yardstick)."""
    import torch
    N, p_pos, p_m, p_e = _sources(pos, mass, eps)
    T = N if targets is None else targets.numel()
    p_t = None if targets is None else _dev(targets, torch.int64, "targets")
    if out_acc is None:
        out_acc = torch.empty((3, T), dtype=torch.float64, device=pos.device)
    if potential and out_pot is None:
        out_pot = torch.empty((T,), dtype=torch.float64, device=pos.device)
    p_acc = _dev(out_acc, torch.float64, "out_acc", 3 * T)
    p_pot = _dev(out_pot, torch.float64, "out_pot", T) if potential else None
    _check(lib().steps_cyl_forces_f64(p_pos, p_m, p_e, N, float(L), int(n_img), p_t, T, p_acc,
                                      p_pot, _stream(stream, pos.device)))
    return out_acc, (out_pot if potential else None)
