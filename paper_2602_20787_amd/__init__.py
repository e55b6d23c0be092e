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
    "steps_cyl_forces_noalloc", "STEPS_NOALLOC_MAX_N",
    "steps_cyl_forces_workspace", "steps_cyl_forces_ws", "steps_cyl_forces_ex_ws", "steps_cyl_forces_f64_ws",
    "steps_cyl_forces_learned_ws", "steps_cyl_forces_learned_ex_ws", "steps_cyl_forces_table_ws",
    "STEPS_PATH_EXACT", "STEPS_PATH_LEARNED", "STEPS_PATH_TABLE", "STEPS_PATH_F64",
    "steps_cyl_last_error", "steps_cyl_version",
    "STEPS_SUM_COMPENSATED", "STEPS_SUM_PLAIN", "STEPS_SUM_PAIRWISE", "STEPS_MAX_NIMG", "STEPS_MAX_N", "STEPS_MLP_PARAMS",
    "steps_cyl_mlp_create", "steps_cyl_mlp_destroy", "steps_cyl_mlp_get_params",
    "steps_cyl_mlp_set_params", "steps_cyl_mlp_forward", "steps_cyl_mlp_grad",
    "steps_cyl_mlp_samples", "steps_cyl_mlp_train", "steps_cyl_mlp_save", "steps_cyl_mlp_load",
    "Mlp", "steps_cyl_forces_learned", "steps_cyl_forces_learned_ex",
    "KdkParams", "steps_cyl_kdk_factors", "steps_cyl_history_factors", "steps_cyl_compensation", "steps_cyl_kdk_step",
    "CorrectionTable", "steps_cyl_table_create", "steps_cyl_table_destroy",
    "steps_cyl_table_values", "steps_cyl_forces_table", "steps_cyl_table_create_ewald",
    "steps_cyl_table_values_f64", "steps_cyl_table_info", "STEPS_EWALD_BESSEL", "STEPS_EWALD_PRINTED",
    "Octree", "steps_cyl_tree_create", "steps_cyl_tree_destroy", "steps_cyl_tree_forces",
    "steps_cyl_tree_calibrate", "steps_cyl_tree_set_correction", "steps_cyl_tree_info",
    "steps_cyl_tree_cells",
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
STEPS_SUM_PAIRWISE = 2
STEPS_MAX_NIMG = 4096
STEPS_MAX_N = 1 << 29
STEPS_MLP_PARAMS = 12802
STEPS_NOALLOC_MAX_N = 1 << 20
STEPS_PATH_EXACT = 0
STEPS_PATH_LEARNED = 1
STEPS_PATH_TABLE = 2
STEPS_PATH_F64 = 3


class StepsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int
_F64 = ctypes.c_double
_SZ = ctypes.c_size_t

class TrainCfg(ctypes.Structure):
    """Mirror of steps_cyl_train_cfg."""
    _fields_ = [
        ("train_in", ctypes.c_void_p), ("n_train", ctypes.c_int64),
        ("val_in", ctypes.c_void_p), ("n_val", ctypes.c_int64),
        ("steps", ctypes.c_int64), ("batch", ctypes.c_int64),
        ("lr", ctypes.c_float), ("lr_min", ctypes.c_float),
        ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float),
        ("seed", ctypes.c_uint64), ("eval_every", ctypes.c_int64),
        ("history", ctypes.c_void_p), ("history_len", ctypes.c_int64),
    ]


class KdkParams(ctypes.Structure):
    """Mirror of steps_cyl_kdk_params."""
    _fields_ = [
        ("a_begin", ctypes.c_double), ("a_end", ctypes.c_double), ("H0", ctypes.c_double),
        ("Omega_m", ctypes.c_double), ("Omega_L", ctypes.c_double), ("Omega_r", ctypes.c_double),
        ("Omega_k", ctypes.c_double), ("w0", ctypes.c_double), ("wa", ctypes.c_double),
        ("R_cyl", ctypes.c_double), ("rho0", ctypes.c_double),
        ("compensate", ctypes.c_int), ("n_img", ctypes.c_int), ("net", ctypes.c_void_p),
        ("factors", ctypes.c_void_p), ("table", ctypes.c_void_p), ("table_order", ctypes.c_int),
        ("tree", ctypes.c_void_p), ("theta", ctypes.c_double), ("tree_shift", ctypes.c_double),
        ("tree_angle", ctypes.c_double), ("tree_correct", ctypes.c_int),
    ]


_PP = ctypes.POINTER(ctypes.c_void_p)

_SIGNATURES = {
    "steps_cyl_forces": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _VP, _VP],
    "steps_cyl_forces_ex": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _I64, _I32, _VP, _VP, _VP],
    "steps_cyl_forces_f64": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _I64, _VP, _VP, _VP],
    "steps_cyl_mlp_create": [_VP, _PP],
    "steps_cyl_mlp_get_params": [_VP, _VP],
    "steps_cyl_mlp_set_params": [_VP, _VP],
    "steps_cyl_mlp_forward": [_VP, _VP, _VP, _I64, _VP],
    "steps_cyl_mlp_grad": [_VP, _VP, _VP, _I64, _VP, _VP, _VP],
    "steps_cyl_mlp_samples": [_VP, _I64, _VP, _VP, _VP],
    "steps_cyl_mlp_train": [_VP, ctypes.POINTER(TrainCfg), _VP],
    "steps_cyl_mlp_save": [_VP, ctypes.c_char_p],
    "steps_cyl_mlp_load": [ctypes.c_char_p, _PP],
    "steps_cyl_forces_learned": [_VP, _VP, _VP, _I64, _F64, _VP, _VP, _VP, _VP],
    "steps_cyl_forces_learned_ex": [_VP, _VP, _VP, _I64, _F64, _VP, _VP, _I64, _I32, _VP, _VP, _VP],
    "steps_cyl_kdk_factors": [ctypes.POINTER(KdkParams), _VP],
    "steps_cyl_history_factors": [_VP, _VP, _I64, _I32, _F64, _F64, _VP],
    "steps_cyl_compensation": [_VP, _I64, _F64, _F64, _F64, _VP, _VP],
    "steps_cyl_kdk_step": [_VP, _VP, _VP, _VP, _I64, _F64, ctypes.POINTER(KdkParams), _VP, _VP],
    "steps_cyl_table_create": [_I32, _I32, _F64, _I32, _VP, _PP],
    "steps_cyl_table_values": [_VP, _VP],
    "steps_cyl_table_create_ewald": [_I32, _I32, _F64, _F64, _I32, _I32, _I32, _VP, _PP],
    "steps_cyl_table_values_f64": [_VP, _VP],
    "steps_cyl_table_info": [_VP, _VP, _VP, _VP, _VP],
    "steps_cyl_tree_create": [_I32, _I32, _PP],
    "steps_cyl_tree_forces": [_VP, _VP, _VP, _VP, _I64, _F64, _F64, _VP, _I32, _F64, _F64, _F64, _I32,
                              _VP, _VP],
    "steps_cyl_tree_calibrate": [_VP, _VP, _VP, _VP, _I64, _F64, _F64, _VP, _I32, _F64, _VP, _VP,
                                 _I32, _I32, _VP, _VP],
    "steps_cyl_tree_set_correction": [_VP, _VP, _I32, _F64],
    "steps_cyl_tree_info": [_VP, _VP, _VP, _VP],
    "steps_cyl_tree_cells": [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP],
    "steps_cyl_forces_table": [_VP, _VP, _VP, _I64, _F64, _VP, _I32, _VP, _I64, _VP, _VP, _VP],
    "steps_cyl_forces_noalloc": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _VP, _VP],
    "steps_cyl_forces_workspace": [_I32, _I64, _I32, _I64, _I32, _VP, _I32, _I32, ctypes.POINTER(ctypes.c_size_t)],
    "steps_cyl_forces_ws": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _VP, _VP, _SZ, _VP],
    "steps_cyl_forces_ex_ws": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _I64, _I32, _VP, _VP, _VP, _SZ, _VP],
    "steps_cyl_forces_f64_ws": [_VP, _VP, _VP, _I64, _F64, _I32, _VP, _I64, _VP, _VP, _VP, _SZ, _VP],
    "steps_cyl_forces_learned_ws": [_VP, _VP, _VP, _I64, _F64, _VP, _VP, _VP, _VP, _SZ, _VP],
    "steps_cyl_forces_learned_ex_ws": [_VP, _VP, _VP, _I64, _F64, _VP, _VP, _I64, _I32, _VP, _VP, _VP, _SZ,
                                       _VP],
    "steps_cyl_forces_table_ws": [_VP, _VP, _VP, _I64, _F64, _VP, _I32, _VP, _I64, _VP, _VP, _VP, _SZ, _VP],
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
        L.steps_cyl_mlp_destroy.argtypes = [_VP]
        L.steps_cyl_mlp_destroy.restype = None
        L.steps_cyl_table_destroy.argtypes = [_VP]
        L.steps_cyl_table_destroy.restype = None
        L.steps_cyl_tree_destroy.argtypes = [_VP]
        L.steps_cyl_tree_destroy.restype = None
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


def _ws_args(workspace):
    """(device pointer, bytes) of a caller's workspace tensor."""
    import torch
    if not isinstance(workspace, torch.Tensor) or workspace.device.type != "cuda":
        raise TypeError("workspace must be a device (cuda) tensor")
    if not workspace.is_contiguous():
        raise ValueError("workspace must be contiguous")
    return workspace.data_ptr(), workspace.numel() * workspace.element_size()


def _call(name, args, stream, workspace):
    """The C entry point `name` (or its _ws form with the workspace inserted
    before the stream)."""
    if workspace is None:
        _check(getattr(lib(), name)(*args, stream))
    else:
        _check(getattr(lib(), name + "_ws")(*args, *_ws_args(workspace), stream))


def steps_cyl_forces_workspace(path, N, n_img=0, n_targets=0, mode=STEPS_SUM_PAIRWISE, table=None, order=0,
                               potential=True):
    """Bytes of device workspace the _ws form of a force call needs on the
    current device (n_targets 0: targets None)."""
    b = ctypes.c_size_t()
    h = None if table is None else (table.handle if hasattr(table, "handle") else table)
    _check(lib().steps_cyl_forces_workspace(int(path), int(N), int(n_img), int(n_targets), int(mode), h,
                                            int(order), 1 if potential else 0, ctypes.byref(b)))
    return b.value


def steps_cyl_forces(pos, mass, eps, L, n_img, out_acc=None, out_pot=None, potential=True,
                     stream=None, workspace=None):
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
    _call("steps_cyl_forces", (p_pos, p_m, p_e, N, float(L), int(n_img), p_acc, p_pot),
          _stream(stream, pos.device), workspace)
    return out_acc, (out_pot if potential else None)


def steps_cyl_forces_noalloc(pos, mass, eps, L, n_img, out_acc=None, out_pot=None, potential=True,
                             stream=None):
    """:func:`steps_cyl_forces` in the library's static device scratch (no
    allocation by the library; N <= STEPS_NOALLOC_MAX_N; calls on one device
    must not overlap)."""
    import torch
    N, p_pos, p_m, p_e = _sources(pos, mass, eps)
    if out_acc is None:
        out_acc = torch.empty((3, N), dtype=torch.float32, device=pos.device)
    if potential and out_pot is None:
        out_pot = torch.empty((N,), dtype=torch.float32, device=pos.device)
    p_acc = _dev(out_acc, torch.float32, "out_acc", 3 * N)
    p_pot = _dev(out_pot, torch.float32, "out_pot", N) if potential else None
    _check(lib().steps_cyl_forces_noalloc(p_pos, p_m, p_e, N, float(L), int(n_img), p_acc, p_pot,
                                          _stream(stream, pos.device)))
    return out_acc, (out_pot if potential else None)


def steps_cyl_forces_ws(pos, mass, eps, L, n_img, workspace, **kw):
    """:func:`steps_cyl_forces` in a caller-owned device workspace (a
    contiguous device tensor of at least steps_cyl_forces_workspace bytes)."""
    return steps_cyl_forces(pos, mass, eps, L, n_img, workspace=workspace, **kw)


def steps_cyl_forces_ex(pos, mass, eps, L, n_img, targets=None, mode=STEPS_SUM_COMPENSATED,
                        out_acc=None, out_pot=None, potential=True, stream=None, workspace=None):
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
    _call("steps_cyl_forces_ex", (p_pos, p_m, p_e, N, float(L), int(n_img), p_t, T, int(mode), p_acc, p_pot),
          _stream(stream, pos.device), workspace)
    return out_acc, (out_pot if potential else None)


def steps_cyl_forces_ex_ws(pos, mass, eps, L, n_img, workspace, **kw):
    return steps_cyl_forces_ex(pos, mass, eps, L, n_img, workspace=workspace, **kw)


def steps_cyl_forces_f64(pos, mass, eps, L, n_img, targets=None, out_acc=None, out_pot=None,
                         potential=True, stream=None, workspace=None):
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
    _call("steps_cyl_forces_f64", (p_pos, p_m, p_e, N, float(L), int(n_img), p_t, T, p_acc, p_pot),
          _stream(stream, pos.device), workspace)
    return out_acc, (out_pot if potential else None)


def steps_cyl_forces_f64_ws(pos, mass, eps, L, n_img, workspace, **kw):
    return steps_cyl_forces_f64(pos, mass, eps, L, n_img, workspace=workspace, **kw)


# ---------------------------------------------------------------- network
def _host_f32(a, n, name):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != n:
        raise ValueError(f"{name} must hold {n} values")
    return a


def steps_cyl_mlp_create(init_params):
    """Handle (int) of a network made from 12802 host parameters."""
    p = _host_f32(init_params, STEPS_MLP_PARAMS, "init_params")
    h = ctypes.c_void_p()
    _check(lib().steps_cyl_mlp_create(p.ctypes.data, ctypes.byref(h)))
    return h.value


def steps_cyl_mlp_destroy(handle):
    if handle:
        lib().steps_cyl_mlp_destroy(handle)


def steps_cyl_mlp_get_params(handle):
    import numpy as np
    out = np.empty(STEPS_MLP_PARAMS, dtype=np.float32)
    _check(lib().steps_cyl_mlp_get_params(handle, out.ctypes.data))
    return out


def steps_cyl_mlp_set_params(handle, params):
    p = _host_f32(params, STEPS_MLP_PARAMS, "params")
    _check(lib().steps_cyl_mlp_set_params(handle, p.ctypes.data))


def steps_cyl_mlp_forward(handle, features, out=None, stream=None):
    """Outputs (2, B) FP32 for device features (2, B) FP32."""
    import torch
    B = features.shape[1]
    p_in = _dev(features, torch.float32, "features", 2 * B)
    if out is None:
        out = torch.empty((2, B), dtype=torch.float32, device=features.device)
    p_out = _dev(out, torch.float32, "out", 2 * B)
    _check(lib().steps_cyl_mlp_forward(handle, p_in, p_out, B, _stream(stream, features.device)))
    return out


def steps_cyl_mlp_grad(handle, features, targets, stream=None):
    """(gradient (12802,) FP32, loss () FP32) on device for one batch."""
    import torch
    B = features.shape[1]
    p_in = _dev(features, torch.float32, "features", 2 * B)
    p_t = _dev(targets, torch.float32, "targets", 2 * B)
    g = torch.empty((STEPS_MLP_PARAMS,), dtype=torch.float32, device=features.device)
    loss = torch.empty((), dtype=torch.float32, device=features.device)
    _check(lib().steps_cyl_mlp_grad(handle, p_in, p_t, B, g.data_ptr(), loss.data_ptr(),
                                    _stream(stream, features.device)))
    return g, loss


def steps_cyl_mlp_samples(inputs, stream=None):
    """(features, targets), each (2, n) FP32, for device inputs (2, n) FP64
    holding |d|/L and rho/L."""
    import torch
    n = inputs.shape[1]
    p_in = _dev(inputs, torch.float64, "inputs", 2 * n)
    F = torch.empty((2, n), dtype=torch.float32, device=inputs.device)
    T = torch.empty((2, n), dtype=torch.float32, device=inputs.device)
    _check(lib().steps_cyl_mlp_samples(p_in, n, F.data_ptr(), T.data_ptr(),
                                       _stream(stream, inputs.device)))
    return F, T


def steps_cyl_mlp_train(handle, train_in, steps, batch, lr=1e-3, lr_min=1e-5, beta1=0.9,
                        beta2=0.999, adam_eps=1e-8, seed=0, val_in=None, eval_every=0,
                        stream=None):
    """Adam training on device inputs (2, n) FP64; returns the recorded
    history as an (k, 3) array of (step, batch loss, validation loss)."""
    import numpy as np
    import torch
    n = train_in.shape[1]
    cfg = TrainCfg()
    cfg.train_in = _dev(train_in, torch.float64, "train_in", 2 * n)
    cfg.n_train = n
    if val_in is not None:
        cfg.val_in = _dev(val_in, torch.float64, "val_in")
        cfg.n_val = val_in.shape[1]
    cfg.steps, cfg.batch = int(steps), int(batch)
    cfg.lr, cfg.lr_min = float(lr), float(lr_min)
    cfg.beta1, cfg.beta2, cfg.adam_eps = float(beta1), float(beta2), float(adam_eps)
    cfg.seed = int(seed)
    cfg.eval_every = int(eval_every)
    k = (int(steps) // int(eval_every) + 1) if eval_every else 0
    hist = np.zeros((max(k, 1), 3), dtype=np.float32)
    cfg.history = hist.ctypes.data if k else None
    cfg.history_len = k
    _check(lib().steps_cyl_mlp_train(handle, ctypes.byref(cfg), _stream(stream, train_in.device)))
    return hist[: (hist[:, 0] > 0).sum()] if k else hist[:0]


def steps_cyl_mlp_save(handle, path):
    _check(lib().steps_cyl_mlp_save(handle, os.fsencode(path)))


def steps_cyl_mlp_load(path):
    h = ctypes.c_void_p()
    _check(lib().steps_cyl_mlp_load(os.fsencode(path), ctypes.byref(h)))
    return h.value


class Mlp:
    """Owning wrapper of a network handle."""

    def __init__(self, handle):
        self.handle = handle

    @classmethod
    def create(cls, params):
        return cls(steps_cyl_mlp_create(params))

    @classmethod
    def load(cls, path):
        return cls(steps_cyl_mlp_load(path))

    def close(self):
        if self.handle:
            steps_cyl_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        return steps_cyl_mlp_get_params(self.handle)

    def set_params(self, p):
        steps_cyl_mlp_set_params(self.handle, p)

    def forward(self, features, **kw):
        return steps_cyl_mlp_forward(self.handle, features, **kw)

    def grad(self, features, targets, **kw):
        return steps_cyl_mlp_grad(self.handle, features, targets, **kw)

    def train(self, train_in, steps, batch, **kw):
        return steps_cyl_mlp_train(self.handle, train_in, steps, batch, **kw)

    def save(self, path):
        steps_cyl_mlp_save(self.handle, path)


def _handle(net):
    return net.handle if isinstance(net, Mlp) else net


def steps_cyl_forces_learned(pos, mass, eps, L, net, out_acc=None, out_pot=None, potential=True,
                             stream=None, workspace=None):
    """Learned-correction accelerations (3, N) FP32 and near-image
    potentials (N,) FP32 of all particles; ``net`` an :class:`Mlp` or handle."""
    import torch
    N, p_pos, p_m, p_e = _sources(pos, mass, eps)
    if out_acc is None:
        out_acc = torch.empty((3, N), dtype=torch.float32, device=pos.device)
    if potential and out_pot is None:
        out_pot = torch.empty((N,), dtype=torch.float32, device=pos.device)
    p_acc = _dev(out_acc, torch.float32, "out_acc", 3 * N)
    p_pot = _dev(out_pot, torch.float32, "out_pot", N) if potential else None
    _call("steps_cyl_forces_learned", (p_pos, p_m, p_e, N, float(L), _handle(net), p_acc, p_pot),
          _stream(stream, pos.device), workspace)
    return out_acc, (out_pot if potential else None)


def steps_cyl_forces_learned_ws(pos, mass, eps, L, net, workspace, **kw):
    return steps_cyl_forces_learned(pos, mass, eps, L, net, workspace=workspace, **kw)


def steps_cyl_forces_learned_ex(pos, mass, eps, L, net, targets=None, mode=STEPS_SUM_COMPENSATED,
                                out_acc=None, out_pot=None, potential=True, stream=None, workspace=None):
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
    _call("steps_cyl_forces_learned_ex", (p_pos, p_m, p_e, N, float(L), _handle(net), p_t, T, int(mode), p_acc,
                                          p_pot), _stream(stream, pos.device), workspace)
    return out_acc, (out_pot if potential else None)


def steps_cyl_forces_learned_ex_ws(pos, mass, eps, L, net, workspace, **kw):
    return steps_cyl_forces_learned_ex(pos, mass, eps, L, net, workspace=workspace, **kw)


# ---------------------------------------------------------------- time integration
def kdk_params(a_begin, a_end, H0, Omega_m, Omega_L, Omega_r=0.0, Omega_k=0.0, w0=-1.0, wa=0.0,
               R_cyl=1.0, rho0=0.0, compensate=True, n_img=8, net=None, factors=None, table=None,
               table_order=2, tree=None, theta=0.5, tree_shift=0.0, tree_angle=0.0, tree_correct=False):
    arr = None
    if factors is not None:
        arr = (ctypes.c_double * 3)(*[float(x) for x in factors])
    p = KdkParams(a_begin, a_end, H0, Omega_m, Omega_L, Omega_r, Omega_k, w0, wa, R_cyl, rho0,
                  1 if compensate else 0, int(n_img), _handle(net) if net is not None else None,
                  ctypes.cast(arr, ctypes.c_void_p) if arr is not None else None,
                  (table.handle if isinstance(table, CorrectionTable) else table) if table is not None
                  else None, int(table_order),
                  (tree.handle if isinstance(tree, Octree) else tree) if tree is not None else None,
                  float(theta), float(tree_shift), float(tree_angle), 1 if tree_correct else 0)
    p._factors = arr   # the struct points into it: keep it alive as long as the struct
    return p


def steps_cyl_history_factors(t, a, order, a_begin, a_end):
    """(K1, D, K2) of one step on a tabulated history (host computation)."""
    import numpy as np
    t = np.ascontiguousarray(t, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = (ctypes.c_double * 3)()
    _check(lib().steps_cyl_history_factors(t.ctypes.data, a.ctypes.data, t.size, int(order),
                                           float(a_begin), float(a_end),
                                           ctypes.cast(out, ctypes.c_void_p)))
    return tuple(out)


def steps_cyl_kdk_factors(params):
    """(K1, D, K2) of one step (host computation)."""
    out = (ctypes.c_double * 3)()
    _check(lib().steps_cyl_kdk_factors(ctypes.byref(params), ctypes.cast(out, ctypes.c_void_p)))
    return tuple(out)


def steps_cyl_compensation(pos, R_cyl, Z, rho0, out=None, stream=None):
    import torch
    N = pos.shape[1]
    p = _dev(pos, torch.float64, "pos", 3 * N)
    if out is None:
        out = torch.empty((3, N), dtype=torch.float64, device=pos.device)
    _check(lib().steps_cyl_compensation(p, N, float(R_cyl), float(Z), float(rho0),
                                        _dev(out, torch.float64, "out", 3 * N),
                                        _stream(stream, pos.device)))
    return out


def steps_cyl_kdk_step(pos, mom, mass, eps, L, params, acc, stream=None):
    """One KDK step in place on device tensors pos, mom (3, N) FP64 and
    acc (3, N) FP32 (pair acceleration at pos on entry and on return)."""
    import torch
    N, p_pos, p_m, p_e = _sources(pos, mass, eps)
    p_mom = _dev(mom, torch.float64, "mom", 3 * N)
    p_acc = _dev(acc, torch.float32, "acc", 3 * N)
    _check(lib().steps_cyl_kdk_step(p_pos, p_mom, p_m, p_e, N, float(L), ctypes.byref(params),
                                    p_acc, _stream(stream, pos.device)))


# ---------------------------------------------------------------- correction table
def steps_cyl_table_create(n_delta=128, n_rho=144, rho_max=6.4, n_far=1024, stream=None):
    import torch
    h = ctypes.c_void_p()
    _check(lib().steps_cyl_table_create(int(n_delta), int(n_rho), float(rho_max), int(n_far),
                                        _stream(stream, torch.device("cuda:0")), ctypes.byref(h)))
    return h.value


def steps_cyl_table_destroy(handle):
    if handle:
        lib().steps_cyl_table_destroy(handle)


def steps_cyl_table_values(handle, n_delta, n_rho):
    """Nodes as an FP32 array (n_rho + 3, n_delta + 3, 2)."""
    import numpy as np
    out = np.empty((n_rho + 3, n_delta + 3, 2), dtype=np.float32)
    _check(lib().steps_cyl_table_values(handle, out.ctypes.data))
    return out


STEPS_EWALD_BESSEL = 0
STEPS_EWALD_PRINTED = 1


def steps_cyl_table_create_ewald(n_delta=128, n_rho=144, rho_max=6.4, alpha=2.0, n_max=5, m_max=12,
                                 kernel=STEPS_EWALD_BESSEL, stream=None):
    import torch
    h = ctypes.c_void_p()
    _check(lib().steps_cyl_table_create_ewald(int(n_delta), int(n_rho), float(rho_max), float(alpha),
                                              int(n_max), int(m_max), int(kernel),
                                              _stream(stream, torch.device("cuda:0")), ctypes.byref(h)))
    return h.value


def steps_cyl_table_values_f64(handle, n_delta, n_rho):
    """Nodes as an FP64 array (n_rho + 3, n_delta + 3, 2)."""
    import numpy as np
    out = np.empty((n_rho + 3, n_delta + 3, 2), dtype=np.float64)
    _check(lib().steps_cyl_table_values_f64(handle, out.ctypes.data))
    return out


def steps_cyl_table_info(handle):
    """(n_delta, n_rho, rho_max, n_far); n_far = -1 for a complete table."""
    nd, nr, nf = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rm = ctypes.c_double()
    _check(lib().steps_cyl_table_info(handle, ctypes.byref(nd), ctypes.byref(nr), ctypes.byref(rm),
                                      ctypes.byref(nf)))
    return nd.value, nr.value, rm.value, nf.value


class CorrectionTable:
    """Owning wrapper of a table handle: a band table of the images
    2 <= |n| <= n_far, or (``CorrectionTable.ewald``) a complete table."""

    def __init__(self, n_delta=128, n_rho=144, rho_max=6.4, n_far=1024, _handle=None):
        if _handle is None:
            _handle = steps_cyl_table_create(n_delta, n_rho, rho_max, n_far)
        self.handle = _handle
        self.n_delta, self.n_rho, self.rho_max, self.n_far = steps_cyl_table_info(_handle)
        self.complete = self.n_far < 0

    @classmethod
    def ewald(cls, n_delta=128, n_rho=144, rho_max=6.4, alpha=2.0, n_max=5, m_max=12,
              kernel=STEPS_EWALD_BESSEL):
        return cls(_handle=steps_cyl_table_create_ewald(n_delta, n_rho, rho_max, alpha, n_max, m_max,
                                                        kernel))

    def close(self):
        if self.handle:
            steps_cyl_table_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def values(self):
        return steps_cyl_table_values(self.handle, self.n_delta, self.n_rho)

    def values_f64(self):
        return steps_cyl_table_values_f64(self.handle, self.n_delta, self.n_rho)


def steps_cyl_forces_table(pos, mass, eps, L, table, order=2, targets=None, out_acc=None,
                           out_pot=None, potential=True, stream=None, workspace=None):
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
    h = table.handle if isinstance(table, CorrectionTable) else table
    _call("steps_cyl_forces_table", (p_pos, p_m, p_e, N, float(L), h, int(order), p_t, T, p_acc, p_pot),
          _stream(stream, pos.device), workspace)
    return out_acc, (out_pot if potential else None)


def steps_cyl_forces_table_ws(pos, mass, eps, L, table, workspace, **kw):
    return steps_cyl_forces_table(pos, mass, eps, L, table, workspace=workspace, **kw)


# ---------------------------------------------------------------- octree
def steps_cyl_tree_create(leaf_size=16, quadrupole=False):
    h = ctypes.c_void_p()
    _check(lib().steps_cyl_tree_create(int(leaf_size), 1 if quadrupole else 0, ctypes.byref(h)))
    return h.value


def steps_cyl_tree_destroy(handle):
    if handle:
        lib().steps_cyl_tree_destroy(handle)


def _table_handle(table):
    return table.handle if isinstance(table, CorrectionTable) else table


def steps_cyl_tree_forces(tree, pos, mass, eps, L, R_dom, table, order=1, theta=0.5, shift=0.0,
                          angle=0.0, correct=False, out_acc=None, stream=None):
    import torch
    N, p_pos, p_m, p_e = _sources(pos, mass, eps)
    if out_acc is None:
        out_acc = torch.empty((3, N), dtype=torch.float32, device=pos.device)
    p_acc = _dev(out_acc, torch.float32, "out_acc", 3 * N)
    h = tree.handle if isinstance(tree, Octree) else tree
    _check(lib().steps_cyl_tree_forces(h, p_pos, p_m, p_e, N, float(L), float(R_dom), _table_handle(table),
                                       int(order), float(theta), float(shift), float(angle),
                                       1 if correct else 0, p_acc, _stream(stream, pos.device)))
    return out_acc


def steps_cyl_tree_calibrate(tree, pos, mass, eps, L, R_dom, table, order, theta, shifts, angles,
                             n_bins, stream=None):
    """Measures and stores the radial correction; returns it (host FP64)."""
    import numpy as np
    N, p_pos, p_m, p_e = _sources(pos, mass, eps)
    sh = np.ascontiguousarray(shifts, dtype=np.float64)
    an = np.ascontiguousarray(angles, dtype=np.float64)
    if sh.shape != an.shape:
        raise ValueError("shifts and angles differ in length")
    out = np.zeros(int(n_bins), dtype=np.float64)
    h = tree.handle if isinstance(tree, Octree) else tree
    _check(lib().steps_cyl_tree_calibrate(h, p_pos, p_m, p_e, N, float(L), float(R_dom),
                                          _table_handle(table), int(order), float(theta),
                                          sh.ctypes.data, an.ctypes.data, sh.size, int(n_bins),
                                          out.ctypes.data, _stream(stream, pos.device)))
    return out


def steps_cyl_tree_set_correction(tree, corr, R_dom):
    import numpy as np
    c = np.ascontiguousarray(corr if corr is not None else [], dtype=np.float64)
    h = tree.handle if isinstance(tree, Octree) else tree
    _check(lib().steps_cyl_tree_set_correction(h, c.ctypes.data if c.size else None, c.size,
                                               float(R_dom)))


def steps_cyl_tree_info(tree):
    """(cells, cell interactions, particle interactions) of the last walk."""
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    h = tree.handle if isinstance(tree, Octree) else tree
    _check(lib().steps_cyl_tree_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def steps_cyl_tree_cells(tree, N):
    """Cells of the last build (depth-first) and the particles' key order."""
    import numpy as np
    n = steps_cyl_tree_info(tree)[0]
    out = {k: np.empty(n, dtype=np.int32) for k in ("level", "start", "count", "skip", "leaf")}
    out["mass"] = np.empty(n, dtype=np.float64)
    out["com"] = np.empty((3, n), dtype=np.float64)
    out["order"] = np.empty(int(N), dtype=np.int32)
    h = tree.handle if isinstance(tree, Octree) else tree
    _check(lib().steps_cyl_tree_cells(h, out["level"].ctypes.data, out["start"].ctypes.data,
                                      out["count"].ctypes.data, out["skip"].ctypes.data,
                                      out["leaf"].ctypes.data, out["mass"].ctypes.data,
                                      out["com"].ctypes.data, out["order"].ctypes.data))
    return out


class Octree:
    """Owning wrapper of a tree handle."""

    def __init__(self, leaf_size=16, quadrupole=False):
        self.leaf_size, self.quadrupole = leaf_size, bool(quadrupole)
        self.handle = steps_cyl_tree_create(leaf_size, quadrupole)

    def close(self):
        if self.handle:
            steps_cyl_tree_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
