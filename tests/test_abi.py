"""The C-ABI library loads, exports every entry point its header declares,
and rejects invalid arguments on the host before any device work."""
import ctypes
import math
import os
import re

import pytest

import paper_2602_20787_amd as sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "steps_cyl.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(steps_cyl_\w+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    assert "steps_cyl_forces" in syms and len(syms) >= 5


def test_library_exports_every_declared_symbol():
    L = sc.lib()
    for name in declared_symbols():
        assert hasattr(L, name), f"{name} not exported by {sc.library_path}"


def test_version_and_error_strings():
    assert "gfx950" in sc.steps_cyl_version()
    assert isinstance(sc.steps_cyl_last_error(), str)


P = 8  # a non-null dummy address: never dereferenced because validation fails first


@pytest.mark.parametrize("args,msg", [
    ((None, P, P, 10, 1.0, 8, P, None, None), "non-null"),
    ((P, None, P, 10, 1.0, 8, P, None, None), "non-null"),
    ((P, P, None, 10, 1.0, 8, P, None, None), "non-null"),
    ((P, P, P, 10, 1.0, 8, None, None, None), "out_acc"),
    ((P, P, P, 0, 1.0, 8, P, None, None), "N=0"),
    ((P, P, P, -5, 1.0, 8, P, None, None), "N=-5"),
    ((P, P, P, 2 ** 31, 1.0, 8, P, None, None), "N="),
    ((P, P, P, 2 ** 29 + 1, 1.0, 8, P, None, None), "N=536870913"),
    ((P, P, P, 10, 0.0, 8, P, None, None), "L must"),
    ((P, P, P, 10, -1.0, 8, P, None, None), "L must"),
    ((P, P, P, 10, math.nan, 8, P, None, None), "L must"),
    ((P, P, P, 10, math.inf, 8, P, None, None), "L must"),
    ((P, P, P, 10, 1.0, -1, P, None, None), "n_img=-1"),
    ((P, P, P, 10, 1.0, 4097, P, None, None), "n_img=4097"),
])
def test_forces_rejects_invalid_arguments(args, msg):
    rc = sc.lib().steps_cyl_forces(*args)
    assert rc == sc.STEPS_EINVAL
    assert msg in sc.steps_cyl_last_error()


@pytest.mark.parametrize("fn", ["steps_cyl_forces_ex", "steps_cyl_forces_f64"])
def test_subset_entry_points_reject_invalid_arguments(fn):
    f = getattr(sc.lib(), fn)
    extra = (0,) if fn == "steps_cyl_forces_ex" else ()
    # targets NULL but n_targets != N
    assert f(P, P, P, 10, 1.0, 8, None, 9, *extra, P, None, None) == sc.STEPS_EINVAL
    assert "n_targets must equal N" in sc.steps_cyl_last_error()
    # n_targets = 0
    assert f(P, P, P, 10, 1.0, 8, P, 0, *extra, P, None, None) == sc.STEPS_EINVAL
    # missing output
    assert f(P, P, P, 10, 1.0, 8, P, 3, *extra, None, None, None) == sc.STEPS_EINVAL


def test_particle_count_cap_keeps_soa_offsets_in_int32():
    # the kernels address component c of particle i at c*N + i in 32-bit
    # arithmetic (c <= 3); the cap keeps the largest offset representable
    assert sc.STEPS_MAX_N == 2 ** 29
    assert 3 * sc.STEPS_MAX_N + (sc.STEPS_MAX_N - 1) <= 2 ** 31 - 1
    text = open(HEADER).read()
    assert "#define STEPS_MAX_N (1LL << 29)" in text


def test_forces_ex_rejects_unknown_mode():
    rc = sc.lib().steps_cyl_forces_ex(P, P, P, 10, 1.0, 8, None, 10, 7, P, None, None)
    assert rc == sc.STEPS_EINVAL and "mode=7" in sc.steps_cyl_last_error()


def test_no_device_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc = sc.lib().steps_cyl_forces(P, P, P, 10, 1.0, 8, P, None, None)
    assert rc == sc.STEPS_ENODEV


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(sc, "_lib", None)
    monkeypatch.setattr(sc, "library_path", "/nonexistent/libsteps_cyl.so")
    with pytest.raises(RuntimeError, match="missing"):
        sc.lib()


def test_binding_checks_tensor_arguments():
    import torch
    x = torch.zeros(3, 4, dtype=torch.float64)
    with pytest.raises(ValueError, match="device"):
        sc.steps_cyl_forces(x, torch.zeros(4, dtype=torch.float64),
                            torch.zeros(4, dtype=torch.float64), 1.0, 8)


# ---------------------------------------------------------------- network files
def _write(path, blob):
    with open(path, "wb") as f:
        f.write(blob)


def _valid_blob(params):
    import struct

    import numpy as np
    p = np.asarray(params, dtype=np.float32)
    body = p.tobytes()
    h = 1469598103934665603
    for b in body:
        h ^= b
        h = (h * 1099511628211) % (1 << 64)
    return b"SCYLMLP1" + struct.pack("<II", 1, p.size) + body + struct.pack("<Q", h)


@pytest.mark.parametrize("kind", ["missing", "magic", "version", "count", "truncated", "extra",
                                  "checksum", "nan"])
def test_mlp_load_rejects_bad_files(tmp_path, kind):
    import numpy as np

    import synth
    p = synth.mlp_init(seed=1)
    blob = _valid_blob(p)
    path = tmp_path / "net.bin"
    if kind == "magic":
        blob = b"XCYLMLP1" + blob[8:]
    elif kind == "version":
        blob = blob[:8] + b"\x02\x00\x00\x00" + blob[12:]
    elif kind == "count":
        blob = blob[:12] + b"\x00\x00\x00\x00" + blob[16:]
    elif kind == "truncated":
        blob = blob[:-100]
    elif kind == "extra":
        blob = blob + b"\x00"
    elif kind == "checksum":
        blob = blob[:-8] + bytes([blob[-8] ^ 1]) + blob[-7:]
    elif kind == "nan":
        q = p.copy()
        q[5] = np.nan
        blob = _valid_blob(q)
    if kind != "missing":
        _write(path, blob)
    h = ctypes.c_void_p()
    rc = sc.lib().steps_cyl_mlp_load(os.fsencode(str(path)), ctypes.byref(h))
    assert rc == sc.STEPS_EIO, sc.steps_cyl_last_error()
    assert not h.value


def test_mlp_load_accepts_a_valid_file_up_to_the_device(tmp_path):
    import torch

    import synth
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    path = tmp_path / "net.bin"
    _write(path, _valid_blob(synth.mlp_init(seed=2)))
    h = ctypes.c_void_p()
    assert sc.lib().steps_cyl_mlp_load(os.fsencode(str(path)), ctypes.byref(h)) == sc.STEPS_ENODEV


def test_mlp_create_rejects_bad_arguments():
    import numpy as np
    h = ctypes.c_void_p()
    assert sc.lib().steps_cyl_mlp_create(None, ctypes.byref(h)) == sc.STEPS_EINVAL
    p = np.zeros(sc.STEPS_MLP_PARAMS, dtype=np.float32)
    p[17] = np.inf
    assert sc.lib().steps_cyl_mlp_create(p.ctypes.data, ctypes.byref(h)) == sc.STEPS_EINVAL
    assert sc.lib().steps_cyl_mlp_create(p.ctypes.data, None) == sc.STEPS_EINVAL


def test_mlp_calls_reject_null_handles():
    L = sc.lib()
    assert L.steps_cyl_mlp_forward(None, P, P, 10, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_mlp_grad(None, P, P, 10, P, None, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_mlp_train(None, None, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_mlp_save(None, b"/tmp/x") == sc.STEPS_EINVAL
    assert L.steps_cyl_mlp_samples(None, 4, P, P, None) == sc.STEPS_EINVAL
    L.steps_cyl_mlp_destroy(None)


@pytest.mark.parametrize("args", [
    (1, 8, 6.4, 1024), (8, 5000, 6.4, 1024), (8, 8, 0.0, 1024), (8, 8, float("nan"), 1024),
    (8, 8, 6.4, 1), (8, 8, 6.4, (1 << 24) + 1),
])
def test_table_create_rejects_bad_arguments(args):
    h = ctypes.c_void_p()
    assert sc.lib().steps_cyl_table_create(*args, None, ctypes.byref(h)) == sc.STEPS_EINVAL
    assert sc.lib().steps_cyl_table_create(8, 8, 6.4, 1024, None, None) == sc.STEPS_EINVAL


@pytest.mark.parametrize("args,msg", [
    ((8, 8, 3.9, 2.0, 5, 12, 0), "rho_max >= 4"),
    ((8, 8, 6.4, 0.0, 5, 12, 0), "alpha"),
    ((8, 8, 6.4, 65.0, 5, 12, 0), "alpha"),
    ((8, 8, 6.4, 2.0, 0, 12, 0), "n_max"),
    ((8, 8, 6.4, 2.0, 5, -1, 0), "m_max"),
    ((8, 8, 6.4, 2.0, 5, 2000, 0), "m_max"),
    ((8, 8, 6.4, 2.0, 5, 12, 2), "kernel"),
    ((1, 8, 6.4, 2.0, 5, 12, 0), "grid"),
])
def test_ewald_table_create_rejects_bad_arguments(args, msg):
    h = ctypes.c_void_p()
    assert sc.lib().steps_cyl_table_create_ewald(*args, None, ctypes.byref(h)) == sc.STEPS_EINVAL
    assert msg in sc.steps_cyl_last_error()


def test_table_calls_reject_null_handles():
    L = sc.lib()
    P = ctypes.c_void_p(64)
    assert L.steps_cyl_table_values(None, P) == sc.STEPS_EINVAL
    assert L.steps_cyl_table_values_f64(None, P) == sc.STEPS_EINVAL
    assert L.steps_cyl_table_info(None, None, None, None, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_forces_table(P, P, P, 10, 1.0, None, 1, None, 10, P, None, None) == sc.STEPS_EINVAL
    L.steps_cyl_table_destroy(None)


def test_tree_calls_reject_bad_arguments():
    L = sc.lib()
    P = ctypes.c_void_p(64)
    h = ctypes.c_void_p()
    assert L.steps_cyl_tree_create(0, 0, ctypes.byref(h)) == sc.STEPS_EINVAL
    assert L.steps_cyl_tree_create(65, 0, ctypes.byref(h)) == sc.STEPS_EINVAL
    assert L.steps_cyl_tree_create(16, 2, ctypes.byref(h)) == sc.STEPS_EINVAL
    assert L.steps_cyl_tree_create(16, 0, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_tree_create(16, 1, ctypes.byref(h)) == sc.STEPS_OK   # host object only
    t = h.value
    f = L.steps_cyl_tree_forces
    assert f(None, P, P, P, 10, 1.0, 3.0, P, 1, 0.5, 0.0, 0.0, 0, P, None) == sc.STEPS_EINVAL
    assert f(t, P, P, P, 10, 1.0, 3.0, None, 1, 0.5, 0.0, 0.0, 0, P, None) == sc.STEPS_EINVAL
    assert f(t, P, P, P, 0, 1.0, 3.0, P, 1, 0.5, 0.0, 0.0, 0, P, None) == sc.STEPS_EINVAL
    assert f(t, P, P, P, 10, 1.0, -3.0, P, 1, 0.5, 0.0, 0.0, 0, P, None) == sc.STEPS_EINVAL
    assert f(t, P, P, P, 10, 1.0, 3.0, P, 3, 0.5, 0.0, 0.0, 0, P, None) == sc.STEPS_EINVAL
    assert f(t, P, P, P, 10, 1.0, 3.0, P, 1, -0.5, 0.0, 0.0, 0, P, None) == sc.STEPS_EINVAL
    assert f(t, P, P, P, 10, 1.0, 3.0, P, 1, 0.5, float("nan"), 0.0, 0, P, None) == sc.STEPS_EINVAL
    assert f(t, P, P, P, 10, 1.0, 3.0, P, 1, 0.5, 0.0, 0.0, 1, P, None) == sc.STEPS_EINVAL
    assert "no radial correction" in sc.steps_cyl_last_error()
    c = L.steps_cyl_tree_calibrate
    assert c(t, P, P, P, 10, 1.0, 3.0, P, 1, 0.5, None, P, 2, 8, None, None) == sc.STEPS_EINVAL
    assert c(t, P, P, P, 10, 1.0, 3.0, P, 1, 0.5, P, P, 0, 8, None, None) == sc.STEPS_EINVAL
    assert c(t, P, P, P, 10, 1.0, 3.0, P, 1, 0.5, P, P, 2, 300, None, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_tree_set_correction(t, None, 4, 3.0) == sc.STEPS_EINVAL
    assert L.steps_cyl_tree_set_correction(t, None, 0, 3.0) == sc.STEPS_OK
    assert L.steps_cyl_tree_info(None, None, None, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_tree_cells(None, None, None, None, None, None, None, None, None) == sc.STEPS_EINVAL
    L.steps_cyl_tree_destroy(t)
    L.steps_cyl_tree_destroy(None)


def test_pairwise_mode_needs_every_particle():
    rc = sc.lib().steps_cyl_forces_ex(P, P, P, 10, 1.0, 8, P, 10, sc.STEPS_SUM_PAIRWISE, P, None, None)
    assert rc == sc.STEPS_EINVAL and "targets NULL" in sc.steps_cyl_last_error()


def test_workspace_query_rejects_invalid_arguments():
    L = sc.lib()
    b = ctypes.c_size_t(123)
    assert L.steps_cyl_forces_workspace(0, 10, 8, 0, 2, None, 0, 1, None) == sc.STEPS_EINVAL
    assert "bytes" in sc.steps_cyl_last_error()
    for args, msg in [((9, 10, 8, 0, 2, None, 0, 1), "path=9"),
                      ((0, 0, 8, 0, 2, None, 0, 1), "N=0"),
                      ((0, 2 ** 29 + 1, 8, 0, 2, None, 0, 1), "N="),
                      ((0, 10, 8, -1, 2, None, 0, 1), "n_targets=-1"),
                      ((0, 10, 4097, 0, 2, None, 0, 1), "n_img=4097"),
                      ((0, 10, 8, 0, 7, None, 0, 1), "mode=7"),
                      ((0, 10, 8, 5, 2, None, 0, 1), "STEPS_SUM_PAIRWISE"),
                      ((1, 10, 8, 5, 2, None, 0, 1), "STEPS_SUM_PAIRWISE"),
                      ((2, 10, 8, 0, 0, None, 1, 1), "table"),
                      ((2, 10, 8, 0, 0, P, 3, 1), "order=3")]:
        assert L.steps_cyl_forces_workspace(*args, ctypes.byref(b)) == sc.STEPS_EINVAL, args
        assert msg in sc.steps_cyl_last_error(), (args, sc.steps_cyl_last_error())
        assert b.value == 0


@pytest.mark.parametrize("fn,args", [
    ("steps_cyl_forces_ws", (None, P, P, 10, 1.0, 8, P, None, P, 64, None)),
    ("steps_cyl_forces_ws", (P, P, P, 0, 1.0, 8, P, None, P, 64, None)),
    ("steps_cyl_forces_ex_ws", (P, P, P, 10, 1.0, 8, None, 9, 0, P, None, P, 64, None)),
    ("steps_cyl_forces_ex_ws", (P, P, P, 10, 1.0, 8, P, 3, 2, P, None, P, 64, None)),
    ("steps_cyl_forces_f64_ws", (P, P, P, 10, 1.0, 8, P, 0, P, None, P, 64, None)),
    ("steps_cyl_forces_learned_ws", (P, P, P, 10, 1.0, None, P, None, P, 64, None)),
    ("steps_cyl_forces_learned_ex_ws", (P, P, P, 10, 1.0, P, P, 3, 5, P, None, P, 64, None)),
    ("steps_cyl_forces_table_ws", (P, P, P, 10, 1.0, P, 3, None, 10, P, None, P, 64, None)),
])
def test_workspace_entry_points_reject_invalid_arguments(fn, args):
    # validated on the host before the device check and any use of the workspace
    assert getattr(sc.lib(), fn)(*args) == sc.STEPS_EINVAL


def test_noalloc_rejects_sizes_beyond_its_static_scratch():
    # checked on the host before the device check: N above STEPS_NOALLOC_MAX_N
    L = sc.lib()
    assert sc.STEPS_NOALLOC_MAX_N == 2 ** 20
    assert L.steps_cyl_forces_noalloc(P, P, P, 2 ** 20 + 1, 1.0, 8, P, None, None) == sc.STEPS_EINVAL
    assert "static scratch" in sc.steps_cyl_last_error()
    assert L.steps_cyl_forces_noalloc(P, P, P, 0, 1.0, 8, P, None, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_forces_noalloc(None, P, P, 10, 1.0, 8, P, None, None) == sc.STEPS_EINVAL
