"""The C-ABI library loads and exports every symbol that include/mpm.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2303_02346_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("mpm_create", "mpm_step", "mpm_step_backward", "mpm_set_actions", "mpm_set_state",
              "mpm_workspace_bytes", "mpm_destroy", "mpm_strerror", "mpm_loss_blob"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmpm.so not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_host_validation_without_gpu():
    """Pure host paths: workspace sizing and argument checks."""
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmpm.so not built")
    L = _lib.lib()
    assert L.mpm_workspace_bytes(None) == 0
    m = (_lib.MpmMaterial * 1)(_lib.MpmMaterial(0, 1.0, 1.0, 0.0, 30.0, 0.0, 1e-6, 1e-6))
    r = (ctypes.c_float * 1)(0.0)
    p = (ctypes.c_float * 3)(0.5, 0.5, 0.5)
    R = (ctypes.c_float * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    d = _lib.MpmDesc(32, 1e-4, (ctypes.c_float * 3)(0, -9.8, 0), 3, 100, 1,
                     ctypes.cast(m, ctypes.POINTER(_lib.MpmMaterial)), 1, None,
                     ctypes.cast(r, ctypes.POINTER(ctypes.c_float)), ctypes.cast(p, ctypes.POINTER(ctypes.c_float)),
                     ctypes.cast(R, ctypes.POINTER(ctypes.c_float)), 3.0, 0.5, 10, 4, 1)
    ws = L.mpm_workspace_bytes(ctypes.byref(d))
    assert ws > 0 and ws % 256 == 0
    d.n_grid = 4
    assert L.mpm_workspace_bytes(ctypes.byref(d)) == 0
    d.n_grid = 32
    d.n_scenes = 2          # two scenes need offsets
    assert L.mpm_workspace_bytes(ctypes.byref(d)) == 0
    d.n_scenes = 1
    out = ctypes.c_void_p()
    assert L.mpm_create(ctypes.byref(d), None, 0, None, ctypes.byref(out)) == _lib.MPM_EINVAL
    assert L.mpm_create(ctypes.byref(d), ctypes.c_void_p(256), 16, None, ctypes.byref(out)) == _lib.MPM_EWORKSPACE
    assert L.mpm_step(None, 1) == _lib.MPM_EINVAL
    assert L.mpm_strerror(_lib.MPM_EDOMAIN).startswith(b"simulation")


def gas_declared_functions():
    src = open(os.path.join(ROOT, "include", "gas.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gas_[a-z_]+)\s*\(", src)))


def test_library_exports_every_gas_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmpm.so not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    names = gas_declared_functions()
    for n in ("gas_create", "gas_step", "gas_step_backward", "gas_set_state", "gas_set_actions", "gas_destroy"):
        assert n in names
    for n in names:
        assert hasattr(L, n), n
    assert set(_lib.GAS_EXPORTS) == set(names)


def test_gas_host_validation_without_gpu():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmpm.so not built")
    L = _lib.lib()
    assert L.gas_workspace_bytes(None) == 0
    src = (ctypes.c_float * 2)(0.0, 1.0)
    d = _lib.GasDesc()
    d.nx = d.ny = d.nz = 32
    d.h, d.dt, d.buoyancy, d.t_amb = 1.0 / 32, 5e-3, 1.0, 1.0
    d.n_scalars = 2
    d.src = ctypes.cast(src, ctypes.POINTER(ctypes.c_float))
    d.emit_sigma, d.emit_kappa, d.emit_speed = 0.05, 0.5, 2.0
    d.horizon, d.ckpt_every, d.requires_grad, d.mg_cycles = 10, 4, 1, 8
    ws = L.gas_workspace_bytes(ctypes.byref(d))
    assert ws > 0 and ws % 256 == 0
    d.nz = 30            # not a multiple of 4
    assert L.gas_workspace_bytes(ctypes.byref(d)) == 0
    d.nz = 32
    d.emit_kappa = 1.5   # blend weight above 1
    assert L.gas_workspace_bytes(ctypes.byref(d)) == 0
    d.emit_kappa = 0.5
    out = ctypes.c_void_p()
    assert L.gas_create(ctypes.byref(d), None, 0, None, ctypes.byref(out)) == _lib.MPM_EINVAL
    assert L.gas_create(ctypes.byref(d), ctypes.c_void_p(256), 16, None, ctypes.byref(out)) == _lib.MPM_EWORKSPACE
