"""ctypes binding of libmpm.so (include/mpm.h): argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm.so")

MPM_OK, MPM_EINVAL, MPM_EWORKSPACE, MPM_EHIP, MPM_EDOMAIN, MPM_ESTATE = 0, -1, -2, -3, -4, -5


class MpmMaterial(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("mu", ctypes.c_float), ("lambda_", ctypes.c_float),
                ("viscosity", ctypes.c_float), ("friction_deg", ctypes.c_float), ("cohesion", ctypes.c_float),
                ("p_vol", ctypes.c_float), ("p_mass", ctypes.c_float), ("yield_stress", ctypes.c_float),
                ("theta_c", ctypes.c_float), ("theta_s", ctypes.c_float)]


class MpmState(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("F", ctypes.c_void_p), ("J", ctypes.c_void_p), ("mat", ctypes.c_void_p)]


class MpmDesc(ctypes.Structure):
    _fields_ = [("n_grid", ctypes.c_int32), ("dt", ctypes.c_float), ("gravity", ctypes.c_float * 3),
                ("bound", ctypes.c_int32), ("n_particles", ctypes.c_int32), ("n_materials", ctypes.c_int32),
                ("materials", ctypes.POINTER(MpmMaterial)), ("n_scenes", ctypes.c_int32),
                ("scene_offsets", ctypes.POINTER(ctypes.c_int64)), ("cyl_radius", ctypes.POINTER(ctypes.c_float)),
                ("cyl_pos0", ctypes.POINTER(ctypes.c_float)), ("cyl_rot0", ctypes.POINTER(ctypes.c_float)),
                ("contact_band", ctypes.c_float), ("contact_friction", ctypes.c_float),
                ("horizon", ctypes.c_int32), ("ckpt_every", ctypes.c_int32), ("requires_grad", ctypes.c_int32)]


EXPORTS = ["mpm_workspace_bytes", "mpm_create", "mpm_set_state", "mpm_set_actions", "mpm_step",
           "mpm_step_backward", "mpm_loss_blob", "mpm_clock", "mpm_last_error_bits", "mpm_timing_enable",
           "mpm_timing_read", "mpm_set_option", "mpm_get_option", "mpm_sort_snapshot", "mpm_autotune", "mpm_log_samples", "mpm_set_closure",
           "mpm_closure_stats", "mpm_mlp_state_bytes", "mpm_mlp_scratch_bytes", "mpm_mlp_init", "mpm_mlp_train",
           "mpm_mlp_grad", "mpm_mlp_grad_noalloc", "mpm_mlp_predict", "mpm_mlp_params", "mpm_destroy", "mpm_strerror"]

class GasDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("h", ctypes.c_float),
                ("dt", ctypes.c_float), ("buoyancy", ctypes.c_float), ("t_amb", ctypes.c_float),
                ("n_scalars", ctypes.c_int32), ("src", ctypes.POINTER(ctypes.c_float)),
                ("emit_sigma", ctypes.c_float), ("emit_kappa", ctypes.c_float), ("emit_speed", ctypes.c_float),
                ("emit_pos0", ctypes.c_float * 3), ("emit_rot0", ctypes.c_float * 9), ("horizon", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("requires_grad", ctypes.c_int32), ("mg_cycles", ctypes.c_int32),
                ("pressure_solver", ctypes.c_int32)]


class GasState(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("w", ctypes.c_void_p), ("s", ctypes.c_void_p)]


GAS_EXPORTS = ["gas_workspace_bytes", "gas_create", "gas_set_state", "gas_set_actions", "gas_step",
               "gas_step_backward", "gas_sensor_loss", "gas_enable_stats", "gas_solver_residual", "gas_timing_enable",
               "gas_timing_read", "gas_last_error_bits", "gas_clock", "gas_destroy"]

MPM_OPT_GRAPH, MPM_OPT_PART_THREADS, MPM_OPT_PART_WGS, MPM_OPT_GRID_WGS, MPM_OPT_ADJOINT, MPM_OPT_N_KEYS = 1, 2, 3, 4, 5, 6
MPM_OPT_SHARE_CHUNKS = 7

_lib = None


class MpmError(RuntimeError):
    def __init__(self, status: int, where: str, bits: int = 0):
        self.status = status
        self.bits = bits
        super().__init__(f"{where}: {lib().mpm_strerror(status).decode()} (status {status}, error bits {bits})")


def lib():
    """Load libmpm.so.  There is no fallback: a missing library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2303_02346_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    L.mpm_workspace_bytes.argtypes = [ctypes.POINTER(MpmDesc)]
    L.mpm_workspace_bytes.restype = ctypes.c_size_t
    L.mpm_create.argtypes = [ctypes.POINTER(MpmDesc), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.mpm_set_state.argtypes = [vp, ctypes.POINTER(MpmState)]
    L.mpm_set_actions.argtypes = [vp, i32, i32, vp]
    L.mpm_step.argtypes = [vp, i32]
    L.mpm_step_backward.argtypes = [vp, ctypes.POINTER(MpmState), vp, ctypes.POINTER(MpmState)]
    L.mpm_loss_blob.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_float, vp, ctypes.POINTER(MpmState)]
    L.mpm_clock.argtypes = [vp, ctypes.POINTER(i32)]
    L.mpm_last_error_bits.argtypes = [vp, ctypes.POINTER(i32)]
    L.mpm_timing_enable.argtypes = [vp, i32]
    L.mpm_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), ctypes.c_char_p, i32]
    L.mpm_set_option.argtypes = [vp, i32, i32]
    L.mpm_get_option.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.mpm_autotune.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.mpm_sort_snapshot.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(i32)]
    u64, i64 = ctypes.c_uint64, ctypes.c_int64
    L.mpm_log_samples.argtypes = [vp, vp, u64, vp]
    L.mpm_set_closure.argtypes = [vp, vp, ctypes.c_float]
    L.mpm_closure_stats.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    L.mpm_mlp_state_bytes.argtypes = []
    L.mpm_mlp_state_bytes.restype = ctypes.c_size_t
    L.mpm_mlp_scratch_bytes.argtypes = [i32]
    L.mpm_mlp_scratch_bytes.restype = ctypes.c_size_t
    L.mpm_mlp_init.argtypes = [vp, vp, i64, vp, u64, vp]
    L.mpm_mlp_train.argtypes = [vp, vp, i64, i32, i32, ctypes.c_float, u64, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.mpm_mlp_grad.argtypes = [vp, vp, i64, i32, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.mpm_mlp_grad_noalloc.argtypes = [vp, vp, i64, i32, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.mpm_mlp_predict.argtypes = [vp, vp, i64, vp, vp]
    L.mpm_mlp_params.argtypes = [vp, vp, vp, vp]
    L.mpm_destroy.argtypes = [vp]
    L.mpm_strerror.argtypes = [ctypes.c_int]
    L.mpm_strerror.restype = ctypes.c_char_p
    gp = ctypes.POINTER(GasState)
    L.gas_workspace_bytes.argtypes = [ctypes.POINTER(GasDesc)]
    L.gas_workspace_bytes.restype = ctypes.c_size_t
    L.gas_create.argtypes = [ctypes.POINTER(GasDesc), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.gas_set_state.argtypes = [vp, gp]
    L.gas_set_actions.argtypes = [vp, i32, i32, vp]
    L.gas_step.argtypes = [vp, i32]
    L.gas_step_backward.argtypes = [vp, gp, vp, gp]
    L.gas_sensor_loss.argtypes = [vp, i32, vp, vp, vp, gp]
    L.gas_enable_stats.argtypes = [vp, i32]
    L.gas_solver_residual.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.gas_timing_enable.argtypes = [vp, i32]
    L.gas_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(i64)]
    L.gas_last_error_bits.argtypes = [vp, ctypes.POINTER(i32)]
    L.gas_clock.argtypes = [vp, ctypes.POINTER(i32)]
    L.gas_destroy.argtypes = [vp]
    for name in GAS_EXPORTS:
        if name != "gas_workspace_bytes":
            getattr(L, name).restype = ctypes.c_int
    for name in EXPORTS:
        if name not in ("mpm_workspace_bytes", "mpm_strerror", "mpm_mlp_state_bytes", "mpm_mlp_scratch_bytes"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(status: int, where: str, ctx=None):
    if status != MPM_OK:
        bits = 0
        if ctx is not None and status == MPM_EDOMAIN:
            b = ctypes.c_int32(0)
            lib().mpm_last_error_bits(ctx, ctypes.byref(b))
            bits = b.value
        raise MpmError(status, where, bits)
