"""Python front end of the gas step (include/gas.h): torch supplies device
memory and the stream; every step runs in the library's HIP kernels.

GasSim       -- one gas context over a torch-allocated packed state
                (u | v | w | scalars, FP32).
GasRollout   -- torch.autograd.Function: actions -> final packed state,
                backward through gas_step_backward.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from .scenes import GasScene


class GasSim:
    """A gas context for one GasScene.  The state lives in ``self.buf`` (one
    float32 vector: u, v, w, then the scalars); ``u``, ``v``, ``w``, ``s``
    are views with the grid shapes."""

    def __init__(self, sc: GasScene, requires_grad: bool = False, ckpt_every: int = 16,
                 horizon: Optional[int] = None, mg_cycles: int = 6, solver: str = "spectral",
                 device: str = "cuda"):
        self.sc = sc
        self.device = torch.device(device)
        nx, ny, nz = (int(a) for a in sc.n)
        self.n = (nx, ny, nz)
        self.K = int(sc.s.shape[0])
        self.horizon = int(horizon if horizon is not None else sc.horizon)
        self.requires_grad = requires_grad
        self._src = (ctypes.c_float * self.K)(*[float(x) for x in sc.src])
        d = _lib.GasDesc()
        d.nx, d.ny, d.nz = nx, ny, nz
        d.h, d.dt, d.buoyancy, d.t_amb = sc.h, sc.dt, sc.buoyancy, sc.t_amb
        d.n_scalars = self.K
        d.src = ctypes.cast(self._src, ctypes.POINTER(ctypes.c_float))
        d.emit_sigma, d.emit_kappa, d.emit_speed = sc.emit_sigma, sc.emit_kappa, sc.emit_speed
        for k in range(3):
            d.emit_pos0[k] = float(sc.emit_pos0[k])
        for k in range(9):
            d.emit_rot0[k] = float(sc.emit_rot0[k])
        d.horizon = self.horizon
        d.ckpt_every = ckpt_every
        d.requires_grad = 1 if requires_grad else 0
        d.mg_cycles = mg_cycles
        if solver not in ("spectral", "multigrid"):
            raise ValueError("solver must be 'spectral' or 'multigrid'")
        d.pressure_solver = 0 if solver == "spectral" else 1
        self.desc = d
        L = _lib.lib()
        ws = L.gas_workspace_bytes(ctypes.byref(d))
        if ws == 0:
            raise ValueError("invalid gas description")
        self.ws_bytes = int(ws)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.Stream(self.device)
        ctx = ctypes.c_void_p()
        _lib.check(L.gas_create(ctypes.byref(d), ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(self.ws_bytes),
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)), "gas_create")
        self.ctx = ctx
        self.sizes = [(nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1), self.K * nx * ny * nz]
        self.buf = torch.zeros(sum(self.sizes), dtype=torch.float32, device=self.device)
        self.actions = torch.zeros(self.horizon, 6, dtype=torch.float32, device=self.device)
        acts = np.zeros((self.horizon, 6))
        acts[: min(sc.horizon, self.horizon)] = sc.actions[: self.horizon]
        self.actions.copy_(torch.from_numpy(acts))
        self.reset()

    # views ------------------------------------------------------------------
    def split(self, buf: torch.Tensor):
        nx, ny, nz = self.n
        a, b, c, _ = self.sizes
        return (buf[:a].view(nx + 1, ny, nz), buf[a:a + b].view(nx, ny + 1, nz),
                buf[a + b:a + b + c].view(nx, ny, nz + 1), buf[a + b + c:].view(self.K, nx, ny, nz))

    def struct(self, buf: torch.Tensor) -> _lib.GasState:
        u, v, w, s = self.split(buf)
        return _lib.GasState(u.data_ptr(), v.data_ptr(), w.data_ptr(), s.data_ptr())

    def pack(self, u, v, w, s) -> torch.Tensor:
        return torch.cat([torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).reshape(-1)
                          for a in (u, v, w, s)]).to(self.device)

    def _sync_in(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _check(self, status: int, where: str):
        if status != _lib.MPM_OK:
            bits = ctypes.c_int32(0)
            if status == _lib.MPM_EDOMAIN:
                _lib.lib().gas_last_error_bits(self.ctx, ctypes.byref(bits))
            raise _lib.MpmError(status, where, bits.value)

    # calls ------------------------------------------------------------------
    def load(self, u=None, v=None, w=None, s=None):
        sc = self.sc
        self.buf.copy_(self.pack(sc.u if u is None else u, sc.v if v is None else v,
                                 sc.w if w is None else w, sc.s if s is None else s))

    def reset(self):
        self.load()
        self._sync_in()
        self._state = self.struct(self.buf)
        self._check(_lib.lib().gas_set_state(self.ctx, ctypes.byref(self._state)), "gas_set_state")
        self.set_actions(self.actions)

    def set_actions(self, actions: torch.Tensor, t0: int = 0):
        a = actions.to(self.device, torch.float32).reshape(-1, 6).contiguous()
        self._sync_in()
        _lib.check(_lib.lib().gas_set_actions(self.ctx, t0, a.shape[0], ctypes.c_void_p(a.data_ptr())),
                   "gas_set_actions")
        self._act_keep = a

    def step(self, n: int):
        self._sync_in()
        self._check(_lib.lib().gas_step(self.ctx, int(n)), "gas_step")

    def clock(self) -> int:
        t = ctypes.c_int32(0)
        _lib.check(_lib.lib().gas_clock(self.ctx, ctypes.byref(t)), "gas_clock")
        return t.value

    def backward(self, grad: torch.Tensor, want_grad0: bool = False):
        """grad: packed dL/d(state at t).  Returns dL/d(actions) (t, 6) and
        optionally dL/d(state at 0) (packed)."""
        T = self.clock()
        g = grad.to(self.device, torch.float32).contiguous()
        gs = self.struct(g)
        ga = torch.zeros(T, 6, dtype=torch.float32, device=self.device)
        g0 = torch.zeros_like(self.buf) if want_grad0 else None
        g0s = self.struct(g0) if want_grad0 else None
        self._sync_in()
        self._check(_lib.lib().gas_step_backward(self.ctx, ctypes.byref(gs), ctypes.c_void_p(ga.data_ptr()),
                                                ctypes.byref(g0s) if g0s is not None else None), "gas_step_backward")
        return (ga, g0) if want_grad0 else ga

    def sensor_loss(self, cells=None, targets=None, want_grad: bool = True):
        cells = torch.as_tensor(self.sc.sensors if cells is None else cells).to(self.device, torch.int32)
        targets = torch.as_tensor(self.sc.targets if targets is None else targets).to(self.device, torch.float32)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        g = torch.zeros_like(self.buf) if want_grad else None
        gs = self.struct(g) if want_grad else None
        self._sync_in()
        self._check(_lib.lib().gas_sensor_loss(self.ctx, int(cells.numel()), ctypes.c_void_p(cells.data_ptr()),
                                              ctypes.c_void_p(targets.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
                                              ctypes.byref(gs) if gs is not None else None), "gas_sensor_loss")
        return (loss, g) if want_grad else loss

    def enable_stats(self, on: bool = True):
        _lib.check(_lib.lib().gas_enable_stats(self.ctx, 1 if on else 0), "gas_enable_stats")

    def residual(self) -> float:
        r = ctypes.c_double(0.0)
        _lib.check(_lib.lib().gas_solver_residual(self.ctx, ctypes.byref(r)), "gas_solver_residual")
        return r.value

    def timing(self, on: bool):
        _lib.check(_lib.lib().gas_timing_enable(self.ctx, 1 if on else 0), "gas_timing_enable")

    def timing_read(self):
        a, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
        na, nb = ctypes.c_int64(0), ctypes.c_int64(0)
        _lib.check(_lib.lib().gas_timing_read(self.ctx, ctypes.byref(a), ctypes.byref(na), ctypes.byref(b),
                                              ctypes.byref(nb)), "gas_timing_read")
        return a.value, na.value, b.value, nb.value

    def state_numpy(self):
        u, v, w, s = self.split(self.buf.double().cpu())
        return {"u": u.numpy(), "v": v.numpy(), "w": w.numpy(), "s": s.numpy()}

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            _lib.lib().gas_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GasRollout(torch.autograd.Function):
    """actions (T, 6) -> final packed state; backward: gas_step_backward."""

    @staticmethod
    def forward(ctx, actions: torch.Tensor, sim: GasSim):
        if not sim.requires_grad:
            raise ValueError("GasRollout needs a GasSim created with requires_grad=True")
        sim.reset()
        sim.set_actions(actions.detach())
        sim.step(actions.shape[0])
        ctx.sim = sim
        return sim.buf.clone()

    @staticmethod
    def backward(ctx, g):
        return ctx.sim.backward(g.contiguous()), None
