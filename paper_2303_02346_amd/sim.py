"""Python front end of libmpm: torch supplies device memory and the stream,
every step of the simulation runs in the library's HIP kernels.

Simulator     -- one context (one scene, or many independent scenes batched
                 in one launch) over torch-allocated buffers.
MpmRollout    -- torch.autograd.Function: actions -> final positions and
                 velocities, backward through mpm_step_backward.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Union

import numpy as np
import torch

from . import _lib
from .scenes import Scene, concat_scenes

STATE_ROWS = 25   # x(3) v(3) C(9) F(9) J(1), each row of length N


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Simulator:
    """A libmpm context for one scene or a batch of independent scenes.

    The state lives in ``self.buf`` (float32, shape (25, N), rows x, v, C, F,
    J) on the GPU; ``x``, ``v`` ... are views.  All arithmetic happens in the
    library; this class only allocates and passes pointers.
    """

    def __init__(self, scenes: Union[Scene, Sequence[Scene]], requires_grad: bool = False, ckpt_every: int = 16,
                 horizon: Optional[int] = None, device: str = "cuda", graph: bool = False, adjoint: str = "tiled"):
        if isinstance(scenes, Scene):
            scenes = [scenes]
        self.scenes = list(scenes)
        sc0 = self.scenes[0]
        for sc in self.scenes:
            if sc.n_grid != sc0.n_grid or sc.dt != sc0.dt:
                raise ValueError("batched scenes must share n_grid and dt")
        self.device = torch.device(device)
        self.S = len(self.scenes)
        arrs, offs, mats = concat_scenes(self.scenes)
        self.N = int(offs[-1])
        self.offsets = offs
        self.horizon = int(horizon if horizon is not None else max(sc.horizon for sc in self.scenes))
        self._mats = (_lib.MpmMaterial * len(mats))()
        for i, m in enumerate(mats):
            self._mats[i] = _lib.MpmMaterial(m.kind, m.mu, m.lam, m.viscosity, m.friction_deg, m.cohesion, m.p_vol, m.p_mass,
                                             m.yield_stress, m.theta_c, m.theta_s)
        self._offs = (ctypes.c_int64 * (self.S + 1))(*[int(o) for o in offs])
        self._rad = (ctypes.c_float * self.S)(*[float(sc.cyl_radius) for sc in self.scenes])
        self._pos = (ctypes.c_float * (3 * self.S))(*np.concatenate([np.asarray(sc.cyl_pos0, np.float64) for sc in self.scenes]).tolist())
        self._rot = (ctypes.c_float * (9 * self.S))(*np.concatenate([np.asarray(sc.cyl_rot0, np.float64).reshape(-1) for sc in self.scenes]).tolist())
        d = _lib.MpmDesc()
        d.n_grid = sc0.n_grid
        d.dt = sc0.dt
        for k in range(3):
            d.gravity[k] = sc0.gravity[k]
        d.bound = sc0.bound
        d.n_particles = self.N
        d.n_materials = len(mats)
        d.materials = ctypes.cast(self._mats, ctypes.POINTER(_lib.MpmMaterial))
        d.n_scenes = self.S
        d.scene_offsets = ctypes.cast(self._offs, ctypes.POINTER(ctypes.c_int64)) if self.S > 1 else None
        d.cyl_radius = ctypes.cast(self._rad, ctypes.POINTER(ctypes.c_float))
        d.cyl_pos0 = ctypes.cast(self._pos, ctypes.POINTER(ctypes.c_float))
        d.cyl_rot0 = ctypes.cast(self._rot, ctypes.POINTER(ctypes.c_float))
        d.contact_band = sc0.contact_band
        d.contact_friction = sc0.contact_friction
        d.horizon = self.horizon
        d.ckpt_every = ckpt_every
        d.requires_grad = 1 if requires_grad else 0
        self.desc = d
        self.requires_grad = requires_grad
        L = _lib.lib()
        ws = L.mpm_workspace_bytes(ctypes.byref(d))
        if ws == 0:
            raise ValueError("invalid scene description")
        self.ws_bytes = int(ws)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        # the library works on a stream of its own (default priority); every
        # call first waits for torch's current stream and returns synchronised
        self.stream = torch.cuda.Stream(self.device)
        ctx = ctypes.c_void_p()
        _lib.check(L.mpm_create(ctypes.byref(d), ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(self.ws_bytes),
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)), "mpm_create")
        self.ctx = ctx
        self.buf = torch.zeros(STATE_ROWS, self.N, dtype=torch.float32, device=self.device)
        self.mat = torch.from_numpy(arrs["mat"].astype(np.uint8)).to(self.device)
        self._init_arrays = arrs
        self.actions = torch.zeros(self.horizon, self.S, 6, dtype=torch.float32, device=self.device)
        acts = np.zeros((self.horizon, self.S, 6))
        for s, sc in enumerate(self.scenes):
            acts[: sc.horizon, s] = sc.actions[: self.horizon]
        self.actions.copy_(torch.from_numpy(acts))
        self.reset()
        if graph:
            self.set_option(_lib.MPM_OPT_GRAPH, 1)
        if adjoint not in ("tiled", "plain"):
            raise ValueError("adjoint must be 'tiled' or 'plain'")
        self.set_option(_lib.MPM_OPT_ADJOINT, 1 if adjoint == "plain" else 0)

    def _sync_in(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def set_option(self, key: int, value: int):
        _lib.check(_lib.lib().mpm_set_option(self.ctx, int(key), int(value)), "mpm_set_option")

    def get_option(self, key: int) -> int:
        v = ctypes.c_int32(0)
        _lib.check(_lib.lib().mpm_get_option(self.ctx, int(key), ctypes.byref(v)), "mpm_get_option")
        return v.value

    def autotune(self, n_steps: int = 20, cache: Optional[str] = None):
        """Pick the fastest launch shape (native autotuner, mpm_autotune) for
        this workload; with `cache`, results are stored in / read from a JSON
        file keyed by the workload's shape and the device."""
        import json, os
        key = f"{torch.cuda.get_device_name(self.device)}|N={self.N}|S={self.S}|n={self.desc.n_grid}|steps={n_steps}"
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            best = table[key]
            self.set_option(_lib.MPM_OPT_PART_THREADS, best["part_threads"])
            self.set_option(_lib.MPM_OPT_PART_WGS, best["part_wgs"])
            self.set_option(_lib.MPM_OPT_GRID_WGS, best["grid_wgs"])
            self.set_option(_lib.MPM_OPT_SHARE_CHUNKS, best.get("share_chunks", 2))
            return best
        self._sync_in()
        out = (ctypes.c_int32 * 5)()
        _lib.check(_lib.lib().mpm_autotune(self.ctx, int(n_steps), out), "mpm_autotune", self.ctx)
        best = {"part_threads": out[0], "part_wgs": out[1], "grid_wgs": out[2], "us_per_step": out[3],
                "share_chunks": out[4]}
        if cache:
            table[key] = best
            d = os.path.dirname(os.path.abspath(cache))
            os.makedirs(d, exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return best

    # ---- views -------------------------------------------------------------
    @property
    def x(self):
        return self.buf[0:3]

    @property
    def v(self):
        return self.buf[3:6]

    @property
    def C(self):
        return self.buf[6:15]

    @property
    def F(self):
        return self.buf[15:24]

    @property
    def J(self):
        return self.buf[24]

    def state_struct(self, buf: Optional[torch.Tensor] = None, with_mat: bool = True) -> _lib.MpmState:
        b = self.buf if buf is None else buf
        return _lib.MpmState(b[0].data_ptr(), b[3].data_ptr(), b[6].data_ptr(), b[15].data_ptr(), b[24].data_ptr(),
                             self.mat.data_ptr() if with_mat else None)

    # ---- calls -------------------------------------------------------------
    def load(self, arrs=None):
        """Copy initial particle arrays (host, float64 from the scene
        generator) into the device state, FP32."""
        a = self._init_arrays if arrs is None else arrs
        N = self.N
        host = np.empty((STATE_ROWS, N), np.float32)
        host[0:3] = a["x"].T
        host[3:6] = a["v"].T
        host[6:15] = a["C"].reshape(N, 9).T
        host[15:24] = a["F"].reshape(N, 9).T
        host[24] = a["J"]
        self.buf.copy_(torch.from_numpy(host))

    def reset(self, arrs=None):
        self.load(arrs)
        self.set_state()
        self.set_actions(self.actions)

    def set_state(self):
        self._sync_in()
        self._state = self.state_struct()
        _lib.check(_lib.lib().mpm_set_state(self.ctx, ctypes.byref(self._state)), "mpm_set_state", self.ctx)

    def set_actions(self, actions: torch.Tensor, t0: int = 0):
        a = actions.to(self.device, torch.float32).reshape(-1, self.S, 6).contiguous()
        self._sync_in()
        self._act_keep = a
        _lib.check(_lib.lib().mpm_set_actions(self.ctx, t0, a.shape[0], ctypes.c_void_p(a.data_ptr())), "mpm_set_actions", self.ctx)

    def step(self, n: int):
        self._sync_in()
        _lib.check(_lib.lib().mpm_step(self.ctx, int(n)), "mpm_step", self.ctx)

    def clock(self) -> int:
        t = ctypes.c_int32(0)
        _lib.check(_lib.lib().mpm_clock(self.ctx, ctypes.byref(t)), "mpm_clock")
        return t.value

    def backward(self, grad_x: torch.Tensor, grad_v: torch.Tensor, want_grad0: bool = False):
        """grad_x, grad_v: (3, N) adjoints of the current state.  Returns
        dL/d(actions) (t, S, 6) and optionally dL/d(state_0) (25, N)."""
        T = self.clock()
        # persistent argument buffers, so that a graph-mode context replays
        # its captured backward (the capture is keyed by these pointers)
        bufs = getattr(self, "_bwd_bufs", None)
        if bufs is None or bufs[1].shape[0] != T:
            gT = torch.zeros(STATE_ROWS, self.N, dtype=torch.float32, device=self.device)
            ga = torch.zeros(T, self.S, 6, dtype=torch.float32, device=self.device)
            g0 = torch.zeros_like(gT)
            self._bwd_bufs = bufs = (gT, ga, g0)
        gT, ga, g0 = bufs
        gT[0:3] = grad_x
        gT[3:6] = grad_v
        gs = self.state_struct(gT, with_mat=False)
        g0s = self.state_struct(g0, with_mat=False) if want_grad0 else None
        self._sync_in()
        _lib.check(_lib.lib().mpm_step_backward(self.ctx, ctypes.byref(gs), ctypes.c_void_p(ga.data_ptr()),
                                                ctypes.byref(g0s) if g0s is not None else None),
                   "mpm_step_backward", self.ctx)
        return (ga.clone(), g0.clone()) if want_grad0 else ga.clone()

    def loss_blob(self, mu, sigma: float, want_grad: bool = True):
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        mu_c = (ctypes.c_float * 3)(*[float(m) for m in mu])
        g = torch.zeros(STATE_ROWS, self.N, dtype=torch.float32, device=self.device) if want_grad else None
        gs = self.state_struct(g, with_mat=False) if want_grad else None
        self._sync_in()
        _lib.check(_lib.lib().mpm_loss_blob(self.ctx, mu_c, ctypes.c_float(sigma), ctypes.c_void_p(loss.data_ptr()),
                                            ctypes.byref(gs) if gs is not None else None), "mpm_loss_blob", self.ctx)
        return (loss, g) if want_grad else loss

    def log_samples(self, buf: Optional[torch.Tensor], count: Optional[torch.Tensor] = None):
        """Log exact cone-case projections into buf (float32, (cap, 9));
        count is a device uint64 tensor of one element.  None stops."""
        L = _lib.lib()
        if buf is None:
            _lib.check(L.mpm_log_samples(self.ctx, None, 0, None), "mpm_log_samples")
            return
        _lib.check(L.mpm_log_samples(self.ctx, ctypes.c_void_p(buf.data_ptr()), ctypes.c_uint64(buf.shape[0]),
                                     ctypes.c_void_p(count.data_ptr())), "mpm_log_samples")

    def set_closure(self, mlp=None, tol: float = 1e-3):
        """Use a trained closure.MLP for the sand cone return (None: exact)."""
        ptr = ctypes.c_void_p(mlp.state.data_ptr()) if mlp is not None else None
        _lib.check(_lib.lib().mpm_set_closure(self.ctx, ptr, ctypes.c_float(tol)), "mpm_set_closure")

    def closure_stats(self):
        a, f = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _lib.check(_lib.lib().mpm_closure_stats(self.ctx, ctypes.byref(a), ctypes.byref(f)), "mpm_closure_stats")
        return a.value, f.value

    def sort_snapshot(self, which: int = 0):
        """Integer outputs of the block sort (mpm_sort_snapshot): which = 0
        sorts the current state and returns (ids, keys, list) as numpy
        arrays, list rows {key, offset, count}; which = 2 the same with the
        rows in key order; which = 1 returns the ids of the buffer the last
        forward call left."""
        L = _lib.lib()
        ids = torch.empty(self.N, dtype=torch.int32, device=self.device)
        self._sync_in()
        if which == 1:
            _lib.check(L.mpm_sort_snapshot(self.ctx, 1, ctypes.c_void_p(ids.data_ptr()), None, None, None),
                       "mpm_sort_snapshot", self.ctx)
            return ids.cpu().numpy().view(np.uint32)
        keys = torch.empty(self.N, dtype=torch.int32, device=self.device)
        nk = self.get_option(_lib.MPM_OPT_N_KEYS)
        lst = torch.empty(nk, 4, dtype=torch.int32, device=self.device)
        nl = ctypes.c_int32(0)
        _lib.check(L.mpm_sort_snapshot(self.ctx, which, ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(keys.data_ptr()),
                                       ctypes.c_void_p(lst.data_ptr()), ctypes.byref(nl)), "mpm_sort_snapshot", self.ctx)
        return (ids.cpu().numpy().view(np.uint32), keys.cpu().numpy().view(np.uint32),
                lst[: nl.value, :3].cpu().numpy())

    def timing(self, enable: bool):
        _lib.check(_lib.lib().mpm_timing_enable(self.ctx, 1 if enable else 0), "mpm_timing_enable")

    def timing_read(self):
        """(total ms, launches, kernel name) of the timed kernel since the last read."""
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        name = ctypes.create_string_buffer(64)
        _lib.check(_lib.lib().mpm_timing_read(self.ctx, ctypes.byref(ms), ctypes.byref(n), name, 64), "mpm_timing_read")
        return ms.value, n.value, name.value.decode()

    def positions(self) -> np.ndarray:
        return self.x.T.double().cpu().numpy()

    def state_numpy(self):
        b = self.buf.double().cpu().numpy()
        N = self.N
        return {"x": b[0:3].T.copy(), "v": b[3:6].T.copy(), "C": b[6:15].T.reshape(N, 3, 3).copy(),
                "F": b[15:24].T.reshape(N, 3, 3).copy(), "J": b[24].copy()}

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            _lib.lib().mpm_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MpmRollout(torch.autograd.Function):
    """actions (T, S, 6) -> (x_T, v_T) each (3, N); the backward runs the
    hand-written adjoint with checkpoint recompute (mpm_step_backward)."""

    @staticmethod
    def forward(ctx, actions: torch.Tensor, sim: Simulator):
        if not sim.requires_grad:
            raise ValueError("MpmRollout needs a Simulator created with requires_grad=True")
        sim.load()
        sim.set_state()
        sim.set_actions(actions.detach())
        sim.step(actions.shape[0])
        ctx.sim = sim
        return sim.x.clone(), sim.v.clone()

    @staticmethod
    def backward(ctx, gx, gv):
        sim = ctx.sim
        gx = torch.zeros(3, sim.N, device=sim.device) if gx is None else gx.contiguous()
        gv = torch.zeros(3, sim.N, device=sim.device) if gv is None else gv.contiguous()
        ga = sim.backward(gx, gv)
        return ga, None


class BlobLoss(torch.autograd.Function):
    """Blob loss of the simulator's current state (HIP kernel), with dL/dx."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, sim: Simulator, mu, sigma: float):
        loss, g = sim.loss_blob(mu, sigma, want_grad=True)
        ctx.save_for_backward(g[0:3].clone())
        return loss[0]

    @staticmethod
    def backward(ctx, gl):
        (gx,) = ctx.saved_tensors
        return gl * gx, None, None, None
