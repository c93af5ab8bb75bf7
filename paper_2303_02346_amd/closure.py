"""Learned closure of the Drucker-Prager cone return: sample generation from
the simulator's own exact projections, training and evaluation.  All
arithmetic runs in libmpm (HIP); torch holds the buffers."""
from __future__ import annotations

import ctypes
from typing import List, Optional

import numpy as np
import torch

from . import _lib, scenes

RECORD = 9   # log sigma_tr (3, descending), alpha, c, kappa, projected log sigma (3)


class MLP:
    """Device state of the 6-64-64-3 closure network (libmpm layout)."""

    def __init__(self, device="cuda"):
        L = _lib.lib()
        self.device = torch.device(device)
        self.state = torch.zeros(int(L.mpm_mlp_state_bytes()) // 4, dtype=torch.float32, device=self.device)
        self._scratch = None
        self._batch = 0

    def _scr(self, batch):
        if self._scratch is None or self._batch != batch:
            nbytes = int(_lib.lib().mpm_mlp_scratch_bytes(batch))
            self._scratch = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=self.device)
            self._batch = batch
        return ctypes.c_void_p(self._scratch.data_ptr())

    def init(self, samples: torch.Tensor, seed: int = 0, params: Optional[np.ndarray] = None):
        s = torch.cuda.current_stream(self.device)
        p = None
        if params is not None:
            pa = np.ascontiguousarray(params, np.float32)
            p = pa.ctypes.data_as(ctypes.c_void_p)
        _lib.check(_lib.lib().mpm_mlp_init(ctypes.c_void_p(self.state.data_ptr()), ctypes.c_void_p(samples.data_ptr()),
                                           samples.shape[0], p, ctypes.c_uint64(seed), ctypes.c_void_p(s.cuda_stream)),
                   "mpm_mlp_init")

    def train(self, samples: torch.Tensor, epochs: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0) -> List[float]:
        s = torch.cuda.current_stream(self.device)
        hist = (ctypes.c_double * epochs)()
        _lib.check(_lib.lib().mpm_mlp_train(ctypes.c_void_p(self.state.data_ptr()), ctypes.c_void_p(samples.data_ptr()),
                                            samples.shape[0], batch, epochs, ctypes.c_float(lr), ctypes.c_uint64(seed),
                                            self._scr(batch), hist, ctypes.c_void_p(s.cuda_stream)), "mpm_mlp_train")
        return list(hist)

    def grad(self, samples: torch.Tensor, batch: int):
        s = torch.cuda.current_stream(self.device)
        g = torch.zeros(4803, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double(0)
        _lib.check(_lib.lib().mpm_mlp_grad(ctypes.c_void_p(self.state.data_ptr()), ctypes.c_void_p(samples.data_ptr()),
                                           samples.shape[0], batch, self._scr(batch), ctypes.c_void_p(g.data_ptr()),
                                           ctypes.byref(loss), ctypes.c_void_p(s.cuda_stream)), "mpm_mlp_grad")
        return loss.value, g

    def predict(self, records: torch.Tensor) -> torch.Tensor:
        s = torch.cuda.current_stream(self.device)
        y = torch.zeros(records.shape[0], 3, dtype=torch.float32, device=self.device)
        _lib.check(_lib.lib().mpm_mlp_predict(ctypes.c_void_p(self.state.data_ptr()), ctypes.c_void_p(records.data_ptr()),
                                              records.shape[0], ctypes.c_void_p(y.data_ptr()),
                                              ctypes.c_void_p(s.cuda_stream)), "mpm_mlp_predict")
        return y

    def params(self):
        """(FP32 parameter vector, normalisation dict, BF16-rounded weights as
        float32 vector) on the host."""
        p = np.zeros(4803, np.float32)
        blob = (ctypes.c_uint8 * 16384)()
        s = torch.cuda.current_stream(self.device)
        _lib.check(_lib.lib().mpm_mlp_params(ctypes.c_void_p(self.state.data_ptr()), p.ctypes.data_as(ctypes.c_void_p),
                                             blob, ctypes.c_void_p(s.cuda_stream)), "mpm_mlp_params")
        raw = bytes(blob)
        f = np.frombuffer(raw, np.float32, count=18 + 64 + 64 + 16)
        norm = {"in_mean": f[0:6].copy(), "in_std": f[6:12].copy(), "out_mean": f[12:15].copy(), "out_std": f[15:18].copy()}
        off = 4 * (18 + 64 + 64 + 16)
        w = np.frombuffer(raw, np.uint16, count=64 * 16 + 64 * 64 + 16 * 64, offset=off).astype(np.uint32) << 16
        w = w.view(np.float32)
        W1 = w[: 64 * 16].reshape(64, 16)[:, :6]
        W2 = w[64 * 16: 64 * 16 + 64 * 64].reshape(64, 64)
        W3 = w[64 * 16 + 64 * 64:].reshape(16, 64)[:3]
        pb = p.copy()
        pb[0:384] = W1.reshape(-1)
        pb[448:448 + 4096] = W2.reshape(-1)
        pb[4608:4608 + 192] = W3.reshape(-1)
        return p, norm, pb


def sand_scene(seed: int, n_particles: int = 60_000, n_grid: Optional[int] = None, steps: int = 100):
    """Seeded sand-impact scene: four boxes resting on the floor band from
    the first step, moving down at 0.5..2 m/s with a sideways drift.  Per box,
    the friction angle is drawn from [20, 40] deg, the Poisson ratio from
    [0.2, 0.35] (E = 1e3), and the cohesion is 0 for half of the boxes and
    drawn from [0, 0.01] for the others.  Without n_grid the grid is one of
    64^3, 128^3, 256^3; dt = 6.4e-3 / n_grid keeps the elastic CFL number
    at 0.21.  The impact drives the cone-case returns."""
    rng = np.random.default_rng(np.random.SeedSequence([20230302, 5, seed]))
    if n_grid is None:
        n_grid = int(rng.choice([64, 128, 256]))
    dx = 1.0 / n_grid
    dt = 6.4e-3 / n_grid
    boxes = []
    per = n_particles // 4
    for b in range(4):
        E = 1e3
        nu = rng.uniform(0.2, 0.35)
        mu, lam = scenes.lame(E, nu)
        coh = 0.0 if rng.random() < 0.5 else rng.uniform(0, 0.01)
        m = scenes.Material(scenes.SAND, mu, lam, 1.0, friction_deg=rng.uniform(20, 40), cohesion=coh)
        lo = np.array([0.12 + 0.2 * b, 3 * dx, rng.uniform(0.15, 0.6)])
        side = np.array([0.15, 0.25, 0.2])
        pos = lo + side * rng.random((per, 3))
        boxes.append((pos, m, float(np.prod(side))))
    sc = scenes._assemble(n_grid, dt, boxes, np.zeros((steps, 6)), cyl_radius=0.0)
    sc.v[:, 1] = -rng.uniform(0.5, 2.0)
    sc.v[:, 0] = rng.uniform(-0.3, 0.3)
    sc.name = f"sand{seed}"
    return sc


def generate_samples(target: int, device="cuda", n_scenes: int = 32, steps: int = 100, window: int = 8,
                     seed: int = 0) -> torch.Tensor:
    """Cone-case samples of the exact projection from seeded sand rollouts:
    each scene contributes at most target / n_scenes records, logged during a
    window of `window` steps that starts at a seeded step of its rollout, so
    that the set spans materials, grids and impact stages.  Scenes are drawn
    (up to 16 n_scenes of them) until the target is reached."""
    from .sim import Simulator
    rng = np.random.default_rng(np.random.SeedSequence([20230302, 7, seed]))
    buf = torch.zeros(target, RECORD, dtype=torch.float32, device=device)
    quota = -(-target // n_scenes)
    have = 0
    for s in range(16 * n_scenes):
        if have >= target:
            break
        sc = sand_scene(s, steps=steps)
        sim = Simulator(sc)
        t0 = int(rng.integers(0, steps - window + 1))
        if t0 > 0:
            sim.step(t0)
        cap = min(quota, target - have)
        cnt = torch.zeros(1, dtype=torch.int64, device=device)
        sim.log_samples(buf[have:have + cap], cnt)
        sim.step(window)
        sim.log_samples(None)
        have += min(int(cnt.item()), cap)
        sim.close()
    return buf[:have]
