"""FP64 CPU oracle of the gas step: incompressible advection-projection on a
Cartesian grid, and its gradient.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the HIP gas path is checked against.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the HIP path: plain PyTorch
CPU ops in float64 (gradients by reverse-mode autograd), and one sparse
direct solve from scipy for the pressure.

What the paper fixes and what this module follows:
  * FluidEngine simulates gas (smoke, air) as an incompressible fluid on a
    Cartesian grid with the advection-projection scheme of Stam 1999
    (section 3.2, "Gas"): each step advects the velocity and the carried
    quantities semi-Lagrangian (trace each grid point back through the
    velocity field for one step, interpolate there), then projects the
    velocity onto its divergence-free part by a pressure solve.
  * A gas field holds a velocity field and advected quantity fields such as
    smoke density and temperature (section 3.1); the air-circulation state
    is velocity plus temperature per cell (section 4.2).
  * The projection has a hand-written gradient (section 3.3); with the exact
    projection on a staggered grid the gradient is the projection itself.
  * The agent is driven by a 6-vector of translational and angular velocity
    (section 4.2); in the air-circulation task it turns an air conditioner
    that blows cool air (section 4.1).  The sensor loss is the sum of the
    absolute temperature errors at sensor cells (Appendix, air circulation).
Readings of what the paper leaves open (staggered grid, closed walls,
trilinear interpolation with clamped back-traces, the emitter as a Gaussian
blend towards an outflow velocity and source values, buoyancy, the order of
the step's parts) are stated in the design notes and restated below.

Parity status: pinned by tests/test_oracle_gas.py against closed forms
(linear fields are interpolated exactly and translated exactly by a uniform
flow), the projector identities (P^2 = P, P self-adjoint, D P u = 0, P G phi
= 0, divergence-free fields unchanged), a dense pseudo-inverse on tiny grids,
and central finite differences of whole rollouts.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np
import scipy.sparse
import scipy.sparse.linalg
import torch

from oracle.mpm_oracle import integrate_pose

DT = torch.float64
COMPS = ("u", "v", "w")


@dataclass
class GasParams:
    n: Tuple[int, int, int]     # cells per axis (nx, ny, nz)
    h: float                    # cell size
    dt: float
    buoyancy: float             # beta: v += dt beta (T - T_amb) (T = scalar 0)
    t_amb: float
    emit_sigma: float           # Gaussian radius of the emitter
    emit_kappa: float           # blend weight at the emitter centre (0..1)
    emit_speed: float           # outflow speed along the emitter's local y axis
    src: torch.Tensor = field(default=None)   # (K,) source values of the scalars


# ----------------------------------------------------------------------------
# Staggered (MAC) grid: u on x-faces, v on y-faces, w on z-faces, scalars at
# cell centres.  Component q has dims shape(q) and grid point (i, j, k) at
# (origin(q) + (i, j, k)) * h.
# ----------------------------------------------------------------------------
def shape(q: str, n) -> Tuple[int, int, int]:
    nx, ny, nz = n
    return {"u": (nx + 1, ny, nz), "v": (nx, ny + 1, nz), "w": (nx, ny, nz + 1), "c": (nx, ny, nz)}[q]


def origin(q: str) -> torch.Tensor:
    o = {"u": (0.0, 0.5, 0.5), "v": (0.5, 0.0, 0.5), "w": (0.5, 0.5, 0.0), "c": (0.5, 0.5, 0.5)}[q]
    return torch.tensor(o, dtype=DT)


def points(q: str, p: GasParams) -> torch.Tensor:
    d = shape(q, p.n)
    ii = torch.stack(torch.meshgrid(*[torch.arange(m, dtype=DT) for m in d], indexing="ij"), -1).reshape(-1, 3)
    return (ii + origin(q)) * p.h


def interp(f: torch.Tensor, q: str, x: torch.Tensor, p: GasParams) -> torch.Tensor:
    """Trilinear interpolation of grid q's values f (dims shape(q)) at
    positions x (M, 3).  Grid coordinates are clamped into [0, dim - 1] per
    axis first (a back-trace that leaves the grid samples its boundary)."""
    d = shape(q, p.n)
    g = x / p.h - origin(q)
    gs, i0s, fr = [], [], []
    for a in range(3):
        ga = g[:, a].clamp(0.0, d[a] - 1.0)
        i0 = torch.clamp(torch.floor(ga), max=d[a] - 2).long()
        i0s.append(i0)
        fr.append(ga - i0.to(DT))
    out = torch.zeros(x.shape[0], dtype=DT)
    for di in (0, 1):
        for dj in (0, 1):
            for dk in (0, 1):
                w = (fr[0] if di else 1 - fr[0]) * (fr[1] if dj else 1 - fr[1]) * (fr[2] if dk else 1 - fr[2])
                out = out + w * f[i0s[0] + di, i0s[1] + dj, i0s[2] + dk]
    return out


def velocity_at(vel: Dict[str, torch.Tensor], x: torch.Tensor, p: GasParams) -> torch.Tensor:
    return torch.stack([interp(vel[q], q, x, p) for q in COMPS], -1)


# ----------------------------------------------------------------------------
# The parts of one step
# ----------------------------------------------------------------------------
def advect(state: Dict[str, torch.Tensor], p: GasParams) -> Dict[str, torch.Tensor]:
    """Semi-Lagrangian advection (Stam 1999) of u, v, w and the scalars by the
    velocity of the step's start: q'(x) = q(x - dt U(x))."""
    vel = {q: state[q] for q in COMPS}
    out = {}
    for q in COMPS + ("c",):
        x = points(q, p)
        xb = x - p.dt * velocity_at(vel, x, p)
        if q == "c":
            s = state["s"]
            out["s"] = torch.stack([interp(s[k], "c", xb, p).reshape(p.n) for k in range(s.shape[0])], 0)
        else:
            out[q] = interp(state[q], q, xb, p).reshape(shape(q, p.n))
    return out


def emitter_weight(x: torch.Tensor, c: torch.Tensor, p: GasParams) -> torch.Tensor:
    return p.emit_kappa * torch.exp(-((x - c) ** 2).sum(-1) / (2.0 * p.emit_sigma ** 2))


def emit(state, c, R, p: GasParams):
    """The agent's emitter at pose (c, R): every grid value moves towards its
    source value by the Gaussian weight chi(x) = kappa exp(-|x - c|^2 / 2 sigma^2):
    velocities towards emit_speed * R e_y, scalars towards src."""
    d = p.emit_speed * R[:, 1]
    out = dict(state)
    for a, q in enumerate(COMPS):
        chi = emitter_weight(points(q, p), c, p).reshape(shape(q, p.n))
        out[q] = state[q] + chi * (d[a] - state[q])
    chi = emitter_weight(points("c", p), c, p).reshape(p.n)
    out["s"] = state["s"] + chi[None] * (p.src[:, None, None, None] - state["s"])
    return out


def buoyancy(state, p: GasParams):
    """v += dt beta (T - T_amb) on the interior y-faces, T the mean of the two
    cells the face separates (scalar 0 is the temperature)."""
    T = state["s"][0]
    Tf = 0.5 * (T[:, 1:, :] + T[:, :-1, :])
    v = state["v"]
    inner = v[:, 1:-1, :] + p.dt * p.buoyancy * (Tf - p.t_amb)
    out = dict(state)
    out["v"] = torch.cat([v[:, :1, :], inner, v[:, -1:, :]], 1)
    return out


def zero_walls(state):
    """Closed walls: the normal velocity on the domain's boundary faces is zero."""
    out = dict(state)
    u, v, w = state["u"], state["v"], state["w"]
    out["u"] = torch.cat([torch.zeros_like(u[:1]), u[1:-1], torch.zeros_like(u[:1])], 0)
    out["v"] = torch.cat([torch.zeros_like(v[:, :1]), v[:, 1:-1], torch.zeros_like(v[:, :1])], 1)
    out["w"] = torch.cat([torch.zeros_like(w[:, :, :1]), w[:, :, 1:-1], torch.zeros_like(w[:, :, :1])], 2)
    return out


# ----------------------------------------------------------------------------
# Exact projection on the staggered grid with closed walls.  Divergence D at
# cells, gradient G = -D^T on the interior faces, pressure Laplacian L = D G
# (the 7-point Neumann Laplacian); P u = u - G L^+ D u.  P is the orthogonal
# projector onto the divergence-free fields, so its adjoint is P itself.
# ----------------------------------------------------------------------------
def divergence(u, v, w, h):
    return ((u[1:] - u[:-1]) + (v[:, 1:] - v[:, :-1]) + (w[:, :, 1:] - w[:, :, :-1])) / h


def gradient(phi, h):
    """G phi on the interior faces (zero on the boundary faces)."""
    nx, ny, nz = phi.shape
    gu = torch.zeros(nx + 1, ny, nz, dtype=DT)
    gv = torch.zeros(nx, ny + 1, nz, dtype=DT)
    gw = torch.zeros(nx, ny, nz + 1, dtype=DT)
    gu[1:-1] = (phi[1:] - phi[:-1]) / h
    gv[:, 1:-1] = (phi[:, 1:] - phi[:, :-1]) / h
    gw[:, :, 1:-1] = (phi[:, :, 1:] - phi[:, :, :-1]) / h
    return gu, gv, gw


def laplacian_matrix(n, h) -> scipy.sparse.csr_matrix:
    """L = D G as a sparse matrix over the cells (row-major (i, j, k))."""
    nx, ny, nz = n
    N = nx * ny * nz
    idx = np.arange(N).reshape(n)
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    for a in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[a] = slice(0, n[a] - 1)
        hi[a] = slice(1, n[a])
        i0, i1 = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        rows += [i0, i1]
        cols += [i1, i0]
        vals += [np.ones(i0.size), np.ones(i0.size)]
        np.add.at(diag, i0, -1.0)
        np.add.at(diag, i1, -1.0)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    L = scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return L / (h * h)


_FACTORS = {}


def _pinned_factor(n, h):
    """Sparse LU of L with its first equation replaced by phi[0] = 0 (the
    same matrix every step: factorised once per grid)."""
    key = (tuple(n), float(h))
    if key not in _FACTORS:
        L = laplacian_matrix(n, h).tolil()
        L[0, :] = 0.0
        L[0, 0] = 1.0
        _FACTORS[key] = scipy.sparse.linalg.splu(L.tocsc())
    return _FACTORS[key]


DIRECT_MAX_CELLS = 48 ** 3


def solve_pressure(b: np.ndarray, n, h) -> np.ndarray:
    """A solution of L phi = b for a b with zero sum (the Neumann problem is
    singular; phi is fixed up to a constant, which G does not see).  Grids up
    to 48^3: sparse LU with phi[0] = 0; larger ones: conjugate gradients on
    the consistent semi-definite system -L phi = -b to a relative residual of
    1e-12 (the factorisation of a 128^3 Laplacian does not fit)."""
    if int(np.prod(n)) <= DIRECT_MAX_CELLS:
        bb = b.ravel().copy()
        bb[0] = 0.0
        return _pinned_factor(n, h).solve(bb).reshape(n)
    A = -laplacian_matrix(n, h)
    phi, info = scipy.sparse.linalg.cg(A, -b.ravel(), rtol=1e-12, atol=0.0, maxiter=20000)
    if info != 0:
        raise RuntimeError(f"pressure CG did not converge (info {info})")
    return phi.reshape(n)


def project_np(u, v, w, h):
    b = divergence(u, v, w, h)
    b = b - b.mean()            # (zero up to rounding with closed walls)
    phi = torch.from_numpy(solve_pressure(b.detach().numpy(), tuple(b.shape), h))
    gu, gv, gw = gradient(phi, h)
    return u - gu, v - gv, w - gw


class Projection(torch.autograd.Function):
    """P u for a (u, v, w) whose boundary faces are zero (the step closes the
    walls first).  On that subspace P is self-adjoint, so the backward is P
    applied to the output gradient with its boundary faces zeroed (the
    gradient of the boundary-face inputs is dropped by the walls anyway)."""

    @staticmethod
    def forward(ctx, u, v, w, h):
        ctx.h = h
        with torch.no_grad():
            return project_np(u, v, w, h)

    @staticmethod
    def backward(ctx, gu, gv, gw):
        z = zero_walls({"u": gu, "v": gv, "w": gw})
        pu, pv, pw = project_np(z["u"].contiguous(), z["v"].contiguous(), z["w"].contiguous(), ctx.h)
        return pu, pv, pw, None


def project(state, p: GasParams):
    out = dict(state)
    out["u"], out["v"], out["w"] = Projection.apply(state["u"], state["v"], state["w"], p.h)
    return out


def step(state, c, R, p: GasParams):
    """advect -> emitter -> buoyancy -> closed walls -> projection."""
    st = advect(state, p)
    st = emit(st, c, R, p)
    st = buoyancy(st, p)
    st = zero_walls(st)
    return project(st, p)


def rollout(state0, actions, c0, R0, p: GasParams, steps: Optional[int] = None):
    T = steps if steps is not None else actions.shape[0]
    cs, Rs = integrate_pose(c0, R0, actions[:T], p.dt)
    st = state0
    for t in range(T):
        st = step(st, cs[t], Rs[t], p)
    return st


def sensor_loss(s, cells: torch.Tensor, targets: torch.Tensor) -> torch.Tensor:
    """Sum over sensors of |T(cell) - target| (scalar 0 is the temperature)."""
    T = s[0].reshape(-1)
    return (T[cells] - targets).abs().sum()


# ----------------------------------------------------------------------------
# Seeded scenes (paper_2303_02346_amd.scenes.GasScene)
# ----------------------------------------------------------------------------
def params_from_scene(sc) -> GasParams:
    return GasParams(n=tuple(sc.n), h=sc.h, dt=sc.dt, buoyancy=sc.buoyancy, t_amb=sc.t_amb,
                     emit_sigma=sc.emit_sigma, emit_kappa=sc.emit_kappa, emit_speed=sc.emit_speed,
                     src=torch.tensor(sc.src, dtype=DT))


def state_from_scene(sc, requires_grad=False):
    st = {k: torch.tensor(np.asarray(getattr(sc, k)), dtype=DT) for k in ("u", "v", "w", "s")}
    if requires_grad:
        for t in st.values():
            t.requires_grad_(True)
    return st


def rollout_scene(sc, steps=None, actions=None, state=None, params=None):
    p = params or params_from_scene(sc)
    st = state if state is not None else state_from_scene(sc)
    acts = actions if actions is not None else torch.tensor(sc.actions, dtype=DT)
    c0 = torch.tensor(sc.emit_pos0, dtype=DT)
    R0 = torch.tensor(sc.emit_rot0, dtype=DT).reshape(3, 3)
    return rollout(st, acts, c0, R0, p, steps=steps)
