"""FP64 CPU oracle of the MLS-MPM time step and its gradient.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the HIP path is checked against.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path never does.  It shares no code with the HIP path: it is written in plain
PyTorch CPU ops in float64, and its gradient comes from reverse-mode autograd
plus one custom backward (isotropic functions of F through the SVD).

What the paper fixes and what this module follows:
  * FluidEngine simulates elastic, plastic and liquid materials with MLS-MPM
    (section 3.2, citing Hu et al. 2018): particle-to-grid transfer carrying
    the material stress, grid operations that apply boundary conditions and
    coupling, grid-to-particle transfer.  The transfer formulas are those of
    MLS-MPM / APIC with quadratic B-splines.
  * Corotated elasticity (section 3.2); here the fixed-corotated form of
    Stomakhin et al. 2012.
  * Liquids reuse the corotated model with mu = 0 and a deformation gradient
    reset to a diagonal (section 3.2): only J = det F is kept; viscosity is an
    explicit Newtonian term.
  * Granular material (Drucker-Prager on Hencky strain, Klar et al. 2016) is
    not in the paper; it follows that published method.
  * SDF-particle contact on the grid with surface normals and Coulomb
    friction (section 3.2, Stomakhin et al. 2013), softened by the blend
    v = alpha v_c + (1 - alpha) v with alpha = min(exp(-d), 1) inside a
    distance threshold (section 5.1, "Soft Contact Model").
  * The manipulator is driven by a 6-vector of translational and angular
    velocity (section 4.2).
  * Gradients through SVD are hand-derived (section 3.3, Appendix A).
Readings of points the paper leaves open (units of d in the blend, band
width, friction coefficient, wall semantics, order inside the grid update)
are listed in the design notes and restated where used below.

Parity status: every function here is pinned by tests under tests/ against
closed forms, conservation laws, library routines (LAPACK SVD, scipy polar,
scipy rotations), brute-force loops and central finite differences.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch
import torch.utils.checkpoint

DT = torch.float64
ELASTIC, LIQUID, SAND, VONMISES, BOX, RIGID = 0, 1, 2, 3, 4, 5


class OracleDomainError(RuntimeError):
    """Raised when a particle stencil leaves the grid, a value becomes
    non-finite, or a sand singular value is not positive."""


# ----------------------------------------------------------------------------
# Quadratic B-spline transfer weights (MLS-MPM, Hu et al. 2018)
# ----------------------------------------------------------------------------
OFFSETS = torch.tensor([[i, j, k] for i in range(3) for j in range(3) for k in range(3)], dtype=DT)


def bspline(x: torch.Tensor, dx: float):
    """Quadratic B-spline weights of the 3x3x3 nodes around each particle.

    base = floor(x/dx - 1/2), f = x/dx - base in [1/2, 3/2), per axis
    w0 = (3/2 - f)^2 / 2, w1 = 3/4 - (f - 1)^2, w2 = (f - 1/2)^2 / 2.
    Returns base (N,3) long, f (N,3), W (N,27) node weights and
    dpos (N,27,3) = x_i - x_p.
    """
    X = x / dx
    base = torch.floor(X - 0.5).detach()
    f = X - base
    w = torch.stack([0.5 * (1.5 - f) ** 2, 0.75 - (f - 1.0) ** 2, 0.5 * (f - 0.5) ** 2], dim=1)  # (N,3k,3axis)
    o = OFFSETS.long()
    W = w[:, o[:, 0], 0] * w[:, o[:, 1], 1] * w[:, o[:, 2], 2]                  # (N,27)
    dpos = (OFFSETS[None, :, :] - f[:, None, :]) * dx                               # (N,27,3)
    return base.long(), f, W, dpos


def node_index(base: torch.Tensor, n: int) -> torch.Tensor:
    """Linear indices (N,27) of the stencil nodes, layout (i*n + j)*n + k."""
    idx = base[:, None, :] + OFFSETS.long()[None, :, :]
    return (idx[..., 0] * n + idx[..., 1]) * n + idx[..., 2]


# ----------------------------------------------------------------------------
# Signed SVD and isotropic matrix functions with a hand-written derivative
# ----------------------------------------------------------------------------
def signed_svd(F: np.ndarray):
    """F = U diag(s) V^T with U, V proper rotations; the sign of det F is
    carried by the smallest singular value (LAPACK SVD plus sign fix).
    A non-finite F is an invalid state: it is reported, not decomposed."""
    if not np.isfinite(F).all():
        raise OracleDomainError("non-finite deformation gradient")
    U, s, Vt = np.linalg.svd(F)
    V = np.swapaxes(Vt, -1, -2).copy()
    U = U.copy()
    s = s.copy()
    du = np.linalg.det(U) < 0
    U[du, :, 2] *= -1.0
    s[du, 2] *= -1.0
    dv = np.linalg.det(V) < 0
    V[dv, :, 2] *= -1.0
    s[dv, 2] *= -1.0
    return U, s, V


class IsotropicMap(torch.autograd.Function):
    """Phi(F) = U diag(g(sigma)) V^T for an isotropic map g of the singular values.

    Backward, with M = U^T Phibar V:
      diagonal:     Abar_kk = sum_i M_ii dg_i/dsigma_k
      off-diagonal: Abar_ij = s_ij (M_ij + M_ji)/2 + t_ij (M_ij - M_ji)/2
        s_ij = (g_i - g_j)/(sigma_i - sigma_j)  (limit dg_i/dsigma_i - dg_i/dsigma_j)
        t_ij = (g_i + g_j)/(sigma_i + sigma_j)
      Fbar = U Abar V^T.
    These are the derivative formulas of isotropic matrix functions; they stay
    finite at repeated singular values, where the plain SVD derivative does not.
    """

    @staticmethod
    def forward(ctx, F, gfun):
        Fn = F.detach().numpy()
        U, s, V = signed_svd(Fn)
        st = torch.from_numpy(s)
        g, dg = gfun(st)
        ctx.save_for_backward(torch.from_numpy(U), st, torch.from_numpy(V), g, dg)
        return torch.from_numpy(U) @ torch.diag_embed(g) @ torch.from_numpy(V).transpose(-1, -2)

    @staticmethod
    def backward(ctx, Gbar):
        U, s, V, g, dg = ctx.saved_tensors
        M = U.transpose(-1, -2) @ Gbar @ V
        A = torch.zeros_like(M)
        diagM = torch.diagonal(M, dim1=-2, dim2=-1)
        A_diag = torch.einsum("ni,nik->nk", diagM, dg)
        for i in range(3):
            A[:, i, i] = A_diag[:, i]
        for i in range(3):
            for j in range(3):
                if i == j:
                    continue
                d = s[:, i] - s[:, j]
                scale = torch.maximum(torch.ones_like(d), torch.maximum(s[:, i].abs(), s[:, j].abs()))
                near = d.abs() <= 1e-6 * scale
                dsafe = torch.where(near, torch.ones_like(d), d)
                s_ij = torch.where(near, dg[:, i, i] - dg[:, i, j], (g[:, i] - g[:, j]) / dsafe)
                t_ij = (g[:, i] + g[:, j]) / (s[:, i] + s[:, j])
                A[:, i, j] = s_ij * 0.5 * (M[:, i, j] + M[:, j, i]) + t_ij * 0.5 * (M[:, i, j] - M[:, j, i])
        return U @ A @ V.transpose(-1, -2), None


def g_rotation(s):
    """g = 1: Phi(F) = U V^T = R, the rotation of the polar decomposition F = R S."""
    return torch.ones_like(s), torch.zeros(s.shape + (3,), dtype=s.dtype)


def polar_rotation(F: torch.Tensor) -> torch.Tensor:
    return IsotropicMap.apply(F, g_rotation)


# ----------------------------------------------------------------------------
# Constitutive models: Kirchhoff stress tau = P F^T
# ----------------------------------------------------------------------------
def stress_fixed_corotated(F, mu, lam):
    """Fixed corotated (Stomakhin et al. 2012): tau = 2 mu (F - R) F^T + lam J (J - 1) I."""
    R = polar_rotation(F)
    J = torch.linalg.det(F)
    I = torch.eye(3, dtype=DT)
    return 2.0 * mu[:, None, None] * (F - R) @ F.transpose(-1, -2) + (lam * J * (J - 1.0))[:, None, None] * I


def stress_liquid(J, C, lam, eta):
    """Liquid: pressure from J (the mu = 0 limit of the corotated model) and a
    Newtonian viscous term: tau = lam J (J - 1) I + eta J (C + C^T)."""
    I = torch.eye(3, dtype=DT)
    return (lam * J * (J - 1.0))[:, None, None] * I + (eta * J)[:, None, None] * (C + C.transpose(-1, -2))


def make_g_hencky(mu, lam):
    """First Piola stress of Hencky elasticity as an isotropic map:
    P = U diag((2 mu eps_i + lam tr eps)/sigma_i) V^T with eps = log sigma,
    so that tau = P F^T = U diag(2 mu eps + lam tr eps) U^T."""
    def g(s):
        if torch.any(s <= 0):
            raise OracleDomainError("sand singular value <= 0")
        eps = torch.log(s)
        tr = eps.sum(-1, keepdim=True)
        h = 2.0 * mu[:, None] * eps + lam[:, None] * tr
        gv = h / s
        # d g_i / d s_k = (2 mu delta_ik / s_k + lam / s_k) / s_i - delta_ik h_i / s_i^2
        eye = torch.eye(3, dtype=DT)
        dh = (2.0 * mu[:, None, None] * eye + lam[:, None, None]) / s[:, None, :]
        dg = dh / s[:, :, None] - eye * (h / s ** 2)[:, :, None]
        return gv, dg
    return g


def stress_sand(F, mu, lam):
    P = IsotropicMap.apply(F, make_g_hencky(mu, lam))
    return P @ F.transpose(-1, -2)


# ----------------------------------------------------------------------------
# Drucker-Prager projection in log-strain space (Klar et al. 2016)
# ----------------------------------------------------------------------------
def dp_alpha(friction_deg):
    sphi = math.sin(math.radians(friction_deg))
    return math.sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi)


def dp_project(eps: torch.Tensor, alpha, kappa, cohesion):
    """Return-map a log-strain eps (N,3) onto the Drucker-Prager cone.

    eps_s = eps - c; t = tr eps_s; dev = eps_s - t/3.
    t > 0 -> apex: eps_s' = 0.  Else dgamma = |dev| + kappa alpha t;
    dgamma <= 0 -> inside (unchanged); else eps_s' = eps_s - dgamma dev/|dev|.
    eps' = eps_s' + c.  Returns (eps', case) with case 0 inside, 1 apex, 2 cone.
    """
    c = cohesion[:, None]
    es = eps - c
    t = es.sum(-1, keepdim=True)
    dev = es - t / 3.0
    ndev = torch.linalg.norm(dev, dim=-1, keepdim=True)
    dgam = ndev + (kappa * alpha)[:, None] * t
    apex = (t > 0)
    inside = (~apex) & (dgam <= 0)
    cone = (~apex) & (~inside)
    nsafe = torch.where(ndev > 0, ndev, torch.ones_like(ndev))
    es_cone = es - dgam * dev / nsafe
    out = torch.where(apex, torch.zeros_like(es), torch.where(inside, es, es_cone)) + c
    case = torch.where(apex[:, 0], 1, torch.where(inside[:, 0], 0, 2))
    return out, case


def dp_jacobian(eps, alpha, kappa, cohesion):
    """d eps'/d eps of dp_project (N,3,3), per case."""
    c = cohesion[:, None]
    es = eps - c
    t = es.sum(-1, keepdim=True)
    dev = es - t / 3.0
    ndev = torch.linalg.norm(dev, dim=-1, keepdim=True)
    dgam = ndev + (kappa * alpha)[:, None] * t
    N = eps.shape[0]
    eye = torch.eye(3, dtype=DT).expand(N, 3, 3)
    ones = torch.ones(N, 3, 3, dtype=DT)
    apex = (t[:, 0] > 0)
    inside = (~apex) & (dgam[:, 0] <= 0)
    nsafe = torch.where(ndev > 0, ndev, torch.ones_like(ndev))
    nh = dev / nsafe
    ka = (kappa * alpha)[:, None, None]
    # eps' = t/3 1 + c - ka t nh  with  d nh/d eps = (I - nh nh^T - 11^T/3)/|dev|
    dnh = (eye - nh[:, :, None] * nh[:, None, :] - ones / 3.0) / nsafe[:, :, None]
    Jc = ones / 3.0 - ka * (nh[:, :, None] * torch.ones(N, 1, 3, dtype=DT)) - ka * t[:, :, None] * dnh
    Jm = torch.where(apex[:, None, None], torch.zeros_like(eye), torch.where(inside[:, None, None], eye, Jc))
    return Jm


def make_g_dp(alpha, kappa, cohesion):
    """Projected deformation as an isotropic map of the trial F:
    F' = U diag(exp(P(log sigma))) V^T."""
    def g(s):
        if torch.any(s <= 0):
            raise OracleDomainError("sand singular value <= 0")
        eps = torch.log(s)
        ep, _ = dp_project(eps, alpha, kappa, cohesion)
        gv = torch.exp(ep)
        Jm = dp_jacobian(eps, alpha, kappa, cohesion)
        dg = gv[:, :, None] * Jm / s[:, None, :]
        return gv, dg
    return g


# ----------------------------------------------------------------------------
# Von Mises projection in log-strain space (section 3.2: the non-Newtonian
# liquid is an elastoplastic continuum whose plastic part follows the von
# Mises criterion).  Hencky elasticity as for sand; with dev = eps - tr/3, the
# yield surface is |dev| = rho, rho = yield stress / (2 mu).
# ----------------------------------------------------------------------------
def vm_project(eps: torch.Tensor, rho):
    """|dev| <= rho -> unchanged (case 0); else eps' = tr/3 + rho dev/|dev|
    (case 2): the trace is kept and the deviatoric part is scaled back onto
    the yield surface along its own direction."""
    t = eps.sum(-1, keepdim=True)
    dev = eps - t / 3.0
    ndev = torch.linalg.norm(dev, dim=-1, keepdim=True)
    yielding = ndev > rho[:, None]
    nsafe = torch.where(ndev > 0, ndev, torch.ones_like(ndev))
    out = torch.where(yielding, t / 3.0 + rho[:, None] * dev / nsafe, eps)
    case = torch.where(yielding[:, 0], 2, 0)
    return out, case


def vm_jacobian(eps, rho):
    """d eps'/d eps of vm_project (N,3,3): identity inside; when yielding
    11^T/3 + (rho/|dev|)(I - nh nh^T - 11^T/3)."""
    t = eps.sum(-1, keepdim=True)
    dev = eps - t / 3.0
    ndev = torch.linalg.norm(dev, dim=-1, keepdim=True)
    N = eps.shape[0]
    eye = torch.eye(3, dtype=DT).expand(N, 3, 3)
    ones = torch.ones(N, 3, 3, dtype=DT)
    yielding = ndev[:, 0] > rho
    nsafe = torch.where(ndev > 0, ndev, torch.ones_like(ndev))
    nh = dev / nsafe
    Jy = ones / 3.0 + (rho[:, None, None] / nsafe[:, :, None]) * (eye - nh[:, :, None] * nh[:, None, :] - ones / 3.0)
    return torch.where(yielding[:, None, None], Jy, eye)


def make_g_vm(rho):
    """Projected deformation as an isotropic map of the trial F:
    F' = U diag(exp(P_vm(log sigma))) V^T."""
    def g(s):
        if torch.any(s <= 0):
            raise OracleDomainError("plastic singular value <= 0")
        eps = torch.log(s)
        ep, _ = vm_project(eps, rho)
        gv = torch.exp(ep)
        dg = gv[:, :, None] * vm_jacobian(eps, rho) / s[:, None, :]
        return gv, dg
    return g


# ----------------------------------------------------------------------------
# Box yield (section 3.2's plastic material, Stomakhin et al. 2013): after
# each update the singular values of F are clamped to [1 - theta_c,
# 1 + theta_s]; the corotated stress acts on the clamped F.  No hardening.
# ----------------------------------------------------------------------------
def make_g_box(lo, hi):
    """F' = U diag(clamp(sigma, lo, hi)) V^T as an isotropic map."""
    def g(s):
        if torch.any(s <= 0):
            raise OracleDomainError("plastic singular value <= 0")
        gv = torch.minimum(torch.maximum(s, lo[:, None]), hi[:, None])
        inside = ((s > lo[:, None]) & (s < hi[:, None])).to(DT)
        dg = torch.diag_embed(inside)
        return gv, dg
    return g


# ----------------------------------------------------------------------------
# Rigid bodies represented by particles (section 3.2): the body's particles
# are first updated as an elastic (corotated) solid; then the object-level
# rigid transformation is computed and imposed.  Shape matching: centroid c
# and rotation R = polar(sum m (x - c) r^T) of the rest offsets r; positions
# c + R r; velocities the rigid field v_cm + w x (R r) with the body's linear
# momentum and its angular momentum L = sum m (x - c) x (v - v_cm) about c
# (w = R I_rest^-1 R^T L); C = [w]x; F = R.
# ----------------------------------------------------------------------------
def rigid_project(st, b, p: "Params"):
    i = b["idx"]
    m = p.mass[i]
    M = m.sum()
    x, v = st["x"][i], st["v"][i]
    c = (m[:, None] * x).sum(0) / M
    vcm = (m[:, None] * v).sum(0) / M
    A = (m[:, None, None] * (x - c)[:, :, None] * b["r"][:, None, :]).sum(0)
    R = polar_rotation(A[None])[0]
    L = (m[:, None] * torch.cross(x - c, v - vcm, dim=-1)).sum(0)
    w = R @ (b["Iinv"] @ (R.T @ L))
    q = b["r"] @ R.T
    out = dict(st)
    out["x"] = st["x"].index_put((i,), c + q)
    out["v"] = st["v"].index_put((i,), vcm + torch.cross(w.expand_as(q), q, dim=-1))
    W = skew(w)
    out["C"] = st["C"].index_put((i,), W.expand(i.numel(), 3, 3))
    out["F"] = st["F"].index_put((i,), R.expand(i.numel(), 3, 3))
    return out


# ----------------------------------------------------------------------------
# Scene parameters (oracle-side copy of the inputs)
# ----------------------------------------------------------------------------
@dataclass
class Params:
    n_grid: int
    dt: float
    gravity: torch.Tensor
    bound: int
    kind: torch.Tensor        # (N,) long
    mu: torch.Tensor          # (N,)
    lam: torch.Tensor
    eta: torch.Tensor
    alpha: torch.Tensor
    kappa: torch.Tensor
    cohesion: torch.Tensor
    yield_radius: torch.Tensor   # von Mises: yield stress / (2 mu)
    box_lo: torch.Tensor         # Box yield: 1 - theta_c
    box_hi: torch.Tensor         # Box yield: 1 + theta_s
    vol: torch.Tensor
    mass: torch.Tensor
    cyl_radius: float
    contact_band: float
    friction: float
    idx_el: torch.Tensor = field(default=None)
    idx_liq: torch.Tensor = field(default=None)
    idx_sand: torch.Tensor = field(default=None)
    idx_vm: torch.Tensor = field(default=None)
    idx_box: torch.Tensor = field(default=None)
    # rigid bodies (one per rigid material): particle indices, rest offsets
    # from the body's mass-weighted rest centroid, inverse rest inertia
    rigid: list = field(default=None)

    @property
    def dx(self):
        return 1.0 / self.n_grid


def params_from_scene(sc) -> Params:
    mat = np.asarray(sc.mat)
    def per(attr):
        return torch.tensor([getattr(sc.materials[m], attr) for m in range(len(sc.materials))], dtype=DT)[torch.from_numpy(mat).long()]
    kind = torch.tensor([sc.materials[m].kind for m in range(len(sc.materials))])[torch.from_numpy(mat).long()]
    mu, lam = per("mu"), per("lam")
    phi = [sc.materials[m].friction_deg for m in range(len(sc.materials))]
    alpha = torch.tensor([dp_alpha(p) for p in phi], dtype=DT)[torch.from_numpy(mat).long()]
    kappa = torch.where(mu > 0, (3.0 * lam + 2.0 * mu) / (2.0 * torch.where(mu > 0, mu, torch.ones_like(mu))), torch.zeros_like(mu))
    def per_opt(attr):
        return torch.tensor([getattr(sc.materials[m], attr, 0.0) for m in range(len(sc.materials))],
                            dtype=DT)[torch.from_numpy(mat).long()]
    ys = per_opt("yield_stress")
    yrad = torch.where(mu > 0, ys / (2.0 * torch.where(mu > 0, mu, torch.ones_like(mu))), torch.zeros_like(mu))
    p = Params(n_grid=sc.n_grid, dt=sc.dt, gravity=torch.tensor(sc.gravity, dtype=DT), bound=sc.bound,
               kind=kind, mu=mu, lam=lam, eta=per("viscosity"), alpha=alpha, kappa=kappa,
               cohesion=per("cohesion"), yield_radius=yrad,
               box_lo=1.0 - per_opt("theta_c"), box_hi=1.0 + per_opt("theta_s"),
               vol=per("p_vol"), mass=per("p_mass"),
               cyl_radius=sc.cyl_radius, contact_band=sc.contact_band, friction=sc.contact_friction)
    p.idx_el = torch.nonzero(kind == ELASTIC)[:, 0]
    p.idx_liq = torch.nonzero(kind == LIQUID)[:, 0]
    p.idx_sand = torch.nonzero(kind == SAND)[:, 0]
    p.idx_vm = torch.nonzero(kind == VONMISES)[:, 0]
    p.idx_box = torch.nonzero(kind == BOX)[:, 0]
    p.rigid = []
    x0 = torch.tensor(np.asarray(sc.x), dtype=DT)
    matl = torch.from_numpy(mat).long()
    for m in range(len(sc.materials)):
        if sc.materials[m].kind != RIGID:
            continue
        idx = torch.nonzero(matl == m)[:, 0]
        if idx.numel() == 0:
            continue
        w = p.mass[idx]
        X = x0[idx]
        r = X - (w[:, None] * X).sum(0) / w.sum()
        I = (w[:, None, None] * ((r * r).sum(-1)[:, None, None] * torch.eye(3, dtype=DT) - r[:, :, None] * r[:, None, :])).sum(0)
        p.rigid.append({"idx": idx, "r": r, "Iinv": torch.linalg.inv(I)})
    return p


def state_from_scene(sc, requires_grad=False) -> Dict[str, torch.Tensor]:
    st = {k: torch.tensor(np.asarray(getattr(sc, k)), dtype=DT) for k in ("x", "v", "C", "F", "J")}
    if requires_grad:
        for t in st.values():
            t.requires_grad_(True)
    return st


# ----------------------------------------------------------------------------
# The three phases of one step
# ----------------------------------------------------------------------------
def kirchhoff_stress(st, p: Params):
    N = st["x"].shape[0]
    tau = torch.zeros(N, 3, 3, dtype=DT)
    if p.idx_el.numel():
        i = p.idx_el
        tau = tau.index_put((i,), stress_fixed_corotated(st["F"][i], p.mu[i], p.lam[i]))
    if p.idx_liq.numel():
        i = p.idx_liq
        tau = tau.index_put((i,), stress_liquid(st["J"][i], st["C"][i], p.lam[i], p.eta[i]))
    if p.idx_sand.numel():
        i = p.idx_sand
        tau = tau.index_put((i,), stress_sand(st["F"][i], p.mu[i], p.lam[i]))
    if p.idx_vm.numel():
        i = p.idx_vm
        tau = tau.index_put((i,), stress_sand(st["F"][i], p.mu[i], p.lam[i]))   # Hencky as well
    if p.idx_box.numel():
        i = p.idx_box
        tau = tau.index_put((i,), stress_fixed_corotated(st["F"][i], p.mu[i], p.lam[i]))
    for b in p.rigid:
        i = b["idx"]
        tau = tau.index_put((i,), stress_fixed_corotated(st["F"][i], p.mu[i], p.lam[i]))
    return tau


def check_stencil(base, n):
    if torch.any(base < 0) or torch.any(base + 2 > n - 1):
        raise OracleDomainError("particle stencil outside the grid")


def p2g(st, p: Params):
    """Particle-to-grid (APIC momentum + MLS force).

    A_p = -dt V_p (4/dx^2) tau_p + m_p C_p
    m_i  += w_ip m_p
    mv_i += w_ip (m_p v_p + A_p (x_i - x_p))
    Returns dense grid mass (n^3,) and momentum (n^3,3).
    """
    n, dx, dt = p.n_grid, p.dx, p.dt
    base, f, W, dpos = bspline(st["x"], dx)
    check_stencil(base, n)
    tau = kirchhoff_stress(st, p)
    A = -(dt * p.vol * 4.0 / dx ** 2)[:, None, None] * tau + p.mass[:, None, None] * st["C"]
    idx = node_index(base, n).reshape(-1)
    mom = (p.mass[:, None] * st["v"])[:, None, :] + torch.einsum("pab,pnb->pna", A, dpos)  # (N,27,3)
    m = torch.zeros(n ** 3, dtype=DT).index_add(0, idx, (W * p.mass[:, None]).reshape(-1))
    mv = torch.zeros(n ** 3, 3, dtype=DT).index_add(0, idx, (W[:, :, None] * mom).reshape(-1, 3))
    return m, mv


def skew(w):
    z = torch.zeros_like(w[..., 0])
    return torch.stack([torch.stack([z, -w[..., 2], w[..., 1]], -1),
                        torch.stack([w[..., 2], z, -w[..., 0]], -1),
                        torch.stack([-w[..., 1], w[..., 0], z], -1)], -2)


def cylinder_contact(xi, vg, c, R, u, w, p: Params):
    """Soft SDF contact of grid velocities vg at node positions xi with an
    infinite cylinder (axis R e_y through c, radius r) moving rigidly with
    velocity u and angular velocity w.

    d = |P(x - c)| - r with P = I - a a^T;  inside the band d < band*dx:
      n = P(x - c)/|P(x - c)|  (R e_x on the axis)
      v_co = u + w x (x - c);  v_rel = vg - v_co;  vn = v_rel . n
      vn < 0: vt = v_rel - vn n; |vt| <= -mu vn -> v_rel' = 0,
              else v_rel' = vt + mu vn vt/|vt|;  v_c = v_rel' + v_co
      vn >= 0: v_c = vg
      alpha = min(exp(-d/dx), 1);  v = alpha v_c + (1 - alpha) vg
    """
    dx = p.dx
    a = R[:, 1]
    r = xi - c
    rp = r - (r @ a)[:, None] * a[None, :]
    dist = torch.linalg.norm(rp, dim=-1)
    d = dist - p.cyl_radius
    band = d < p.contact_band * dx
    on_axis = dist <= 0
    dsafe = torch.where(on_axis, torch.ones_like(dist), dist)
    nrm = torch.where(on_axis[:, None], R[:, 0][None, :].expand_as(rp), rp / dsafe[:, None])
    vco = u[None, :] + torch.cross(w[None, :].expand_as(r), r, dim=-1)
    vrel = vg - vco
    vn = (vrel * nrm).sum(-1)
    vt = vrel - vn[:, None] * nrm
    vtn = torch.linalg.norm(vt, dim=-1)
    stick = vtn <= -p.friction * vn
    vtn_safe = torch.where(stick | (vtn <= 0), torch.ones_like(vtn), vtn)
    vrel2 = torch.where(stick[:, None], torch.zeros_like(vt), vt + (p.friction * vn / vtn_safe)[:, None] * vt)
    vc = torch.where((vn < 0)[:, None], vrel2 + vco, vg)
    alpha = torch.clamp(torch.exp(-d / dx), max=1.0)
    out = alpha[:, None] * vc + (1.0 - alpha[:, None]) * vg
    return torch.where(band[:, None], out, vg)


def grid_update(m, mv, pose_c, pose_R, action, p: Params):
    """Grid operations, in this order on every node with m > 0:
    v = mv/m; v += dt g; cylinder soft contact; slip walls (a band of
    ``bound`` nodes on each face zeroes the velocity component pointing out
    of the domain).  Returns v (n^3,3); nodes with m = 0 get v = 0."""
    n, dx, dt = p.n_grid, p.dx, p.dt
    act = torch.nonzero(m > 0)[:, 0]
    ma = m[act]
    vg = mv[act] / ma[:, None] + dt * p.gravity[None, :]
    ii = torch.stack([act // (n * n), (act // n) % n, act % n], -1)
    if p.cyl_radius > 0:
        xi = ii.to(DT) * dx
        vg = cylinder_contact(xi, vg, pose_c, pose_R, action[:3], action[3:], p)
    lo = (ii < p.bound) & (vg < 0)
    hi = (ii > n - 1 - p.bound) & (vg > 0)
    vg = torch.where(lo | hi, torch.zeros_like(vg), vg)
    v = torch.zeros(n ** 3, 3, dtype=DT).index_put((act,), vg)
    return v


def g2p(st, vgrid, p: Params):
    """Grid-to-particle: v' = sum w v_i; C' = (4/dx^2) sum w v_i (x_i - x_p)^T;
    x' = x + dt v'; F_tr = (I + dt C') F; elastic F' = F_tr; liquid
    J' = J det(I + dt C'); sand F' = Drucker-Prager projection of F_tr;
    von Mises F' = von Mises projection of F_tr; Box yield F' = F_tr with its
    singular values clamped."""
    n, dx, dt = p.n_grid, p.dx, p.dt
    base, f, W, dpos = bspline(st["x"], dx)
    idx = node_index(base, n)
    vi = vgrid[idx]                                                   # (N,27,3)
    v_new = (W[:, :, None] * vi).sum(1)
    C_new = (4.0 / dx ** 2) * torch.einsum("pn,pna,pnb->pab", W, vi, dpos)
    x_new = st["x"] + dt * v_new
    I = torch.eye(3, dtype=DT)
    Mdef = I + dt * C_new
    F_tr = Mdef @ st["F"]
    F_new = F_tr
    J_new = st["J"]
    if p.idx_liq.numel():
        i = p.idx_liq
        J_new = J_new.index_put((i,), st["J"][i] * torch.linalg.det(Mdef[i]))
        F_new = F_new.index_put((i,), st["F"][i])      # liquids keep F = I; only J evolves
    if p.idx_sand.numel():
        i = p.idx_sand
        F_new = F_new.index_put((i,), IsotropicMap.apply(F_tr[i], make_g_dp(p.alpha[i], p.kappa[i], p.cohesion[i])))
    if p.idx_vm.numel():
        i = p.idx_vm
        F_new = F_new.index_put((i,), IsotropicMap.apply(F_tr[i], make_g_vm(p.yield_radius[i])))
    if p.idx_box.numel():
        i = p.idx_box
        F_new = F_new.index_put((i,), IsotropicMap.apply(F_tr[i], make_g_box(p.box_lo[i], p.box_hi[i])))
    out = {"x": x_new, "v": v_new, "C": C_new, "F": F_new, "J": J_new}
    for b in p.rigid:
        out = rigid_project(out, b, p)
    for k, t in out.items():
        if not torch.isfinite(t).all():
            raise OracleDomainError(f"non-finite {k}")
    return out


# ----------------------------------------------------------------------------
# Manipulator kinematics
# ----------------------------------------------------------------------------
def integrate_pose(c0, R0, actions, dt):
    """c_{n+1} = c_n + dt u_n;  R_{n+1} = exp(dt [w_n]x) R_n.
    Returns lists of (c_n, R_n) for n = 0..T."""
    cs, Rs = [c0], [R0]
    for t in range(actions.shape[0]):
        cs.append(cs[-1] + dt * actions[t, :3])
        Rs.append(torch.linalg.matrix_exp(dt * skew(actions[t, 3:])) @ Rs[-1])
    return cs, Rs


def step(st, c, R, action, p: Params):
    m, mv = p2g(st, p)
    v = grid_update(m, mv, c, R, action, p)
    return g2p(st, v, p)


def rollout(sc, actions: Optional[torch.Tensor] = None, state=None, steps: Optional[int] = None,
            checkpoint_every: int = 0, params: Optional[Params] = None):
    """Run ``steps`` steps (default: the scene horizon).  Returns the final
    state dict.  With checkpoint_every > 0 the autograd graph is recomputed
    per step (torch.utils.checkpoint) to bound memory."""
    p = params or params_from_scene(sc)
    st = state if state is not None else state_from_scene(sc)
    if actions is None:
        actions = torch.tensor(sc.actions, dtype=DT)
    T = steps if steps is not None else actions.shape[0]
    cs, Rs = integrate_pose(torch.tensor(sc.cyl_pos0, dtype=DT), torch.tensor(sc.cyl_rot0, dtype=DT), actions[:T], p.dt)
    keys = ("x", "v", "C", "F", "J")
    for t in range(T):
        if checkpoint_every:
            def fn(x, v, C, F, J, c, R, a):
                o = step({"x": x, "v": v, "C": C, "F": F, "J": J}, c, R, a, p)
                return tuple(o[k] for k in keys)
            outs = torch.utils.checkpoint.checkpoint(fn, *[st[k] for k in keys], cs[t], Rs[t], actions[t], use_reentrant=False)
            st = dict(zip(keys, outs))
        else:
            st = step(st, cs[t], Rs[t], actions[t], p)
    return st


def blob_loss(x, liquid_mask, mu_g, sigma_g):
    """Expected squared distance of the liquid particles to a Gaussian blob
    N(mu_g, sigma_g^2 I): mean_p |x_p - mu_g|^2 + 3 sigma_g^2."""
    xl = x[liquid_mask]
    return ((xl - mu_g) ** 2).sum(-1).mean() + 3.0 * sigma_g ** 2


def loss_and_action_grad(sc, steps=None, checkpoint_every=1):
    """Config-3 style gradient: L(x_T) w.r.t. the per-step 6-DoF actions."""
    p = params_from_scene(sc)
    acts = torch.tensor(sc.actions, dtype=DT, requires_grad=True)
    st = rollout(sc, actions=acts, steps=steps, checkpoint_every=checkpoint_every, params=p)
    liq = p.kind == LIQUID
    L = blob_loss(st["x"], liq, torch.tensor(sc.target_mu, dtype=DT), sc.target_sigma)
    L.backward()
    return L.detach(), acts.grad.detach()
