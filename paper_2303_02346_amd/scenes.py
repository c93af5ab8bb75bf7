"""Seeded synthetic scenes for the MLS-MPM step.

This module only draws inputs: particle boxes, materials, the cylinder
trajectory and the loss target.  It holds none of the method's arithmetic
(no transfer, stress, contact or projection).  Both the FP64 CPU oracle (via
the tests) and the HIP path are fed from the arrays built here; the HIP path
receives an FP32 cast.

Shapes follow the paper's task setting: 6-DoF end-effector velocity actions
(section 4.2), Table 4 material constants, substeps of order 1e-4 s
(Appendix B.1) and ~1e5 particles on a 64^3 grid.  The task meshes and goal
patterns of the paper are not available; seeded boxes of particles and a
seeded Gaussian target blob stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

ELASTIC = 0   # fixed-corotated elastic solid
LIQUID = 1    # weakly compressible liquid, J-based pressure + Newtonian viscosity
SAND = 2      # Hencky elasticity + Drucker-Prager plasticity
VONMISES = 3  # Hencky elasticity + von Mises plasticity (the non-Newtonian ice cream)
BOX = 4       # corotated elasticity + Box yield (the plastic material, Stomakhin 2013)
RIGID = 5     # rigid body from particles: corotated update, then the object-level rigid projection

# Table 4 (Appendix B.1) constants used by the synthetic scenes.
WATER_LAMBDA = 277.78
SOLID_MU = 416.67
SOLID_LAMBDA = 277.78


ICE_CREAM_YIELD = 5.0   # not in Table 4; deviatoric flow from |dev log strain| = 0.006


def ice_cream():
    """Table 4's non-Newtonian ice cream (mu 416.67, lambda 277.78, rho 0.5)
    as a von Mises elastoplastic continuum."""
    return Material(VONMISES, SOLID_MU, SOLID_LAMBDA, 0.5, yield_stress=ICE_CREAM_YIELD)


def plasticine():
    """A Box-yield plastic with Table 4's solid constants (mu 416.67,
    lambda 277.78, rho 1) and Stomakhin et al.'s critical compression and
    stretch (2.5e-2, 7.5e-3)."""
    return Material(BOX, SOLID_MU, SOLID_LAMBDA, 1.0, theta_c=2.5e-2, theta_s=7.5e-3)


def rigid_object():
    """Table 4's rigid object (mu 416.67, lambda 277.78, rho 5.0)."""
    return Material(RIGID, SOLID_MU, SOLID_LAMBDA, 5.0)


def lame(E: float, nu: float):
    """Lame parameters from Young's modulus and Poisson ratio (input recipe)."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


@dataclasses.dataclass
class Material:
    kind: int
    mu: float = 0.0
    lam: float = 0.0
    rho: float = 1.0
    viscosity: float = 0.0
    friction_deg: float = 30.0
    cohesion: float = 0.0
    yield_stress: float = 0.0   # von Mises yield stress (Kirchhoff)
    theta_c: float = 0.0        # Box yield: critical compression
    theta_s: float = 0.0        # Box yield: critical stretch
    p_vol: float = 0.0    # initial particle volume V_p = V_box / N_box
    p_mass: float = 0.0   # m_p = rho * V_p


@dataclasses.dataclass
class Scene:
    n_grid: int
    dt: float
    x: np.ndarray                  # (N,3) float64
    v: np.ndarray                  # (N,3)
    C: np.ndarray                  # (N,3,3)
    F: np.ndarray                  # (N,3,3)
    J: np.ndarray                  # (N,)
    mat: np.ndarray                # (N,) int32 index into materials
    materials: List[Material]
    actions: np.ndarray            # (T,6): ux uy uz wx wy wz, world frame
    gravity: tuple = (0.0, -9.8, 0.0)
    bound: int = 3                 # slip-wall band, in nodes
    cyl_radius: float = 0.05       # <= 0 disables the manipulator
    cyl_pos0: np.ndarray = dataclasses.field(default_factory=lambda: np.array([0.5, 0.5, 0.5]))
    cyl_rot0: np.ndarray = dataclasses.field(default_factory=lambda: np.eye(3))
    contact_band: float = 3.0      # contact threshold epsilon, in cells
    contact_friction: float = 0.5  # Coulomb coefficient
    target_mu: Optional[np.ndarray] = None
    target_sigma: float = 0.05
    name: str = ""

    @property
    def n(self) -> int:
        return self.x.shape[0]

    @property
    def horizon(self) -> int:
        return self.actions.shape[0]

    def copy(self) -> "Scene":
        return dataclasses.replace(
            self, x=self.x.copy(), v=self.v.copy(), C=self.C.copy(), F=self.F.copy(),
            J=self.J.copy(), mat=self.mat.copy(), actions=self.actions.copy(),
            materials=[dataclasses.replace(m) for m in self.materials])


def _rngs(config_id: int, n: int = 4):
    ss = np.random.SeedSequence(20230302 + config_id)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def _box_particles(rng, lo, hi, count):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    return lo + (hi - lo) * rng.random((count, 3))


def _assemble(n_grid, dt, boxes, actions, **kw) -> Scene:
    """boxes: list of (positions (k,3), Material, box_volume)."""
    xs, mats, materials = [], [], []
    for idx, (pos, m, vol) in enumerate(boxes):
        m = dataclasses.replace(m)
        m.p_vol = vol / pos.shape[0]
        m.p_mass = m.rho * m.p_vol
        materials.append(m)
        xs.append(pos)
        mats.append(np.full(pos.shape[0], idx, np.int32))
    x = np.concatenate(xs, 0)
    N = x.shape[0]
    return Scene(n_grid=n_grid, dt=dt, x=x, v=np.zeros((N, 3)), C=np.zeros((N, 3, 3)),
                 F=np.tile(np.eye(3), (N, 1, 1)), J=np.ones(N), mat=np.concatenate(mats),
                 materials=materials, actions=actions, **kw)


def smooth_actions(rng, T: int, dt: float, u_mean=(0.0, 0.0, 0.0),
                   amp_u: float = 0.5, amp_w: float = 2.0) -> np.ndarray:
    """Seeded smooth 6-DoF velocity trajectory: per component a sum of three
    sines with random amplitude and phase over the horizon T*dt."""
    Th = T * dt
    t = np.arange(T) * dt
    out = np.zeros((T, 6))
    for k in range(6):
        amp = amp_u if k < 3 else amp_w
        A = rng.uniform(-amp, amp, 3)
        ph = rng.uniform(0.0, 2.0 * math.pi, 3)
        for m in range(3):
            out[:, k] += A[m] * np.sin(2.0 * math.pi * (m + 1) * t / Th + ph[m])
    out[:, :3] += np.asarray(u_mean)
    return out


def config1(n_particles: int = 4096, steps: int = 100, affine: bool = False) -> Scene:
    """4096 fixed-corotated particles (E=5e3, nu=0.2, rho=1) uniform in
    [0.3,0.5]^3, 32^3 grid, dt=1e-4, 100 steps, no manipulator.
    ``affine`` gives the particles a seeded affine velocity (rotation plus
    shear, |v| ~ 0.5) so that the stress path is exercised."""
    r_geo, r_pos, r_traj, r_aff = _rngs(1)
    mu, lam = lame(5e3, 0.2)
    pos = _box_particles(r_pos, [0.3] * 3, [0.5] * 3, n_particles)
    sc = _assemble(32, 1e-4, [(pos, Material(ELASTIC, mu, lam, 1.0), 0.2 ** 3)],
                   np.zeros((steps, 6)), cyl_radius=0.0, name="c1b" if affine else "c1")
    if affine:
        w = r_aff.uniform(-1, 1, 3)
        w *= 2.0 / np.linalg.norm(w)
        S = r_aff.uniform(-1, 1, (3, 3))
        S = 0.5 * (S + S.T)
        S *= 1.5 / np.linalg.norm(S)
        G = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]) + S
        sc.v = (sc.x - 0.4) @ G.T
        sc.C = np.tile(G, (sc.n, 1, 1))
    return sc


def _two_box_scene(cfg_id: int, n_particles: int, n_grid: int, dt: float, steps: int,
                   side: float = 0.2, second: "Material" = None) -> Scene:
    r_geo, r_pos, r_traj, r_tgt = _rngs(cfg_id)
    dx = 1.0 / n_grid
    y0 = 5 * dx                       # two cells above the 3-node floor band
    # liquid box and sand box side by side along x, seeded x/z placement
    while True:
        xl = r_geo.uniform(0.1 + 0.05 + dx, 0.9 - 2 * side - 0.02)
        gap = r_geo.uniform(0.02, 0.9 - (xl + 2 * side))
        zl = r_geo.uniform(0.1, 0.9 - side)
        zs = r_geo.uniform(0.1, 0.9 - side)
        if xl + 2 * side + gap <= 0.9:
            break
    n_liq = n_particles // 2
    n_sand = n_particles - n_liq
    liq_lo = np.array([xl, y0, zl])
    sand_lo = np.array([xl + side + gap, y0, zs])
    pl = _box_particles(r_pos, liq_lo, liq_lo + side, n_liq)
    ps = _box_particles(r_pos, sand_lo, sand_lo + side, n_sand)
    liquid = Material(LIQUID, 0.0, WATER_LAMBDA, 1.0, viscosity=0.1)
    sand = Material(SAND, SOLID_MU, SOLID_LAMBDA, 1.0, friction_deg=30.0, cohesion=0.0) if second is None else second
    acts = smooth_actions(r_traj, steps, dt, u_mean=(0.5, 0.0, 0.0))
    # cylinder one cell from the liquid box's -x face, moving into the box on average
    c0 = np.array([xl - 0.05 - dx, 0.5, zl + 0.5 * side])
    sc = _assemble(n_grid, dt, [(pl, liquid, side ** 3), (ps, sand, side ** 3)], acts,
                   cyl_radius=0.05, cyl_pos0=c0, cyl_rot0=np.eye(3))
    sc.target_mu = np.array([r_tgt.uniform(0.3, 0.7), r_tgt.uniform(0.1, 0.3), r_tgt.uniform(0.3, 0.7)])
    sc.target_sigma = 0.05
    return sc


def config2(n_particles: int = 250_000, steps: int = 200, sand_stir: float = 0.0) -> Scene:
    """250k particles (half liquid, half Drucker-Prager sand) in two seeded
    cubes of side 0.2, kinematic cylinder r=0.05, 128^3, dt=5e-5.

    The sand of config 2 falls freely for its 200 steps (it starts two cells
    above the floor band), so all its returns are of the elastic case.  With
    sand_stir > 0 the sand box instead starts with a seeded smooth velocity
    field of that amplitude (m/s): per component a plane wave
    A sin(k.x + phase) with |k| = 2 pi / 0.2 in a seeded direction, which
    compresses, stretches and shears the sand, so that apex, inside and cone
    returns all occur within a few steps."""
    sc = _two_box_scene(2, n_particles, 128, 5e-5, steps)
    sc.name = "c2"
    if sand_stir > 0.0:
        rng = np.random.default_rng(np.random.SeedSequence(20230302 + 2, spawn_key=(9,)))
        sand = sc.mat == 1
        xs = sc.x[sand]
        v = np.zeros_like(xs)
        for a in range(3):
            d = rng.normal(size=3)
            k = 2.0 * math.pi / 0.2 * d / np.linalg.norm(d)
            v[:, a] = sand_stir * np.sin(xs @ k + rng.uniform(0.0, 2.0 * math.pi))
        sc.v[sand] = v
        sc.name = "c2stir"
    return sc


def rigid_config2(n_particles: int = 250_000, steps: int = 200) -> Scene:
    """Config-2 geometry with the sand box replaced by a rigid body of
    Table 4's rigid object (rho 5.0): water pushed by the cylinder towards a
    rigid cube; 250k particles, 128^3, dt=5e-5."""
    sc = _two_box_scene(2, n_particles, 128, 5e-5, steps, second=rigid_object())
    sc.name = "c2r"
    return sc


def config3(n_particles: int = 100_000, steps: int = 64) -> Scene:
    """Config-2 scene at 100k particles on 96^3 over 64 steps, with a seeded
    Gaussian target blob for the loss."""
    sc = _two_box_scene(3, n_particles, 96, 5e-5, steps)
    sc.name = "c3"
    return sc


def config4(n_scenes: int = 64, steps: int = 100, n_min: int = 10_000, n_max: int = 200_000,
            scale: float = 1.0) -> List[Scene]:
    """Independent 64^3 scenes with log-uniform particle counts in
    [n_min, n_max], 1-3 seeded boxes each of elastic, liquid or sand,
    dt=1e-4.  ``scale`` multiplies the counts (for small test versions)."""
    r_geo, r_pos, r_traj, r_cnt = _rngs(4)
    scenes = []
    n_grid, dt = 64, 1e-4
    dx = 1.0 / n_grid
    for s in range(n_scenes):
        Ns = int(math.floor(math.exp(r_cnt.uniform(math.log(n_min), math.log(n_max))) * scale))
        Ns = max(Ns, 8)
        nbox = int(r_geo.integers(1, 4))
        counts = np.full(nbox, Ns // nbox)
        counts[0] += Ns - counts.sum()
        boxes = []
        for b in range(nbox):
            kind = int(r_geo.integers(0, 3))
            side = 0.16
            lo = np.array([0.12 + b * 0.26, 5 * dx, r_geo.uniform(0.12, 0.72)])
            pos = _box_particles(r_pos, lo, lo + side, int(counts[b]))
            if kind == ELASTIC:
                m = Material(ELASTIC, SOLID_MU, SOLID_LAMBDA, 0.5)
            elif kind == LIQUID:
                m = Material(LIQUID, 0.0, WATER_LAMBDA, 1.0, viscosity=0.1)
            else:
                m = Material(SAND, SOLID_MU, SOLID_LAMBDA, 1.0, friction_deg=30.0)
            boxes.append((pos, m, side ** 3))
        acts = smooth_actions(r_traj, steps, dt, u_mean=(0.3, 0.0, 0.0))
        c0 = np.array([0.06, 0.5, r_geo.uniform(0.3, 0.7)])
        sc = _assemble(n_grid, dt, boxes, acts, cyl_radius=0.05, cyl_pos0=c0)
        sc.name = f"c4s{s}"
        scenes.append(sc)
    return scenes


def paper_point(n_particles: int = 100_000, steps: int = 200) -> Scene:
    """The paper's operating point (section 4.2, App. B.1): about 1e5
    particles on a 64^3 grid at substeps of 1e-4 s.  Three boxes of Table 4
    materials (water, a viscous liquid, an elastic solid) on the floor band
    and the cylinder stirring the water with a seeded trajectory."""
    r_geo, r_pos, r_traj, r_tgt = _rngs(6)
    n_grid, dt = 64, 1e-4
    dx = 1.0 / n_grid
    per = [n_particles // 3] * 3
    per[0] += n_particles - sum(per)
    side = 0.2
    mats = [Material(LIQUID, 0.0, WATER_LAMBDA, 1.0),
            Material(LIQUID, 0.0, WATER_LAMBDA, 1.0, viscosity=0.1),
            Material(ELASTIC, SOLID_MU, SOLID_LAMBDA, 1.0)]
    boxes = []
    for b in range(3):
        lo = np.array([0.12 + 0.27 * b, 3 * dx, r_geo.uniform(0.2, 0.6)])
        boxes.append((_box_particles(r_pos, lo, lo + side, per[b]), mats[b], side ** 3))
    acts = smooth_actions(r_traj, steps, dt, u_mean=(0.0, 0.0, 0.3))
    c0 = np.array([0.22, 0.5, boxes[0][0][:, 2].mean()])
    return _assemble(n_grid, dt, boxes, acts, cyl_radius=0.05, cyl_pos0=c0, name="paper64")


def config5(n_particles: int = 1_000_000, steps: int = 100) -> Scene:
    """1M sand particles in a 0.2x0.3x0.2 box hitting the floor of a 256^3
    grid at 1 m/s (its base is inside the wall band from the first step),
    dt=2.5e-5."""
    r_geo, r_pos, r_traj, r_tgt = _rngs(5)
    n_grid, dt = 256, 2.5e-5
    dx = 1.0 / n_grid
    lo = np.array([0.4, 3 * dx, 0.4])
    pos = _box_particles(r_pos, lo, lo + np.array([0.2, 0.3, 0.2]), n_particles)
    sand = Material(SAND, SOLID_MU, SOLID_LAMBDA, 1.0, friction_deg=30.0)
    sc = _assemble(n_grid, dt, [(pos, sand, 0.2 * 0.3 * 0.2)], np.zeros((steps, 6)),
                   cyl_radius=0.0, name="c5")
    sc.v[:, 1] = -1.0
    return sc


def tiny(n_particles: int = 125, n_grid: int = 16, steps: int = 10, seed: int = 0,
         kinds=(ELASTIC, LIQUID, SAND), with_cylinder: bool = True, dt: float = 2e-4,
         velocity: float = 0.3) -> Scene:
    """Small seeded scene for gradient and parity tests: one box per material
    kind, random initial velocities, optional cylinder inside the contact band."""
    rng = np.random.default_rng(np.random.SeedSequence([20230302, 99, seed]))
    dx = 1.0 / n_grid
    boxes = []
    k = len(kinds)
    per = [n_particles // k] * k
    per[0] += n_particles - sum(per)
    for b, kind in enumerate(kinds):
        side = 0.22
        lo = np.array([0.3 + 0.0 * b, 0.25 + 0.25 * (b % 2), 0.2 + 0.22 * b])
        lo = np.minimum(lo, 0.75 - side)
        pos = _box_particles(rng, lo, lo + side, per[b])
        if kind == ELASTIC:
            m = Material(ELASTIC, SOLID_MU, SOLID_LAMBDA, 1.0)
        elif kind == LIQUID:
            m = Material(LIQUID, 0.0, WATER_LAMBDA, 1.0, viscosity=0.1)
        elif kind == VONMISES:
            m = ice_cream()
        elif kind == BOX:
            m = plasticine()
        elif kind == RIGID:
            m = rigid_object()
        else:
            m = Material(SAND, SOLID_MU, SOLID_LAMBDA, 1.0, friction_deg=30.0, cohesion=0.0)
        boxes.append((pos, m, side ** 3))
    acts = smooth_actions(rng, steps, dt, u_mean=(0.5, 0.0, 0.0), amp_u=0.5, amp_w=2.0)
    sc = _assemble(n_grid, dt, boxes, acts, cyl_radius=0.08 if with_cylinder else 0.0,
                   cyl_pos0=np.array([0.2, 0.5, 0.45]))
    sc.v = rng.uniform(-velocity, velocity, (sc.n, 3))
    sc.target_mu = np.array([0.5, 0.3, 0.5])
    sc.name = f"tiny{seed}"
    return sc


def concat_scenes(scenes: List[Scene]):
    """Concatenate independent scenes for a batched launch: returns the
    particle arrays, the per-scene offsets and the per-scene material tables
    (material indices are made global)."""
    offs = [0]
    mats = []
    parts = {k: [] for k in ("x", "v", "C", "F", "J", "mat")}
    for sc in scenes:
        base = len(mats)
        mats.extend(sc.materials)
        for k in parts:
            a = getattr(sc, k)
            parts[k].append(a + base if k == "mat" else a)
        offs.append(offs[-1] + sc.n)
    out = {k: np.concatenate(v, 0) for k, v in parts.items()}
    return out, np.asarray(offs, np.int64), mats


# ----------------------------------------------------------------------------
# Gas (section 3.2's advection-projection gas; the air-circulation task)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class GasScene:
    n: tuple                       # cells per axis (nx, ny, nz)
    h: float                       # cell size
    dt: float
    u: np.ndarray                  # (nx+1, ny, nz) x-face velocities
    v: np.ndarray                  # (nx, ny+1, nz)
    w: np.ndarray                  # (nx, ny, nz+1)
    s: np.ndarray                  # (K, nx, ny, nz) scalars; 0 = temperature, 1 = smoke density
    actions: np.ndarray            # (T, 6) emitter velocities ux uy uz wx wy wz (world frame)
    src: tuple = (0.0, 1.0)        # emitter source values of the scalars (cool air, smoke)
    buoyancy: float = 1.0          # v += dt beta (T - T_amb)
    t_amb: float = 1.0
    emit_sigma: float = 0.04
    emit_kappa: float = 0.5
    emit_speed: float = 2.0
    emit_pos0: tuple = (0.15, 0.6, 0.5)
    # local y axis (the outflow direction) along +x
    emit_rot0: tuple = (0.0, 1.0, 0.0, -1.0, 0.0, 0.0, 0.0, 0.0, 1.0)
    sensors: np.ndarray = None     # (M,) flat cell indices of temperature sensors
    targets: np.ndarray = None     # (M,) target temperatures
    name: str = "gas"

    @property
    def horizon(self):
        return self.actions.shape[0]


def gas_room(n=128, steps: int = 100, seed: int = 0, dt: float = 5e-3, velocity: float = 0.5,
             n_scalars: int = 2, translate: bool = False, **kw) -> GasScene:
    """A closed room of warm air (T = 1 with seeded smooth variations) and a
    cool-air emitter near the -x wall that swings about the vertical axis
    (the air-circulation task of section 4.1 on the 128^3 gas grid of
    section 4.2).  The initial velocity is a seeded smooth field (not
    divergence-free: the first projection removes its divergent part).  27
    temperature sensors sit on a 3x3x3 lattice with seeded cool/warm targets.
    translate: also move the emitter (small seeded translational velocities).
    n: cells per axis, or (nx, ny, nz) for a box of cell size 1 / max(n);
    other keyword arguments override GasScene fields (emitter, buoyancy)."""
    dims = tuple(int(a) for a in n) if hasattr(n, "__len__") else (int(n),) * 3
    cube = dims[0] == dims[1] == dims[2]
    rng = np.random.default_rng(np.random.SeedSequence([20230302, 77, dims[0], seed] if cube else
                                                       [20230302, 77, *dims, seed]))
    h = 1.0 / max(dims)

    def smooth(shape, amp):
        # sum of a few seeded low-frequency modes sampled on the grid points
        idx = np.meshgrid(*[np.arange(m, dtype=np.float64) for m in shape], indexing="ij")
        out = np.zeros(shape)
        for _ in range(4):
            k = rng.integers(1, 4, 3)
            ph = rng.uniform(0, 2 * math.pi, 3)
            a = rng.uniform(-amp, amp)
            out += a * np.sin(math.pi * k[0] * idx[0] / shape[0] + ph[0]) * \
                np.sin(math.pi * k[1] * idx[1] / shape[1] + ph[1]) * np.sin(math.pi * k[2] * idx[2] / shape[2] + ph[2])
        return out

    nx, ny, nz = dims
    u = smooth((nx + 1, ny, nz), velocity)
    v = smooth((nx, ny + 1, nz), velocity)
    w = smooth((nx, ny, nz + 1), velocity)
    u[0] = u[-1] = 0.0
    v[:, 0] = v[:, -1] = 0.0
    w[:, :, 0] = w[:, :, -1] = 0.0
    s = np.zeros((n_scalars,) + dims)
    s[0] = 1.0 + 0.05 * smooth(dims, 1.0)
    acts = smooth_actions(rng, steps, dt, amp_u=0.2 if translate else 0.0, amp_w=2.0)
    acts[:, 3] = 0.0
    acts[:, 5] = 0.0                       # the air conditioner turns about y only
    if not translate:
        acts[:, :3] = 0.0
    lat = [[int(round(f * d)) for f in (0.2, 0.5, 0.8)] for d in dims]
    sensors = np.array([(i * ny + j) * nz + k for i in lat[0] for j in lat[1] for k in lat[2]], np.int64)
    targets = np.where(rng.random(sensors.size) < 0.5, 0.0, 1.0)
    sc = GasScene(n=dims, h=h, dt=dt, u=u, v=v, w=w, s=s, actions=acts, sensors=sensors, targets=targets,
                  src=(0.0, 1.0)[:n_scalars] if n_scalars <= 2 else tuple([0.0, 1.0] + [0.5] * (n_scalars - 2)),
                  name=f"gas{nx}x{ny}x{nz}_{seed}")
    for k, val in kw.items():
        if not hasattr(sc, k):
            raise TypeError(f"unknown GasScene field {k}")
        setattr(sc, k, val)
    return sc
