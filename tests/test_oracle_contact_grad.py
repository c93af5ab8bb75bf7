"""Pins of the oracle's manipulator contact, pose integration, liquid J
update and gradients (CPU only).

Contact special cases follow the soft contact model (section 5.1) with
Coulomb friction (section 3.2); the pose is checked against scipy's rotation
vectors; gradients against central finite differences on tiny scenes.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import mpm_oracle as O
from paper_2303_02346_amd import scenes

DT = torch.float64


def contact_params(friction):
    p = O.params_from_scene(scenes.tiny(n_particles=3, n_grid=32))
    p.friction = friction
    p.cyl_radius = 0.1
    return p


def _nodes_near(dist_cells, n=32, c=(0.5, 0.5, 0.5), r=0.1, m=64, seed=0):
    """m node-like points at a given signed distance (in cells) from the
    surface of a vertical cylinder, with their outward normals."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0, 2 * math.pi, m)
    y = rng.uniform(0.3, 0.7, m)
    nrm = np.stack([np.cos(th), np.zeros(m), np.sin(th)], -1)
    rad = r + dist_cells / n
    x = np.array(c) + rad * nrm
    x[:, 1] = y
    return torch.tensor(x, dtype=DT), torch.tensor(nrm, dtype=DT)


def test_contact_frictionless_removes_normal_approach():
    p = contact_params(0.0)
    xi, nrm = _nodes_near(-0.5)                      # inside: alpha = 1
    rng = np.random.default_rng(1)
    vg = torch.tensor(rng.normal(0, 1, (64, 3)), dtype=DT)
    c = torch.tensor([0.5, 0.5, 0.5], dtype=DT)
    out = O.cylinder_contact(xi, vg, c, torch.eye(3, dtype=DT), torch.zeros(3, dtype=DT), torch.zeros(3, dtype=DT), p)
    vn = (vg * nrm).sum(-1)
    ref = torch.where((vn < 0)[:, None], vg - vn[:, None] * nrm, vg)
    assert torch.allclose(out, ref, atol=1e-14)


def test_contact_sticky_and_separating():
    p = contact_params(1e6)
    xi, nrm = _nodes_near(-0.2)
    rng = np.random.default_rng(2)
    vg = torch.tensor(rng.normal(0, 1, (64, 3)), dtype=DT)
    c = torch.tensor([0.5, 0.5, 0.5], dtype=DT)
    u = torch.tensor([0.3, -0.1, 0.2], dtype=DT)
    w = torch.tensor([0.0, 0.0, 0.0], dtype=DT)
    out = O.cylinder_contact(xi, vg, c, torch.eye(3, dtype=DT), u, w, p)
    vn = ((vg - u) * nrm).sum(-1)
    # approaching nodes take the collider velocity, separating ones are untouched
    assert torch.allclose(out[vn < 0], u.expand(int((vn < 0).sum()), 3), atol=1e-14)
    assert torch.allclose(out[vn >= 0], vg[vn >= 0], atol=0)


def test_contact_outside_band_and_blend():
    p = contact_params(0.0)
    c = torch.tensor([0.5, 0.5, 0.5], dtype=DT)
    rng = np.random.default_rng(3)
    vg = -torch.tensor(np.abs(rng.normal(0, 1, (64, 3))), dtype=DT)
    xi, nrm = _nodes_near(3.2)
    out = O.cylinder_contact(xi, vg, c, torch.eye(3, dtype=DT), torch.zeros(3, dtype=DT), torch.zeros(3, dtype=DT), p)
    assert torch.equal(out, vg)
    xi, nrm = _nodes_near(1.5)
    vg = -2.0 * nrm + torch.tensor([0.0, 0.4, 0.0], dtype=DT)     # pure approach plus tangent
    out = O.cylinder_contact(xi, vg, c, torch.eye(3, dtype=DT), torch.zeros(3, dtype=DT), torch.zeros(3, dtype=DT), p)
    a = math.exp(-1.5)
    ref = a * torch.tensor([0.0, 0.4, 0.0], dtype=DT) + (1 - a) * vg
    assert torch.allclose(out, ref, atol=1e-12)


def test_contact_galilean_and_rotation_equivariance():
    """A cylinder moving with u, acting on vg + u, gives the stationary result
    plus u; rotating the whole configuration rotates the result."""
    p = contact_params(0.5)
    rng = np.random.default_rng(4)
    xi, nrm = _nodes_near(0.7, seed=5)
    vg = torch.tensor(rng.normal(0, 1, (64, 3)), dtype=DT)
    c = torch.tensor([0.5, 0.5, 0.5], dtype=DT)
    z = torch.zeros(3, dtype=DT)
    base = O.cylinder_contact(xi, vg, c, torch.eye(3, dtype=DT), z, z, p)
    u = torch.tensor([0.2, 0.7, -0.4], dtype=DT)
    moved = O.cylinder_contact(xi, vg + u, c, torch.eye(3, dtype=DT), u, z, p)
    assert torch.allclose(moved, base + u, atol=1e-13)
    Q = torch.tensor(Rotation.from_rotvec([0.3, -0.5, 0.2]).as_matrix(), dtype=DT)
    xr = (xi - c) @ Q.T + c
    rot = O.cylinder_contact(xr, vg @ Q.T, c, Q, z, z, p)
    assert torch.allclose(rot, base @ Q.T, atol=1e-13)


def test_contact_rigid_rotation_collider_velocity():
    """A spinning cylinder with infinite friction drags approaching nodes to
    u + w x (x - c)."""
    p = contact_params(1e9)
    xi, nrm = _nodes_near(-0.3, seed=6)
    c = torch.tensor([0.5, 0.5, 0.5], dtype=DT)
    w = torch.tensor([0.0, 3.0, 0.0], dtype=DT)
    vg = -1.0 * nrm
    out = O.cylinder_contact(xi, vg, c, torch.eye(3, dtype=DT), torch.zeros(3, dtype=DT), w, p)
    ref = torch.cross(w.expand(64, 3), xi - c, dim=-1)
    assert torch.allclose(out, ref, atol=1e-13)


def test_pose_integration_matches_rotvec():
    T, dt = 50, 1e-3
    w = np.array([0.7, -1.2, 2.0])
    acts = torch.tensor(np.tile(np.concatenate([[0.1, 0.2, -0.3], w]), (T, 1)), dtype=DT)
    R0 = torch.tensor(Rotation.from_rotvec([0.1, 0.0, 0.2]).as_matrix(), dtype=DT)
    c0 = torch.tensor([0.5, 0.5, 0.5], dtype=DT)
    cs, Rs = O.integrate_pose(c0, R0, acts, dt)
    ref = Rotation.from_rotvec(T * dt * w).as_matrix() @ R0.numpy()
    assert np.allclose(Rs[-1].numpy(), ref, atol=1e-14)
    assert np.allclose(cs[-1].numpy(), c0.numpy() + T * dt * np.array([0.1, 0.2, -0.3]), atol=1e-15)


def test_liquid_uniform_dilation_J():
    """A uniform dilation v = s (x - x0) has C' = s I, so each step
    multiplies J by (1 + dt s)^3 exactly."""
    sc = scenes.tiny(n_particles=100, n_grid=24, kinds=(scenes.LIQUID,), with_cylinder=False)
    p = O.params_from_scene(sc)
    p.gravity = torch.zeros(3, dtype=DT)
    n, dx = p.n_grid, p.dx
    s = 0.8
    st = O.state_from_scene(sc)
    lin = torch.arange(n ** 3)
    xi = torch.stack([lin // (n * n), (lin // n) % n, lin % n], -1).to(DT) * dx
    vgrid = s * (xi - 0.5)
    out = O.g2p(st, vgrid, p)
    assert torch.allclose(out["C"], s * torch.eye(3, dtype=DT).expand(sc.n, 3, 3), atol=1e-11)
    assert torch.allclose(out["J"], torch.full((sc.n,), (1 + p.dt * s) ** 3, dtype=DT), atol=1e-14)


def test_liquid_pressure_pushes_outward():
    """A compressed liquid box (J < 1) gains outward momentum at its faces."""
    sc = scenes.tiny(n_particles=400, n_grid=24, kinds=(scenes.LIQUID,), with_cylinder=False)
    sc.v[:] = 0
    sc.J[:] = 0.95
    sc.gravity = (0.0, 0.0, 0.0)
    st = O.rollout(sc, steps=2)
    x0 = torch.tensor(sc.x, dtype=DT)
    cen = x0.mean(0)
    radial = ((x0 - cen) * st["v"]).sum(-1)
    assert radial.mean() > 0


# ---------------------------------------------------------------------------
# Gradients by central finite differences
# ---------------------------------------------------------------------------
def _generic_loss(st, wx, wv):
    return (st["x"] * wx).sum() + (st["v"] * wv).sum()


@pytest.mark.parametrize("seed,kinds", [(0, None), (1, None), (2, (scenes.VONMISES, scenes.LIQUID)),
                                        (3, (scenes.BOX, scenes.LIQUID))])
def test_rollout_gradient_fd(seed, kinds):
    """d L / d actions and d L / d x_0 by autograd against central FD in
    float64 on a tiny scene with the cylinder in contact (5 steps): all three
    base materials, or the von Mises ice cream or the Box-yield plastic with
    water."""
    kw = {} if kinds is None else {"kinds": kinds, "velocity": 3.0}
    sc = scenes.tiny(n_particles=45, n_grid=16, steps=5, seed=seed, **kw)
    rng = np.random.default_rng(100 + seed)
    wx = torch.tensor(rng.normal(0, 1, (sc.n, 3)), dtype=DT)
    wv = torch.tensor(rng.normal(0, 1, (sc.n, 3)), dtype=DT) * 1e-2
    p = O.params_from_scene(sc)
    acts = torch.tensor(sc.actions, dtype=DT, requires_grad=True)
    st0 = O.state_from_scene(sc, requires_grad=True)
    L = _generic_loss(O.rollout(sc, actions=acts, state=st0, params=p), wx, wv)
    L.backward()
    def Lof(a, x0):
        st = O.state_from_scene(sc)
        st["x"] = x0
        return _generic_loss(O.rollout(sc, actions=a, state=st, params=p), wx, wv).item()
    a0 = torch.tensor(sc.actions, dtype=DT)
    x0 = torch.tensor(sc.x, dtype=DT)
    eps = 1e-6
    ga = acts.grad
    assert ga.abs().max() > 0
    for (t, k) in [(0, 0), (1, 3), (2, 1), (4, 5), (3, 2), (0, 4)]:
        ap, am = a0.clone(), a0.clone()
        ap[t, k] += eps
        am[t, k] -= eps
        num = (Lof(ap, x0) - Lof(am, x0)) / (2 * eps)
        assert abs(num - ga[t, k].item()) <= 1e-6 * max(1.0, abs(num)), (t, k, num, ga[t, k].item())
    gx = st0["x"].grad
    for (q, a) in [(0, 0), (7, 1), (20, 2), (33, 0), (44, 1)]:
        xp, xm = x0.clone(), x0.clone()
        xp[q, a] += eps
        xm[q, a] -= eps
        num = (Lof(a0, xp) - Lof(a0, xm)) / (2 * eps)
        assert abs(num - gx[q, a].item()) <= 1e-6 * max(1.0, abs(num)), (q, a, num, gx[q, a].item())


def test_blob_loss_gradient_with_checkpointing_matches_plain():
    sc = scenes.tiny(n_particles=45, n_grid=16, steps=4, seed=3)
    L1, g1 = O.loss_and_action_grad(sc, checkpoint_every=1)
    L0, g0 = O.loss_and_action_grad(sc, checkpoint_every=0)
    assert abs(L1.item() - L0.item()) < 1e-15
    assert torch.allclose(g1, g0, atol=1e-14)


def test_blob_loss_closed_form():
    x = torch.tensor([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [5.0, 5.0, 5.0]], dtype=DT)
    mask = torch.tensor([True, True, False])
    L = O.blob_loss(x, mask, torch.tensor([0.5, 0.0, 0.0], dtype=DT), 0.1)
    assert abs(L.item() - (0.25 + 3 * 0.01)) < 1e-15


# ---------------------------------------------------------------------------
# rigid bodies represented by particles
# ---------------------------------------------------------------------------
def _rigid_scene(steps=6, **kw):
    return scenes.tiny(n_particles=200, n_grid=24, steps=steps, seed=3, kinds=(scenes.RIGID, scenes.LIQUID),
                       velocity=1.0, **kw)


def test_rigid_projection_keeps_shape_and_momenta():
    """After the projection the body is its rest shape moved rigidly, its
    velocities are a rigid field, and its linear and angular momentum
    (about the centroid) equal those of the elastic state it came from."""
    sc = _rigid_scene()
    p = O.params_from_scene(sc)
    b = p.rigid[0]
    i = b["idx"]
    rng = np.random.default_rng(50)
    st = O.state_from_scene(sc)
    st["x"] = st["x"] + torch.tensor(rng.normal(0, 1e-3, (sc.n, 3)), dtype=DT)   # a deformed elastic state
    st["v"] = torch.tensor(rng.normal(0, 0.5, (sc.n, 3)), dtype=DT)
    out = O.rigid_project(st, b, p)
    m = p.mass[i][:, None]
    x0, v0, x1, v1 = st["x"][i], st["v"][i], out["x"][i], out["v"][i]
    X = torch.tensor(sc.x, dtype=DT)[i]
    d1 = (x1[:, None] - x1[None]).norm(dim=-1)
    d0 = (X[:, None] - X[None]).norm(dim=-1)
    assert (d1 - d0).abs().max() < 1e-15
    c0 = (m * x0).sum(0) / m.sum()
    c1 = (m * x1).sum(0) / m.sum()
    assert torch.allclose(c0, c1, atol=1e-15)
    assert torch.allclose((m * v1).sum(0), (m * v0).sum(0), atol=1e-14)
    L0 = (m * torch.cross(x0 - c0, v0 - (m * v0).sum(0) / m.sum(), dim=-1)).sum(0)
    L1 = (m * torch.cross(x1 - c1, v1, dim=-1)).sum(0)
    assert torch.allclose(L1, L0, atol=1e-15)
    W = out["C"][i[0]]
    w = torch.stack([W[2, 1], W[0, 2], W[1, 0]])
    assert torch.allclose(W, -W.T, atol=0)
    assert torch.allclose(v1 - (m * v1).sum(0) / m.sum(), torch.cross(w.expand_as(x1), x1 - c1, dim=-1), atol=1e-15)
    R = out["F"][i[0]]
    assert torch.allclose(R @ R.T, torch.eye(3, dtype=DT), atol=1e-14) and abs(torch.linalg.det(R) - 1) < 1e-14


def test_rigid_body_in_free_fall():
    """A rigid body alone, at rest, without collider: it falls as a point
    mass, x_n = X + g dt^2 n (n + 1) / 2, and keeps its shape exactly."""
    sc = scenes.tiny(n_particles=120, n_grid=24, steps=20, seed=4, kinds=(scenes.RIGID,), velocity=0.0,
                     with_cylinder=False)
    st = O.rollout(sc)
    n, dt = 20, sc.dt
    ref = torch.tensor(sc.x, dtype=DT) + torch.tensor([0.0, -9.8, 0.0], dtype=DT) * dt * dt * n * (n + 1) / 2
    assert torch.allclose(st["x"], ref, atol=1e-13)


def test_rigid_rollout_gradient_fd():
    """Action and initial-position gradients through a rigid body in contact
    with water and the cylinder, autograd against central FD (float64)."""
    sc = scenes.tiny(n_particles=60, n_grid=16, steps=5, seed=5, kinds=(scenes.RIGID, scenes.LIQUID), velocity=1.0)
    rng = np.random.default_rng(105)
    wx = torch.tensor(rng.normal(0, 1, (sc.n, 3)), dtype=DT)
    wv = torch.tensor(rng.normal(0, 1, (sc.n, 3)), dtype=DT) * 1e-2
    p = O.params_from_scene(sc)
    acts = torch.tensor(sc.actions, dtype=DT, requires_grad=True)
    st0 = O.state_from_scene(sc, requires_grad=True)
    L = _generic_loss(O.rollout(sc, actions=acts, state=st0, params=p), wx, wv)
    L.backward()
    def Lof(a, x0):
        st = O.state_from_scene(sc)
        st["x"] = x0
        return _generic_loss(O.rollout(sc, actions=a, state=st, params=p), wx, wv).item()
    a0 = torch.tensor(sc.actions, dtype=DT)
    x0 = torch.tensor(sc.x, dtype=DT)
    eps = 1e-6
    for (t, k) in [(0, 0), (1, 3), (2, 1), (4, 5)]:
        ap, am = a0.clone(), a0.clone()
        ap[t, k] += eps
        am[t, k] -= eps
        num = (Lof(ap, x0) - Lof(am, x0)) / (2 * eps)
        assert abs(num - acts.grad[t, k].item()) <= 1e-6 * max(1.0, abs(num))
    for (q, a) in [(0, 0), (10, 1), (29, 2), (31, 0), (50, 1)]:
        xp, xm = x0.clone(), x0.clone()
        xp[q, a] += eps
        xm[q, a] -= eps
        num = (Lof(a0, xp) - Lof(a0, xm)) / (2 * eps)
        assert abs(num - st0["x"].grad[q, a].item()) <= 1e-6 * max(1.0, abs(num)), (q, a)
