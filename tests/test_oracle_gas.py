"""CPU pins of the gas oracle (advection-projection, section 3.2's gas
following Stam 1999): closed forms, the projector identities, a dense
pseudo-inverse on a tiny grid, and finite differences of whole rollouts."""
import math

import numpy as np
import pytest
import torch

from oracle import gas_oracle as G

DT = torch.float64


def params(n=(8, 8, 8), dt=5e-3, buoyancy=0.0, kappa=0.5, sigma=0.15, speed=2.0, src=(0.0, 1.0)):
    return G.GasParams(n=n, h=1.0 / max(n), dt=dt, buoyancy=buoyancy, t_amb=1.0, emit_sigma=sigma,
                       emit_kappa=kappa, emit_speed=speed, src=torch.tensor(src, dtype=DT))


def rand_state(p, seed, scale=1.0, K=2):
    g = torch.Generator().manual_seed(seed)
    st = {q: scale * torch.randn(*G.shape(q, p.n), generator=g, dtype=DT) for q in G.COMPS}
    st["s"] = 1.0 + 0.1 * torch.randn(K, *p.n, generator=g, dtype=DT)
    return G.zero_walls(st)


def test_interp_reproduces_linear_functions():
    p = params(n=(6, 7, 5))
    a = torch.tensor([0.3, -1.2, 2.1], dtype=DT)
    for q in ("u", "v", "w", "c"):
        X = G.points(q, p)
        f = (X @ a + 0.7).reshape(G.shape(q, p.n))
        # interior points of the grid's own interpolation box
        lo = (G.origin(q)) * p.h
        hi = (G.origin(q) + torch.tensor(G.shape(q, p.n), dtype=DT) - 1) * p.h
        g = torch.Generator().manual_seed(1)
        x = lo + (hi - lo) * torch.rand(200, 3, generator=g, dtype=DT)
        assert torch.allclose(G.interp(f, q, x, p), x @ a + 0.7, atol=1e-13)
        # outside: the value at the clamped point
        xo = x + torch.tensor([10.0, 0.0, 0.0], dtype=DT)
        xc = torch.minimum(xo, hi)
        assert torch.allclose(G.interp(f, q, xo, p), xc @ a + 0.7, atol=1e-13)


def test_uniform_flow_translates_linear_scalar_exactly():
    """Advection by a uniform velocity U0 of a linear scalar field gives
    s(x - dt U0) wherever the back-trace stays inside the cell grid."""
    p = params(n=(10, 10, 10), dt=0.01)
    U0 = torch.tensor([0.8, -0.5, 0.3], dtype=DT)
    st = {"u": torch.full(G.shape("u", p.n), U0[0].item(), dtype=DT),
          "v": torch.full(G.shape("v", p.n), U0[1].item(), dtype=DT),
          "w": torch.full(G.shape("w", p.n), U0[2].item(), dtype=DT)}
    a = torch.tensor([1.5, 0.4, -2.0], dtype=DT)
    X = G.points("c", p)
    st["s"] = (X @ a).reshape(1, *p.n)
    out = G.advect(st, p)
    xb = X - p.dt * U0
    lo, hi = 0.5 * p.h, (10 - 0.5) * p.h
    inside = ((xb >= lo) & (xb <= hi)).all(-1)
    assert inside.sum() > 500
    assert torch.allclose(out["s"].reshape(-1)[inside], (xb @ a)[inside], atol=1e-13)
    # the uniform velocity itself is carried unchanged
    for q in G.COMPS:
        assert torch.allclose(out[q], st[q], atol=1e-14)


def test_zero_velocity_advection_is_identity():
    p = params()
    st = rand_state(p, 3)
    for q in G.COMPS:
        st[q] = torch.zeros_like(st[q])
    out = G.advect(st, p)
    assert torch.allclose(out["s"], st["s"], atol=1e-15)


def _inner(a, b):
    return sum((a[q] * b[q]).sum() for q in G.COMPS)


def test_projection_identities():
    p = params(n=(8, 6, 7))
    a, b = rand_state(p, 5), rand_state(p, 6)
    Pa, Pb = G.project(a, p), G.project(b, p)
    # divergence-free, walls closed
    div = G.divergence(Pa["u"], Pa["v"], Pa["w"], p.h)
    assert div.abs().max() < 1e-10 * G.divergence(a["u"], a["v"], a["w"], p.h).abs().max()
    assert Pa["u"][0].abs().max() == 0 and Pa["v"][:, -1].abs().max() == 0
    # idempotent and self-adjoint on wall-closed fields
    PPa = G.project(Pa, p)
    for q in G.COMPS:
        assert torch.allclose(PPa[q], Pa[q], atol=1e-11)
    assert abs(_inner(Pa, b) - _inner(a, Pb)) < 1e-10 * abs(_inner(a, b))
    # gradients of a cell field are removed entirely
    phi = torch.randn(*p.n, generator=torch.Generator().manual_seed(7), dtype=DT)
    gu, gv, gw = G.gradient(phi, p.h)
    Pg = G.project({"u": gu, "v": gv, "w": gw}, p)
    for q in G.COMPS:
        assert Pg[q].abs().max() < 1e-9 * gu.abs().max()


def test_projection_equals_dense_pseudo_inverse_formula():
    """P u = u - G L^+ D u with L^+ from a dense pseudo-inverse (4^3 grid)."""
    p = params(n=(4, 4, 4))
    st = rand_state(p, 8)
    b = G.divergence(st["u"], st["v"], st["w"], p.h).reshape(-1)
    L = torch.tensor(G.laplacian_matrix(p.n, p.h).toarray(), dtype=DT)
    phi = (torch.linalg.pinv(L) @ b).reshape(p.n)
    gu, gv, gw = G.gradient(phi, p.h)
    P = G.project(st, p)
    for q, g in zip(G.COMPS, (gu, gv, gw)):
        assert torch.allclose(P[q], st[q] - g, atol=1e-11)


def test_projection_backward_is_the_projection():
    """Autograd through walls + projection equals the explicit adjoint of the
    linear map (a dense Jacobian built column by column)."""
    p = params(n=(4, 4, 4))
    st = rand_state(p, 9)
    sizes = [st[q].numel() for q in G.COMPS]
    def f(flat):
        parts = torch.split(flat, sizes)
        s = {q: parts[i].reshape(st[q].shape) for i, q in enumerate(G.COMPS)}
        o = G.project(G.zero_walls(s), p)
        return torch.cat([o[q].reshape(-1) for q in G.COMPS])
    x0 = torch.cat([st[q].reshape(-1) for q in G.COMPS])
    n = x0.numel()
    J = torch.stack([f(torch.eye(n, dtype=DT)[i]) for i in range(n)], 1)   # linear: columns = images of e_i
    gout = torch.randn(n, generator=torch.Generator().manual_seed(10), dtype=DT)
    x = x0.clone().requires_grad_(True)
    (f(x) * gout).sum().backward()
    assert torch.allclose(x.grad, J.T @ gout, atol=1e-10)


def test_emitter_and_buoyancy_closed_forms():
    p = params(n=(8, 8, 8), kappa=1.0, buoyancy=2.0)
    st = rand_state(p, 11)
    c = (G.points("c", p)[100]).clone()          # a cell centre
    R = torch.eye(3, dtype=DT)
    out = G.emit(st, c, R, p)
    # kappa = 1: the cell at the centre takes the source values exactly
    for k in range(2):
        assert abs(out["s"][k].reshape(-1)[100].item() - p.src[k].item()) < 1e-15
    # far cells keep their values up to the Gaussian tail
    far = ((G.points("c", p) - c) ** 2).sum(-1) > (6 * p.emit_sigma) ** 2
    assert torch.allclose(out["s"][0].reshape(-1)[far], st["s"][0].reshape(-1)[far], atol=1e-6)
    # buoyancy of a uniform temperature: interior v-faces shift by dt beta (T - T_amb)
    st["s"][0] = 0.25
    b = G.buoyancy(st, p)
    assert torch.allclose(b["v"][:, 1:-1] - st["v"][:, 1:-1],
                          torch.full_like(st["v"][:, 1:-1], p.dt * 2.0 * (0.25 - 1.0)), atol=1e-15)
    assert torch.equal(b["v"][:, 0], st["v"][:, 0])


def _rollout_loss(p, st0, acts, c0, R0, wq, ws):
    st = G.rollout(st0, acts, c0, R0, p)
    return sum((wq[q] * st[q]).sum() for q in G.COMPS) + (ws * st["s"]).sum()


def test_rollout_gradient_fd():
    """Action and initial-state gradients through 3 steps (advection with
    clamped back-traces, emitter, buoyancy, projection): autograd against
    central differences in float64."""
    p = params(n=(8, 8, 8), dt=0.01, buoyancy=1.5)
    st0 = rand_state(p, 12, scale=0.5)
    st0 = G.project(st0, p)
    g = torch.Generator().manual_seed(13)
    acts = 0.5 * torch.randn(3, 6, generator=g, dtype=DT)
    c0 = torch.tensor([0.3, 0.5, 0.45], dtype=DT)
    R0 = torch.tensor([[0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 1.0]], dtype=DT)
    wq = {q: torch.randn(*G.shape(q, p.n), generator=g, dtype=DT) for q in G.COMPS}
    ws = torch.randn(2, *p.n, generator=g, dtype=DT)
    A = acts.clone().requires_grad_(True)
    s0 = {k: v.clone().requires_grad_(True) for k, v in st0.items()}
    L = _rollout_loss(p, s0, A, c0, R0, wq, ws)
    L.backward()
    eps = 1e-6
    for (t, k) in [(0, 0), (0, 4), (1, 3), (2, 1), (1, 5)]:
        ap, am = acts.clone(), acts.clone()
        ap[t, k] += eps
        am[t, k] -= eps
        num = (_rollout_loss(p, st0, ap, c0, R0, wq, ws) - _rollout_loss(p, st0, am, c0, R0, wq, ws)).item() / (2 * eps)
        assert abs(num - A.grad[t, k].item()) <= 1e-6 * max(1.0, abs(num)), (t, k, num, A.grad[t, k].item())
    for (q, idx) in [("u", (3, 4, 2)), ("v", (2, 5, 6)), ("w", (5, 1, 4)), ("s", (0, 3, 3, 3)), ("s", (1, 6, 2, 5))]:
        sp = {k: v.clone() for k, v in st0.items()}
        sm = {k: v.clone() for k, v in st0.items()}
        sp[q][idx] += eps
        sm[q][idx] -= eps
        num = (_rollout_loss(p, sp, acts, c0, R0, wq, ws) - _rollout_loss(p, sm, acts, c0, R0, wq, ws)).item() / (2 * eps)
        assert abs(num - s0[q].grad[idx].item()) <= 1e-6 * max(1.0, abs(num)), (q, idx, num, s0[q].grad[idx].item())


def test_sensor_loss():
    s = torch.zeros(2, 4, 4, 4, dtype=DT)
    s[0] = torch.arange(64, dtype=DT).reshape(4, 4, 4)
    cells = torch.tensor([0, 5, 63])
    targets = torch.tensor([1.0, 5.0, 60.0], dtype=DT)
    assert G.sensor_loss(s, cells, targets).item() == 1.0 + 0.0 + 3.0


def test_cg_pressure_path_equals_direct_path():
    """The conjugate-gradient solve used for grids too large to factorise
    gives the direct solve's projection (32^3, both paths forced)."""
    p = params(n=(32, 32, 32))
    st = rand_state(p, 14)
    a = G.project(st, p)
    old = G.DIRECT_MAX_CELLS
    try:
        G.DIRECT_MAX_CELLS = 0
        b = G.project(st, p)
    finally:
        G.DIRECT_MAX_CELLS = old
    for q in G.COMPS:
        assert torch.allclose(a[q], b[q], atol=1e-10 * a[q].abs().max().item())
