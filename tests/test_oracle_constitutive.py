"""Pins of the oracle's constitutive models, SVD/polar routines, their
hand-written derivatives and the Drucker-Prager return map (CPU only).

References: LAPACK SVD (numpy), scipy's polar decomposition, closed forms at
special deformations, and central finite differences.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import torch
from scipy.spatial.transform import Rotation

from oracle import mpm_oracle as O

DT = torch.float64
MU, LAM = 416.67, 277.78


def rand_F(rng, n, strain=0.2):
    return np.eye(3) + rng.normal(0, strain, (n, 3, 3))


def test_signed_svd_properties():
    rng = np.random.default_rng(0)
    F = rand_F(rng, 200, 0.5)
    F[:20] = F[:20] @ np.diag([1, 1, -1])          # some inverted F
    U, s, V = O.signed_svd(F)
    assert np.allclose(U @ (s[:, :, None] * np.swapaxes(V, -1, -2)), F, atol=1e-13)
    assert np.allclose(np.linalg.det(U), 1.0) and np.allclose(np.linalg.det(V), 1.0)
    assert np.all(np.sign(s[:, 2]) == np.sign(np.linalg.det(F)))
    assert np.all(s[:, 0] >= s[:, 1]) and np.all(s[:, 1] >= np.abs(s[:, 2]))


def test_polar_matches_scipy():
    rng = np.random.default_rng(1)
    F = rand_F(rng, 50, 0.3)
    F = F[np.linalg.det(F) > 0]
    R = O.polar_rotation(torch.tensor(F)).numpy()
    for q in range(F.shape[0]):
        u, pmat = scipy.linalg.polar(F[q])
        assert np.allclose(R[q], u, atol=1e-12)
        S = R[q].T @ F[q]
        assert np.allclose(S, S.T, atol=1e-12)
        assert np.all(np.linalg.eigvalsh(0.5 * (S + S.T)) > 0)


def test_fixed_corotated_closed_forms():
    n = 40
    mu = torch.full((n,), 2083.33, dtype=DT)
    lam = torch.full((n,), 1388.89, dtype=DT)
    Rs = torch.tensor(Rotation.random(n, random_state=2).as_matrix(), dtype=DT)
    assert O.stress_fixed_corotated(Rs, mu, lam).abs().max() < 1e-9       # tau(R) = 0
    s = torch.linspace(0.8, 1.2, n, dtype=DT)
    tau = O.stress_fixed_corotated(s[:, None, None] * torch.eye(3, dtype=DT), mu, lam)
    ref = (2 * mu * s * (s - 1) + lam * s ** 3 * (s ** 3 - 1))[:, None, None] * torch.eye(3, dtype=DT)
    assert torch.allclose(tau, ref, atol=1e-9)
    rng = np.random.default_rng(3)
    F = torch.tensor(rand_F(rng, n, 0.3), dtype=DT)
    F = F[torch.linalg.det(F) > 0]
    t = O.stress_fixed_corotated(F, mu[: F.shape[0]], lam[: F.shape[0]])
    assert torch.allclose(t, t.transpose(-1, -2), atol=1e-9)
    # rotating the deformation rotates the stress: tau(Q F) = Q tau(F) Q^T
    Q = torch.tensor(Rotation.random(F.shape[0], random_state=4).as_matrix(), dtype=DT)
    t2 = O.stress_fixed_corotated(Q @ F, mu[: F.shape[0]], lam[: F.shape[0]])
    assert torch.allclose(t2, Q @ t @ Q.transpose(-1, -2), atol=1e-8)


def test_hencky_closed_forms():
    n = 30
    mu = torch.full((n,), MU, dtype=DT)
    lam = torch.full((n,), LAM, dtype=DT)
    rng = np.random.default_rng(5)
    sig = torch.tensor(rng.uniform(0.7, 1.3, (n, 3)), dtype=DT)
    tau = O.stress_sand(torch.diag_embed(sig), mu, lam)
    e = torch.log(sig)
    ref = torch.diag_embed(2 * MU * e + LAM * e.sum(-1, keepdim=True))
    assert torch.allclose(tau, ref, atol=1e-10)
    Q = torch.tensor(Rotation.random(n, random_state=6).as_matrix(), dtype=DT)
    Q2 = torch.tensor(Rotation.random(n, random_state=7).as_matrix(), dtype=DT)
    # tau(Q diag Q2^T) = Q tau(diag) Q^T: the stress depends on the left frame only
    tau2 = O.stress_sand(Q @ torch.diag_embed(sig) @ Q2.transpose(-1, -2), mu, lam)
    assert torch.allclose(tau2, Q @ ref @ Q.transpose(-1, -2), atol=1e-9)
    assert O.stress_sand(Q, mu, lam).abs().max() < 1e-10


def test_liquid_pressure_and_viscosity_split():
    """The viscous term vanishes for a rigid rotation C = [w]x and the
    pressure vanishes at J = 1."""
    n = 10
    rng = np.random.default_rng(8)
    w = torch.tensor(rng.normal(0, 1, (n, 3)), dtype=DT)
    Jv = torch.tensor(rng.uniform(0.9, 1.1, n), dtype=DT)
    lam = torch.full((n,), 277.78, dtype=DT)
    eta = torch.full((n,), 0.1, dtype=DT)
    tau = O.stress_liquid(Jv, O.skew(w), lam, eta)
    assert torch.allclose(tau, (lam * Jv * (Jv - 1))[:, None, None] * torch.eye(3, dtype=DT), atol=1e-13)
    tau1 = O.stress_liquid(torch.ones(n, dtype=DT), O.skew(w), lam, eta)
    assert tau1.abs().max() < 1e-14


def fd_check(fun, F, gbar, eps=1e-6):
    """Central finite difference of <gbar, fun(F)> against autograd."""
    Ft = F.clone().requires_grad_(True)
    out = (fun(Ft) * gbar).sum()
    (g,) = torch.autograd.grad(out, Ft)
    num = torch.zeros_like(F)
    for q in range(F.shape[0]):
        for a in range(3):
            for b in range(3):
                Fp = F.clone(); Fp[q, a, b] += eps
                Fm = F.clone(); Fm[q, a, b] -= eps
                num[q, a, b] = ((fun(Fp) * gbar).sum() - (fun(Fm) * gbar).sum()) / (2 * eps)
    return g, num


SPECIAL = [np.eye(3), np.diag([1.2, 1.2, 0.8]), np.diag([1.1, 0.9, 0.9])]


@pytest.mark.parametrize("which", ["rotation", "hencky"])
def test_isotropic_map_derivative_fd(which):
    rng = np.random.default_rng(9)
    F = np.concatenate([rand_F(rng, 4, 0.15), np.stack(SPECIAL)], 0)
    Q = Rotation.random(F.shape[0], random_state=10).as_matrix()
    F = torch.tensor(Q @ F, dtype=DT)           # rotate so the special points are not diagonal
    n = F.shape[0]
    mu = torch.full((n,), MU, dtype=DT)
    lam = torch.full((n,), LAM, dtype=DT)
    gbar = torch.tensor(rng.normal(0, 1, (n, 3, 3)), dtype=DT)
    if which == "rotation":
        fun = O.polar_rotation
    else:
        fun = lambda X: O.stress_sand(X, mu, lam)
    g, num = fd_check(fun, F, gbar)
    assert torch.allclose(g, num, atol=5e-7 * max(1.0, num.abs().max().item()))


def test_polar_derivative_at_identity_is_skew_part():
    """At F = I, RS = F with R^T R = I and S symmetric gives dR = (dF - dF^T)/2."""
    rng = np.random.default_rng(11)
    dF = torch.tensor(rng.normal(0, 1, (3, 3)), dtype=DT)
    F = torch.eye(3, dtype=DT)[None].clone().requires_grad_(True)
    R = O.polar_rotation(F)
    jac = torch.zeros(3, 3, 3, 3, dtype=DT)
    for a in range(3):
        for b in range(3):
            (g,) = torch.autograd.grad(R[0, a, b], F, retain_graph=True)
            jac[a, b] = g[0]
    dR = torch.einsum("abij,ij->ab", jac, dF)
    assert torch.allclose(dR, 0.5 * (dF - dF.T), atol=1e-14)


# ---------------------------------------------------------------------------
# Drucker-Prager return map
# ---------------------------------------------------------------------------
def dp_setup(n, phi=30.0, coh=0.0):
    alpha = torch.full((n,), O.dp_alpha(phi), dtype=DT)
    kappa = torch.full((n,), (3 * LAM + 2 * MU) / (2 * MU), dtype=DT)
    c = torch.full((n,), coh, dtype=DT)
    return alpha, kappa, c


def test_dp_alpha_value():
    assert abs(O.dp_alpha(30.0) - 0.3265986323710904) < 1e-15


@pytest.mark.parametrize("coh", [0.0, 0.01])
def test_dp_projection_properties(coh):
    rng = np.random.default_rng(12)
    n = 20000
    eps = torch.tensor(rng.normal(0, 0.05, (n, 3)), dtype=DT)
    alpha, kappa, c = dp_setup(n, coh=coh)
    ep, case = O.dp_project(eps, alpha, kappa, c)
    es, eps_s = ep - coh, eps - coh
    tr, tr0 = es.sum(-1), eps_s.sum(-1)
    dev = es - tr[:, None] / 3
    dev0 = eps_s - tr0[:, None] / 3
    yieldf = dev.norm(dim=-1) + kappa * alpha * tr
    inside, apex, cone = case == 0, case == 1, case == 2
    assert inside.any() and apex.any() and cone.any()
    assert torch.allclose(ep[inside], eps[inside], rtol=0, atol=1e-16)
    assert torch.allclose(ep[apex], torch.full_like(ep[apex], coh), atol=0)
    assert yieldf[cone].abs().max() < 1e-15                   # lands on the cone
    assert torch.allclose(tr[cone], tr0[cone], atol=1e-16)    # volume preserved
    cosang = (dev[cone] * dev0[cone]).sum(-1) / (dev[cone].norm(dim=-1) * dev0[cone].norm(dim=-1))
    assert torch.allclose(cosang, torch.ones_like(cosang), atol=1e-12)   # direction kept
    assert (yieldf[inside] <= 1e-15).all()
    ep2, case2 = O.dp_project(ep, alpha, kappa, c)             # idempotent
    assert torch.allclose(ep2, ep, atol=1e-15)


def test_dp_projection_is_continuous_across_cases():
    rng = np.random.default_rng(13)
    n = 4000
    alpha, kappa, c = dp_setup(n)
    eps = torch.tensor(rng.normal(0, 0.05, (n, 3)), dtype=DT)
    d = torch.tensor(rng.normal(0, 1, (n, 3)), dtype=DT) * 1e-9
    e1, c1 = O.dp_project(eps, alpha, kappa, c)
    e2, c2 = O.dp_project(eps + d, alpha, kappa, c)
    # a Lipschitz map: a 1e-9 perturbation moves the result by O(1e-9) even
    # where the case changes
    assert ((e1 - e2).norm(dim=-1) <= 5e-9 * (1 + kappa * alpha)).all()


def test_dp_jacobian_fd():
    rng = np.random.default_rng(14)
    n = 300
    alpha, kappa, c = dp_setup(n)
    eps = torch.tensor(rng.normal(0, 0.05, (n, 3)), dtype=DT)
    Jm = O.dp_jacobian(eps, alpha, kappa, c)
    h = 1e-7
    for k in range(3):
        ep_p, cp = O.dp_project(eps + h * torch.eye(3, dtype=DT)[k], alpha, kappa, c)
        ep_m, cm = O.dp_project(eps - h * torch.eye(3, dtype=DT)[k], alpha, kappa, c)
        same = (cp == cm)
        num = (ep_p - ep_m) / (2 * h)
        assert torch.allclose(Jm[same][:, :, k], num[same], atol=1e-6)


def test_dp_isotropic_map_derivative_fd():
    """Derivative of F_tr -> U exp(P(log sigma)) V^T in all three cases and at
    repeated singular values."""
    rng = np.random.default_rng(15)
    sig = np.array([[1.05, 0.98, 0.97],          # cone (deviatoric, compressive)
                    [1.01, 1.01, 0.95],          # cone, repeated pair
                    [1.02, 1.01, 1.005],         # apex (expanded)
                    [0.999, 0.998, 0.997],       # inside
                    [0.99, 0.99, 0.99],          # inside, triple
                    [1.04, 0.97, 0.97]])         # cone, repeated pair
    n = sig.shape[0]
    U = Rotation.random(n, random_state=16).as_matrix()
    V = Rotation.random(n, random_state=17).as_matrix()
    F = torch.tensor(U @ (sig[:, :, None] * np.swapaxes(V, -1, -2)), dtype=DT)
    alpha, kappa, c = dp_setup(n)
    _, case = O.dp_project(torch.log(torch.tensor(sig)), alpha, kappa, c)
    assert set(case.tolist()) == {0, 1, 2}
    g = O.make_g_dp(alpha, kappa, c)
    fun = lambda X: O.IsotropicMap.apply(X, g)
    gbar = torch.tensor(rng.normal(0, 1, (n, 3, 3)), dtype=DT)
    ga, num = fd_check(fun, F, gbar, eps=1e-7)
    assert torch.allclose(ga, num, atol=2e-6)


# ---------------------------------------------------------------------------
# von Mises return in log strain (the non-Newtonian ice cream)
# ---------------------------------------------------------------------------
def test_vm_projection_closed_form():
    """Pure shear trial strain (a, -a, 0): |dev| = sqrt(2) a; beyond the
    radius the return is rho (1, -1, 0)/sqrt(2); a pure dilation never yields."""
    rho = torch.tensor([0.006, 0.006], dtype=DT)
    eps = torch.tensor([[0.01, -0.01, 0.0], [0.003, -0.003, 0.0]], dtype=DT)
    ep, case = O.vm_project(eps, rho)
    assert case.tolist() == [2, 0]
    assert torch.allclose(ep[0], torch.tensor([0.006, -0.006, 0.0], dtype=DT) / math.sqrt(2.0), atol=1e-17)
    assert torch.equal(ep[1], eps[1])
    dil = torch.full((1, 3), 0.2, dtype=DT)
    ep2, case2 = O.vm_project(dil, rho[:1])
    assert case2.item() == 0 and torch.equal(ep2, dil)


def test_vm_projection_properties():
    rng = np.random.default_rng(31)
    n = 20000
    eps = torch.tensor(rng.normal(0, 0.01, (n, 3)), dtype=DT)
    rho = torch.tensor(rng.uniform(0.002, 0.01, n), dtype=DT)
    ep, case = O.vm_project(eps, rho)
    y = case == 2
    assert y.any() and (~y).any()
    tr, tr0 = ep.sum(-1), eps.sum(-1)
    dev, dev0 = ep - tr[:, None] / 3, eps - tr0[:, None] / 3
    assert torch.allclose(tr, tr0, atol=1e-16)                                   # trace kept
    assert (dev[y].norm(dim=-1) - rho[y]).abs().max() < 1e-16                     # on the surface
    cosang = (dev[y] * dev0[y]).sum(-1) / (dev[y].norm(dim=-1) * dev0[y].norm(dim=-1))
    assert torch.allclose(cosang, torch.ones_like(cosang), atol=1e-12)           # direction kept
    assert torch.equal(ep[~y], eps[~y])
    ep2, _ = O.vm_project(ep, rho * (1 + 1e-12))                                 # idempotent
    assert torch.allclose(ep2, ep, atol=1e-16)
    d = torch.tensor(rng.normal(0, 1, (n, 3)), dtype=DT) * 1e-9                  # Lipschitz across the surface
    e3, _ = O.vm_project(eps + d, rho)
    assert ((e3 - ep).norm(dim=-1) <= 2e-9 * (1 + d.norm(dim=-1) / 1e-9)).all()


def test_vm_jacobian_fd():
    rng = np.random.default_rng(32)
    n = 400
    eps = torch.tensor(rng.normal(0, 0.01, (n, 3)), dtype=DT)
    rho = torch.full((n,), 0.006, dtype=DT)
    Jm = O.vm_jacobian(eps, rho)
    h = 1e-8
    for k in range(3):
        ep_p, cp = O.vm_project(eps + h * torch.eye(3, dtype=DT)[k], rho)
        ep_m, cm = O.vm_project(eps - h * torch.eye(3, dtype=DT)[k], rho)
        same = cp == cm
        num = (ep_p - ep_m) / (2 * h)
        assert torch.allclose(Jm[same][:, :, k], num[same], atol=1e-6)


def test_vm_isotropic_map_derivative_fd():
    """Derivative of F_tr -> U exp(P_vm(log sigma)) V^T, yielding and not,
    at distinct and repeated singular values."""
    rng = np.random.default_rng(33)
    sig = np.array([[1.02, 0.99, 0.985],        # yields
                    [1.01, 1.01, 0.98],         # yields, repeated pair
                    [1.002, 1.0, 0.999],        # inside
                    [0.99, 0.99, 0.99],         # inside, triple
                    [1.03, 0.98, 0.98]])        # yields, repeated pair
    n = sig.shape[0]
    U = Rotation.random(n, random_state=34).as_matrix()
    V = Rotation.random(n, random_state=35).as_matrix()
    F = torch.tensor(U @ (sig[:, :, None] * np.swapaxes(V, -1, -2)), dtype=DT)
    rho = torch.full((n,), 0.006, dtype=DT)
    _, case = O.vm_project(torch.log(torch.tensor(sig)), rho)
    assert set(case.tolist()) == {0, 2}
    fun = lambda X: O.IsotropicMap.apply(X, O.make_g_vm(rho))
    gbar = torch.tensor(rng.normal(0, 1, (n, 3, 3)), dtype=DT)
    ga, num = fd_check(fun, F, gbar, eps=1e-7)
    assert torch.allclose(ga, num, atol=2e-6)


# ---------------------------------------------------------------------------
# Box yield (the plastic material): clamped singular values
# ---------------------------------------------------------------------------
def test_box_clamp_closed_forms():
    lo = torch.tensor([0.975], dtype=DT)
    hi = torch.tensor([1.0075], dtype=DT)
    g = O.make_g_box(lo, hi)
    gv, dg = g(torch.tensor([[1.02, 1.0, 0.95]], dtype=DT))
    assert torch.equal(gv, torch.tensor([[1.0075, 1.0, 0.975]], dtype=DT))
    assert torch.equal(torch.diagonal(dg[0]), torch.tensor([0.0, 1.0, 0.0], dtype=DT))
    # a rotation is untouched; a uniform stretch beyond the limit comes back to it
    R = torch.tensor(Rotation.random(1, random_state=40).as_matrix(), dtype=DT)
    assert torch.allclose(O.IsotropicMap.apply(R, g), R, atol=1e-14)
    Fs = 1.1 * R
    assert torch.allclose(O.IsotropicMap.apply(Fs, g), 1.0075 * R, atol=1e-14)


def test_box_isotropic_map_derivative_fd():
    rng = np.random.default_rng(41)
    sig = np.array([[1.02, 0.99, 0.96],          # stretch and compression clamped
                    [1.001, 1.0, 0.999],         # inside
                    [1.001, 1.001, 0.99],        # inside, repeated pair
                    [1.03, 1.03, 0.98],          # clamped repeated pair
                    [0.97, 0.96, 0.95]])         # all compressed
    n = sig.shape[0]
    U = Rotation.random(n, random_state=42).as_matrix()
    V = Rotation.random(n, random_state=43).as_matrix()
    F = torch.tensor(U @ (sig[:, :, None] * np.swapaxes(V, -1, -2)), dtype=DT)
    lo = torch.full((n,), 0.975, dtype=DT)
    hi = torch.full((n,), 1.0075, dtype=DT)
    fun = lambda X: O.IsotropicMap.apply(X, O.make_g_box(lo, hi))
    gbar = torch.tensor(rng.normal(0, 1, (n, 3, 3)), dtype=DT)
    ga, num = fd_check(fun, F, gbar, eps=1e-7)
    assert torch.allclose(ga, num, atol=2e-6)
