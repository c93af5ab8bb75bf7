"""GPU parity of the gas step (section 3.2's advection-projection after Stam
1999; the air-circulation setting of section 4.1) through the C ABI, against
the FP64 oracle on the same seeded scenes.

Tolerances: FP32 advection and an exact FP32 pressure solve (spectral by
default, on the matrix cores; the multigrid alternative at 6 V-cycles
reaches the FP32 residual floor) against the oracle's exact projection in
FP64: fields 2e-4 relative after several steps; gradients 2e-3 relative.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import gas_oracle as G
from paper_2303_02346_amd import scenes

pytestmark = pytest.mark.gpu

DT = torch.float64
MPM_ERR_NONFINITE = 2


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def gas_sim(sc, **kw):
    from paper_2303_02346_amd.gas import GasSim
    return GasSim(sc, **kw)


def compare(g, ref, tol_v=2e-4, tol_s=2e-5):
    e = {q: rel(g[q], ref[q].detach().numpy()) for q in ("u", "v", "w", "s")}
    say("  rel err " + " ".join(f"{q} {e[q]:.2e}" for q in e))
    assert e["u"] <= tol_v and e["v"] <= tol_v and e["w"] <= tol_v and e["s"] <= tol_s


@pytest.mark.parametrize("n", [16, 32])
def test_gas_steps_vs_oracle(n):
    """Several steps (moving and turning emitter, buoyancy) against the
    oracle, with the default (spectral) solver."""
    sc = scenes.gas_room(n=n, steps=6, seed=1, translate=True)
    say(f"gas {n}^3, 6 steps")
    sim = gas_sim(sc)
    sim.enable_stats(True)
    sim.step(6)
    say(f"  last pressure residual {sim.residual():.2e}")
    compare(sim.state_numpy(), G.rollout_scene(sc, steps=6))


def test_gas_projection_is_divergence_free_and_walls_closed():
    sc = scenes.gas_room(n=64, steps=3, seed=2)
    say("gas 64^3: divergence after 3 steps")
    sim = gas_sim(sc)
    sim.enable_stats(True)
    sim.step(3)
    g = sim.state_numpy()
    div = G.divergence(*(torch.from_numpy(g[q]) for q in ("u", "v", "w")), sc.h).numpy()
    scale = max(np.abs(g[q]).max() for q in ("u", "v", "w")) / sc.h
    say(f"  max |div| / (|u|/h) {np.abs(div).max() / scale:.2e}, residual {sim.residual():.2e}")
    assert np.abs(div).max() <= 1e-4 * scale
    assert np.abs(g["u"][0]).max() == 0 and np.abs(g["u"][-1]).max() == 0
    assert np.abs(g["v"][:, 0]).max() == 0 and np.abs(g["w"][:, :, -1]).max() == 0


def test_gas_full_size_step_vs_oracle():
    """The bench workload (128^3, 2 scalars) for one step against the oracle
    (its pressure by conjugate gradients to 1e-12)."""
    sc = scenes.gas_room(n=128, steps=1, seed=0)
    say("gas 128^3, 1 step")
    sim = gas_sim(sc)
    sim.enable_stats(True)
    sim.step(1)
    say(f"  pressure residual {sim.residual():.2e}")
    compare(sim.state_numpy(), G.rollout_scene(sc, steps=1))


def _seeds(sim, seed):
    rng = np.random.default_rng(seed)
    return torch.tensor(rng.normal(0, 1, sim.buf.numel()), dtype=torch.float32)


@pytest.mark.parametrize("ckpt", [16, 3])
def test_gas_gradient_vs_oracle(ckpt):
    """Seeded adjoints on the whole final state: gradients with respect to
    the actions (emitter translation and rotation) and the initial state
    against oracle autograd, one checkpoint segment or several."""
    sc = scenes.gas_room(n=16, steps=5, seed=3, translate=True)
    say(f"gas gradient 16^3, 5 steps, checkpoint every {ckpt}")
    sim = gas_sim(sc, requires_grad=True, ckpt_every=ckpt)
    sim.step(5)
    wflat = _seeds(sim, 30)
    ga, g0 = sim.backward(wflat.to(sim.device), want_grad0=True)
    # oracle
    p = G.params_from_scene(sc)
    acts = torch.tensor(sc.actions, dtype=DT, requires_grad=True)
    st0 = G.state_from_scene(sc, requires_grad=True)
    st = G.rollout_scene(sc, actions=acts, state=st0, params=p)
    wq = [t.double() for t in sim.split(wflat)]
    L = sum((w * st[q]).sum() for w, q in zip(wq[:3], ("u", "v", "w"))) + (wq[3] * st["s"]).sum()
    L.backward()
    ea = rel(ga.double().cpu().numpy(), acts.grad.numpy())
    g0s = [t.double().cpu().numpy() for t in sim.split(g0)]
    e0 = {q: rel(g0s[i], st0[q].grad.numpy()) for i, q in enumerate(("u", "v", "w", "s"))}
    say(f"  actions rel {ea:.2e}; initial state " + " ".join(f"{q} {e0[q]:.2e}" for q in e0))
    assert ea <= 2e-3
    assert all(e <= 2e-3 for e in e0.values())


def test_gas_sensor_loss_and_its_gradient():
    sc = scenes.gas_room(n=32, steps=4, seed=4)
    say("gas sensor loss, 32^3, 4 steps")
    sim = gas_sim(sc, requires_grad=True, ckpt_every=2)
    sim.step(4)
    loss, g = sim.sensor_loss()
    ga = sim.backward(g)
    p = G.params_from_scene(sc)
    acts = torch.tensor(sc.actions, dtype=DT, requires_grad=True)
    st = G.rollout_scene(sc, actions=acts, params=p)
    L = G.sensor_loss(st["s"], torch.from_numpy(sc.sensors), torch.tensor(sc.targets, dtype=DT))
    L.backward()
    ea = rel(ga.double().cpu().numpy(), acts.grad.numpy())
    say(f"  loss gpu {loss.item():.6f} ref {L.item():.6f}; actions rel {ea:.2e}")
    assert abs(loss.item() - L.item()) <= 1e-4 * abs(L.item())
    assert ea <= 2e-3


def test_gas_box_grid_one_scalar_vs_oracle():
    """A non-cubic box (24 x 16 x 32 cells: axis lengths below the
    transform's 64-value chunks, zero-padded) with one scalar, against the
    oracle."""
    sc = scenes.gas_room(n=(24, 16, 32), steps=4, seed=5, n_scalars=1, translate=True)
    say("gas 24x16x32, one scalar, 4 steps")
    sim = gas_sim(sc)
    sim.step(4)
    compare(sim.state_numpy(), G.rollout_scene(sc, steps=4))


def test_gas_four_scalars_no_emitter_long_backtraces_vs_oracle():
    """Four scalars, the emitter switched off (kappa = 0), no buoyancy, and a
    step long enough that back-traces cross several cells (and leave the
    grid near the walls)."""
    sc = scenes.gas_room(n=16, steps=3, seed=6, n_scalars=4, velocity=3.0, dt=0.05, emit_kappa=0.0, buoyancy=0.0)
    say("gas 16^3, 4 scalars, kappa 0, CFL > 1")
    u = np.abs(sc.u).max()
    say(f"  max |u| dt / h = {u * sc.dt / sc.h:.2f}")
    sim = gas_sim(sc)
    sim.step(3)
    compare(sim.state_numpy(), G.rollout_scene(sc, steps=3))


def test_gas_nonfinite_is_reported():
    """A NaN temperature spreads through buoyancy; the step reports it as
    MPM_EDOMAIN with the non-finite bit (nothing is clamped or hidden)."""
    from paper_2303_02346_amd import _lib
    sc = scenes.gas_room(n=16, steps=2, seed=7)
    sc.s[0, 8, 8, 8] = np.nan
    sim = gas_sim(sc)
    with pytest.raises(_lib.MpmError) as e:
        sim.step(1)
    assert e.value.status == _lib.MPM_EDOMAIN and (e.value.bits & MPM_ERR_NONFINITE) != 0


def test_gas_rollout_autograd_function_matches_direct_backward():
    """GasRollout (torch.autograd.Function over gas_step / gas_step_backward)
    gives the direct backward's action gradient."""
    from paper_2303_02346_amd.gas import GasRollout
    sc = scenes.gas_room(n=16, steps=4, seed=8, translate=True)
    sim = gas_sim(sc, requires_grad=True, ckpt_every=2)
    w = _seeds(sim, 31).to(sim.device)
    acts = torch.tensor(sc.actions, dtype=torch.float32, device=sim.device, requires_grad=True)
    out = GasRollout.apply(acts, sim)
    (out * w).sum().backward()
    sim.reset()
    sim.step(4)
    ga = sim.backward(w)
    e = rel(acts.grad.double().cpu().numpy(), ga.double().cpu().numpy())
    say(f"  autograd vs direct backward rel {e:.2e}")
    assert e <= 1e-6


@pytest.mark.parametrize("n", [(16, 16, 16), (24, 16, 32)], ids=["cube", "box"])
def test_gas_spectral_and_multigrid_solvers_agree(n):
    """The exact spectral pressure solve (default) and the multigrid solver
    give the same steps, forward and backward."""
    sc = scenes.gas_room(n=n, steps=4, seed=9, translate=True)
    say(f"gas {n}: spectral vs multigrid, 4 steps with gradients")
    out = {}
    for solver in ("spectral", "multigrid"):
        sim = gas_sim(sc, requires_grad=True, ckpt_every=2, solver=solver)
        sim.enable_stats(True)
        sim.step(4)
        res = sim.residual()
        ga = sim.backward(_seeds(sim, 32).to(sim.device))
        out[solver] = (sim.buf.double().cpu().numpy(), ga.double().cpu().numpy(), res)
    e = rel(out["spectral"][0], out["multigrid"][0])
    eg = rel(out["spectral"][1], out["multigrid"][1])
    say(f"  residual spectral {out['spectral'][2]:.1e} multigrid {out['multigrid'][2]:.1e}; "
        f"state rel {e:.2e}, action gradient rel {eg:.2e}")
    assert out["spectral"][2] <= 1e-5 and e <= 1e-4 and eg <= 1e-3


def test_gas_long_axes_vs_oracle():
    """Axes longer than 128 cells (132 along x, 136 along z) take the axis
    transform's wider output split (64 outputs per workgroup) with ragged
    last chunks; a thin y axis (12) the narrow one."""
    sc = scenes.gas_room(n=(132, 12, 136), steps=3, seed=10, n_scalars=1, translate=True)
    say("gas 132x12x136, one scalar, 3 steps")
    sim = gas_sim(sc)
    sim.enable_stats(True)
    sim.step(3)
    say(f"  pressure residual {sim.residual():.2e}")
    compare(sim.state_numpy(), G.rollout_scene(sc, steps=3))
