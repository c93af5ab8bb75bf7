"""GPU tests of the batched multi-scene launch, the HIP-graph replay and the
launch-shape autotuner.

Batched scenes are independent (the batched oracle is one oracle run per
scene), so every scene of a batched launch must match its own oracle run
and its own single-scene launch to FP32 rounding.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O
from paper_2303_02346_amd import scenes, _lib

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def sim_of(sc, **kw):
    from paper_2303_02346_amd.sim import Simulator
    return Simulator(sc, **kw)


def small_batch(n_scenes=5, steps=20):
    sc = scenes.config4(n_scenes=n_scenes, steps=steps, scale=0.02)
    return sc


def test_batched_matches_per_scene_oracle():
    scs = small_batch()
    say(f"batched {len(scs)} scenes, sizes {[s.n for s in scs]}")
    sim = sim_of(scs)
    sim.step(20)
    x = sim.positions()
    for s, sc in enumerate(scs):
        lo, hi = sim.offsets[s], sim.offsets[s + 1]
        ref = O.rollout(sc, steps=20)["x"].numpy()
        e = rel(x[lo:hi], ref)
        say(f"  scene {s} ({sc.n} particles) rel err {e:.2e}")
        assert e <= 1e-5


def test_batched_equals_single_scene_launches():
    scs = small_batch(n_scenes=4, steps=15)
    sim = sim_of(scs)
    sim.step(15)
    xb = sim.positions()
    for s, sc in enumerate(scs):
        one = sim_of(sc)
        one.step(15)
        e = rel(xb[sim.offsets[s]:sim.offsets[s + 1]], one.positions())
        say(f"  scene {s}: batched vs single rel diff {e:.2e}")
        assert e <= 1e-6


@pytest.mark.parametrize("threads", [128, 256])
def test_particle_workgroup_sizes(threads):
    sc = scenes.tiny(n_particles=600, n_grid=32, steps=30, seed=5, dt=1e-4)
    sim = sim_of(sc)
    sim.set_option(_lib.MPM_OPT_PART_THREADS, threads)
    sim.set_option(_lib.MPM_OPT_PART_WGS, 512)
    sim.step(30)
    e = rel(sim.positions(), O.rollout(sc, steps=30)["x"].numpy())
    say(f"  {threads} threads per workgroup: rel err {e:.2e}")
    assert e <= 1e-5


def test_graph_replays_match_eager():
    """Replay one captured call several times, with eager work and
    synchronisation between replays, and compare each replay with an eager
    run of the same call."""
    sc = scenes.tiny(n_particles=800, n_grid=32, steps=12, seed=6, dt=1e-4)
    eager = sim_of(sc)
    eager.step(12)
    ref = eager.state_numpy()
    g = sim_of(sc, graph=True)
    for rep in range(4):
        g.reset()
        g.step(12)
        torch.cuda.synchronize()
        out = g.state_numpy()
        tmp = torch.randn(1000, device="cuda").sum().item()   # eager work between replays
        ex = rel(out["x"], ref["x"])
        ev = rel(out["v"], ref["v"])
        say(f"  replay {rep}: rel diff x {ex:.2e} v {ev:.2e}")
        assert ex <= 1e-6 and ev <= 1e-4


def test_graph_replay_at_other_start_times():
    """A call captured at t = 0 is replayed at later clock values: the
    device-side clock selects the right actions."""
    sc = scenes.tiny(n_particles=400, n_grid=32, steps=12, seed=7, dt=1e-4)
    eager = sim_of(sc)
    for _ in range(3):
        eager.step(4)
    g = sim_of(sc, graph=True)
    for _ in range(3):
        g.step(4)
    e = rel(g.positions(), eager.positions())
    say(f"  graph chunks vs eager chunks rel diff {e:.2e}")
    assert e <= 1e-6


def test_autotuner_keeps_state_and_picks_a_valid_shape(tmp_path):
    sc = scenes.tiny(n_particles=2000, n_grid=32, steps=40, seed=8, dt=1e-4)
    sim = sim_of(sc)
    before = sim.buf.clone()
    best = sim.autotune(n_steps=10, cache=str(tmp_path / "tune.json"))
    say(f"  autotune: {best}")
    assert torch.equal(before, sim.buf)
    assert sim.clock() == 0
    assert best["part_threads"] in (128, 256, 512) and best["part_wgs"] >= 64 and best["grid_wgs"] >= 64
    assert best["share_chunks"] in (0, 1, 2)
    assert sim.get_option(_lib.MPM_OPT_PART_WGS) == best["part_wgs"]
    assert sim.get_option(_lib.MPM_OPT_SHARE_CHUNKS) == best["share_chunks"]
    again = sim.autotune(n_steps=10, cache=str(tmp_path / "tune.json"))
    assert again == best
    sim.step(40)
    e = rel(sim.positions(), O.rollout(sc, steps=40)["x"].numpy())
    say(f"  after autotune rel err {e:.2e}")
    assert e <= 1e-5


def test_graph_cache_follows_rebound_state_arrays():
    """A captured call bakes in every state pointer.  Rebinding only v (a
    separate tensor, same x and mat) must drop the captured graph: the
    graph-mode result with the rebound v equals an eager run."""
    import ctypes
    sc = scenes.tiny(n_particles=500, n_grid=32, steps=10, seed=9, dt=1e-4)
    eager = sim_of(sc)
    eager.step(5)
    ref = eager.state_numpy()
    g = sim_of(sc, graph=True)
    g.step(5)                      # captures the call with the packed buffer's v rows
    g.reset()
    v2 = g.buf[3:6].clone()        # v rebound to a tensor of its own
    b = g.buf
    st = _lib.MpmState(b[0].data_ptr(), v2.data_ptr(), b[6].data_ptr(), b[15].data_ptr(), b[24].data_ptr(),
                       g.mat.data_ptr())
    g._sync_in()
    _lib.check(_lib.lib().mpm_set_state(g.ctx, ctypes.byref(st)), "mpm_set_state", g.ctx)
    g.set_actions(g.actions)
    g.step(5)
    torch.cuda.synchronize()
    out = g.state_numpy()
    ex = rel(out["x"], ref["x"])
    ev = rel(v2.T.double().cpu().numpy(), ref["v"])
    say(f"  rebound v under graph mode: rel diff x {ex:.2e}, v (the rebound tensor) {ev:.2e}")
    assert ex <= 1e-6 and ev <= 1e-5


@pytest.mark.timeout(900)
def test_config4_full_size_batched_vs_single_and_oracle():
    """The full config-4 batch (64 scenes, 3.8M particles, 64^3 each) in the
    autotuned launch: after 2 steps every scene equals its own single-scene
    launch on x, v, C and F or J (Frobenius and per particle), and three
    scenes (smallest, median, largest) match the oracle."""
    from parity import compare_states, liquid_mask, state_errors
    scs = scenes.config4(steps=4)
    say(f"config 4 full size: {len(scs)} scenes, {sum(s.n for s in scs)} particles")
    sim = sim_of(scs)
    tune = sim.autotune(n_steps=2)
    say(f"  launch {tune}")
    sim.reset()
    sim.step(2)
    gb = sim.state_numpy()
    worst = {}
    for s, sc in enumerate(scs):
        lo, hi = sim.offsets[s], sim.offsets[s + 1]
        one = sim_of(sc)
        one.step(2)
        g1 = one.state_numpy()
        one.close()
        part = {k: v[lo:hi] for k, v in gb.items()}
        e = state_errors(part, g1, liquid_mask(sc), n_grid=sc.n_grid)
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
        assert e["x"] <= 1e-6 and e["x_max"] <= 1e-5, (s, e)
        assert e["v"] <= 1e-4 and e["C"] <= 1e-3 and e["v_max"] <= 1e-3 and e["C_max"] <= 1e-2, (s, e)
        assert e["F"] <= 1e-5 and e["J"] <= 1e-5 and e["F_max"] <= 1e-4 and e["J_max"] <= 1e-4, (s, e)
    say("  batched vs single, worst over scenes: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    sizes = np.array([sc.n for sc in scs])
    for s in (int(sizes.argmin()), int(np.argsort(sizes)[len(sizes) // 2]), int(sizes.argmax())):
        sc = scs[s]
        ref = {k: v.detach().numpy() for k, v in O.rollout(sc, steps=2).items()}
        part = {k: v[sim.offsets[s]:sim.offsets[s + 1]] for k, v in gb.items()}
        say(f"  scene {s} ({sc.n} particles) vs oracle")
        compare_states(part, ref, liquid_mask(sc), tol_x=1e-6, tol=1e-3, tol_FJ=1e-5, n_grid=sc.n_grid)
