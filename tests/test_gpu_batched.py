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
    assert sim.get_option(_lib.MPM_OPT_PART_WGS) == best["part_wgs"]
    again = sim.autotune(n_steps=10, cache=str(tmp_path / "tune.json"))
    assert again == best
    sim.step(40)
    e = rel(sim.positions(), O.rollout(sc, steps=40)["x"].numpy())
    say(f"  after autotune rel err {e:.2e}")
    assert e <= 1e-5
