#!/usr/bin/env python
"""Benchmark of the MLS-MPM step on one MI355X.

Workload: the two-material scene of 250k particles (125k weakly compressible
viscous liquid, 125k Drucker-Prager sand) on a 128^3 grid, dt = 5e-5, with a
kinematic cylinder driven by a smooth 6-DoF velocity trajectory.  One step is
one MLS-MPM substep (P2G with stress, grid update with gravity, walls and
soft contact, G2P with F/J update and plastic projection).

Prints one JSON line: forward particle-steps/s as ``value`` (K steps in one
call, replayed from the call's captured HIP graph, the library's production
mode; the same call run eagerly with its kernels event-timed is reported as
``timed_call``), the forward+backward rate (checkpointed adjoint, blob loss) in ``fwd_bwd``, the
dominant kernel against the HBM roofline in ``roofline``, and the FP64 CPU
oracle timed on a bounded sample in ``cpu_baseline``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # MI355X dense FP32 (vector and matrix)
METRIC = "MPM particle-steps/s fwd and fwd+bwd, 250k particles 128^3 grid; % HBM roofline"

# Algorithmic bytes per unit, FP32 SoA state read once and written once.
BYTES_SOLID = 193      # x v C F read + write (96 + 96) + 1 B material tag
BYTES_LIQUID = 129     # x v C J read + write (64 + 64) + 1 B tag
BYTES_NODE = 56        # active node: P2G write m,mv 16; grid read 16, write v 12; G2P read 12
# per-kernel algorithmic bytes: (bytes per solid particle, per liquid particle, per active node)
KERNEL_BYTES = {
    "k_p2g_plain": (97, 65, 16),      # read x v C F|J + tag; write m, mv
    "k_g2p2g": (193, 129, 28),        # read + write the particle state; write m,mv and read v per node
}


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_g2p2g_config2_traffic.md")
TRAFFIC_SOURCES = ["mpm_fast.hip", "mpm_fast.h", "mpm_blocks.h", "mpm_phys.h", "mpm_math.h", "mpm_internal.h", "mpm_transfer.h"]
GAS_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_axis_gas128_traffic.md")
BATCHED_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_g2p2g_config4_traffic.md")
GAS_TRAFFIC_SOURCES = ["gas.hip"]


def counted_traffic(summary=None, sources=None):
    """HBM bytes per launch from a committed counter summary (default: the
    fused MPM kernel's), or None when the kernel's sources have changed
    since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(summary or TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m_b = re.search(r"traffic_bytes_per_launch:\s*(\d+)", text)
    m_h = re.search(r"source-sha256:\s*([0-9a-f]+)", text)
    if not m_b or not m_h:
        return None
    h = hashlib.sha256()
    for f in (sources or TRAFFIC_SOURCES):
        with open(os.path.join(ROOT, "paper_2303_02346_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m_b.group(1)) if h.hexdigest()[:16] == m_h.group(1) else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def active_nodes(x, n):
    import numpy as np
    base = np.floor(x * n - 0.5).astype(np.int64)
    offs = np.array([[i, j, k] for i in range(3) for j in range(3) for k in range(3)])
    idx = base[:, None, :] + offs[None]
    lin = (idx[..., 0] * n + idx[..., 1]) * n + idx[..., 2]
    return int(np.unique(lin.reshape(-1)).size)


def cpu_baseline(sc, steps):
    import torch
    from oracle import mpm_oracle as O
    p = O.params_from_scene(sc)
    st = O.state_from_scene(sc)
    t0 = time.perf_counter()
    O.rollout(sc, state=st, steps=steps, params=p)
    dt = time.perf_counter() - t0
    return {"value": sc.n * steps / dt, "unit": "particle-steps/s", "cores": torch.get_num_threads(),
            "kind": "oracle", "sample": f"config-2 scene (250k particles, 128^3), first {steps} steps, FP64 torch-CPU",
            "seconds": dt}


def fused_bytes(scs):
    """Algorithmic bytes per launch of the fused kernel over the scenes of a
    batch: the particle state read and written (193 B per solid, 129 B per
    liquid particle) plus 28 B per active node (the tile write and the
    velocity read), active nodes counted at the initial positions."""
    import numpy as np
    from paper_2303_02346_amd import scenes
    total = 0
    for sc in scs:
        kinds = np.array([m.kind for m in sc.materials])[sc.mat]
        n_liq = int((kinds == scenes.LIQUID).sum())
        total += BYTES_SOLID * (sc.n - n_liq) + BYTES_LIQUID * n_liq + 28 * active_nodes(sc.x, sc.n_grid)
    return total


def bench_batched(torch, steps=100):
    """Config 4: 64 independent 64^3 scenes of log-uniform size in one
    launch (graph-captured, autotuned) against the same scenes run one
    after another, each in its own launch.  At 3.8M particles its state
    (about 300 MB) exceeds the 256 MB last-level cache, so its fused kernel
    is also reported against the HBM roofline, event-timed in an eager run
    of the same steps, with the HBM bytes counted per launch by rocprofv3
    (the committed counter summary, while its sources are unchanged)."""
    from paper_2303_02346_amd import scenes
    from paper_2303_02346_amd.sim import Simulator
    scs = scenes.config4(steps=steps)
    n_tot = sum(sc.n for sc in scs)
    log(f"[bench] batched: {len(scs)} scenes, {n_tot} particles")
    sim = Simulator(scs, graph=True)
    tune = sim.autotune(n_steps=min(10, steps))
    sim.reset()
    sim.step(steps)
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    # the same launch with every block in a single workgroup (no block
    # shared by two), against the tuned choice
    from paper_2303_02346_amd import _lib
    sim.set_option(_lib.MPM_OPT_SHARE_CHUNKS, 0)
    sim.reset()
    sim.step(steps)
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t_u = time.perf_counter() - t0
    sim.set_option(_lib.MPM_OPT_SHARE_CHUNKS, tune["share_chunks"])
    # the same steps eager, with the fused kernel's launches event-timed
    sim.reset()
    sim.timing(True)
    sim.step(steps)
    torch.cuda.synchronize()
    k_ms, k_n, k_name = sim.timing_read()
    sim.timing(False)
    sim.close()
    singles = [Simulator(sc, graph=True) for sc in scs]
    for s1 in singles:
        s1.step(steps)
        s1.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s1 in singles:
        s1.step(steps)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    for s1 in singles:
        s1.close()
    roof = None
    if k_n:
        b = fused_bytes(scs)
        avg = k_ms / k_n * 1e-3
        ach = b / avg / 1e9
        roof = {"bound": "hbm", "kernel": k_name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "avg_us": round(avg * 1e6, 2), "algorithmic_bytes_per_launch": b,
                "traffic": counted_traffic(BATCHED_TRAFFIC_SUMMARY)}
    out = {"scenes": len(scs), "particles": n_tot, "steps": steps, "launch": tune,
           "batched_rate": n_tot * steps / t_b, "sequential_rate": n_tot * steps / t_s,
           "unshared_blocks_rate": n_tot * steps / t_u,
           "speedup": t_s / t_b, "unit": "particle-steps/s", "roofline": roof}
    log(f"[bench] batched {out['batched_rate']:.3e} (no shared blocks {out['unshared_blocks_rate']:.3e}) vs "
        f"sequential {out['sequential_rate']:.3e} particle-steps/s (x{out['speedup']:.2f}); fused kernel {roof['avg_us'] if roof else None} us, "
        f"{roof['frac'] if roof else None} of HBM peak")
    return out


def bench_closure(torch, steps=100, n_samples=10_000_000, epochs=16):
    """Config 5: 1M sand particles on 256^3 with the learned cone return
    against the exact return (step time, fallback rate, accuracy)."""
    import numpy as np
    from paper_2303_02346_amd import scenes
    from paper_2303_02346_amd.closure import MLP, generate_samples
    from paper_2303_02346_amd.sim import Simulator
    t0 = time.perf_counter()
    samples = generate_samples(n_samples)
    t_gen = time.perf_counter() - t0
    perm = torch.randperm(samples.shape[0], device=samples.device)
    samples = samples[perm].contiguous()
    n_tr = int(0.95 * samples.shape[0])
    train, held = samples[:n_tr].contiguous(), samples[n_tr:].contiguous()
    net = MLP()
    net.init(train, seed=0)
    t0 = time.perf_counter()
    hist = net.train(train, epochs=epochs, batch=8192, lr=2e-3)
    t_train = time.perf_counter() - t0
    y = net.predict(held)
    err = (y - held[:, 6:9]).abs().max(1).values
    sc = scenes.config5(steps=steps)
    times = {}
    pos = {}
    stats = None
    for mode in ("exact", "learned"):
        sim = Simulator(sc, horizon=steps, graph=True)
        if mode == "learned":
            sim.set_closure(net, tol=1e-3)
        sim.step(steps)
        sim.reset()
        if mode == "learned":
            sim.closure_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        times[mode] = time.perf_counter() - t0
        pos[mode] = sim.positions()
        if mode == "learned":
            stats = sim.closure_stats()
        sim.close()
    dx = float(np.linalg.norm(pos["learned"] - pos["exact"]) / np.linalg.norm(pos["exact"]))
    out = {"particles": sc.n, "steps": steps, "samples": int(samples.shape[0]), "sample_seconds": t_gen,
           "train_seconds": t_train, "train_loss": hist, "heldout_err_inf_median": float(err.median()),
           "heldout_err_inf_p99": float(err.quantile(0.99)) if err.numel() < 16_000_000 else None,
           "exact_ms_per_step": times["exact"] * 1e3 / steps, "learned_ms_per_step": times["learned"] * 1e3 / steps,
           "speedup": times["exact"] / times["learned"], "accepted": stats[0], "fallback": stats[1],
           "position_rel_diff": dx}
    log(f"[bench] closure: exact {out['exact_ms_per_step']:.3f} ms/step, learned {out['learned_ms_per_step']:.3f} "
        f"ms/step (x{out['speedup']:.2f}); accepted {stats[0]}, fallback {stats[1]}; position diff {dx:.2e}")
    return out


def bench_paper_point(torch, steps=200):
    """The paper's operating point: ~1e5 particles on 64^3, substeps of
    1e-4 s; reported as substeps/s and as frames/s at 10 substeps per frame
    (the paper's real-time statement is 60 frames/s on an RTX 3090)."""
    from paper_2303_02346_amd import scenes
    from paper_2303_02346_amd.sim import Simulator
    sc = scenes.paper_point(steps=steps)
    sim = Simulator(sc, graph=True)
    tune = sim.autotune(n_steps=20)
    sim.reset()
    sim.step(steps)
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    # one call per frame of 10 substeps, as a Gym-style loop steps the
    # environment: each call imports the state, steps and exports it, and
    # returns after its read of the error word
    frames = steps // 10
    sim.reset()
    sim.step(10)
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(frames):
        sim.step(10)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    sim.close()
    out = {"particles": sc.n, "n_grid": sc.n_grid, "dt": sc.dt, "steps": steps, "launch": tune,
           "ms_per_substep": t * 1e3 / steps, "particle_steps_per_s": sc.n * steps / t,
           "frames_per_s_at_10_substeps": steps / t / 10.0,
           "one_call_per_frame": {"frames": frames, "ms_per_frame": tf * 1e3 / frames, "frames_per_s": frames / tf}}
    log(f"[bench] paper operating point: {out['ms_per_substep']:.4f} ms/substep, "
        f"{out['frames_per_s_at_10_substeps']:.0f} frames/s at 10 substeps per frame; one call per frame "
        f"{tf * 1e3 / frames:.3f} ms ({frames / tf:.0f} frames/s)")
    return out


def bench_rigid(torch, steps=100, bwd_steps=32):
    """Rigid bodies from particles at config-2 size: the sand cube replaced
    by a rigid cube (scenes.rigid_config2).  Such scenes step on the unfused
    sorted path (P2G, grid, G2P, projection, sort); forward and
    forward+backward (tiled adjoint, checkpoint every 16) rates."""
    from paper_2303_02346_amd import scenes
    from paper_2303_02346_amd.sim import Simulator
    sc = scenes.rigid_config2(steps=max(steps, bwd_steps))
    sim = Simulator(sc, horizon=steps)
    sim.step(10)
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    sim.close()
    simg = Simulator(sc, requires_grad=True, ckpt_every=16, horizon=bwd_steps)
    wx = torch.ones(3, sc.n, device="cuda")
    for rep in range(2):
        simg.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        simg.step(bwd_steps)
        ga = simg.backward(wx, torch.zeros_like(wx))
        torch.cuda.synchronize()
        t_fb = time.perf_counter() - t0
    simg.close()
    out = {"workload": "config-2 geometry, 125k water + 125k rigid-cube particles, 128^3, dt=5e-5",
           "particles": sc.n, "steps": steps, "ms_per_step": t * 1e3 / steps, "particle_steps_per_s": sc.n * steps / t,
           "fwd_bwd_steps": bwd_steps, "fwd_bwd_ms_per_step": t_fb * 1e3 / bwd_steps,
           "fwd_bwd_particle_steps_per_s": sc.n * bwd_steps / t_fb, "grad_norm": float(ga.norm().item())}
    log(f"[bench] rigid body scene: forward {out['ms_per_step']:.3f} ms/step, "
        f"fwd+bwd {out['fwd_bwd_ms_per_step']:.3f} ms/step")
    return out


def bench_gas(torch, n=128, steps=20, bwd_steps=8):
    """The gas solver (section 3.2's advection-projection) on the 128^3
    grid of the air-circulation task: forward steps, forward+backward, and
    the roofline of the spectral pressure solve's axis transform (the
    dominant kernel, six launches per step).  One launch transforms every
    grid line along one axis (here as a dense FP32 contraction with the
    n x n transform matrix on the matrix cores, 2 n flops per cell, also
    reported); the method's work is the separable transform, which reads and
    writes 8 B per cell, so the launch is priced against HBM.
    The six launches of a solve run back to back inside one HIP event pair;
    the average per launch is that time over six."""
    from paper_2303_02346_amd import scenes
    from paper_2303_02346_amd.gas import GasSim
    sc = scenes.gas_room(n=n, steps=max(steps, bwd_steps) + 2, seed=0)
    cells = n ** 3
    sim = GasSim(sc, horizon=steps + 2)
    sim.step(2)
    sim.reset()
    torch.cuda.synchronize()
    sim.timing(True)
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    adv_ms, adv_n, sm_ms, sm_n = sim.timing_read()
    sim.timing(False)
    sim.enable_stats(True)
    sim.reset()
    sim.step(1)
    res = sim.residual()
    sim.close()
    simg = GasSim(sc, requires_grad=True, ckpt_every=16, horizon=bwd_steps)
    w = torch.ones_like(simg.buf)
    for rep in range(2):
        simg.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        simg.step(bwd_steps)
        simg.backward(w)
        torch.cuda.synchronize()
        t_fb = time.perf_counter() - t0
    simg.close()
    sm_avg = sm_ms / max(sm_n, 1) * 1e-3
    ax_flops = 2.0 * n * cells
    ax_bytes = 8.0 * cells
    # the method's work is a separable transform: one read and one write of
    # every cell per axis pass, 8 B per cell, priced against HBM
    ach = ax_bytes / sm_avg / 1e9 if sm_n else None
    adv_avg = adv_ms / max(adv_n, 1) * 1e-3
    # advection reads the state once and writes it once at best: 8 B per value
    adv_bytes = 8.0 * sim_values(n, sc.s.shape[0])
    out = {"workload": f"gas room {n}^3 (velocity + temperature + smoke), emitter turning about y, dt=5e-3",
           "cells": cells, "steps": steps, "ms_per_step": t * 1e3 / steps, "cell_steps_per_s": cells * steps / t,
           "fwd_bwd_steps": bwd_steps, "fwd_bwd_ms_per_step": t_fb * 1e3 / bwd_steps,
           "pressure_solver": "spectral (DCT-II axis transforms)", "pressure_rel_residual": res,
           "advect": {"avg_us": round(adv_avg * 1e6, 2), "algorithmic_bytes_per_launch": int(adv_bytes),
                      "achieved_GBps": round(adv_bytes / adv_avg / 1e9, 1) if adv_n else None,
                      "frac_of_hbm": round(adv_bytes / adv_avg / 1e9 / HBM_PEAK_GBS, 4) if adv_n else None},
           "roofline": {"bound": "hbm", "kernel": "k_axis (the six transforms of a solve, per launch)", "dtype": "f32",
                        "achieved": round(ach, 1) if ach else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4) if ach else None,
                        "avg_us": round(sm_avg * 1e6, 2), "algorithmic_bytes_per_launch": int(ax_bytes),
                        "dense_matrix_flops_per_launch": int(ax_flops),
                        "dense_matrix_TFLOPs": round(ax_flops / sm_avg / 1e12, 2) if sm_n else None,
                        "traffic": counted_traffic(GAS_TRAFFIC_SUMMARY, GAS_TRAFFIC_SOURCES) if n == 128 else None}}
    log(f"[bench] gas {n}^3: forward {out['ms_per_step']:.3f} ms/step ({out['cell_steps_per_s']:.3e} cell-steps/s), "
        f"fwd+bwd {out['fwd_bwd_ms_per_step']:.3f} ms/step; axis transform {out['roofline']['avg_us']} us "
        f"({out['roofline']['frac']} of HBM peak), advection {out['advect']['avg_us']} us "
        f"({out['advect']['frac_of_hbm']} of HBM peak); residual {res:.1e}")
    return out


def sim_values(n, n_scalars):
    """Values of the gas state on an n^3 grid: three staggered velocity
    components ((n + 1) n^2 each) and the cell scalars."""
    return 3 * (n + 1) * n * n + n_scalars * n ** 3


def copy_ceiling(torch, mb=1024, reps=10):
    """Measured device-to-device copy rate (bytes read + bytes written per
    second) of a 1 GiB buffer, event-timed: the practical HBM ceiling beside
    the 8 TB/s nominal peak."""
    n = int(mb) * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return {"bytes": 2 * n * 4, "GBps": round(2 * n * 4 / sec / 1e9, 1), "frac_of_peak": round(2 * n * 4 / sec / 1e9 / HBM_PEAK_GBS, 4)}


def copy_calibration(torch, mb):
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    n = int(mb) * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: 3 copies of {n * 4} bytes")
    return n * 4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--bwd-steps", type=int, default=64)
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--adjoint", choices=["tiled", "plain"], default="tiled")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--particles", type=int, default=250_000)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-paper-point", action="store_true")
    ap.add_argument("--no-rigid", action="store_true")
    ap.add_argument("--no-gas", action="store_true")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched leg and print its object (for profiling its kernels)")
    ap.add_argument("--batched-steps", type=int, default=100)
    ap.add_argument("--copy-mb", type=int, default=0, help="first run a device copy of this size (counter scaling)")
    ap.add_argument("--no-closure", action="store_true", help="skip the learned-closure leg (config 5)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not part of this build",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2303_02346_amd import scenes
    from paper_2303_02346_amd.sim import Simulator

    copy_bytes = copy_calibration(torch, args.copy_mb) if args.copy_mb > 0 else None
    if args.only_batched:
        print(json.dumps({"batched": bench_batched(torch, steps=args.batched_steps)}), flush=True)
        return
    ceiling = copy_ceiling(torch)
    log(f"[bench] measured copy ceiling {ceiling['GBps']} GB/s ({ceiling['frac_of_peak']} of 8 TB/s)")
    sc = scenes.config2(n_particles=args.particles, steps=max(args.steps, args.warmup, args.bwd_steps))
    N = sc.n
    kinds = np.array([m.kind for m in sc.materials])[sc.mat]
    n_liq = int((kinds == scenes.LIQUID).sum())
    n_sol = N - n_liq
    n_act = active_nodes(sc.x, sc.n_grid)

    log(f"[bench] forward: {N} particles, {args.warmup} warmup + {args.steps} timed steps")
    sim = Simulator(sc, requires_grad=False, horizon=max(args.steps, args.warmup))
    tune = None
    if not args.no_tune:
        tune = sim.autotune(n_steps=min(20, args.steps))
        log(f"[bench] autotuned launch shape: {tune}")
    # untimed warm-up, then the timed region: K steps in one call, with the
    # dominant kernel's launches bracketed by HIP events on the library's
    # stream (timed calls run without graph capture)
    sim.reset()
    sim.step(args.warmup)
    sim.reset()
    torch.cuda.synchronize()
    sim.timing(True)
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    k_ms, k_launches, k_name = sim.timing_read()
    sim.timing(False)
    fwd_rate = N * args.steps / t_fwd
    log(f"[bench] forward {t_fwd * 1e3 / args.steps:.3f} ms/step, {fwd_rate:.3e} particle-steps/s; "
        f"{k_name} avg {k_ms / max(k_launches, 1) * 1e3:.1f} us over {k_launches} launches")
    # steady state: the timed call above also imports (sorts) and exports the
    # state once; (T(K) - T(1)) / (K - 1) removes that one-time cost
    steady = None
    if args.steps > 1:
        sim.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(1)
        torch.cuda.synchronize()
        t_one = time.perf_counter() - t0
        ms = (t_fwd - t_one) * 1e3 / (args.steps - 1)
        steady = {"ms_per_step": ms, "value": N / (ms * 1e-3), "one_step_call_ms": t_one * 1e3}
        log(f"[bench] forward steady state {ms:.4f} ms/step (a one-step call takes {t_one * 1e3:.3f} ms)")
    graph = None
    if not args.no_graph:
        # the same K steps replayed from a captured HIP graph (untimed per kernel)
        from paper_2303_02346_amd import _lib
        sim.set_option(_lib.MPM_OPT_GRAPH, 1)
        sim.reset()
        sim.step(args.steps)
        sim.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(args.steps)
        torch.cuda.synchronize()
        t_g = time.perf_counter() - t0
        graph = {"value": N * args.steps / t_g, "ms_per_step": t_g * 1e3 / args.steps}
        log(f"[bench] forward, graph replay: {t_g * 1e3 / args.steps:.3f} ms/step")

    per = KERNEL_BYTES.get(k_name)
    roof = None
    if per is not None and k_launches > 0:
        bytes_launch = per[0] * n_sol + per[1] * n_liq + per[2] * n_act
        avg_s = k_ms / k_launches * 1e-3
        ach = bytes_launch / avg_s / 1e9
        traffic = counted_traffic() if k_name == "k_g2p2g" else None
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": k_name,
                "avg_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": int(bytes_launch),
                "frac_of_copy_ceiling": round(ach / ceiling["GBps"], 4)}
    # the headline: the graph replay of the K-step call when it ran, else the
    # event-timed eager call (the same work either way)
    t_head = graph["ms_per_step"] * 1e-3 * args.steps if graph else t_fwd
    step_bytes = BYTES_SOLID * n_sol + BYTES_LIQUID * n_liq + BYTES_NODE * n_act
    step_frac = step_bytes / (t_head / args.steps) / 1e9 / HBM_PEAK_GBS

    fwd_bwd = None
    if not args.no_bwd:
        T = args.bwd_steps
        log(f"[bench] forward+backward: {T} steps, checkpoint every 16, {args.adjoint} adjoint")
        simg = Simulator(sc, requires_grad=True, ckpt_every=16, horizon=T, graph=not args.no_graph,
                         adjoint=args.adjoint)
        for rep in range(2):
            simg.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            simg.step(T)
            loss, g = simg.loss_blob(sc.target_mu, sc.target_sigma)
            ga = simg.backward(g[0:3], torch.zeros_like(g[0:3]))
            torch.cuda.synchronize()
            t_fb = time.perf_counter() - t0
        simg.close()
        fb_bytes = 680.0 * N * T
        fwd_bwd = {"value": N * T / t_fb, "unit": "particle-steps/s", "steps": T, "ckpt_every": 16,
                   "adjoint": args.adjoint,
                   "ms_per_step": t_fb * 1e3 / T, "loss": float(loss.item()),
                   "grad_norm": float(ga.norm().item()),
                   "hbm_frac_algorithmic": round(fb_bytes / t_fb / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"[bench] fwd+bwd {t_fb * 1e3 / T:.3f} ms/step, {N * T / t_fb:.3e} particle-steps/s")
        if args.adjoint == "tiled":
            # the same with a record of every step kept by the forward
            # (ckpt_every = 0): the backward recomputes nothing
            simr = Simulator(sc, requires_grad=True, ckpt_every=0, horizon=T, graph=not args.no_graph)
            for rep in range(2):
                simr.reset()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                simr.step(T)
                loss_r, g = simr.loss_blob(sc.target_mu, sc.target_sigma)
                ga_r = simr.backward(g[0:3], torch.zeros_like(g[0:3]))
                torch.cuda.synchronize()
                t_r = time.perf_counter() - t0
            simr.close()
            fwd_bwd["no_recompute"] = {"ckpt_every": 0, "value": N * T / t_r, "ms_per_step": t_r * 1e3 / T,
                                       "loss": float(loss_r.item()), "grad_norm": float(ga_r.norm().item())}
            log(f"[bench] fwd+bwd with every step's record kept {t_r * 1e3 / T:.3f} ms/step, "
                f"{N * T / t_r:.3e} particle-steps/s")

    batched = None
    if not args.no_batched:
        batched = bench_batched(torch, steps=args.batched_steps)

    paper = None if args.no_paper_point else bench_paper_point(torch)

    rigid = None if args.no_rigid else bench_rigid(torch)
    gas = None if args.no_gas else bench_gas(torch)

    closure = None if args.no_closure else bench_closure(torch)

    cpu = None
    if not args.no_cpu:
        log(f"[bench] CPU oracle sample: {args.cpu_steps} steps")
        cpu = cpu_baseline(sc, args.cpu_steps)
        log(f"[bench] CPU oracle {cpu['value']:.3e} particle-steps/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC, "value": N * args.steps / t_head, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_head * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "config 2: 250k particles (125k liquid + 125k Drucker-Prager sand) in two seeded boxes, "
                               "128^3 grid, dt=5e-5, kinematic cylinder r=0.05 with seeded smooth 6-DoF trajectory",
                   "n_particles": N, "n_grid": sc.n_grid, "dt": sc.dt, "active_nodes": n_act},
        "step_hbm_frac_algorithmic": round(step_frac, 4),
        "launch": tune,
        "timed_call": {"value": fwd_rate, "ms_per_step": t_fwd * 1e3 / args.steps,
                       "mode": "eager, fused kernel launches bracketed by HIP events"},
        "steady_state": steady,
        "graph_replay": graph,
        "copy_ceiling": ceiling,
        "fwd_bwd": fwd_bwd,
        "batched": batched,
        "paper_point": paper,
        "rigid": rigid,
        "gas": gas,
        "closure": closure,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
