"""Write the FP64 oracle's config-3 loss and action gradient to
tests/golden/c3_oracle_grad.json.

Calls only the oracle (oracle/mpm_oracle.py) on the seeded config-3 scene
(100k particles, 96^3, 64 steps, blob loss), with per-step recompute to bound
memory.  Run from the repository root:  python tests/golden/make_c3_oracle_grad.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mpm_oracle as O  # noqa: E402
from paper_2303_02346_amd import scenes  # noqa: E402


def fd_directions(sc, g, n_dirs=4, eps=1e-3):
    """Central differences of the oracle loss along seeded unit directions
    in action space (eps = 1e-3), beside the oracle's own adjoint."""
    import numpy as np
    import torch
    p = O.params_from_scene(sc)
    liq = p.kind == O.LIQUID
    mu = torch.tensor(sc.target_mu, dtype=O.DT)
    a0 = torch.tensor(sc.actions, dtype=O.DT)
    rng = np.random.default_rng(20230302)
    out = []
    for k in range(n_dirs):
        d = rng.normal(0, 1, a0.shape)
        d /= np.linalg.norm(d)
        vals = []
        for sgn in (1, -1):
            st = O.rollout(sc, actions=a0 + sgn * eps * torch.tensor(d), params=p)
            vals.append(float(O.blob_loss(st["x"], liq, mu, sc.target_sigma)))
        out.append({"direction": d.tolist(), "eps": eps, "fd": (vals[0] - vals[1]) / (2 * eps),
                    "adjoint": float((g.numpy() * d).sum())})
        print(f"direction {k}: fd {out[-1]['fd']:.6e} adjoint {out[-1]['adjoint']:.6e}", flush=True)
    return out


def main():
    sc = scenes.config3()
    t0 = time.time()
    L, g = O.loss_and_action_grad(sc, checkpoint_every=1)
    fd = fd_directions(sc, g) if "--no-fd" not in sys.argv else []
    out = {"scene": "config 3: 100k particles (50k liquid + 50k sand), 96^3, dt=5e-5, 64 steps, blob loss",
           "target_mu": sc.target_mu.tolist(), "target_sigma": sc.target_sigma, "loss": float(L),
           "grad_actions": g.numpy().tolist(), "fd": fd, "oracle_seconds": time.time() - t0}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle_grad.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: loss {float(L):.10f}, |g| {float(g.norm()):.6e}, {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
