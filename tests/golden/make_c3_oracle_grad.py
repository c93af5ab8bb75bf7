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


def main():
    sc = scenes.config3()
    t0 = time.time()
    L, g = O.loss_and_action_grad(sc, checkpoint_every=1)
    out = {"scene": "config 3: 100k particles (50k liquid + 50k sand), 96^3, dt=5e-5, 64 steps, blob loss",
           "target_mu": sc.target_mu.tolist(), "target_sigma": sc.target_sigma, "loss": float(L),
           "grad_actions": g.numpy().tolist(), "oracle_seconds": time.time() - t0}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle_grad.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: loss {float(L):.10f}, |g| {float(g.norm()):.6e}, {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
