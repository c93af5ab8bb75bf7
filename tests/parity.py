"""Element-wise comparison of a GPU particle state with the FP64 oracle's.

Every field is judged two ways:
  - the Frobenius ratio ||Q_gpu - Q_ref|| / ||Q_ref|| over all particles;
  - the largest per-particle error: for positions the per-particle relative
    error |x_gpu,p - x_ref,p| / |x_ref,p| (positions lie inside the unit
    cube, away from the origin by the wall band), for v, C, F and J the
    per-particle error norm divided by the largest per-particle norm of the
    reference field.
A single wrong particle therefore fails the second figure even when the
Frobenius ratio over hundreds of thousands of particles hides it.
"""
import numpy as np

from paper_2303_02346_amd import scenes


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def liquid_mask(sc):
    kinds = np.array([m.kind for m in sc.materials])
    return kinds[sc.mat] == scenes.LIQUID


def _rows(a):
    a = np.asarray(a, np.float64)
    return a.reshape(a.shape[0], -1)


def _max_scaled(a, b):
    """Largest per-particle error norm over the largest reference norm."""
    a, b = _rows(a), _rows(b)
    if a.shape[0] == 0:
        return 0.0
    err = np.linalg.norm(a - b, axis=1)
    return float(err.max() / max(np.linalg.norm(b, axis=1).max(), 1e-30))


def state_errors(gpu, ref, liquid, n_grid=None):
    """With n_grid, C is judged against the larger of its own size and the
    velocity-gradient scale |v|/dx: where the reference C is round-off (a
    body in free fall), its own size is no scale."""
    solid = ~liquid
    xg, xr = _rows(gpu["x"]), _rows(ref["x"])
    Cg, Cr = _rows(gpu["C"]), _rows(ref["C"])
    if n_grid is None:
        eC, eC_max = rel(Cg, Cr), _max_scaled(Cg, Cr)
    else:
        vr = _rows(ref["v"])
        fro = max(np.linalg.norm(Cr), np.linalg.norm(vr) * n_grid, 1e-30)
        top = max(np.linalg.norm(Cr, axis=1).max(), np.linalg.norm(vr, axis=1).max() * n_grid, 1e-30)
        eC = float(np.linalg.norm(Cg - Cr) / fro)
        eC_max = float(np.linalg.norm(Cg - Cr, axis=1).max() / top)
    e = {
        "x": rel(xg, xr),
        "x_max": float((np.linalg.norm(xg - xr, axis=1) / np.linalg.norm(xr, axis=1)).max()),
        "v": rel(gpu["v"], ref["v"]), "v_max": _max_scaled(gpu["v"], ref["v"]),
        "C": eC, "C_max": eC_max,
        "F": rel(gpu["F"][solid], ref["F"][solid]) if solid.any() else 0.0,
        "F_max": _max_scaled(gpu["F"][solid], ref["F"][solid]) if solid.any() else 0.0,
        "J": rel(gpu["J"][liquid], ref["J"][liquid]) if liquid.any() else 0.0,
        "J_max": _max_scaled(gpu["J"][liquid][:, None], ref["J"][liquid][:, None]) if liquid.any() else 0.0,
    }
    return e


def compare_states(gpu, ref, liquid, tol_x=1e-5, tol=1e-3, tol_x_max=None, tol_max=None, tol_FJ=None,
                   tol_FJ_max=None, n_grid=None):
    """Assert both the Frobenius and the per-particle figures.  Defaults:
    per-particle gates ten times the Frobenius gates; F and J gates ten times
    the position gate."""
    e = state_errors(gpu, ref, liquid, n_grid)
    tol_x_max = 10 * tol_x if tol_x_max is None else tol_x_max
    tol_max = 10 * tol if tol_max is None else tol_max
    tol_FJ = 10 * tol_x if tol_FJ is None else tol_FJ
    tol_FJ_max = 10 * tol_FJ if tol_FJ_max is None else tol_FJ_max
    say("  Frobenius x {x:.2e} v {v:.2e} C {C:.2e} F {F:.2e} J {J:.2e} | "
        "per particle x {x_max:.2e} v {v_max:.2e} C {C_max:.2e} F {F_max:.2e} J {J_max:.2e}".format(**e))
    assert e["x"] <= tol_x and e["x_max"] <= tol_x_max, e
    assert e["v"] <= tol and e["C"] <= tol, e
    assert e["v_max"] <= tol_max and e["C_max"] <= tol_max, e
    assert e["F"] <= tol_FJ and e["J"] <= tol_FJ, e
    assert e["F_max"] <= tol_FJ_max and e["J_max"] <= tol_FJ_max, e
    return e


def dp_cases(F_old, C_new, dt, alpha, kappa, cohesion):
    """Drucker-Prager case of each sand particle's trial state
    F_tr = (I + dt C_new) F_old: 0 inside the cone, 1 apex (tension),
    2 cone (flow).  Counted from the singular values in FP64 with the
    textbook case split of the log-strain return (trace beyond the apex,
    else yield function f = |dev| + kappa alpha tr)."""
    I = np.eye(3)
    Ft = (I[None] + dt * C_new) @ F_old
    s = np.linalg.svd(Ft, compute_uv=False)
    e = np.log(s) - cohesion[:, None]
    t = e.sum(1)
    dev = e - t[:, None] / 3.0
    f = np.linalg.norm(dev, axis=1) + kappa * alpha * t
    return np.where(t > 0, 1, np.where(f <= 0, 0, 2))


def oracle_rollout_coverage(O, sc, steps):
    """The oracle's rollout (the same steps as O.rollout), step by step, also
    counting over the window (a) the Drucker-Prager cases of the sand trial
    states and (b) the particles inside the contact band by at least one
    cell (d < (band - 1) dx from the cylinder's surface), whose stencils
    then hold nodes inside the band.  Returns (state as numpy, case counts
    [inside, apex, cone], band particle-steps)."""
    import torch
    p = O.params_from_scene(sc)
    st = O.state_from_scene(sc)
    acts = torch.tensor(sc.actions, dtype=torch.float64)
    cs, Rs = O.integrate_pose(torch.tensor(sc.cyl_pos0, dtype=torch.float64),
                              torch.tensor(sc.cyl_rot0, dtype=torch.float64), acts[:steps], p.dt)
    sand = (p.kind == O.SAND).numpy()
    al, ka, co = p.alpha.numpy()[sand], p.kappa.numpy()[sand], p.cohesion.numpy()[sand]
    cases = np.zeros(3, np.int64)
    band = 0
    for t in range(steps):
        if sc.cyl_radius > 0:
            x = st["x"].numpy()
            a = Rs[t].numpy()[:, 1]
            r = x - cs[t].numpy()
            rp = r - (r @ a)[:, None] * a[None, :]
            d = np.linalg.norm(rp, axis=1) - sc.cyl_radius
            band += int((d < (sc.contact_band - 1.0) * p.dx).sum())
        new = O.step(st, cs[t], Rs[t], acts[t], p)
        if sand.any():
            c = dp_cases(st["F"].numpy()[sand], new["C"].numpy()[sand], p.dt, al, ka, co)
            cases += np.bincount(c, minlength=3)
        st = new
    return {k: v.detach().numpy() for k, v in st.items()}, cases, band


def ill_conditioned_solids(sc, seed, share=0.5):
    """Give a seeded share of the scene's solid particles an ill-conditioned
    initial F = R1 diag(a, b, c) R2^T (proper rotations, a in [1.05, 1.25],
    b / a in [0.5, 0.9], c / a in [0.14, 0.24]), so that the smallest
    singular value is below a quarter of the largest.  Returns the number of
    particles changed."""
    rng = np.random.default_rng(np.random.SeedSequence([20230302, 77, seed]))
    kinds = np.array([m.kind for m in sc.materials])[sc.mat]
    F = np.array(sc.F, np.float64).reshape(sc.n, 3, 3).copy()
    sel = np.flatnonzero((kinds != scenes.LIQUID) & (rng.random(sc.n) < share))

    def rot(k):
        q = rng.normal(size=(k, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        w, x, y, z = q.T
        return np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                         2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                         2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], 1).reshape(k, 3, 3)

    a = rng.uniform(1.05, 1.25, sel.size)
    b = a * rng.uniform(0.5, 0.9, sel.size)
    c = a * rng.uniform(0.14, 0.24, sel.size)
    s = np.stack([a, b, c], 1)
    F[sel] = rot(sel.size) @ (s[:, :, None] * rot(sel.size).transpose(0, 2, 1))
    sc.F = F.reshape(np.shape(sc.F))
    return int(sel.size)
