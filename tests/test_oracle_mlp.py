"""Pins of the closure network oracle (CPU only): closed-form special
networks, finite differences of the loss gradient, the first Adam step and
the exact-return judge."""
import numpy as np
import torch

from oracle import mlp_oracle as M
from oracle import mpm_oracle as O

NORM0 = {"in_mean": np.zeros(6), "in_std": np.ones(6), "out_mean": np.zeros(3), "out_std": np.ones(3)}


def identity_net():
    """W1 = [I6; 0], W2 = I, W3 = [I3 0]: y = relu(x)[:3]."""
    W1 = np.zeros((64, 6)); W1[:6, :6] = np.eye(6)
    W2 = np.eye(64)
    W3 = np.zeros((3, 64)); W3[:3, :3] = np.eye(3)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(), np.zeros(3)])


def test_parameter_count():
    assert sum(int(np.prod(s)) for s in M.SIZES) == 4803


def trace_shift(u, x):
    """u shifted equally in its three components so that its sum is that of x[:, :3]."""
    return u + ((x[:, :3].sum(1) - u.sum(1)) / 3.0)[:, None]


def test_identity_network_closed_form():
    rng = np.random.default_rng(0)
    x = rng.normal(0, 1, (50, 6))
    y, _ = M.forward(identity_net(), NORM0, x)
    assert np.allclose(y.numpy(), trace_shift(np.maximum(x[:, :3], 0), x), atol=1e-15)
    # non-negative inputs pass through unchanged
    xp = np.abs(x)
    yp, _ = M.forward(identity_net(), NORM0, xp)
    assert np.allclose(yp.numpy(), xp[:, :3], atol=1e-15)


def test_normalisation_is_applied():
    rng = np.random.default_rng(1)
    norm = {"in_mean": rng.normal(0, 1, 6), "in_std": rng.uniform(0.5, 2, 6),
            "out_mean": rng.normal(0, 1, 3), "out_std": rng.uniform(0.5, 2, 3)}
    x = rng.normal(0, 1, (20, 6))
    y, yn = M.forward(identity_net(), norm, x)
    xn = (x - norm["in_mean"]) / norm["in_std"]
    u = np.maximum(xn[:, :3], 0) * norm["out_std"] + norm["out_mean"]
    assert np.allclose(y.numpy(), trace_shift(u, x))
    assert np.allclose(yn.numpy(), (trace_shift(u, x) - norm["out_mean"]) / norm["out_std"])


def test_output_keeps_the_trial_trace():
    """The cone return is deviatoric: any network's output has the trial sum."""
    rng = np.random.default_rng(5)
    p = rng.normal(0, 0.5, 4803)
    x = rng.normal(0, 0.05, (100, 6))
    y, _ = M.forward(p, NORM0, x)
    assert np.allclose(y.numpy().sum(1), x[:, :3].sum(1), atol=1e-13)


def test_loss_gradient_fd():
    rng = np.random.default_rng(2)
    p = rng.normal(0, 0.3, 4803)
    rec = rng.normal(0, 1, (40, 9))
    L, g = M.loss_and_grad(p, NORM0, rec)
    for idx in [0, 100, 383, 384, 500, 3000, 4543, 4550, 4700, 4801]:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[idx] += h
        pm[idx] -= h
        num = (M.loss_and_grad(pp, NORM0, rec)[0] - M.loss_and_grad(pm, NORM0, rec)[0]) / (2 * h)
        assert abs(num - g[idx]) <= 1e-6 * max(1.0, abs(num)), idx


def test_first_adam_step_is_sign_step():
    rng = np.random.default_rng(3)
    g = rng.normal(0, 1, 100)
    p, m, v = M.adam_step(np.zeros(100), np.zeros(100), np.zeros(100), g, 1, lr=1e-2)
    assert np.allclose(p, -1e-2 * np.sign(g), atol=1e-9)


def test_exact_return_and_residual():
    rng = np.random.default_rng(4)
    n = 5000
    e = np.sort(rng.normal(0, 0.03, (n, 3)), axis=1)[:, ::-1]
    alpha = np.full(n, O.dp_alpha(30.0))
    coh = rng.uniform(0, 0.01, n)
    kappa = rng.uniform(2, 4.5, n)
    rec = np.concatenate([e, alpha[:, None], coh[:, None], kappa[:, None], np.zeros((n, 3))], 1)
    ep, case = M.exact_return(rec)
    cone = case == 2
    assert cone.any()
    r = M.yield_residual(ep[cone], rec[cone])
    assert r.max() < 1e-14
    # the trial point itself is far from the cone in the cone case
    r0 = M.yield_residual(rec[cone, 0:3], rec[cone])
    assert np.median(r0) > 1e-4
