"""FP64 CPU oracle of the learned cone-return closure network.

TEST INFRASTRUCTURE ONLY (imported by tests, never by the product path).

The network is the plain definition: with normalised input
xn = (x - in_mean) / in_std,
  h1 = relu(W1 xn + b1), h2 = relu(W2 h1 + b2), u = (W3 h2 + b3) * out_std + out_mean,
and its output keeps the trace of the trial log strain (the Drucker-Prager
cone return moves only the deviatoric part):
  y = u + (x_0 + x_1 + x_2 - u_0 - u_1 - u_2) / 3.
The training loss is the mean squared error of the normalised outputs,
L = mean over samples and outputs of ((y - out_mean) / out_std - (t - out_mean) / out_std)^2.
Its gradient comes from torch autograd in float64.  Parameter vector order:
W1 (64x6) b1 W2 (64x64) b2 W3 (3x64) b3, row-major [out][in].

The closure is judged by the exact Drucker-Prager return of the simulator
oracle (mpm_oracle.dp_project): error and yield residual of the prediction.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mpm_oracle as O

DT = torch.float64
SIZES = [(64, 6), (64,), (64, 64), (64,), (3, 64), (3,)]


def unpack(p):
    p = torch.as_tensor(p, dtype=DT)
    out, o = [], 0
    for shp in SIZES:
        n = int(np.prod(shp))
        out.append(p[o:o + n].reshape(shp))
        o += n
    return out


def forward(p, norm, x):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = torch.as_tensor(x, dtype=DT)
    xn = (x - torch.as_tensor(norm["in_mean"], dtype=DT)) / torch.as_tensor(norm["in_std"], dtype=DT)
    h1 = torch.relu(xn @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    sd = torch.as_tensor(norm["out_std"], dtype=DT)
    mn = torch.as_tensor(norm["out_mean"], dtype=DT)
    u = (h2 @ W3.T + b3) * sd + mn
    y = u + ((x[:, 0:3].sum(1) - u.sum(1)) / 3.0)[:, None]
    return y, (y - mn) / sd


def loss_and_grad(p, norm, records):
    """MSE of the normalised outputs over the records (n x 9) and its
    gradient with respect to the parameter vector."""
    pt = torch.as_tensor(np.asarray(p, np.float64), dtype=DT).clone().requires_grad_(True)
    rec = torch.as_tensor(np.asarray(records, np.float64), dtype=DT)
    y, yn = forward(pt, norm, rec[:, :6])
    tn = (rec[:, 6:9] - torch.as_tensor(norm["out_mean"], dtype=DT)) / torch.as_tensor(norm["out_std"], dtype=DT)
    L = ((yn - tn) ** 2).mean()
    L.backward()
    return float(L), pt.grad.numpy().copy()


def adam_step(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def exact_return(records):
    """Exact cone return of the inputs of each record (log sigma, alpha, c,
    kappa) with the simulator oracle's Drucker-Prager map."""
    rec = torch.as_tensor(np.asarray(records, np.float64), dtype=DT)
    ep, case = O.dp_project(rec[:, 0:3], rec[:, 3], rec[:, 5], rec[:, 4])
    return ep.numpy(), case.numpy()


def yield_residual(eps, records):
    """|f(eps)| + |tr eps - tr eps_trial|, f = |dev(eps - c)| + kappa alpha tr(eps - c)."""
    eps = np.asarray(eps, np.float64)
    rec = np.asarray(records, np.float64)
    es = eps - rec[:, 4:5]
    tr = es.sum(-1)
    dev = es - tr[:, None] / 3
    f = np.linalg.norm(dev, axis=-1) + rec[:, 5] * rec[:, 3] * tr
    return np.abs(f) + np.abs(eps.sum(-1) - rec[:, 0:3].sum(-1))
