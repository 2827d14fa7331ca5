"""Training driver for the learned extrapolation (host orchestration only).

Every computation runs in libnnef's kernels through the C ABI: the sweeps that
generate the trajectories (``nnef_step``), the feature and target rows
(``nnef_learned_rows``) and the training steps (``nnef_mlp_train_step``).
This module only decides which iterates become training rows, draws the
seeded initial weights and row order, and allocates device memory.
"""
from __future__ import annotations

import numpy as np

from . import nnef

N_IN, WIDTH = 8, 128


def init_params(seed=0, s0=1.0):
    """He-initialised parameters (float32, the library's flat layout) with the
    output bias set so that the initial step multiplier is s0."""
    import torch
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 77])))
    w1 = rng.normal(0.0, np.sqrt(2.0 / N_IN), (N_IN, WIDTH))
    b1 = np.zeros(WIDTH)
    w2 = rng.normal(0.0, np.sqrt(2.0 / WIDTH), (WIDTH, WIDTH))
    b2 = np.zeros(WIDTH)
    w3 = rng.normal(0.0, 0.1 * np.sqrt(1.0 / WIDTH), WIDTH)
    b3 = np.array([np.log(np.expm1(s0))])
    flat = np.concatenate([w1.ravel(), b1, w2.ravel(), b2, w3, b3]).astype(np.float32)
    assert flat.size == nnef.nnef_mlp_num_params()
    return torch.from_numpy(flat).to("cuda")


def trajectory_rows(plan, Y, M, init, n_sweeps, horizon, t_every=1, t_min=2):
    """Run ``n_sweeps`` plain sweeps from ``init`` (device factors, not
    modified) and return device (X, tau) training rows for t = t_min,
    t_min + t_every, ... <= n_sweeps - horizon."""
    import torch
    f = [t.clone() for t in init]
    snaps = [[t.clone() for t in f]]
    trace = torch.zeros(n_sweeps + 1, dtype=torch.float64, device="cuda")
    for s in range(n_sweeps):
        plan.step(Y, M, f, n_sweeps=1, loss_trace=trace[s:s + 1])
        snaps.append([t.clone() for t in f])
    plan.loss_device(Y, M, f, trace[n_sweeps:n_sweeps + 1])
    losses = trace.cpu().numpy()   # loss of snaps[t] is losses[t]
    ts = list(range(t_min, n_sweeps - horizon + 1, t_every))
    n_el = sum(plan.numels)
    X = torch.empty((len(ts) * n_el, N_IN), dtype=torch.float32, device="cuda")
    tau = torch.empty(len(ts) * n_el, dtype=torch.float32, device="cuda")
    for i, t in enumerate(ts):
        rel = (losses[t - 1] - losses[t]) / losses[t]
        plan.rows(snaps[t], snaps[t - 1], snaps[t - 2], snaps[t + horizon], rel,
                  X[i * n_el:(i + 1) * n_el], tau[i * n_el:(i + 1) * n_el])
    return X, tau, losses


def train(mlp, X, tau, steps, batch=8192, lr=1e-3, seed=0, report_every=0):
    """``steps`` Adam steps on minibatches drawn without replacement (a fresh
    seeded permutation per epoch).  Returns the minibatch losses reported."""
    import torch
    n = X.shape[0]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 78])))
    per_epoch = max(1, n // batch)
    n_epochs = (steps + per_epoch - 1) // per_epoch
    order = np.concatenate([rng.permutation(n)[:per_epoch * batch] for _ in range(n_epochs)])
    idx = torch.from_numpy(order.astype(np.int32)).to("cuda")
    bsz = min(batch, n)
    losses = torch.zeros(max(1, steps), dtype=torch.float64, device="cuda")
    for k in range(steps):
        mlp.train_step(X, tau, lr, idx=idx[k * bsz:(k + 1) * bsz], d_loss=losses[k:k + 1])
    out = losses.cpu().numpy()
    return out
