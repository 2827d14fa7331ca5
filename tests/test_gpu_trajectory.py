"""Trajectory parity at the benchmark size: CP 'ir,jr,kr->ijk' 256^3, R = 32,
20 % missing, (alpha, beta) = (1, 1) and (0.5, 1), 200 sweeps of Algorithm 1.

* one sweep from the GPU's own state at t in {1, 10, 199} matches the FP64
  oracle's sweep from that state: relative 1e-5 per factor for FP32
  contractions, 1e-2 for BF16 (per-iterate tolerances);
* the FP64 loss (evaluated by the oracle) of the GPU's 200-sweep state is
  within 1e-4 relative of L*, the oracle's own 200-sweep loss from the same
  seeded init (tests/golden/cp3_targets.json, written by the oracle only);
* the GPU's loss trace (FP32 terms, FP64 sums) follows the oracle's recorded
  trajectory at 1e-5 relative for FP32 contractions.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_02759_amd import datagen

from _gpu_util import EPS, assert_step_parity, clamp_init, oracle_sweep, to_dev

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
CHECK_AT = (1, 10, 199)
N_SWEEPS = 200


def _targets(ab):
    with open(os.path.join(HERE, "golden", "cp3_targets.json")) as fh:
        return json.load(fh)["targets"][f"{ab[0]},{ab[1]}"]


def _run(p, prec):
    """200 sweeps on the GPU; returns the states at 0..200 that the checks
    need (FP32 numpy) and the loss trace (loss of theta_t at index t)."""
    import torch
    from paper_2602_02759_amd.nnef import Plan
    plan = Plan(p.model_str, p.mode_sizes, p.ranks, p.alpha, p.beta, eps=EPS, prec=prec)
    Y, M = to_dev(p.Y), to_dev(p.M)
    f = [to_dev(s) for s in clamp_init(p)]
    tr = torch.zeros(N_SWEEPS, dtype=torch.float64, device="cuda:0")
    keep = sorted({t for c in CHECK_AT for t in (c, c + 1)} | {N_SWEEPS})
    states, done = {}, 0
    for t in keep:
        plan.step(Y, M, f, n_sweeps=t - done, loss_trace=tr[done:t])
        done = t
        states[t] = [x.cpu().numpy().copy() for x in f]
    torch.cuda.synchronize()
    plan.close()
    return states, tr.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16_all"])
@pytest.mark.parametrize("ab", [(1.0, 1.0), (0.5, 1.0)])
def test_cp3_full_trajectory(ab, prec):
    print(f"[trajectory] CP 256^3 R=32 ab={ab} {prec}", flush=True)
    p = datagen.cp3(*ab)
    tgt = _targets(ab)
    states, tr = _run(p, prec)
    tol = 1e-5 if prec == "fp32" else 1e-2
    for t in CHECK_AT:
        worst = assert_step_parity(states[t + 1], oracle_sweep(p, states[t]), tol, f"{prec} t={t}")
        print(f"  step parity at t={t}: worst rel {worst:.2e}", flush=True)
    lg = O.loss(p.model_str, [x.astype(np.float64) for x in states[N_SWEEPS]], p.Y, p.M, *ab)
    ls = tgt["L_star"]
    print(f"  200-sweep loss {lg:.10e} vs L* {ls:.10e}: rel {(lg - ls) / ls:+.2e}", flush=True)
    assert abs(lg - ls) <= 1e-4 * ls
    if prec == "fp32":
        for k, v in tgt["loss_by_sweep"].items():
            k = int(k)
            if k < N_SWEEPS:
                assert abs(tr[k] - v) <= 1e-5 * v, (k, tr[k], v)
