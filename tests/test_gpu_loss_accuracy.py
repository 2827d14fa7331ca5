"""Loss accuracy near a fit, where the terms of the (alpha, beta)-divergence
cancel: exact-rank CP data (20 % missing) fitted at its own rank for 300
sweeps on the GPU, then the GPU loss of that state (FP32 terms, FP64 sums)
against the oracle's FP64 loss of the same factors at 1e-5 relative.  The
cases cover every branch of the divergence (App. B): alpha + beta = 1 with
beta > 0 and beta < 0, generic, beta = 0, alpha = -beta, and the specialised
KL, Itakura-Saito and squared-Euclidean forms."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_02759_amd import datagen

from _gpu_util import EPS, clamp_init, to_dev

pytestmark = pytest.mark.gpu

PAIRS = [(0.7, 0.3), (0.7, 0.0), (1.3, 1.0), (0.5, 0.5), (2.0, -1.0), (1.5, -1.5), (1.0, 0.0),
         (1.0, -1.0), (1.0, 1.0), (0.5, 1.0)]


@pytest.mark.parametrize("ab", PAIRS, ids=[f"{a}_{b}" for a, b in PAIRS])
def test_loss_near_fit(ab):
    import torch
    from paper_2602_02759_amd.nnef import Plan
    p = datagen.exact_problem("cp3_exact", "ir,jr,kr->ijk", dict(i=40, j=36, k=32, r=4), *ab,
                              seed=61, missing=0.2)
    plan = Plan(p.model_str, p.mode_sizes, p.ranks, *ab, eps=EPS)
    Y, M = to_dev(p.Y), to_dev(p.M)
    f = [to_dev(s) for s in clamp_init(p)]
    l0 = plan.loss(Y, M, f)
    plan.step(Y, M, f, n_sweeps=300)
    torch.cuda.synchronize()
    fs = [x.cpu().numpy().astype(np.float64) for x in f]
    got = plan.loss(Y, M, f)
    ref = O.loss(p.model_str, fs, p.Y, p.M, *ab)
    yh = O.reconstruct(p.model_str, fs)
    obs = p.M.astype(bool)
    t = np.log(p.Y[obs] / yh[obs])
    print(f"ab={ab}: loss {l0:.4e} -> {ref:.6e} (rms log-residual {np.sqrt(np.mean(t * t)):.1e}); "
          f"GPU {got:.10e} rel {(got - ref) / ref:+.2e}", flush=True)
    assert ref < 1e-3 * l0           # the fit is close: the divergence terms cancel
    assert abs(got - ref) <= 1e-5 * abs(ref)
