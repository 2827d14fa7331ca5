"""Splits and early stopping on the GPU vs the oracle: the loss of each split,
and nnef_fit's stopping state, reason and loss traces."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_02759_amd import datagen

from _gpu_util import EPS, clamp_init, to_dev

pytestmark = pytest.mark.gpu


def _problem():
    p = datagen.cp3(1.0, 0.0, sizes=dict(i=44, j=40, k=36), R=8, seed=97, missing=0.0)
    return p, datagen.split_mask(p.Y.shape, seed=97)


def _plan(p):
    from paper_2602_02759_amd.nnef import Plan
    return Plan(p.model_str, p.mode_sizes, p.ranks, p.alpha, p.beta, eps=EPS)


@pytest.mark.parametrize("value", [1, 2, 3])
def test_split_losses(value):
    p, M = _problem()
    plan = _plan(p)
    s0 = clamp_init(p)
    got = plan.loss_split(to_dev(p.Y), to_dev(M), value, [to_dev(s) for s in s0])
    ref = O.loss(p.model_str, [s.astype(np.float64) for s in s0], p.Y, (M == value).astype(np.uint8),
                 p.alpha, p.beta)
    assert abs(got - ref) <= 1e-5 * ref, (got, ref)


def test_step_fits_mask_value_one_only():
    """nnef_step with a split mask equals nnef_step with the binary training mask."""
    import torch
    p, M = _problem()
    plan = _plan(p)
    Y = to_dev(p.Y)
    a = [to_dev(s) for s in clamp_init(p)]
    b = [t.clone() for t in a]
    plan.step(Y, to_dev(M), a, 3)
    plan.step(Y, to_dev((M == 1).astype(np.uint8)), b, 3)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("opts", [dict(rel_tol=1e-3, patience=5), dict(rel_tol=0.0, patience=2, max_sweeps=120),
                                  dict(rel_tol=1e-3, patience=5, check_every=7)])
def test_fit_matches_oracle(opts):
    import torch
    p, M = _problem()
    plan = _plan(p)
    f = [to_dev(s) for s in clamp_init(p)]
    n = opts.get("max_sweeps", 5000) + 1
    tt = torch.zeros(n, dtype=torch.float64, device="cuda")
    tv = torch.zeros(n, dtype=torch.float64, device="cuda")
    res = plan.fit(to_dev(p.Y), to_dev(M), f, tt, tv, **opts)
    o = {k: v for k, v in opts.items() if k != "check_every"}
    rf, rt, rr, L, V = O.fit_early_stopping(p.model_str, [s.astype(np.float64) for s in clamp_init(p)],
                                            p.Y, M, p.alpha, p.beta, EPS, **o)
    print(f"{opts}: GPU stop {res['stop_sweep']} ({res['reason']}, {res['sweeps_run']} run); "
          f"oracle stop {rt} (reason {rr})")
    assert {"max_sweeps": O.STOP_MAX, "train_tol": O.STOP_TRAIN_TOL,
            "validation": O.STOP_VALIDATION}[res["reason"]] == rr
    assert abs(res["stop_sweep"] - rt) <= 2
    m = min(res["stop_sweep"], rt) + 1
    np.testing.assert_allclose(tt.cpu().numpy()[:m], L[:m], rtol=1e-5)
    np.testing.assert_allclose(tv.cpu().numpy()[:m], V[:m], rtol=1e-5)
    assert res["sweeps_run"] >= res["stop_sweep"]
    if opts.get("check_every", 1) == 1:
        assert res["sweeps_run"] == res["stop_sweep"]
        # the returned factors are the stopping state itself
        fs = [x.cpu().numpy().astype(np.float64) for x in f]
        lt = O.loss(p.model_str, fs, p.Y, (M == 1).astype(np.uint8), p.alpha, p.beta)
        assert abs(lt - res["train_loss"]) <= 1e-5 * lt


def test_fit_losses_equal_the_split_loss_passes():
    """The training and validation losses nnef_fit takes from the fused pass
    of the following sweep (one pack holding both splits) equal the separate
    loss passes over each split of the same state."""
    import torch
    p, M = _problem()
    plan = _plan(p)
    Y, Md = to_dev(p.Y), to_dev(M)
    f = [to_dev(s) for s in clamp_init(p)]
    tt = torch.zeros(6, dtype=torch.float64, device="cuda")
    tv = torch.zeros(6, dtype=torch.float64, device="cuda")
    res = plan.fit(Y, Md, f, tt, tv, max_sweeps=5, rel_tol=0.0, patience=0)
    assert res["stop_sweep"] == 5 and res["reason"] == "max_sweeps" and res["sweeps_run"] == 5
    for value, tr in ((1, tt), (2, tv)):
        sep = plan.loss_split(Y, Md, value, f)
        assert abs(tr[5].item() - sep) <= 1e-6 * sep, (value, tr[5].item(), sep)
