"""The C ABI's enqueue-only calls inside a captured graph: every replay of a
captured nnef_step / nnef_step_learned equals the same call made eagerly, bit
for bit, with unrelated eager work and synchronisations between replays."""
import numpy as np
import pytest

from paper_2602_02759_amd import datagen

from _gpu_util import EPS, clamp_init, to_dev

pytestmark = pytest.mark.gpu


def _setup():
    from paper_2602_02759_amd.nnef import Plan
    p = datagen.cp3(0.5, 1.0, sizes=dict(i=48, j=40, k=36), R=32, seed=22)
    plan = Plan(p.model_str, p.mode_sizes, p.ranks, p.alpha, p.beta, eps=EPS)
    Y, M = to_dev(p.Y), to_dev(p.M)
    init = [to_dev(s) for s in clamp_init(p)]
    return plan, Y, M, init


def _replays(run):
    import torch
    plan, Y, M, init = _setup()
    fe = [t.clone() for t in init]
    fg = [t.clone() for t in init]
    te = torch.zeros(6, dtype=torch.float64, device="cuda")
    tg = torch.zeros(6, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run(plan, Y, M, fg, tg)
    for rep in range(3):
        run(plan, Y, M, fe, te)
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(fe, fg):
            assert torch.equal(a, b), f"replay {rep}"
        assert torch.equal(te, tg), f"replay {rep}"
        x = torch.arange(1 << 16, device="cuda", dtype=torch.float32).sum()
        torch.cuda.synchronize()
        assert x.item() == float((1 << 16) * ((1 << 16) - 1) // 2)


def test_graph_replays_of_step():
    _replays(lambda plan, Y, M, f, tr: plan.step(Y, M, f, 6, loss_trace=tr))


def test_graph_replays_of_learned_step():
    from oracle import mlp as Mlp
    from paper_2602_02759_amd.nnef import Mlp as GMlp
    th = np.zeros(Mlp.N_PARAMS, dtype=np.float32)
    th[-1] = np.log(np.expm1(1.0))  # s = 1: geometric extrapolation
    mlp = GMlp(to_dev(th))
    _replays(lambda plan, Y, M, f, tr: plan.step_learned(mlp, Y, M, f, 6, 3, loss_trace=tr))
