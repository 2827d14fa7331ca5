"""Batched plans (many problems x restarts, persistent launches, graph replay)
vs the FP64 oracle, through the C ABI.

Every run of a batch must match the oracle's sweep from the same state at the
FP32 tolerance (1e-5), whatever its shape, rank class or restart; repeated graph
replays with eager work and synchronisations in between must keep matching.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_02759_amd import datagen

from _gpu_util import EPS, assert_step_parity, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _problems():
    """Mixed widths (16, 32, 64 classes), ragged sizes, KL without a mask and
    squared Euclidean with a mask, 1-3 restarts."""
    specs = [((13, 9, 11, 7), 4, 1.0, 0.0, 0.0, 3),
             ((20, 17, 9, 12), 32, 1.0, 0.0, 0.0, 2),
             ((16, 16, 8, 32), 32, 1.0, 0.0, 0.0, 2),
             ((11, 14, 10, 9), 64, 1.0, 0.0, 0.0, 1),
             ((15, 12, 13, 8), 16, 1.0, 1.0, 0.2, 2)]
    probs = []
    for i, (dims, R, a, b, miss, nr) in enumerate(specs):
        sz = {"i": dims[0], "j": dims[1], "k": dims[2], "l": dims[3], "r": R}
        p = datagen.poisson_problem(f"b{i}", "ir,jr,kr,lr->ijkl", sz, a, b, seed=80 + i,
                                    truth_shape=0.5, missing=miss)
        p.init = [datagen.init_factors(p.model_str, sz, 900 + 10 * i + r) for r in range(nr)]
        probs.append(p)
    return probs


def _batch(probs):
    from paper_2602_02759_amd.nnef import Batch
    desc = [dict(model_str=p.model_str, mode_sizes=p.mode_sizes, ranks=p.ranks, alpha=p.alpha,
                 beta=p.beta, n_restarts=len(p.init), masked=p.M is not None) for p in probs]
    return Batch(desc, eps=EPS)


def _device(probs):
    Ys = [to_dev(p.Y) for p in probs]
    Ms = [to_dev(p.M) if p.M is not None else None for p in probs]
    runs = [(p, [to_dev(np.maximum(f, EPS).astype(np.float32)) for f in init]) for p in probs
            for init in p.init]
    return Ys, Ms, runs


def _check_runs(runs, before, what):
    for r, ((p, f), s0) in enumerate(zip(runs, before)):
        got = [t.cpu().numpy() for t in f]
        ref = O.sweep(p.model_str, [x.astype(np.float64) for x in s0], p.Y, p.M, p.alpha, p.beta, EPS)
        assert_step_parity(got, ref, TOL, f"{what} run {r} ({p.name})")


def test_batched_sweep_matches_oracle_every_run():
    import torch
    probs = _problems()
    b = _batch(probs)
    print(b.describe(), flush=True)
    Ys, Ms, runs = _device(probs)
    facs = [f for _, f in runs]
    for call in range(3):  # first call captures the graph; later calls replay it
        before = [[t.cpu().numpy() for t in f] for f in facs]
        b.step(Ys, Ms, facs, 1)
        torch.cuda.synchronize()
        _check_runs(runs, before, f"call {call}")
        # eager work on the same stream between replays
        plain = torch.ones(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert plain.item() == float(1 << 20)


def test_batched_loss_trace():
    import torch
    probs = _problems()
    b = _batch(probs)
    Ys, Ms, runs = _device(probs)
    facs = [f for _, f in runs]
    before = [[t.cpu().numpy().astype(np.float64) for t in f] for f in facs]
    tr = torch.zeros((2, b.n_runs), dtype=torch.float64, device="cuda")
    b.step(Ys, Ms, facs, 2, loss_trace=tr)
    torch.cuda.synchronize()
    for r, (p, _) in enumerate(runs):
        ref = O.loss(p.model_str, before[r], p.Y, p.M, p.alpha, p.beta)
        assert abs(tr[0, r].item() - ref) <= 1e-5 * ref, (r, tr[0, r].item(), ref)
    assert torch.all(tr[1] <= tr[0] * (1 + 1e-6))


def test_autotune_keeps_parity():
    import torch
    probs = _problems()
    b = _batch(probs)
    Ys, Ms, runs = _device(probs)
    facs = [f for _, f in runs]
    before = [[t.cpu().numpy() for t in f] for f in facs]
    b.autotune(Ys, Ms, facs)
    after = [[t.cpu().numpy() for t in f] for f in facs]
    for x, y in zip(before, after):  # the autotuner does not touch the factors
        for u, v in zip(x, y):
            np.testing.assert_array_equal(u, v)
    print(b.describe(), flush=True)
    b.step(Ys, Ms, facs, 1)
    torch.cuda.synchronize()
    _check_runs(runs, before, "autotuned")


def test_quarter_scale_batched_workload():
    """The 96-descriptor batched CP workload at a quarter of its mode sizes
    (uniform in [8, 40]), 2 restarts each: one sweep of every run vs the
    oracle."""
    import torch
    desc = datagen.cp4_batch_descriptors(lo=8, hi=40)
    probs = [datagen.cp4_problem(d, R, seed=1000 + i, n_restarts=2) for i, (d, R) in enumerate(desc)]
    b = _batch(probs)
    Ys, Ms, runs = _device(probs)
    facs = [f for _, f in runs]
    before = [[t.cpu().numpy() for t in f] for f in facs]
    b.step(Ys, Ms, facs, 1)
    torch.cuda.synchronize()
    _check_runs(runs, before, "quarter-scale")


def test_full_size_batched_workload_sampled():
    """The benchmark's launch configuration: all 96 CP4 problems at full size
    (mode sizes U{32..160}) x 8 restarts in one autotuned batched plan, data
    drawn on the GPU.  After one sweep of all 768 runs, the runs of the three
    smallest problems (first and last restart) are checked against the
    oracle's sweep from the same state; every run stays finite and positive."""
    import torch
    desc = datagen.cp4_batch_descriptors()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    Ys, runs, probs = [], [], []
    for dims, R in desc:
        fs = [torch._standard_gamma(torch.full((d, R), 0.5, device="cuda"), generator=gen) for d in dims]
        lam = torch.einsum("ir,jr,kr,lr->ijkl", *fs).contiguous()
        Ys.append(torch.poisson(lam, generator=gen).contiguous())
        del lam, fs
        for _ in range(8):
            runs.append([torch._standard_gamma(torch.ones((d, R), device="cuda"), generator=gen).clamp_min(EPS)
                         for d in dims])
        probs.append(dict(model_str="ir,jr,kr,lr->ijkl", mode_sizes=dims, ranks=[R], alpha=1.0, beta=0.0,
                          n_restarts=8, masked=False))
    from paper_2602_02759_amd.nnef import Batch
    b = Batch(probs, eps=EPS)
    b.autotune(Ys, None, runs)
    print(b.describe(), flush=True)
    sizes = [int(np.prod(d)) for d, _ in desc]
    picked = sorted(range(len(desc)), key=lambda i: sizes[i])[:3]
    sample = [(i, r) for i in picked for r in (0, 7)]
    before = {(i, r): [t.cpu().numpy() for t in runs[8 * i + r]] for i, r in sample}
    b.step(Ys, None, runs, 1)
    torch.cuda.synchronize()
    for f in runs:
        for t in f:
            assert bool(torch.isfinite(t).all()) and bool((t >= EPS).all())
    for i, r in sample:
        Y = Ys[i].cpu().numpy().astype(np.float64)
        ref = O.sweep("ir,jr,kr,lr->ijkl", [x.astype(np.float64) for x in before[(i, r)]], Y, None, 1.0, 0.0, EPS)
        got = [t.cpu().numpy() for t in runs[8 * i + r]]
        assert_step_parity(got, ref, TOL, f"problem {i} {desc[i]} restart {r}")


def _side_problems():
    """Strings whose blocks need side operands and chain-backs: Tucker (eq. 2.4,
    masked IS), tensor train (eq. 2.6, masked KL), the ICEWS string (a grouped
    column piece [a, r]) and NMF (a transposed operand), batched with a CP
    problem; 1-3 restarts each."""
    probs = [datagen.tucker3(I=30, J=26, K=18, Ra=6, Rb=5, Rc=4, seed=331),
             datagen.tt4(I=13, J=11, K=9, Lm=7, Ra=3, Rb=4, Rc=5, seed=341),
             datagen.poisson_problem("icews_b", "ir,jr,ak,kr,tr->ijat", dict(i=40, j=40, a=16, t=8, r=32, k=4),
                                     1.0, 0.0, seed=351, truth_shape=0.5, missing=0.1),
             datagen.poisson_problem("nmf_b", "ir,rj->ij", dict(i=50, j=37, r=8), 1.0, 0.0, seed=361,
                                     truth_shape=0.5),
             datagen.poisson_problem("cp_b", "ir,jr,kr->ijk", dict(i=21, j=19, k=17, r=12), 0.5, 1.0, seed=371,
                                     truth_shape=0.5, missing=0.2)]
    restarts = [3, 2, 1, 2, 1]
    for i, (p, nr) in enumerate(zip(probs, restarts)):
        p.init = [datagen.init_factors(p.model_str, p.sizes, 950 + 10 * i + r) for r in range(nr)]
    return probs


def test_batched_side_operands_match_oracle():
    """Every run of a batch with side operands (per-run workspaces, chain-backs
    in the captured sequence) matches the oracle's sweep at 1e-5, over three
    calls (capture, then replays with eager work in between), and its loss
    trace matches the oracle's loss of the state it belongs to."""
    import torch
    probs = _side_problems()
    b = _batch(probs)
    d = b.describe()
    print(d, flush=True)
    assert "chain-back" in d
    Ys, Ms, runs = _device(probs)
    facs = [f for _, f in runs]
    for call in range(3):
        before = [[t.cpu().numpy() for t in f] for f in facs]
        tr = torch.zeros((1, b.n_runs), dtype=torch.float64, device="cuda")
        b.step(Ys, Ms, facs, 1, loss_trace=tr if call == 2 else None)
        torch.cuda.synchronize()
        _check_runs(runs, before, f"side-operand call {call}")
        if call == 2:
            for r, (p, _) in enumerate(runs):
                ref = O.loss(p.model_str, [x.astype(np.float64) for x in before[r]], p.Y, p.M, p.alpha, p.beta)
                assert abs(tr[0, r].item() - ref) <= 1e-5 * ref, (r, tr[0, r].item(), ref)
        plain = torch.ones(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert plain.item() == float(1 << 20)
