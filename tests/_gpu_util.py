"""Helpers for the GPU parity tests (imported only by tests marked gpu)."""
import numpy as np

from oracle import oracle as O

EPS = 1e-10


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def gpu_sweeps(plan, p, state, n, Y=None, M=None, trace=False):
    """Run n sweeps on the GPU from float32 ``state``; return float32 factors."""
    import torch
    Yd = to_dev(p.Y) if Y is None else Y
    if isinstance(M, str) and M == "none":
        Md = None
    else:
        Md = (to_dev(p.M) if p.M is not None else None) if M is None else M
    f = [to_dev(s.astype(np.float32)) for s in state]
    tr = torch.zeros(max(n, 1), dtype=torch.float64, device=dev()) if trace else None
    plan.step(Yd, Md, f, n_sweeps=n, loss_trace=tr)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in f]
    return (out, tr.cpu().numpy()) if trace else out


def assert_step_parity(gpu, ref, tol, what=""):
    """Per factor: relative Frobenius error <= tol and an elementwise bound
    |g - r| <= tol * (|r| + 1e-3 max|r|) (a floor for entries near eps)."""
    worst = 0.0
    for i, (g, r) in enumerate(zip(gpu, ref)):
        g = g.astype(np.float64)
        rel = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)
        worst = max(worst, rel)
        assert rel <= tol, f"{what} factor {i}: rel Frobenius {rel:.3e} > {tol:.1e}"
        bound = tol * (np.abs(r) + 1e-3 * np.max(np.abs(r)))
        bad = np.abs(g - r) > bound
        assert not bad.any(), (f"{what} factor {i}: {bad.sum()} elements outside the bound; "
                               f"max excess {np.max(np.abs(g - r) / bound):.2f}x")
    return worst


def oracle_sweep(p, state):
    return O.sweep(p.model_str, [s.astype(np.float64) for s in state], p.Y, p.M, p.alpha, p.beta, EPS)


def clamp_init(p):
    return [np.maximum(t, np.float32(EPS)).astype(np.float32) for t in p.init]
