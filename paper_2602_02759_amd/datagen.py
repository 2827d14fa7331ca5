"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers.  It holds none of the method's
arithmetic (no weights, no updates, no losses) and is the single thing the GPU
library's tests and the FP64 oracle share: both receive the same bytes.

The paper fits count tensors (Poisson, beta = 0) and positive continuous
tensors (Sec. 6, "Datasets" and "Divergences") under 90/5 % Bernoulli holdout
masks (Sec. 6, "Experimental design").  Those datasets are not available, so
synthetic tensors stand in for them: Poisson counts from heavy-tailed Gamma
factors, Gamma-noise continuous data, and Bernoulli missingness.  The true mean
tensor is formed with ``numpy.einsum`` (a library call).

Every generator uses numpy's PCG64 with a documented base seed and separate
child streams for the truth, the noise, the mask and the initial factors.
Y is float32 (counts below 2^24 are exact), the mask is uint8 (1 = observed)
and the initial factors are float32 Gamma(1, 1) draws.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

STREAM_TRUTH, STREAM_NOISE, STREAM_MASK, STREAM_INIT, STREAM_SPLIT = 0, 1, 2, 3, 4


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


@dataclass
class Problem:
    name: str
    model_str: str
    sizes: dict                      # letter -> size, observed and latent
    alpha: float
    beta: float
    Y: np.ndarray                    # float32, axes in output-letter order
    M: np.ndarray | None             # uint8 or None (fully observed)
    init: list                       # float32 factors, axes in subscript order
    truth: list = field(default_factory=list)
    n_sweeps: int = 1
    family: str = "ab"               # "ab" ((alpha, beta) divergence), "negbin", "binomial", "js"
    family_param: float = 0.0        # negative binomial phi, binomial n

    @property
    def operands(self):
        return self.model_str.split("->")[0].split(",")

    @property
    def output(self):
        return self.model_str.split("->")[1]

    @property
    def mode_sizes(self):
        return [self.sizes[ch] for ch in self.output]

    @property
    def ranks(self):
        """Latent sizes in order of first appearance on the left-hand side."""
        out = self.output
        seen = []
        for t in self.operands:
            for ch in t:
                if ch not in out and ch not in seen:
                    seen.append(ch)
        return [self.sizes[ch] for ch in seen]


def _shapes(model_str, sizes):
    ops = model_str.split("->")[0].split(",")
    return [tuple(sizes[ch] for ch in t) for t in ops]


def gamma_factors(model_str, sizes, shape, scale, g):
    return [g.gamma(shape, scale, size=s).astype(np.float64)
            for s in _shapes(model_str, sizes)]


def init_factors(model_str, sizes, seed, shape=1.0, scale=1.0):
    g = rng(seed, STREAM_INIT)
    return [g.gamma(shape, scale, size=s).astype(np.float32)
            for s in _shapes(model_str, sizes)]


def bernoulli_mask(shape, missing, seed):
    if missing <= 0:
        return None
    g = rng(seed, STREAM_MASK)
    return (g.random(size=shape) >= missing).astype(np.uint8)


def split_mask(shape, seed, heldout=0.10, validation=0.05):
    """Split of Sec. 6: each entry is heldout (3) with probability `heldout`,
    else in training; a `validation` fraction of the training entries is
    validation (2); the rest are fitted (1)."""
    u = rng(seed, STREAM_SPLIT).random(size=(2,) + tuple(shape))
    m = np.ones(shape, dtype=np.uint8)
    m[u[1] < validation] = 2
    m[u[0] < heldout] = 3
    return m


def mean_tensor(model_str, factors):
    return np.einsum(model_str, *factors, optimize=True)


def poisson_problem(name, model_str, sizes, alpha, beta, *, seed, truth_shape,
                    truth_scale=1.0, missing=0.0, n_sweeps=1):
    """Y ~ Poisson(einsum(model_str, truth)) with Gamma(shape, scale) truth."""
    gt = rng(seed, STREAM_TRUTH)
    truth = gamma_factors(model_str, sizes, truth_shape, truth_scale, gt)
    lam = mean_tensor(model_str, truth)
    Y = rng(seed, STREAM_NOISE).poisson(lam).astype(np.float32)
    M = bernoulli_mask(Y.shape, missing, seed)
    return Problem(name, model_str, dict(sizes), alpha, beta, Y, M,
                   init_factors(model_str, sizes, seed), truth, n_sweeps)


def gamma_noise_problem(name, model_str, sizes, alpha, beta, *, seed,
                        noise_shape=10.0, missing=0.0, n_sweeps=1):
    """Y = einsum(model_str, truth) * Gamma(k, 1/k) noise, truth ~ Gamma(1, 1)."""
    gt = rng(seed, STREAM_TRUTH)
    truth = gamma_factors(model_str, sizes, 1.0, 1.0, gt)
    mu = mean_tensor(model_str, truth)
    noise = rng(seed, STREAM_NOISE).gamma(noise_shape, 1.0 / noise_shape, size=mu.shape)
    Y = (mu * noise).astype(np.float32)
    Y = np.maximum(Y, np.float32(np.finfo(np.float32).tiny))  # y > 0 for Itakura-Saito
    M = bernoulli_mask(Y.shape, missing, seed)
    return Problem(name, model_str, dict(sizes), alpha, beta, Y, M,
                   init_factors(model_str, sizes, seed), truth, n_sweeps)


def exact_problem(name, model_str, sizes, alpha, beta, *, seed, truth_shape=1.0,
                  missing=0.0, n_sweeps=1):
    """Y = einsum(model_str, truth) exactly (no noise), truth ~ Gamma(shape, 1):
    data of exact rank, so a fit of that rank drives the residuals to zero."""
    truth = gamma_factors(model_str, sizes, truth_shape, 1.0, rng(seed, STREAM_TRUTH))
    Y = np.ascontiguousarray(mean_tensor(model_str, truth), dtype=np.float32)
    M = bernoulli_mask(Y.shape, missing, seed)
    return Problem(name, model_str, dict(sizes), alpha, beta, Y, M,
                   init_factors(model_str, sizes, seed), truth, n_sweeps)


def negbin_problem(name, model_str, sizes, phi, *, seed, truth_shape, missing=0.0):
    """Y ~ NegBinom(mean einsum(model_str, truth), dispersion phi)."""
    truth = gamma_factors(model_str, sizes, truth_shape, 1.0, rng(seed, STREAM_TRUTH))
    lam = mean_tensor(model_str, truth)
    Y = rng(seed, STREAM_NOISE).negative_binomial(phi, phi / (phi + lam)).astype(np.float32)
    M = bernoulli_mask(Y.shape, missing, seed)
    return Problem(name, model_str, dict(sizes), 1.0, 0.0, Y, M, init_factors(model_str, sizes, seed),
                   truth, 1, "negbin", float(phi))


def binomial_problem(name, model_str, sizes, n, *, seed, truth_shape, truth_scale=1.0, missing=0.0):
    """Y ~ Binomial(n, p) with odds p / (1 - p) = einsum(model_str, truth)."""
    truth = gamma_factors(model_str, sizes, truth_shape, truth_scale, rng(seed, STREAM_TRUTH))
    odds = mean_tensor(model_str, truth)
    Y = rng(seed, STREAM_NOISE).binomial(int(n), odds / (1.0 + odds)).astype(np.float32)
    M = bernoulli_mask(Y.shape, missing, seed)
    return Problem(name, model_str, dict(sizes), 1.0, 0.0, Y, M, init_factors(model_str, sizes, seed),
                   truth, 1, "binomial", float(n))


def js_problem(name, model_str, sizes, *, seed, truth_shape, missing=0.0):
    """Poisson counts fitted under the Jensen-Shannon divergence."""
    p = poisson_problem(name, model_str, sizes, 1.0, 0.0, seed=seed, truth_shape=truth_shape,
                        missing=missing)
    p.family = "js"
    return p


# --------------------------------------------------------------------------
# The five workloads.  (alpha, beta) follow the paper's convention (App. B):
# KL = (1, 0), squared Euclidean = (1, 1), Itakura-Saito = (1, -1).
# ``scale`` shrinks every observed mode for oracle-speed parity cases.
# --------------------------------------------------------------------------
def _scaled(n, scale):
    return max(2, int(round(n * scale)))


def nmf_kl(seed=1, I=200, J=150, R=8):
    """NMF 'ir,jr->ij', KL, Y ~ Poisson(W H^T), W, H ~ Gamma(0.5, 1), no mask."""
    return poisson_problem("nmf_kl", "ir,jr->ij", {"i": I, "j": J, "r": R},
                           1.0, 0.0, seed=seed, truth_shape=0.5, n_sweeps=100)


def cp3(alpha=1.0, beta=1.0, seed=2, n=256, R=32, missing=0.2, sizes=None):
    """CP 'ir,jr,kr->ijk', Y ~ Poisson of Gamma(0.3, 1) CP factors, 20 % missing."""
    sz = sizes or {"i": n, "j": n, "k": n}
    sz = dict(sz, r=R)
    return poisson_problem(f"cp3_{n}_a{alpha}_b{beta}", "ir,jr,kr->ijk", sz,
                           alpha, beta, seed=seed, truth_shape=0.3,
                           missing=missing, n_sweeps=200)


def tucker3(seed=3, I=512, J=512, K=128, Ra=32, Rb=32, Rc=16, missing=0.1,
            alpha=1.0, beta=-1.0):
    """Tucker 'ia,jb,kc,abc->ijk' x Gamma(10, 1/10) noise, IS loss, 10 % missing."""
    sz = {"i": I, "j": J, "k": K, "a": Ra, "b": Rb, "c": Rc}
    return gamma_noise_problem("tucker3", "ia,jb,kc,abc->ijk", sz, alpha, beta,
                               seed=seed, missing=missing, n_sweeps=100)


def tt4(seed=5, I=128, J=128, K=96, Lm=64, Ra=16, Rb=16, Rc=16, missing=0.15):
    """Tensor train 'ia,jab,kbc,lc->ijkl', Poisson counts, 15 % missing, KL.

    Cores ~ Gamma(0.5, 1) * 1/4 so that the mean count is about one.
    """
    sz = {"i": I, "j": J, "k": K, "l": Lm, "a": Ra, "b": Rb, "c": Rc}
    return poisson_problem("tt4", "ia,jab,kbc,lc->ijkl", sz, 1.0, 0.0, seed=seed,
                           truth_shape=0.5, truth_scale=0.25, missing=missing,
                           n_sweeps=200)


def cp4_batch_descriptors(n_problems=96, seed=4, lo=32, hi=160,
                          ranks=(4, 8, 16, 32, 64)):
    """Mode sizes iid uniform integers in [lo, hi] and a rank drawn from ``ranks``."""
    g = rng(seed, STREAM_TRUTH)
    out = []
    for _ in range(n_problems):
        dims = [int(v) for v in g.integers(lo, hi + 1, size=4)]
        R = int(g.choice(ranks))
        out.append((dims, R))
    return out


def cp4_problem(dims, R, seed, n_restarts=8):
    """One problem of the batched set: 'ir,jr,kr,lr->ijkl', KL, no mask.

    Factors ~ Gamma(0.5, 1), Y ~ Poisson; ``n_restarts`` Gamma(1, 1) inits.
    """
    sz = {"i": dims[0], "j": dims[1], "k": dims[2], "l": dims[3], "r": R}
    p = poisson_problem(f"cp4_{'x'.join(map(str, dims))}_r{R}", "ir,jr,kr,lr->ijkl",
                        sz, 1.0, 0.0, seed=seed, truth_shape=0.5, n_sweeps=100)
    p.init = [init_factors(p.model_str, sz, seed * 1000 + 17 + r) for r in range(n_restarts)]
    return p


def random_factors(model_str, sizes, seed, shape=1.0):
    return init_factors(model_str, sizes, seed, shape=shape)


# --------------------------------------------------------------------------
# The paper's custom model strings at its data shapes (Sec. 6: Uber pickups
# w x d x h x i x j with a spatial mesh, ICEWS country x country x action x
# time), with synthetic counts standing in for the unavailable datasets.
# Ranks the paper leaves unstated are this generator's choice.
# --------------------------------------------------------------------------
def uber_problem(mesh=100, R=10, K=6, seed=11, missing=0.1):
    """'wr,dr,hr,irk,jrk->wdhij': 27 weeks x 7 days x 24 hours x mesh x mesh."""
    sz = {"w": 27, "d": 7, "h": 24, "i": mesh, "j": mesh, "r": R, "k": K}
    return poisson_problem(f"uber{mesh}", "wr,dr,hr,irk,jrk->wdhij", sz, 1.0, 0.0, seed=seed,
                           truth_shape=0.3, missing=missing, n_sweeps=100)


def icews_problem(R=32, K=8, seed=12, missing=0.1):
    """'ir,jr,ak,kr,tr->ijat': 249 x 249 countries x 20 action types x 228 months."""
    sz = {"i": 249, "j": 249, "a": 20, "t": 228, "r": R, "k": K}
    return poisson_problem("icews", "ir,jr,ak,kr,tr->ijat", sz, 1.0, 0.0, seed=seed,
                           truth_shape=0.3, missing=missing, n_sweeps=100)
