"""FP64 CPU oracle for NNEinFact multiplicative updates.

TEST INFRASTRUCTURE ONLY. This module exists to check the GPU library against
the paper. Only the test-suite, the smoke check in ``__graft_entry__`` and the
CPU-baseline leg of ``bench.py`` may import or call it; the library itself never
does, and shares no code, tables or helpers with it.

Everything here is plain numpy in float64, written from the paper:

* the model string and the einsum reconstruction (Sec. 2, eqs. 2.1-2.3);
* ``swap`` and the numerator/denominator einsums ``einstr_l`` (Sec. 3, eqs.
  3.5-3.6 and the definition of ``einstr_l`` that follows them);
* the (alpha, beta)-divergence, its weight functions a, b and the map g
  (App. B, "Divergences");
* one block update and one sweep of Algorithm 1 (Sec. 3), with the missing-data
  rule of Sec. 6 ("Experimental design").

Library primitive used as a step: ``numpy.einsum`` (contractions; the paper's
own computational primitive).  ``brute_einsum`` is an independent nested-loop
evaluator used only to pin ``numpy.einsum``'s use on tiny inputs.

Readings where the paper is silent or ambiguous (all shared with the GPU path
through the specification, not through code):

* Mask: the weights are multiplied by the mask, A_i = M_i a(y_i, yhat_i) and
  B_i = M_i b(y_i, yhat_i); masked-out data values never enter arithmetic.
  This is Theorem 3.1 applied to the objective restricted to observed entries.
* Zero data with alpha > 0: x^alpha = 0 and x^alpha log x = 0.
* A denominator entry D_u = 0 (every entry that depends on theta_u is missing)
  leaves theta_u unchanged.
* The initial factors are clamped to >= eps before the first sweep.
* One sweep is the loop over l = 1..L of Algorithm 1 in operand order, with the
  reconstruction recomputed before every block.

Parity pins: every function here is checked in ``tests/test_oracle_*.py``
against brute force, closed-form NMF updates, the loss derivative identity,
monotonicity (Theorem 3.1), fixed points and stationarity (Theorem 4.3).
"""
from __future__ import annotations

import itertools
import string
from dataclasses import dataclass

import numpy as np

_LETTERS = set(string.ascii_letters)


# --------------------------------------------------------------------------
# Model strings (Sec. 2, eqs. 2.2-2.3) and swap (Sec. 3)
# --------------------------------------------------------------------------
@dataclass
class Model:
    operands: list  # subscripts of each parameter tensor, in string order
    output: str     # observed modes, in the order of Y's axes
    latent: list    # contracted letters, in order of first appearance

    @property
    def L(self) -> int:
        return len(self.operands)


def parse_model(model_str: str) -> Model:
    """Parse ``i_1 r_1, ..., i_L r_L -> i_1 ... i_M`` (eq. 2.2).

    Letters on the right are observed modes; letters only on the left are
    contracted (summed).  Raises ValueError for strings that are not of this
    family: a missing arrow, a non-letter, a letter repeated inside one operand
    or inside the output, or an output letter used by no operand.
    """
    s = model_str.replace(" ", "")
    if s.count("->") != 1:
        raise ValueError("model string needs exactly one '->'")
    lhs, out = s.split("->")
    ops = lhs.split(",")
    for t in ops + [out]:
        for ch in t:
            if ch not in _LETTERS:
                raise ValueError(f"bad subscript {ch!r}")
        if len(set(t)) != len(t):
            raise ValueError(f"repeated letter in {t!r}")
    if any(len(t) == 0 for t in ops):
        raise ValueError("empty operand")
    used = set("".join(ops))
    for ch in out:
        if ch not in used:
            raise ValueError(f"output letter {ch!r} appears in no operand")
    latent = []
    for t in ops:
        for ch in t:
            if ch not in out and ch not in latent:
                latent.append(ch)
    return Model(ops, out, latent)


def swap(model_str: str, ell: int) -> str:
    """einstr_l: exchange the model output with the l-th operand (Sec. 3).

    ``ell`` is 0-based here.  The l-th operand slot receives the data-shaped
    tensor a(Y, Yhat) (or b), and the result has operand l's subscripts.
    """
    m = parse_model(model_str)
    ops = list(m.operands)
    ops[ell] = m.output
    return ",".join(ops) + "->" + m.operands[ell]


def factor_shapes(model_str: str, sizes: dict) -> list:
    """Shape of every parameter tensor: one axis per subscript letter."""
    m = parse_model(model_str)
    return [tuple(sizes[ch] for ch in t) for t in m.operands]


# --------------------------------------------------------------------------
# Contractions
# --------------------------------------------------------------------------
def einsum(expr: str, *operands):
    """FP64 einsum through the library primitive."""
    return np.einsum(expr, *[np.asarray(o, dtype=np.float64) for o in operands],
                     optimize=True)


def einsum_to(expr: str, out_shape, *operands):
    """einsum whose output may hold letters that no input holds.

    A latent letter that appears in one operand only is summed inside it
    (Sec. 2); in the numerator einsum of that operand (eq. 3.6) the letter is
    then an output letter of no input, and the contraction is the same for
    every value of it.  ``out_shape`` gives its size.
    """
    lhs, out = expr.replace(" ", "").split("->")
    present = set(lhs.replace(",", ""))
    kept = "".join(c for c in out if c in present)
    r = einsum(lhs + "->" + kept, *operands)
    idx = tuple(slice(None) if c in present else None for c in out)
    return np.array(np.broadcast_to(r[idx], tuple(out_shape)))


def brute_einsum(expr: str, *operands, sizes=None):
    """Nested loops over every letter combination (definition of einsum).

    Used only on tiny inputs to pin ``einsum``.  ``sizes`` gives the size of
    output letters that no operand holds.
    """
    lhs, out = expr.replace(" ", "").split("->")
    ops = lhs.split(",")
    size = dict(sizes or {})
    for t, o in zip(ops, operands):
        for ch, n in zip(t, np.shape(o)):
            size[ch] = n
    letters = sorted(size)
    res = np.zeros(tuple(size[ch] for ch in out), dtype=np.float64)
    for combo in itertools.product(*[range(size[ch]) for ch in letters]):
        idx = dict(zip(letters, combo))
        prod = 1.0
        for t, o in zip(ops, operands):
            prod *= float(o[tuple(idx[ch] for ch in t)])
        res[tuple(idx[ch] for ch in out)] += prod
    return res


def reconstruct(model_str: str, factors) -> np.ndarray:
    """Yhat = einsum(model_str, Theta^(1..L))  (eq. 2.3)."""
    return einsum(model_str.replace(" ", ""), *factors)


# --------------------------------------------------------------------------
# (alpha, beta)-divergence (App. B, "Divergences")
# --------------------------------------------------------------------------
def _pow(x, p):
    """x**p with 0**p = 0 for p > 0 (zero data, alpha > 0)."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        return np.power(x, p)


def _xlogx_ratio(coef, x, y):
    """coef * log(x / y), taken as 0 where coef == 0 (0 log 0 = 0)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        v = coef * np.log(x / y)
    return np.where(coef == 0, 0.0, v)


# --------------------------------------------------------------------------
# Other decomposable likelihoods (App. B, after the (alpha, beta) family):
# negative binomial with dispersion phi, binomial odds with n trials (n = 1:
# Bernoulli), and Jensen-Shannon.  Passed in place of (alpha, beta) as
# ``alpha=<Family>``; every function below dispatches on it.
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Family:
    kind: str           # "negbin" | "binomial" | "js"
    param: float = 0.0  # phi (negbin) or n (binomial)


def negbin(phi: float) -> Family:
    return Family("negbin", float(phi))


def binomial(n: float = 1.0) -> Family:
    return Family("binomial", float(n))


def jensen_shannon() -> Family:
    return Family("js")


def _xlogx(x):
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(x > 0, x * np.log(np.where(x > 0, x, 1.0)), 0.0)


def family_loss(x, y, fam: Family):
    """The negative log-likelihood terms (or divergence) the paper gives for
    each family, x the data and y the model (the odds for the binomial)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        if fam.kind == "negbin":    # (phi + x) log(phi + y) - x log y
            return (fam.param + x) * np.log(fam.param + y) - np.where(x > 0, x * np.log(y), 0.0)
        if fam.kind == "binomial":  # n log(1 + y) - x log y
            return fam.param * np.log1p(y) - np.where(x > 0, x * np.log(y), 0.0)
        if fam.kind == "js":        # (x log x + y log y)/2 - ((x+y)/2) log((x+y)/2)
            return 0.5 * (_xlogx(x) + _xlogx(y)) - _xlogx(0.5 * (x + y))
    raise ValueError(fam.kind)


def family_weights(x, y, fam: Family):
    """(a, b) of each family's convex-concave split."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if fam.kind == "negbin":
        return x / y, (fam.param + x) / (fam.param + y)
    if fam.kind == "binomial":
        return x / y, fam.param / (1.0 + y)
    if fam.kind == "js":
        return np.log((x + y) / (2.0 * y)), np.ones_like(y)
    raise ValueError(fam.kind)


def ab_loss(x, y, alpha: float, beta: float):
    """Elementwise D_{alpha,beta}(x, y): x is the data, y the model (App. B).

    The five cases of the definition, in its order.
    """
    if isinstance(alpha, Family):
        return family_loss(x, y, alpha)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    a, b = float(alpha), float(beta)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        if a != 0 and b != 0 and a + b != 0:
            return (1.0 / (a * b)) * (a / (a + b) * _pow(x, a + b)
                                      + b / (a + b) * _pow(y, a + b)
                                      - _pow(x, a) * _pow(y, b))
        if b == 0 and a != 0:
            xa = _pow(x, a)
            return (1.0 / a ** 2) * (_pow(y, a) - xa + a * _xlogx_ratio(xa, x, y))
        if a == -b and a != 0:
            return (1.0 / a ** 2) * (_pow(x, a) / _pow(y, a) - 1.0
                                     + a * np.log(y / x))
        if a == 0 and b != 0:
            yb = _pow(y, b)
            return (1.0 / b ** 2) * (b * _xlogx_ratio(yb, y, x) - yb + _pow(x, b))
        return 0.5 * (np.log(x) - np.log(y)) ** 2


def ab_weights(x, y, alpha: float, beta: float):
    """(a(x, y), b(x, y)) of the decomposability property (App. B).

    alpha != 0: a = x^alpha y^(beta-1), b = y^(alpha+beta-1).
    alpha == 0, beta == 1: a = log(x / y), b = 1.
    alpha == 0, beta != 1: no decomposition is known -> ValueError.
    """
    if isinstance(alpha, Family):
        return family_weights(x, y, alpha)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if alpha != 0:
        return _pow(x, alpha) * _pow(y, beta - 1.0), _pow(y, alpha + beta - 1.0)
    if beta == 1:
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.log(x / y), np.ones_like(y)
    raise ValueError("alpha = 0 with beta != 1 has no multiplicative update")


def update_rule(alpha: float, beta: float):
    """g^{-1} as ('pow', gamma) meaning r**gamma, or ('exp', None) meaning exp(r).

    From the four cases of g(lambda) in App. B with rho = (1 - beta)/alpha:
    rho > 1: g = lambda^(1-beta); rho < 0: g = lambda^(alpha+beta-1);
    0 <= rho <= 1: g = lambda^alpha; alpha = 0, beta = 1: g = log.
    Other families: g = lambda (negative binomial, binomial), g = log (JS).
    """
    if isinstance(alpha, Family):
        return ("exp", None) if alpha.kind == "js" else ("pow", 1.0)
    if alpha == 0:
        if beta == 1:
            return ("exp", None)
        raise ValueError("alpha = 0 with beta != 1 has no multiplicative update")
    rho = (1.0 - beta) / alpha
    if rho > 1:
        return ("pow", 1.0 / (1.0 - beta))
    if rho < 0:
        return ("pow", 1.0 / (alpha + beta - 1.0))
    return ("pow", 1.0 / alpha)


def masked_loss(Y, Yhat, M, alpha, beta) -> float:
    """Sum of D_{alpha,beta}(y_i, yhat_i) over observed entries (eq. 3.1)."""
    if M is None:
        return float(np.sum(ab_loss(Y, Yhat, alpha, beta)))
    m = np.asarray(M).astype(bool)
    return float(np.sum(ab_loss(np.asarray(Y, np.float64)[m], Yhat[m], alpha, beta)))


def loss(model_str, factors, Y, M, alpha, beta) -> float:
    return masked_loss(Y, reconstruct(model_str, factors), M, alpha, beta)


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
def masked_weights(Y, Yhat, M, alpha, beta):
    """A = M * a(Y, Yhat), B = M * b(Y, Yhat) (Alg. 1 with the Sec. 6 mask).

    Missing entries contribute exactly zero, whatever their stored value.
    """
    Y = np.asarray(Y, dtype=np.float64)
    if M is None:
        return ab_weights(Y, Yhat, alpha, beta)
    m = np.asarray(M).astype(bool)
    Ys = np.where(m, Y, 1.0)          # never feed a missing value into arithmetic
    a, b = ab_weights(Ys, np.where(m, Yhat, 1.0), alpha, beta)
    return np.where(m, a, 0.0), np.where(m, b, 0.0)


def numerator_denominator(model_str, factors, ell, Y, M, alpha, beta):
    """(N_l, D_l) = einsum(einstr_l, ..., a(Y,Yhat) | b(Y,Yhat), ...) (Alg. 1)."""
    Yhat = reconstruct(model_str, factors)
    A, B = masked_weights(Y, Yhat, M, alpha, beta)
    es = swap(model_str, ell)
    opsA = list(factors)
    opsA[ell] = A
    opsB = list(factors)
    opsB[ell] = B
    shape = np.shape(factors[ell])
    return einsum_to(es, shape, *opsA), einsum_to(es, shape, *opsB)


def apply_update(theta, N, D, alpha, beta, eps):
    """Theta <- max(eps, Theta * g^{-1}(N / D)) (eq. 3.4); D == 0 keeps theta."""
    theta = np.asarray(theta, dtype=np.float64)
    kind, gamma = update_rule(alpha, beta)
    pos = D > 0
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        r = np.where(pos, N / np.where(pos, D, 1.0), 1.0)
        if kind == "exp":
            step = np.exp(r)
        else:
            step = np.power(r, gamma)
        new = np.maximum(eps, theta * step)
    return np.where(pos, new, theta)


def block_update(model_str, factors, ell, Y, M, alpha, beta, eps):
    """One block of Algorithm 1: rebuild Yhat, then update Theta^(ell)."""
    N, D = numerator_denominator(model_str, factors, ell, Y, M, alpha, beta)
    out = list(factors)
    out[ell] = apply_update(factors[ell], N, D, alpha, beta, eps)
    return out


def sweep(model_str, factors, Y, M, alpha, beta, eps, block_losses=None):
    """One pass of the inner loop of Algorithm 1 over l = 1..L (Gauss-Seidel)."""
    f = [np.asarray(t, dtype=np.float64) for t in factors]
    for ell in range(len(f)):
        f = block_update(model_str, f, ell, Y, M, alpha, beta, eps)
        if block_losses is not None:
            block_losses.append(loss(model_str, f, Y, M, alpha, beta))
    return f


def _slab_bounds(n, n_slabs):
    return [(int(a), int(b)) for a, b in zip(np.linspace(0, n, n_slabs + 1)[:-1],
                                              np.linspace(0, n, n_slabs + 1)[1:]) if b > a]


def _slab_factors(model_str, factors, a, b):
    """The factors restricted to entries whose first observed index lies in [a, b)."""
    m = parse_model(model_str)
    c = m.output[0]
    out = []
    for t, f in zip(m.operands, factors):
        if c in t:
            idx = [slice(None)] * len(t)
            idx[t.index(c)] = slice(a, b)
            f = f[tuple(idx)]
        out.append(f)
    return out


def loss_slabs(model_str, factors, Y, M, alpha, beta, n_slabs) -> float:
    """``loss`` summed slab by slab along the first observed mode (eq. 3.1 is a
    sum over entries), for tensors too large to reconstruct at once."""
    tot = 0.0
    for a, b in _slab_bounds(np.shape(Y)[0], n_slabs):
        fs = _slab_factors(model_str, factors, a, b)
        tot += loss(model_str, fs, Y[a:b], None if M is None else M[a:b], alpha, beta)
    return tot


def sweep_slabs(model_str, factors, Y, M, alpha, beta, eps, n_slabs):
    """``sweep`` with the reconstruction and the numerator and denominator
    einsums of every block evaluated slab by slab along the first observed mode
    (the sums over entries in eqs. 2.1 and 3.6 are additive; an operand that
    holds that mode receives each slab's rows, the others the sum over slabs).
    The same update up to summation order, for tensors too large to hold the
    reconstruction and its weights at once."""
    m = parse_model(model_str)
    c = m.output[0]
    f = [np.asarray(t, dtype=np.float64) for t in factors]
    for ell in range(len(f)):
        N = np.zeros(f[ell].shape)
        D = np.zeros(f[ell].shape)
        t = m.operands[ell]
        for a, b in _slab_bounds(np.shape(Y)[0], n_slabs):
            fs = _slab_factors(model_str, f, a, b)
            n_, d_ = numerator_denominator(model_str, fs, ell, Y[a:b], None if M is None else M[a:b],
                                           alpha, beta)
            if c in t:
                idx = [slice(None)] * len(t)
                idx[t.index(c)] = slice(a, b)
                N[tuple(idx)] = n_
                D[tuple(idx)] = d_
            else:
                N += n_
                D += d_
        f[ell] = apply_update(f[ell], N, D, alpha, beta, eps)
    return f


def fit(model_str, factors, Y, M, alpha, beta, eps=1e-10, n_sweeps=1,
        trace=False):
    """Algorithm 1 for a fixed number of sweeps, from max(eps, Theta_init).

    Returns the factors and, if ``trace``, the loss before the first sweep and
    after every sweep.
    """
    f = [np.maximum(eps, np.asarray(t, dtype=np.float64)) for t in factors]
    losses = [loss(model_str, f, Y, M, alpha, beta)] if trace else None
    for _ in range(n_sweeps):
        f = sweep(model_str, f, Y, M, alpha, beta, eps)
        if trace:
            losses.append(loss(model_str, f, Y, M, alpha, beta))
    return (f, losses) if trace else f


def kkt_residual(model_str, factors, Y, M, alpha, beta, eps):
    """Stationarity residual of the constrained problem (eq. 3.1).

    With r = N/D, the update multiplies theta by g^{-1}(r) (eq. 3.4), whose
    fixed point is r = g(1): 1 for the power updates, 0 for the exponential
    ones (alpha = 0 with beta = 1, and Jensen-Shannon).  The gradient is
    dL/dtheta_u = -s (N_u - g(1) D_u) with s of the sign of alpha for the
    (alpha, beta) family (from eq. 3.6 and dL/dy = (b - a)/alpha) and s > 0
    for the other families.  Interior entries need r = g(1); entries at the
    floor eps need dL/dtheta >= 0, i.e. sign(s) (r - g(1)) <= 0.  Returns the
    largest |r - g(1)| over interior entries plus the largest violation at the
    floor, maximised over blocks.
    """
    kind, _ = update_rule(alpha, beta)
    g1 = 0.0 if kind == "exp" else 1.0
    sgn = -1.0 if (not isinstance(alpha, Family) and alpha < 0) else 1.0
    worst = 0.0
    for ell in range(len(factors)):
        N, D = numerator_denominator(model_str, factors, ell, Y, M, alpha, beta)
        th = np.asarray(factors[ell])
        pos = D > 0
        r = np.where(pos, N / np.where(pos, D, 1.0), g1)
        interior = (th > eps * (1 + 1e-9)) & pos
        at_floor = (~interior) & pos
        v_int = float(np.max(np.abs(r[interior] - g1), initial=0.0))
        v_floor = float(np.max(np.maximum(0.0, sgn * (r[at_floor] - g1)), initial=0.0))
        worst = max(worst, v_int + v_floor)
    return worst


# --------------------------------------------------------------------------
# Train / validation splits and the stopping rule (Sec. 6, "Experimental
# design"; App. B, "Algorithmic Details", stopping criterion)
# --------------------------------------------------------------------------
STOP_MAX, STOP_TRAIN_TOL, STOP_VALIDATION = 0, 1, 2


def stop_reason(t, L, V, patience, rel_tol, max_sweeps):
    """The rule for state t given the losses L[0..t], V[0..t] (V None: no
    validation set): the validation loss rose `patience` times in a row, the
    training loss fell by less than rel_tol relative, or t reached the cap.
    Checked in that order; None if no rule applies."""
    if V is not None and patience > 0 and t >= patience and \
            all(V[t - q] > V[t - q - 1] for q in range(patience)):
        return STOP_VALIDATION
    if t >= 1 and (L[t - 1] - L[t]) < rel_tol * abs(L[t - 1]):
        return STOP_TRAIN_TOL
    if t >= max_sweeps:
        return STOP_MAX
    return None


def fit_early_stopping(model_str, factors, Y, M, alpha, beta, eps=1e-10, max_sweeps=5000,
                       patience=5, rel_tol=1e-6, train_value=1, val_value=2):
    """Algorithm 1 on the entries with mask byte train_value, stopped by the
    rules above.  Returns (factors of the stopping state, t, reason, L, V)."""
    M = np.asarray(M)
    Mt = (M == train_value).astype(np.uint8)
    Mv = (M == val_value).astype(np.uint8) if val_value else None
    f = [np.maximum(np.asarray(t, dtype=np.float64), eps) for t in factors]
    L, V = [], ([] if Mv is not None else None)
    t = 0
    while True:
        L.append(loss(model_str, f, Y, Mt, alpha, beta))
        if V is not None:
            V.append(loss(model_str, f, Y, Mv, alpha, beta))
        r = stop_reason(t, L, V, patience, rel_tol, max_sweeps)
        if r is not None:
            return f, t, r, L, V
        f = sweep(model_str, f, Y, Mt, alpha, beta, eps)
        t += 1
