"""Pins of the oracle's other decomposable likelihoods (App. B: negative
binomial, binomial / Bernoulli odds, Jensen-Shannon) against calculus, closed
matrix forms and Theorem 3.1."""
import numpy as np
import pytest

from oracle import oracle as O

FAMS = [O.negbin(2.5), O.negbin(0.7), O.binomial(1.0), O.binomial(5.0), O.jensen_shannon()]


def _data_for(fam, shape, rng):
    if fam.kind == "binomial":
        return rng.binomial(int(fam.param), 0.4, shape).astype(np.float64)
    if fam.kind == "negbin":
        return rng.negative_binomial(fam.param, fam.param / (fam.param + 3.0), shape).astype(np.float64)
    return rng.gamma(2.0, 1.0, shape)


@pytest.mark.parametrize("fam", FAMS, ids=lambda f: f"{f.kind}{f.param}")
def test_derivative_identity(fam):
    """d/dy D(x, y) = c(1) (g(1) b - a): b - a for g = lambda, c = 1/lambda;
    -a/2 for Jensen-Shannon (g = log, c = 1/2)."""
    rng = np.random.default_rng(1)
    x = rng.uniform(0.0, 4.0, 200)
    y = rng.uniform(0.2, 5.0, 200)
    if fam.kind == "binomial":
        x = rng.uniform(0.0, fam.param, 200)
    h = 1e-6
    fd = (O.ab_loss(x, y + h, fam, None) - O.ab_loss(x, y - h, fam, None)) / (2 * h)
    a, b = O.ab_weights(x, y, fam, None)
    expect = -0.5 * a if fam.kind == "js" else b - a
    np.testing.assert_allclose(fd, expect, rtol=1e-6, atol=1e-8)


def test_js_is_a_symmetric_divergence():
    rng = np.random.default_rng(2)
    x, y = rng.gamma(2, 1, 100), rng.gamma(2, 1, 100)
    js = O.jensen_shannon()
    np.testing.assert_allclose(O.ab_loss(x, y, js, None), O.ab_loss(y, x, js, None), rtol=1e-13)
    np.testing.assert_allclose(O.ab_loss(x, x, js, None), 0.0, atol=1e-14)
    assert np.all(O.ab_loss(x, y, js, None) >= -1e-15)
    # textbook form with the mean m = (x + y)/2
    m = 0.5 * (x + y)
    ref = 0.5 * (x * np.log(x / m) + y * np.log(y / m))
    np.testing.assert_allclose(O.ab_loss(x, y, js, None), ref, rtol=1e-12, atol=1e-14)


def _nmf(rng, I=13, J=11, R=3):
    W = rng.gamma(1.0, 1.0, (I, R))
    H = rng.gamma(1.0, 1.0, (J, R))
    return W, H


@pytest.mark.parametrize("fam", FAMS, ids=lambda f: f"{f.kind}{f.param}")
@pytest.mark.parametrize("masked", [False, True])
def test_nmf_update_matches_matrix_form(fam, masked):
    """W <- W * (A H) / (B H) (or W * exp((A H)/(B H)) for JS), with A, B the
    masked weights of the family, written with matrix products."""
    rng = np.random.default_rng(3)
    W, H = _nmf(rng)
    Y = _data_for(fam, (13, 11), rng)
    M = (rng.uniform(size=Y.shape) > 0.25).astype(np.uint8) if masked else None
    Yh = W @ H.T
    m = np.ones_like(Y) if M is None else M.astype(np.float64)
    if fam.kind == "negbin":
        A, B = m * Y / Yh, m * (fam.param + Y) / (fam.param + Yh)
    elif fam.kind == "binomial":
        A, B = m * Y / Yh, m * fam.param / (1.0 + Yh)
    else:
        A, B = m * np.log((Y + Yh) / (2 * Yh)), m * 1.0
    r = (A @ H) / (B @ H)
    W_ref = np.maximum(1e-10, W * (np.exp(r) if fam.kind == "js" else r))
    got = O.block_update("ir,jr->ij", [W, H], 0, Y, M, fam, None, 1e-10)[0]
    np.testing.assert_allclose(got, W_ref, rtol=1e-12)


def test_large_dispersion_gives_the_poisson_update():
    """phi -> infinity: b -> 1 and the negative binomial update becomes the
    KL (Poisson) update."""
    rng = np.random.default_rng(4)
    W, H = _nmf(rng)
    Y = rng.poisson(2.0, (13, 11)).astype(np.float64)
    nb = O.block_update("ir,jr->ij", [W, H], 0, Y, None, O.negbin(1e9), None, 1e-10)[0]
    kl = O.block_update("ir,jr->ij", [W, H], 0, Y, None, 1.0, 0.0, 1e-10)[0]
    np.testing.assert_allclose(nb, kl, rtol=1e-7)


MODELS = [("ir,jr->ij", dict(i=9, j=8, r=3)), ("ir,jr,kr->ijk", dict(i=6, j=5, k=4, r=3)),
          ("ia,jb,ab->ij", dict(i=7, j=6, a=3, b=2))]


@pytest.mark.parametrize("fam", FAMS, ids=lambda f: f"{f.kind}{f.param}")
@pytest.mark.parametrize("model", MODELS, ids=lambda m: m[0])
def test_monotone_under_every_block(fam, model):
    """Theorem 3.1 for each family: the loss never increases, block by block."""
    ms, sz = model
    rng = np.random.default_rng(5)
    f = [rng.gamma(1.0, 1.0, s) for s in O.factor_shapes(ms, sz)]
    shape = tuple(sz[c] for c in ms.split("->")[1])
    Y = _data_for(fam, shape, rng)
    M = (rng.uniform(size=shape) > 0.2).astype(np.uint8)
    prev = O.loss(ms, f, Y, M, fam, None)
    for _ in range(15):
        bl = []
        f = O.sweep(ms, f, Y, M, fam, None, 1e-10, block_losses=bl)
        for v in bl:
            assert v <= prev + 1e-10 * abs(prev), (fam, ms, v, prev)
            prev = v


@pytest.mark.parametrize("fam", FAMS, ids=lambda f: f"{f.kind}{f.param}")
def test_exact_data_is_a_fixed_point(fam):
    """Data at the family's optimum for the model: y = yhat (negative
    binomial, JS) or y = n yhat / (1 + yhat) (binomial odds)."""
    rng = np.random.default_rng(6)
    ms, sz = "ir,jr,kr->ijk", dict(i=5, j=6, k=4, r=2)
    f = [rng.gamma(2.0, 1.0, s) for s in O.factor_shapes(ms, sz)]
    Yh = O.reconstruct(ms, f)
    Y = fam.param * Yh / (1.0 + Yh) if fam.kind == "binomial" else Yh
    g = O.sweep(ms, f, Y, None, fam, None, 1e-10)
    for a, b in zip(f, g):
        np.testing.assert_allclose(b, a, rtol=1e-12)
