"""Pins for the oracle's (alpha, beta)-divergence, a, b and g (App. B).

* named special cases equal their textbook forms;
* the generic case tends to each special case in the limit;
* d/dy D(x, y) = (b - a)/alpha (alpha != 0), by central differences;
* the decomposability identity of eq. 3.3 holds for the g chosen by
  ``update_rule`` on each branch, with the convex / concave split built here
  from the sign of each term's second derivative.
"""
import numpy as np
import pytest

from oracle import oracle as O

g = np.random.default_rng(7)
X = g.uniform(0.2, 3.0, 50)
Yv = g.uniform(0.2, 3.0, 50)


TEXTBOOK = {
    (1.0, 0.0): lambda x, y: x * np.log(x / y) - x + y,                 # KL
    (1.0, -1.0): lambda x, y: x / y - np.log(x / y) - 1.0,              # Itakura-Saito
    (1.0, 1.0): lambda x, y: 0.5 * (x - y) ** 2,                        # squared Euclidean
    (0.5, 0.5): lambda x, y: 2.0 * (np.sqrt(x) - np.sqrt(y)) ** 2,      # squared Hellinger (x4 scaling)
    (0.0, 1.0): lambda x, y: y * np.log(y / x) - y + x,                 # reverse KL
    (2.0, -1.0): lambda x, y: (x - y) ** 2 / (2.0 * y),                 # Pearson chi^2
    (-1.0, 2.0): lambda x, y: (x - y) ** 2 / (2.0 * x),                 # Neyman chi^2
    (0.0, 0.0): lambda x, y: 0.5 * (np.log(x) - np.log(y)) ** 2,        # log-Euclidean
}


@pytest.mark.parametrize("ab", sorted(TEXTBOOK))
def test_special_cases(ab):
    np.testing.assert_allclose(O.ab_loss(X, Yv, *ab), TEXTBOOK[ab](X, Yv), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("a,b,lim", [(1.3, 1e-7, (1.3, 0.0)), (0.7, -0.7 + 1e-7, (0.7, -0.7)),
                                     (1e-7, 0.6, (0.0, 0.6))])
def test_generic_case_limits(a, b, lim):
    np.testing.assert_allclose(O.ab_loss(X, Yv, a, b), O.ab_loss(X, Yv, *lim), rtol=2e-5, atol=1e-8)


def test_generic_case_double_limit():
    # alpha = beta -> 0 (first-order convergence; 1/(alpha beta) limits how small a step is usable)
    np.testing.assert_allclose(O.ab_loss(X, Yv, 1e-4, 1e-4), O.ab_loss(X, Yv, 0.0, 0.0), rtol=2e-3, atol=1e-6)


def test_zero_data():
    # x = 0 with alpha > 0: x^alpha = 0 and x^alpha log x = 0, so KL(0, y) = y
    np.testing.assert_allclose(O.ab_loss(np.zeros(3), np.array([0.5, 1.0, 2.0]), 1.0, 0.0),
                               [0.5, 1.0, 2.0])
    a, b = O.ab_weights(np.zeros(2), np.array([1.0, 2.0]), 1.0, 0.0)
    assert np.all(a == 0) and np.all(b == 1)


AB_GRID = [(1.0, 0.0), (1.0, 1.0), (0.5, 1.0), (1.0, -1.0), (0.7, 0.0), (1.3, 0.0), (0.7, 1.0),
           (1.3, 1.0), (0.5, 0.5), (2.0, -1.0), (-1.0, 2.0), (0.8, -0.5), (1.2, 0.4), (-0.5, -0.3),
           (0.3, 1.4), (2.5, 0.5)]


@pytest.mark.parametrize("ab", AB_GRID)
def test_weights_are_loss_derivative(ab):
    al, be = ab
    h = 1e-6
    d = (O.ab_loss(X, Yv + h, al, be) - O.ab_loss(X, Yv - h, al, be)) / (2 * h)
    a, b = O.ab_weights(X, Yv, al, be)
    np.testing.assert_allclose(d, (b - a) / al, rtol=1e-6, atol=1e-7)


def test_reverse_kl_weights():
    # alpha = 0, beta = 1: d/dy D = log(y/x) = -a with b = 1 (g = log, c = 1)
    h = 1e-6
    d = (O.ab_loss(X, Yv + h, 0.0, 1.0) - O.ab_loss(X, Yv - h, 0.0, 1.0)) / (2 * h)
    a, b = O.ab_weights(X, Yv, 0.0, 1.0)
    np.testing.assert_allclose(d, -a, rtol=1e-6, atol=1e-7)
    assert O.update_rule(0.0, 1.0) == ("exp", None)
    with pytest.raises(ValueError):
        O.update_rule(0.0, 0.5)


def _split_derivatives(x, y, lam, al, be):
    """d/dy of the convex part at lam*y plus d/dy of the concave part at y.

    For alpha, beta, alpha+beta != 0 the divergence is, up to a term constant
    in y, T1 + T2 with T1 = y^(a+b)/(a(a+b)) and T2 = -x^a y^b/(ab); each term
    is convex or concave in y by the sign of its second derivative.
    """
    h = 1e-6
    t1 = lambda yy: yy ** (al + be) / (al * (al + be))
    t2 = lambda yy: -(x ** al) * yy ** be / (al * be)
    dd = lambda f, yy: (f(yy + h) - 2 * f(yy) + f(yy - h)) / h ** 2
    d1 = lambda f, yy: (f(yy + h) - f(yy - h)) / (2 * h)
    out = 0.0
    for t in (t1, t2):
        convex = np.all(dd(t, y) >= -1e-6)
        out = out + (d1(t, lam * y) if convex else d1(t, y))
    return out


@pytest.mark.parametrize("ab", [p for p in AB_GRID if p[1] != 0 and p[0] + p[1] != 0])
def test_decomposability_identity(ab):
    """eq. 3.3: the split derivative equals c(lambda) [g(lambda) b - a] with g from App. B.

    g(lambda) = lambda^(1/gamma) where gamma comes from ``update_rule``; the
    ratio (split derivative)/(g b - a) must then depend on lambda only.
    """
    al, be = ab
    kind, gamma = O.update_rule(al, be)
    assert kind == "pow"
    a, b = O.ab_weights(X, Yv, al, be)
    for lam in (0.5, 0.9, 1.7, 3.0):
        lhs = _split_derivatives(X, Yv, lam, al, be)
        rhs = lam ** (1.0 / gamma) * b - a
        c = lhs / rhs
        ok = np.abs(rhs) > 1e-3
        assert np.ptp(c[ok]) < 1e-5 * max(1.0, np.max(np.abs(c[ok])))


@pytest.mark.parametrize("ab,gamma", [((1.0, 0.0), 1.0), ((1.0, 1.0), 1.0), ((0.5, 1.0), 2.0),
                                      ((1.0, -1.0), 0.5), ((0.7, 0.0), 1.0), ((1.3, 0.0), 1 / 1.3),
                                      ((0.7, 1.0), 1 / 0.7), ((1.3, 1.0), 1 / 1.3)])
def test_update_exponents(ab, gamma):
    kind, gm = O.update_rule(*ab)
    assert kind == "pow" and abs(gm - gamma) < 1e-15
