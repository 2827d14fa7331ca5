"""Pins of the FP64 MLP oracle (the learned extrapolation has no paper passage;
these check it against calculus and closed forms)."""
import numpy as np
import pytest

from oracle import mlp as Mlp


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    th = rng.normal(0.0, scale, Mlp.N_PARAMS)
    P = Mlp.unpack(th)
    P["b1"][:] = np.abs(P["b1"]) + 0.05   # keep most ReLUs active
    P["b2"][:] = np.abs(P["b2"]) + 0.05
    return th


def _rows(seed, B=37):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, (B, Mlp.N_IN))
    X[:, 7] = 1.0
    return X, rng.normal(0.0, 1.0, B)


def test_layout_size():
    assert Mlp.N_PARAMS == 8 * 128 + 128 + 128 * 128 + 128 + 128 + 1 == 17793


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    th = _params(seed)
    X, tau = _rows(seed + 10)
    loss, g = Mlp.gradient(th, X, tau)
    assert loss == pytest.approx(Mlp.batch_loss(th, X, tau), rel=1e-14)
    rng = np.random.default_rng(seed + 20)
    # every bias and w3 entry, plus random entries of W1 and W2
    idx = list(range(8 * 128, 8 * 128 + 128)) + list(range(Mlp.N_PARAMS - 257, Mlp.N_PARAMS))
    idx += list(rng.choice(8 * 128, 40, replace=False))
    idx += list(8 * 128 + 128 + rng.choice(128 * 128, 80, replace=False))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (Mlp.batch_loss(th + e, X, tau) - Mlp.batch_loss(th - e, X, tau)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd), np.max(np.abs(g))), (i, fd, g[i])


def test_directional_derivative():
    th = _params(5)
    X, tau = _rows(6, 64)
    _, g = Mlp.gradient(th, X, tau)
    d = np.random.default_rng(7).normal(size=th.size)
    h = 1e-6
    fd = (Mlp.batch_loss(th + h * d, X, tau) - Mlp.batch_loss(th - h * d, X, tau)) / (2 * h)
    assert fd == pytest.approx(g @ d, rel=1e-6)


def test_adam_first_steps_closed_form():
    lr, eps = 1e-2, 1e-8
    opt = Mlp.Adam(3, lr=lr, eps=eps)
    g1 = np.array([0.5, -2.0, 0.0])
    t1 = opt.step(np.zeros(3), g1)
    # after bias correction m_hat = g and v_hat = g^2 on the first step
    np.testing.assert_allclose(t1, -lr * g1 / (np.abs(g1) + eps), rtol=1e-12)
    g2 = np.array([1.0, 1.0, 1.0])
    t2 = opt.step(t1, g2)
    m = (0.9 * 0.1 * g1 + 0.1 * g2) / (1 - 0.81)
    v = (0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    np.testing.assert_allclose(t2, t1 - lr * m / (np.sqrt(v) + eps), rtol=1e-12)


def test_constant_network_is_geometric_extrapolation():
    """All weights zero and b3 = log(e - 1): s = softplus(b3) = 1, so the
    proposal is theta_t^2 / theta_{t-1} (one more step of the same ratio)."""
    th = np.zeros(Mlp.N_PARAMS)
    Mlp.unpack(th)["b3"][0] = np.log(np.e - 1.0)
    rng = np.random.default_rng(3)
    a = rng.gamma(1.0, 1.0, (17, 5)) + 0.1
    b = a * rng.uniform(0.8, 1.2, a.shape)
    c = b * rng.uniform(0.8, 1.2, a.shape)
    prop = Mlp.propose(th, c, b, a, 1e-3, 1.0, 1e-10)
    np.testing.assert_allclose(prop, c * c / b, rtol=1e-12)


def test_features_of_a_geometric_trajectory():
    r = 0.97
    th0 = np.array([[1.0, 2.0], [3.0, 4.0]])
    X, sigma = Mlp.features(th0 * r ** 2, th0 * r, th0, 0.01, 2.0, 1e-10)
    assert sigma == pytest.approx(abs(np.log(r)), rel=1e-12)
    np.testing.assert_allclose(X[:, 0], -1.0, rtol=1e-12)
    np.testing.assert_allclose(X[:, 1], -1.0, rtol=1e-12)
    np.testing.assert_allclose(X[:, 2], np.log10(abs(np.log(r))) / 8)
    np.testing.assert_allclose(X[:, 3], (np.log(th0 * r * r).ravel() + np.log(1e10)) / np.log(1e10))
    np.testing.assert_allclose(X[:, 4], -2.0 / 8)
    np.testing.assert_allclose(X[:, 5:], [[2.0, 1.0 / 8, 1.0]] * 4)
    # h more steps of the same ratio: tau = h log r / sigma = -h
    tau = Mlp.targets(th0 * r ** 2, th0 * r ** 7, sigma)
    np.testing.assert_allclose(tau, -5.0, rtol=1e-12)


def test_training_learns_a_constant_multiplier():
    """Rows whose target is 3 x0 (a 3-step geometric extrapolation): Adam on
    the batch loss drives s towards 3."""
    rng = np.random.default_rng(11)
    X = rng.normal(0, 1, (256, 8))
    X[:, 7] = 1.0
    tau = 3.0 * X[:, 0]
    th = _params(12, scale=0.05)
    opt = Mlp.Adam(th.size, lr=3e-3)
    l0 = Mlp.batch_loss(th, X, tau)
    for _ in range(300):
        _, g = Mlp.gradient(th, X, tau)
        th = opt.step(th, g)
    s, _ = Mlp.forward(th, X)
    assert Mlp.batch_loss(th, X, tau) < 1e-3 * l0
    assert np.median(np.abs(s - 3.0)) < 0.05


def test_accept_rule():
    c = np.array([1e-10, 1.0])
    assert Mlp.accept(1.0, 2.0, c, 1e-10)
    assert not Mlp.accept(2.0, 2.0, c, 1e-10)       # equal loss: keep the iterate
    assert not Mlp.accept(3.0, 2.0, c, 1e-10)
    assert not Mlp.accept(1.0, 2.0, np.array([0.0, 1.0]), 1e-10)


def test_targets_are_clipped():
    th = np.array([1.0, 1.0])
    tau = Mlp.targets(th, np.array([1e-10, 1.001]), 0.01)
    assert tau[0] == -64.0
    assert tau[1] == pytest.approx(np.log(1.001) / 0.01)
