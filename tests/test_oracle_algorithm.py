"""Pins for the oracle's Algorithm 1 (Sec. 3) against what the paper fixes.

* NMF special cases reduce to textbook matrix-form updates written here with
  plain matrix products (Lee-Seung KL and Euclidean; Fevotte-Idier IS with
  exponent 1/2), with and without a mask;
* rank-1 worked example (``tests/golden/rank1_kl_nmf.json``) and the rank-1
  Euclidean block update equal to the least-squares solution;
* the loss never increases across a block update (Theorem 3.1) on a grid of
  (alpha, beta) that visits every g-branch, for CP, Tucker, TT and custom
  strings, with a mask; a planted wrong exponent breaks it;
* exactly factorizable data are fixed points (a(y, y) = b(y, y));
* the stationarity residual vanishes along a run (Theorem 4.3);
* masked-out data never enter arithmetic; D = 0 keeps theta; eps floors.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _rand(shape, seed, lo=0.2, hi=1.5):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


# ---------------------------------------------------------------- NMF closed forms
def _nmf_setup(seed, missing=0.0):
    g = np.random.default_rng(seed)
    I, J, R = 7, 6, 3
    W, H = g.uniform(0.2, 1.5, (I, R)), g.uniform(0.2, 1.5, (J, R))
    Y = g.poisson(3.0 * (W @ H.T)).astype(float) + 0.5
    M = (g.random((I, J)) >= missing).astype(np.uint8) if missing else None
    return W, H, Y, M


@pytest.mark.parametrize("missing", [0.0, 0.3])
def test_nmf_kl_lee_seung(missing):
    W, H, Y, M = _nmf_setup(1, missing)
    Mf = np.ones_like(Y) if M is None else M.astype(float)
    Wn = W * ((Mf * Y / (W @ H.T)) @ H) / (Mf @ H)
    Hn = H * ((Mf * Y / (Wn @ H.T)).T @ Wn) / (Mf.T @ Wn)
    f = O.sweep("ir,jr->ij", [W, H], Y, M, 1.0, 0.0, 1e-300)
    np.testing.assert_allclose(f[0], Wn, rtol=1e-13)
    np.testing.assert_allclose(f[1], Hn, rtol=1e-13)


@pytest.mark.parametrize("missing", [0.0, 0.3])
def test_nmf_euclidean_lee_seung(missing):
    W, H, Y, M = _nmf_setup(2, missing)
    Mf = np.ones_like(Y) if M is None else M.astype(float)
    Wn = W * ((Mf * Y) @ H) / ((Mf * (W @ H.T)) @ H)
    Hn = H * ((Mf * Y).T @ Wn) / ((Mf * (Wn @ H.T)).T @ Wn)
    f = O.sweep("ir,jr->ij", [W, H], Y, M, 1.0, 1.0, 1e-300)
    np.testing.assert_allclose(f[0], Wn, rtol=1e-13)
    np.testing.assert_allclose(f[1], Hn, rtol=1e-13)


@pytest.mark.parametrize("missing", [0.0, 0.3])
def test_nmf_itakura_saito_fevotte(missing):
    W, H, Y, M = _nmf_setup(3, missing)
    Mf = np.ones_like(Y) if M is None else M.astype(float)
    V = W @ H.T
    Wn = W * (((Mf * Y / V ** 2) @ H) / ((Mf / V) @ H)) ** 0.5
    V = Wn @ H.T
    Hn = H * (((Mf * Y / V ** 2).T @ Wn) / ((Mf / V).T @ Wn)) ** 0.5
    f = O.sweep("ir,jr->ij", [W, H], Y, M, 1.0, -1.0, 1e-300)
    np.testing.assert_allclose(f[0], Wn, rtol=1e-13)
    np.testing.assert_allclose(f[1], Hn, rtol=1e-13)


def test_rank1_kl_golden():
    gd = json.load(open(os.path.join(HERE, "golden", "rank1_kl_nmf.json")))
    Y = np.array(gd["Y"])
    W0, H0 = np.array(gd["W0"]), np.array(gd["H0"])
    f = O.block_update(gd["model_str"], [W0, H0], 0, Y, None, gd["alpha"], gd["beta"], 1e-10)
    np.testing.assert_allclose(f[0], gd["after_W_block"]["W"], rtol=1e-15)
    f = O.sweep(gd["model_str"], [W0, H0], Y, None, gd["alpha"], gd["beta"], 1e-10)
    np.testing.assert_allclose(f[0], gd["after_sweep"]["W"], rtol=1e-15)
    np.testing.assert_allclose(f[1], gd["after_sweep"]["H"], rtol=1e-15)
    np.testing.assert_allclose(O.reconstruct(gd["model_str"], f), gd["after_sweep"]["Yhat"], rtol=1e-15)
    # the independence model is then a fixed point
    f2 = O.sweep(gd["model_str"], f, Y, None, 1.0, 0.0, 1e-10)
    np.testing.assert_allclose(O.reconstruct(gd["model_str"], f2), gd["after_sweep"]["Yhat"], rtol=1e-14)


def test_rank1_euclidean_is_least_squares_and_power_iteration():
    g = np.random.default_rng(5)
    Y = g.uniform(0.5, 2.0, (6, 5))
    W, H = g.uniform(0.5, 1.0, (6, 1)), g.uniform(0.5, 1.0, (5, 1))
    f = O.block_update("ir,jr->ij", [W, H], 0, Y, None, 1.0, 1.0, 1e-10)
    ls = np.linalg.lstsq(H, Y.T, rcond=None)[0].T          # argmin_W ||Y - W H^T||
    np.testing.assert_allclose(f[0], ls, rtol=1e-12)
    f = O.fit("ir,jr->ij", [W, H], Y, None, 1.0, 1.0, 1e-10, n_sweeps=200)
    U, S, Vt = np.linalg.svd(Y)
    np.testing.assert_allclose(O.reconstruct("ir,jr->ij", f), S[0] * np.outer(U[:, 0], Vt[0]),
                               rtol=1e-10)


# ---------------------------------------------------------------- monotonicity
MODELS = [
    ("ir,jr,kr->ijk", dict(i=5, j=4, k=6, r=3)),
    ("ia,jb,kc,abc->ijk", dict(i=4, j=5, k=3, a=2, b=3, c=2)),
    ("ia,jab,kbc,lc->ijkl", dict(i=3, j=4, k=3, l=4, a=2, b=2, c=2)),
    ("wr,dr,hr,irk,jrk->wdhij", dict(w=2, d=3, h=2, i=3, j=3, r=2, k=2)),
    ("ij,jk,ik->ijk", dict(i=4, j=3, k=5)),
]
AB_BRANCHES = [(1.0, 0.0), (1.0, 1.0), (0.5, 1.0), (1.0, -1.0), (0.7, 0.0), (1.3, 0.0),
               (0.7, 1.0), (1.3, 1.0), (0.5, 0.5), (2.0, -1.0), (-1.0, 2.0), (0.8, -0.5),
               (1.2, 0.4), (0.3, 1.4), (0.0, 1.0), (0.6, 0.4), (0.6, 0.41), (0.6, 0.39),
               (1.0, 1.0001), (1.0, -0.0001)]


def _problem(model_str, sizes, seed, missing=0.25):
    shapes = O.factor_shapes(model_str, sizes)
    truth = [_rand(s, seed + 10 + i) for i, s in enumerate(shapes)]
    g = np.random.default_rng(seed)
    Y = O.reconstruct(model_str, truth) * g.gamma(4.0, 0.25, size=O.reconstruct(model_str, truth).shape)
    M = (g.random(Y.shape) >= missing).astype(np.uint8)
    init = [_rand(s, seed + 20 + i) for i, s in enumerate(shapes)]
    return Y, M, init


@pytest.mark.parametrize("model_str,sizes", MODELS)
@pytest.mark.parametrize("ab", AB_BRANCHES)
def test_monotone_blocks(model_str, sizes, ab):
    Y, M, f = _problem(model_str, sizes, 11)
    prev = O.loss(model_str, f, Y, M, *ab)
    for _ in range(3):
        bl = []
        f = O.sweep(model_str, f, Y, M, ab[0], ab[1], 1e-10, block_losses=bl)
        for v in bl:
            assert v <= prev + 1e-12 * abs(prev), (v, prev)
            prev = v


@pytest.mark.parametrize("ab,wrong", [((0.5, 1.0), ("pow", 4.0)),    # correct gamma is 2
                                      ((-1.0, 2.0), ("pow", 1.0))])  # correct gamma is -1
def test_planted_wrong_exponent_breaks_monotonicity(monkeypatch, ab, wrong):
    """An exponent that overshoots the minimiser of the surrogate (Lemma 4.2)
    loses the descent guarantee; the monotonicity check must catch it on some
    seed.  The mistake is planted in the oracle, on the CPU."""
    monkeypatch.setattr(O, "update_rule", lambda a, b: wrong)
    broken = False
    for seed in range(6):
        Y, M, f = _problem("ir,jr,kr->ijk", dict(i=5, j=4, k=6, r=3), seed)
        prev = O.loss("ir,jr,kr->ijk", f, Y, M, *ab)
        bl = []
        O.sweep("ir,jr,kr->ijk", f, Y, M, ab[0], ab[1], 1e-10, block_losses=bl)
        for v in bl:
            if v > prev * (1 + 1e-9):
                broken = True
            prev = v
    assert broken


# ---------------------------------------------------------------- fixed points / stationarity
@pytest.mark.parametrize("model_str,sizes", MODELS[:4])
@pytest.mark.parametrize("ab", [(1.0, 0.0), (1.0, 1.0), (0.5, 1.0), (1.0, -1.0), (1.3, 1.0)])
def test_exact_data_is_fixed_point(model_str, sizes, ab):
    shapes = O.factor_shapes(model_str, sizes)
    f = [_rand(s, 30 + i) for i, s in enumerate(shapes)]
    Y = O.reconstruct(model_str, f)
    M = (np.random.default_rng(3).random(Y.shape) >= 0.3).astype(np.uint8)
    f2 = O.sweep(model_str, f, Y, M, ab[0], ab[1], 1e-10)
    for a, b in zip(f, f2):
        np.testing.assert_allclose(b, a, rtol=1e-12)


def test_kkt_residual_vanishes():
    sizes = dict(i=6, j=5, k=4, r=2)
    shapes = O.factor_shapes("ir,jr,kr->ijk", sizes)
    truth = [_rand(s, 40 + i) for i, s in enumerate(shapes)]
    Y = O.reconstruct("ir,jr,kr->ijk", truth)
    f = [_rand(s, 50 + i) for i, s in enumerate(shapes)]
    res = []
    for _ in range(4):
        res.append(O.kkt_residual("ir,jr,kr->ijk", f, Y, None, 1.0, 0.0, 1e-10))
        f = O.fit("ir,jr,kr->ijk", f, Y, None, 1.0, 0.0, 1e-10, n_sweeps=150)
    res.append(O.kkt_residual("ir,jr,kr->ijk", f, Y, None, 1.0, 0.0, 1e-10))
    # MU converges sublinearly; the residual must fall monotonically by three decades
    assert all(b < a for a, b in zip(res, res[1:])) and res[-1] < res[0] * 1e-3, res


# ---------------------------------------------------------------- mask, D = 0, eps
def test_masked_values_never_used():
    Y, M, f = _problem("ir,jr,kr->ijk", dict(i=5, j=4, k=6, r=3), 3)
    Yn = Y.copy()
    Yn[M == 0] = np.nan
    a = O.sweep("ir,jr,kr->ijk", f, Y, M, 0.7, 0.3, 1e-10)
    b = O.sweep("ir,jr,kr->ijk", f, Yn, M, 0.7, 0.3, 1e-10)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert np.isfinite(O.loss("ir,jr,kr->ijk", b, Yn, M, 0.7, 0.3))
    ones = np.ones_like(M)
    c = O.sweep("ir,jr,kr->ijk", f, Y, ones, 1.0, 0.0, 1e-10)
    d = O.sweep("ir,jr,kr->ijk", f, Y, None, 1.0, 0.0, 1e-10)
    for x, y in zip(c, d):
        np.testing.assert_array_equal(x, y)


def test_fully_masked_slice_keeps_theta():
    Y, M, f = _problem("ir,jr->ij", dict(i=4, j=5, r=2), 4)
    M[2, :] = 0
    out = O.block_update("ir,jr->ij", f, 0, Y, M, 1.0, 0.0, 1e-10)
    np.testing.assert_array_equal(out[0][2], f[0][2])


def test_eps_floor():
    Y = np.array([[0.0, 0.0], [1.0, 2.0]])
    W, H = np.ones((2, 1)), np.ones((2, 1))
    out = O.block_update("ir,jr->ij", [W, H], 0, Y, None, 1.0, 0.0, 1e-10)
    assert out[0][0, 0] == 1e-10            # N = 0 < D: the floor (proof of Lemma 4.2)
    f = O.fit("ir,jr->ij", [np.full((2, 1), 1e-20), H], Y + 1, None, 1.0, 0.0, 1e-10, n_sweeps=0)
    assert np.all(f[0] == 1e-10)            # init clamped


@pytest.mark.parametrize("ab,c,expected", [((1.0, 0.0), 2.0, 1.0), ((1.0, 0.0), 0.5, 0.0),
                                           ((-1.0, 2.0), 2.0, 0.5), ((-1.0, 2.0), 0.5, 0.0)])
def test_kkt_residual_floor_branch_by_hand(ab, c, expected):
    """'ir,jr->ij' with I = 2, J = 2, R = 1: w1 sits at the floor, w2 = 1 and
    h are interior; y_2j = yhat_2j and y_1j = c yhat_1j.  By hand: the interior
    ratios of block H are 1 + O(eps); at the floor r_w1 = sum_j a_1j h_j /
    sum_j b_1j h_j, which is c for KL (a = y/yhat, b = 1) and 1/c for
    (alpha, beta) = (-1, 2) (a = yhat/y, b = 1).  KKT needs dL/dtheta >= 0 at
    the floor: r <= 1 when alpha > 0, r >= 1 when alpha < 0; the residual is
    the size of the violation."""
    eps = 1e-10
    W = np.array([[eps], [1.0]])
    H = np.array([[1.0], [2.0]])
    Yhat = W @ H.T
    Y = Yhat.copy()
    Y[0] *= c
    got = O.kkt_residual("ir,jr->ij", [W, H], Y, None, *ab, eps)
    assert abs(got - expected) <= 1e-8, got


@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.0, 1.0), (O.jensen_shannon(), None),
                                        (O.negbin(3.0), None)])
def test_kkt_residual_zero_at_exact_fit(alpha, beta):
    """At Y = Yhat every ratio sits at the update's fixed point g(1): 1 for the
    power updates, 0 for the exponential ones (alpha = 0, beta = 1 and
    Jensen-Shannon), so the residual is zero in every family."""
    g = np.random.default_rng(7)
    f = [g.gamma(1.0, 1.0, size=s) + 0.1 for s in ((5, 3), (4, 3), (6, 3))]
    Y = O.reconstruct("ir,jr,kr->ijk", f)
    assert O.kkt_residual("ir,jr,kr->ijk", f, Y, None, alpha, beta, 1e-10) < 1e-12


def test_kkt_residual_floor_reached_by_mu():
    """KL NMF on data with an all-zero row: MU drives that row of W to the floor
    (N = 0 there), which satisfies KKT; the residual still falls toward zero."""
    g = np.random.default_rng(8)
    W0, H0 = g.gamma(1.0, 1.0, size=(6, 2)), g.gamma(1.0, 1.0, size=(5, 2))
    Y = W0 @ H0.T
    Y[2] = 0.0
    f = [g.gamma(1.0, 1.0, size=(6, 2)), g.gamma(1.0, 1.0, size=(5, 2))]
    f = O.fit("ir,jr->ij", f, Y, None, 1.0, 0.0, 1e-10, n_sweeps=2000)
    assert np.all(f[0][2] == 1e-10)
    assert O.kkt_residual("ir,jr->ij", f, Y, None, 1.0, 0.0, 1e-10) < 1e-4


@pytest.mark.parametrize("model_str,sizes,ab", [
    ("ir,jr,kr->ijk", dict(i=7, j=5, k=6, r=3), (1.0, 1.0)),
    ("wr,dr,hr,irk,jrk->wdhij", dict(w=5, d=3, h=4, i=6, j=5, r=3, k=2), (1.0, 0.0)),
    ("ir,jr,ak,kr,tr->ijat", dict(i=7, j=6, a=3, t=4, r=3, k=2), (0.7, 0.3)),
    ("ij,jk,ik->ijk", dict(i=5, j=4, k=3), (1.0, -1.0))])
def test_slab_sweep_equals_sweep(model_str, sizes, ab):
    """The slab-by-slab evaluation (for tensors too large to reconstruct at
    once) gives the same sweep and loss as the whole-tensor one."""
    g = np.random.default_rng(9)
    f = [g.gamma(1.0, 1.0, size=s) for s in O.factor_shapes(model_str, sizes)]
    Y = g.gamma(2.0, 1.0, size=O.reconstruct(model_str, f).shape)
    M = (g.random(Y.shape) > 0.2).astype(np.uint8)
    ref = O.sweep(model_str, f, Y, M, *ab, 1e-10)
    for n_slabs in (1, 3, sizes[model_str.split("->")[1][0]]):
        got = O.sweep_slabs(model_str, f, Y, M, *ab, 1e-10, n_slabs)
        for a, b in zip(got, ref):
            np.testing.assert_allclose(a, b, rtol=1e-12)
        assert abs(O.loss_slabs(model_str, f, Y, M, *ab, n_slabs) - O.loss(model_str, f, Y, M, *ab)) <= \
            1e-12 * O.loss(model_str, f, Y, M, *ab)
