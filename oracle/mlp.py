"""FP64 CPU oracle for the learned extrapolation of multiplicative-update
iterates.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the library.

The paper has no learned component; this is the specification the GPU kernels
follow, written out plainly in float64:

* Features of one factor element at sweep t (from the iterates theta_t,
  theta_{t-1}, theta_{t-2} of the multiplicative updates of Algorithm 1):
  d1 = log theta_t - log theta_{t-1}, d2 = log theta_{t-1} - log theta_{t-2},
  sigma = root mean square of d1 over the factor (plus 1e-30),
  x = [d1/sigma, d2/sigma, log10(sigma)/8, (log theta_t - log eps)/|log eps|,
       log10(max(rel_dec, 1e-30))/8, gamma, log2(K)/8, 1]
  where rel_dec = (loss_{t-1} - loss_t) / loss_t, gamma the update exponent and
  K the factor's contraction width (last-axis size).
* Network: three dense layers 8 -> 128 -> 128 -> 1 with ReLU between them,
  z = w3 . relu(W2^T relu(W1^T x + b1) + b2) + b3, and the step multiplier
  s = softplus(z) >= 0.
* Proposal: log theta' = log theta_t + s d1, theta' = max(eps, exp(.)), so the
  proposal is positive by construction.
* Training rows: target tau = (log theta_{t+h} - log theta_t) / sigma for a
  horizon of h sweeps, clipped to [-64, 64] (elements falling to the eps
  floor would otherwise dominate); row loss (s x0 - tau)^2, averaged over the
  batch.
* Adam (Kingma and Ba, 2015) with bias correction on float32 master weights.

Parameter vector layout (float64 here, float32 on the GPU), in this order:
W1 [8, 128] row-major (input-major), b1 [128], W2 [128, 128] row-major
(input-major: W2[i, j] connects hidden unit i of layer 1 to unit j of layer 2),
b2 [128], w3 [128], b3 [1]: 17 793 values.
"""
from __future__ import annotations

import numpy as np

N_IN = 8
WIDTH = 128
SHAPES = [("W1", (N_IN, WIDTH)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("w3", (WIDTH,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Split the flat parameter vector into named arrays (views)."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(theta, X):
    """Step multipliers s for the rows of X [B, 8]; also the activations."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["w3"] + P["b3"][0]
    return softplus(z), dict(X=X, a1=a1, h1=h1, a2=a2, h2=h2, z=z)


def batch_loss(theta, X, tau):
    s, _ = forward(theta, X)
    r = s * np.asarray(X, dtype=np.float64)[:, 0] - tau
    return float(np.mean(r * r))


def gradient(theta, X, tau):
    """Loss and its gradient with respect to the flat parameter vector,
    by the chain rule written out layer by layer."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    s, c = forward(theta, X)
    x0 = c["X"][:, 0]
    r = s * x0 - tau
    B = len(tau)
    dz = 2.0 * r * x0 * sigmoid(c["z"]) / B           # d loss / d z
    g = {"w3": c["h2"].T @ dz, "b3": np.array([dz.sum()])}
    da2 = np.outer(dz, P["w3"]) * (c["a2"] > 0)
    g["W2"] = c["h1"].T @ da2
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ P["W2"].T) * (c["a1"] > 0)
    g["W1"] = c["X"].T @ da1
    g["b1"] = da1.sum(axis=0)
    flat = np.concatenate([g[name].ravel() for name, _ in SHAPES])
    return float(np.mean(r * r)), flat


class Adam:
    """Adam with bias correction (Kingma and Ba, 2015)."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def features(th_t, th_tm1, th_tm2, rel_dec, gamma, eps):
    """Rows [n, 8] for one factor (any shape; the last axis is its contraction
    width) and the factor's sigma."""
    t = np.log(np.asarray(th_t, dtype=np.float64))
    d1 = (t - np.log(np.asarray(th_tm1, dtype=np.float64))).ravel()
    d2 = (np.log(np.asarray(th_tm1, dtype=np.float64)) - np.log(np.asarray(th_tm2, dtype=np.float64))).ravel()
    sigma = np.sqrt(np.mean(d1 * d1)) + 1e-30
    K = np.shape(th_t)[-1]
    n = d1.size
    X = np.empty((n, N_IN))
    X[:, 0] = d1 / sigma
    X[:, 1] = d2 / sigma
    X[:, 2] = np.log10(sigma) / 8.0
    X[:, 3] = (t.ravel() - np.log(eps)) / abs(np.log(eps))
    X[:, 4] = np.log10(max(rel_dec, 1e-30)) / 8.0
    X[:, 5] = gamma
    X[:, 6] = np.log2(K) / 8.0
    X[:, 7] = 1.0
    return X, sigma


def targets(th_t, th_th, sigma):
    """Training targets tau = clip((log theta_{t+h} - log theta_t) / sigma, -64, 64)."""
    return np.clip((np.log(np.asarray(th_th, dtype=np.float64))
                    - np.log(np.asarray(th_t, dtype=np.float64))).ravel() / sigma, -64.0, 64.0)


def propose(theta, th_t, th_tm1, th_tm2, rel_dec, gamma, eps):
    """The extrapolated factor theta' = max(eps, theta_t exp(s d1))."""
    X, sigma = features(th_t, th_tm1, th_tm2, rel_dec, gamma, eps)
    s, _ = forward(theta, X)
    d1 = X[:, 0] * sigma
    t = np.log(np.asarray(th_t, dtype=np.float64)).ravel()
    return np.maximum(eps, np.exp(t + s * d1)).reshape(np.shape(th_t))


def accept(loss_candidate, loss_current, candidate, eps):
    """A proposal replaces the iterate only if it is >= eps everywhere and its
    loss is strictly lower (both losses in float64)."""
    return bool(np.all(candidate >= eps)) and loss_candidate < loss_current
