"""Amplitude-guess network in FP64.  TEST INFRASTRUCTURE.

A small multilayer perceptron predicts each doubles amplitude t_ij^ab from
three MP2 features of that amplitude: the integral <ij||ab>, the denominator
D_ij^ab and the MP2 pair energy e_ij = sum_{a<b} |<ij||ab>|^2 / D_ij^ab
(so that E_MP2 = sum_{i<j} e_ij).  Features are standardised,
z = (x / s_x, (D - m_D) / s_D, (e - m_e) / s_e); the integral is scaled
without a shift so that its sign flip commutes with the scaling.

    g(z)  = W3 relu(W2 relu(W1 z + b1) + b2) + b3       (3 -> 128 -> 128 -> 1)
    f(z)  = (g(z) - g(z with z_0 negated)) / 2          odd in <ij||ab>
    t     = s_t f(z)

Because <ij||ab> changes sign under i<->j and under a<->b while D and e_ij
do not, the predicted t2 is antisymmetric by construction.  Loss: mean
squared error of f against t / s_t over the unique amplitudes (i<j, a<b).
Optimiser: Adam (Kingma & Ba, 2015) with the usual bias corrections.
"""
from __future__ import annotations

import numpy as np

H = 128
PARAM_SHAPES = (("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (1, H)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)  # 17153


def unique_pairs(n):
    i, j = np.triu_indices(n, 1)
    return i, j


def raw_features(oovv, d2):
    """(x, D, e) for every unique amplitude i<j, a<b, in (ij, ab) row-major
    order of the unique pairs.  oovv: <ij||ab> (real), d2: D_ij^ab."""
    o, v = oovv.shape[0], oovv.shape[2]
    i, j = unique_pairs(o)
    a, b = unique_pairs(v)
    pair_e = np.zeros((o, o))
    x2 = oovv ** 2 / d2
    for p, q in zip(i, j):
        pair_e[p, q] = pair_e[q, p] = x2[p, q][a, b].sum()
    x = oovv[i, j][:, a, b]
    D = d2[i, j][:, a, b]
    e = np.broadcast_to(pair_e[i, j][:, None], x.shape)
    return np.stack([x.ravel(), D.ravel(), e.ravel()], axis=1)


def standardise(raw, stats):
    sx, mD, sD, me, se = stats["sx"], stats["mD"], stats["sD"], stats["me"], stats["se"]
    return np.stack([raw[:, 0] / sx, (raw[:, 1] - mD) / sD, (raw[:, 2] - me) / se], axis=1)


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in PARAM_SHAPES:
        if name.startswith("W"):
            p[name] = rng.normal(size=shape) * np.sqrt(2.0 / shape[1])
        else:
            p[name] = np.zeros(shape)
    return p


def flatten(p):
    return np.concatenate([p[n].ravel() for n, _ in PARAM_SHAPES])


def unflatten(vec):
    out, k = {}, 0
    for n, s in PARAM_SHAPES:
        m = int(np.prod(s))
        out[n] = vec[k:k + m].reshape(s).copy()
        k += m
    return out


def _g(p, z):
    a1 = z @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    return (h2 @ p["W3"].T + p["b3"])[:, 0], (h1, h2)


def forward(p, z):
    """f(z) for rows z (N x 3)."""
    zm = z.copy()
    zm[:, 0] = -zm[:, 0]
    gp, _ = _g(p, z)
    gm, _ = _g(p, zm)
    return 0.5 * (gp - gm)


def loss_and_grad(p, z, y):
    """Mean squared error of f(z) against y and its gradient (dict)."""
    N = z.shape[0]
    zm = z.copy()
    zm[:, 0] = -zm[:, 0]
    Z2 = np.concatenate([z, zm], axis=0)  # rows: +branch then -branch
    a1 = Z2 @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    g = (h2 @ p["W3"].T + p["b3"])[:, 0]
    f = 0.5 * (g[:N] - g[N:])
    r = f - y
    loss = float(np.mean(r ** 2))
    df = 2.0 * r / N
    dg = np.concatenate([0.5 * df, -0.5 * df])
    grad = {"W3": dg[None, :] @ h2, "b3": np.array([dg.sum()])}
    da2 = np.outer(dg, p["W3"][0]) * (a2 > 0)
    grad["W2"] = da2.T @ h1
    grad["b2"] = da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * (a1 > 0)
    grad["W1"] = da1.T @ Z2
    grad["b1"] = da1.sum(axis=0)
    return loss, grad


class Adam:
    def __init__(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = self.v = None
        self.t = 0

    def step(self, params_vec, grad_vec):
        if self.m is None:
            self.m = np.zeros_like(params_vec)
            self.v = np.zeros_like(params_vec)
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad_vec
        self.v = self.b2 * self.v + (1 - self.b2) * grad_vec ** 2
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return params_vec - self.lr * mh / (np.sqrt(vh) + self.eps)


def predict_t2(p, stats, oovv, d2):
    """Full antisymmetric t2[i][j][a][b] from the network."""
    o, v = oovv.shape[0], oovv.shape[2]
    f = forward(p, standardise(raw_features(oovv, d2), stats)) * stats["st"]
    i, j = unique_pairs(o)
    a, b = unique_pairs(v)
    t2 = np.zeros((o, o, v, v))
    blk = f.reshape(i.size, a.size)
    for u, (p_, q_) in enumerate(zip(i, j)):
        m = np.zeros((v, v))
        m[a, b] = blk[u]
        m[b, a] = -blk[u]
        t2[p_, q_] = m
        t2[q_, p_] = -m
    return t2
