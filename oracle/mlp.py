"""FP64 reference of the learned ray proposal (TEST INFRASTRUCTURE).

The proposal is a 4-layer MLP, 18 -> 64 -> 64 -> 64 -> 1 with ReLU, mapping
(azimuth, elevation, 16-value scene code) to a logit per direction bin; the
sampling density over the 128 x 64 azimuth x sin(elevation) grid of equal
solid-angle bins is the softmax of the logits mixed with the uniform density:
q_mix = (1 - beta) softmax(z) + beta / 8192.  The network is trained on
returned-power histograms H_b of uniformly traced rays with the loss
L = -sum_b H_b log softmax(z)_b / sum_b H_b (mean over scenes) and Adam
(Kingma & Ba 2015).  Plain numpy, float64, written from those definitions.

Flat parameter layout (9 601 values): W1 [64][18], b1 [64], W2 [64][64],
b2 [64], W3 [64][64], b3 [64], W4 [1][64], b4 [1].
"""
from __future__ import annotations

import numpy as np

N_AZ, N_EL = 128, 64
N_BINS = N_AZ * N_EL
N_IN, N_H = 18, 64
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_H, N_H)), ("b3", (N_H,)), ("W4", (1, N_H)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(params):
    params = np.asarray(params, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = params[o:o + n].reshape(shape)
        o += n
    return out


def bin_centres():
    """Normalised bin-centre coordinates in [-1, 1]: bin b = ie * N_AZ + ia."""
    b = np.arange(N_BINS)
    ia, ie = b % N_AZ, b // N_AZ
    return 2.0 * (ia + 0.5) / N_AZ - 1.0, 2.0 * (ie + 0.5) / N_EL - 1.0


def features(codes):
    """Inputs [S * N_BINS][18]: (azimuth, elevation) of the bin centre and the
    scene's 16-value code."""
    codes = np.atleast_2d(np.asarray(codes, dtype=np.float64))
    ua, ue = bin_centres()
    S = codes.shape[0]
    X = np.empty((S, N_BINS, N_IN))
    X[:, :, 0] = ua
    X[:, :, 1] = ue
    X[:, :, 2:] = codes[:, None, :]
    return X.reshape(S * N_BINS, N_IN)


def forward(params, X):
    p = unpack(params)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    a3 = h2 @ p["W3"].T + p["b3"]
    h3 = np.maximum(a3, 0.0)
    z = (h3 @ p["W4"].T + p["b4"])[:, 0]
    return z, (X, a1, h1, a2, h2, a3, h3)


def softmax(z):
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(z - z.max())
    return e / e.sum()


def loss_and_grad(params, codes, hist):
    """Mean over scenes of -sum_b H_b log q_b / sum_b H_b, and its gradient."""
    codes = np.atleast_2d(codes)
    hist = np.atleast_2d(np.asarray(hist, dtype=np.float64))
    S = codes.shape[0]
    X = features(codes)
    z, (X, a1, h1, a2, h2, a3, h3) = forward(params, X)
    z = z.reshape(S, N_BINS)
    loss = 0.0
    dz = np.zeros_like(z)
    for s in range(S):
        Hs = hist[s].sum()
        if Hs <= 0:
            continue
        zs = z[s] - z[s].max()
        logq = zs - np.log(np.exp(zs).sum())
        loss += -(hist[s] * logq).sum() / Hs / S
        dz[s] = (np.exp(logq) - hist[s] / Hs) / S
    dz = dz.reshape(-1)
    p = unpack(params)
    g = {}
    g["W4"] = dz[None, :] @ h3
    g["b4"] = np.array([dz.sum()])
    d3 = (dz[:, None] * p["W4"]) * (a3 > 0)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(0)
    d2 = (d3 @ p["W3"]) * (a2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (a1 > 0)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(0)
    grad = np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])
    return loss, grad


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1); t is the 1-based step."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def mixture(z, beta, power=1.0):
    """(1 - beta) softmax(power z) + beta / n: the sampling density of a
    network output z (power < 1 flattens the fitted density)."""
    return (1.0 - beta) * softmax(power * np.asarray(z, dtype=np.float64)) + beta / len(z)


def mixture_cost(z, beta, kappa):
    """(1 - beta) d / sum d + beta / n with d = sqrt(x / (kappa + x)) and
    x = n softmax(z): the density of least variance x work when a ray costs
    kappa mean returns (importance sampling: variance sum_b x_b / q_b, work
    kappa + sum_b q_b x_b per ray, minimised together by Cauchy-Schwarz)."""
    z = np.asarray(z, dtype=np.float64)
    x = len(z) * softmax(z)
    d = np.sqrt(x / (kappa + x))
    return (1.0 - beta) * d / d.sum() + beta / len(z)


def cdf_of(q):
    c = np.concatenate([[0.0], np.cumsum(q)])
    c /= c[-1]
    c[-1] = 1.0
    return c
