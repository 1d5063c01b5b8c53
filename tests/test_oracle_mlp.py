"""Pins of the proposal oracle: backpropagation against central finite
differences, Adam against torch.optim.Adam, the mixture and CDF, and the
training histogram against its definition on a specular plate."""
import math

import numpy as np
import pytest

import scenegen as sg
from oracle import mlp


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, mlp.N_PARAMS)


def test_param_count():
    assert mlp.N_PARAMS == 9601


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = _params(1)
    codes = rng.random((2, 16))
    hist = rng.random((2, mlp.N_BINS)) * (rng.random((2, mlp.N_BINS)) < 0.05)
    loss, g = mlp.loss_and_grad(p, codes, hist)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 40, replace=False), [9600, 9599, 1152, 0]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mlp.loss_and_grad(p + e, codes, hist)
        lm, _ = mlp.loss_and_grad(p - e, codes, hist)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    p0 = rng.normal(size=50)
    t = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.normal(size=50)
        opt.zero_grad()
        t.grad = torch.tensor(g)
        opt.step()
        p, m, v = mlp.adam_step(p, g, m, v, step, 1e-2)
    assert np.allclose(p, t.detach().numpy(), rtol=0, atol=1e-12)


def test_mixture_and_cdf():
    z = np.random.default_rng(3).normal(size=mlp.N_BINS)
    q = mlp.mixture(z, 0.1)
    assert abs(q.sum() - 1) < 1e-12 and q.min() >= 0.1 / mlp.N_BINS - 1e-18
    c = mlp.cdf_of(q)
    assert c[0] == 0 and c[-1] == 1 and np.all(np.diff(c) >= 0)
    assert np.allclose(np.diff(c), q, atol=1e-15)
    assert np.allclose(mlp.mixture(z, 1.0), 1.0 / mlp.N_BINS)


def test_loss_is_cross_entropy_minimum_at_target():
    """The loss is minimised (gradient zero) when softmax(z) equals H / sum H."""
    rng = np.random.default_rng(4)
    H = rng.random(mlp.N_BINS) + 0.1
    q = H / H.sum()
    z = np.log(q)
    # gradient w.r.t. the logits is q - H / sum H = 0
    assert np.abs(mlp.softmax(z) - q).max() < 1e-15


def test_histogram_definition(orc):
    """Specular plate, Tx = Rx: every received path comes from the bins around
    boresight; the histogram mass equals #paths + 0.1 #(first hits on
    objects other than 0) -- here the plate is object 0, so only paths count."""
    R, r = 5.0, 0.25
    sc = sg.plate(R, 1.0, alpha=0.0)
    arr = sg.Array(np.array([[0, 0, 0.5]]), np.array([[0, 0, 0.5]]), r, sg.MODE_PER_TX)
    tp = sg.TraceParams(n_rays=200_000, max_bounces=2, seed=1)
    hits, paths = orc.trace(sc, arr, tp)
    H = orc.histogram(sc, arr, tp, hits, paths)
    assert abs(H.sum() - len(paths)) < 1e-9
    nz = np.nonzero(H)[0]
    ia, ie = nz % 128, nz // 128
    # theta_max = asin(r / 2R) = 1.43 deg; bins are 1.41 deg in azimuth
    assert np.all(np.abs(ia - 63.5) <= 2.5) and np.all(np.abs(ie - 31.5) <= 2.5)
    # a non-ground object adds 0.1 per ray whose first segment hits it
    sc2 = sg.plate(R, 1.0, alpha=0.0)
    sc2.tri_obj = np.array([0, 0], np.int32)
    sc2.obj_alpha = np.array([0.0, 0.0], np.float32)
    sc2.obj_vel = np.zeros((2, 3))
    sc2.tri_obj[:] = 1
    hits, paths = orc.trace(sc2, arr, tp)
    H = orc.histogram(sc2, arr, tp, hits, paths)
    n_hit = int((hits[:, 0] >= 0).sum())
    assert abs(H.sum() - (len(paths) + 0.1 * n_hit)) < 1e-6


def test_cost_aware_density_limits_and_optimality():
    """The cost-aware table: for a large ray cost it is the square-root
    table, for a vanishing one the uniform density, and in between it
    minimises variance x work, V(q) C(q) with V = sum_b x_b / q_b and
    C = kappa + sum_b q_b x_b: checked against the closed-form minimiser of a
    two-bin problem and against random perturbations on the simplex."""
    rng = np.random.default_rng(7)
    z = rng.normal(0, 2.0, mlp.N_BINS)
    q_sqrt = mlp.mixture(z, 0.0, 0.5)
    assert np.abs(mlp.mixture_cost(z, 0.0, 1e12) / q_sqrt - 1).max() < 1e-9
    assert np.abs(mlp.mixture_cost(z, 0.0, 1e-300) * mlp.N_BINS - 1).max() < 1e-12
    # two bins, x = (x1, x2): minimise (x1/q + x2/(1-q)) (k + q x1 + (1-q) x2) over q
    for x1, x2, k in ((3.0, 0.2, 0.5), (1.0, 4.0, 10.0), (0.01, 2.0, 0.001)):
        qs = np.linspace(1e-6, 1 - 1e-6, 2_000_001)
        f = (x1 / qs + x2 / (1 - qs)) * (k + qs * x1 + (1 - qs) * x2)
        q_best = qs[np.argmin(f)]
        d1, d2 = math.sqrt(x1 / (k + x1)), math.sqrt(x2 / (k + x2))
        assert abs(q_best - d1 / (d1 + d2)) < 2e-6
    # random perturbations of the full table never lower V C
    x = mlp.N_BINS * mlp.softmax(z)
    for kappa in (0.01, 1.0, 100.0):
        q = mlp.mixture_cost(z, 0.0, kappa)
        vc = lambda p: float(np.sum(x / p) * (kappa + np.sum(p * x)))
        base = vc(q)
        for _ in range(20):
            d = rng.normal(size=q.size) * q * 0.05
            d -= q * d.sum() / q.sum()
            assert vc(q + d) >= base * (1 - 1e-12)
