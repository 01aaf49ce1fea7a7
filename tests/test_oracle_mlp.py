"""Pins of the predictor network oracle: GELU against the normal CDF, gradients against
central finite differences, Adam's first step against its closed form."""

import numpy as np
from scipy.stats import norm

from oracle import mlp


def _params(seed, scale=0.3):
    r = np.random.default_rng(seed)
    return {k: r.standard_normal(s) * scale for k, s in mlp.PARAM_SHAPES.items()}


def test_param_count():
    assert mlp.N_PARAMS == 25090


def test_gelu_is_x_times_normal_cdf():
    a = np.linspace(-6, 6, 101)
    assert np.max(np.abs(mlp.gelu(a) - a * norm.cdf(a))) < 1e-14
    h = 1e-6
    fd = (mlp.gelu(a + h) - mlp.gelu(a - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(a))) < 1e-8


def test_gradients_match_finite_differences():
    p = _params(0)
    r = np.random.default_rng(1)
    x = r.standard_normal((5, mlp.IN))
    y = r.standard_normal((5, mlp.OUT))
    g = mlp.backward(p, x, y)
    flat = mlp.flatten(p)
    gflat = mlp.flatten(g)
    idx = r.choice(flat.size, size=60, replace=False)
    h = 1e-6
    for i in idx:
        fp = flat.copy(); fp[i] += h
        fm = flat.copy(); fm[i] -= h
        fd = (mlp.loss(mlp.unflatten(fp), x, y) - mlp.loss(mlp.unflatten(fm), x, y)) / (2 * h)
        assert abs(fd - gflat[i]) < 1e-7 * max(1.0, abs(fd)), i


def test_adam_first_step_moves_by_lr_sign():
    p = _params(2)
    g = _params(3)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    p0 = {k: a.copy() for k, a in p.items()}
    lr = 1e-3
    mlp.adam_step(p, g, m, v, step=1, lr=lr)
    for k in p:
        # m^ = g, v^ = g^2  ->  step = lr g / (|g| + eps)
        assert np.allclose(p0[k] - p[k], lr * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12, atol=1e-15)
