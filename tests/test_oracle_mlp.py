"""Pins of the predictor network oracle: GELU against the normal CDF, gradients against
central finite differences, Adam's first three steps against Kingma & Ba's Algorithm 1
unrolled by hand, and its bias correction against the constant-gradient invariant."""

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


def test_adam_three_steps_match_unrolled_algorithm():
    # Algorithm 1 of Kingma & Ba with beta1 = 0.9, beta2 = 0.999 and zero initial moments,
    # unrolled: m_t = sum_i (1 - b1) b1^(t-i) g_i, v_t = sum_i (1 - b2) b2^(t-i) g_i^2,
    # p_t = p_(t-1) - lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps)
    p = _params(4)
    gs = [_params(5 + i) for i in range(3)]
    lr, eps = 2e-3, 1e-8
    m = {k: np.zeros_like(a) for k, a in p.items()}
    v = {k: np.zeros_like(a) for k, a in p.items()}
    expect = {k: a.copy() for k, a in p.items()}
    mcoef = [[0.1], [0.09, 0.1], [0.081, 0.09, 0.1]]
    vcoef = [[1e-3], [0.999e-3, 1e-3], [0.998001e-3, 0.999e-3, 1e-3]]
    c1 = [0.1, 0.19, 0.271]
    c2 = [1e-3, 1.999e-3, 2.997001e-3]
    for t in range(3):
        mlp.adam_step(p, gs[t], m, v, step=t + 1, lr=lr)
        for k in p:
            mt = sum(c * gs[i][k] for i, c in enumerate(mcoef[t]))
            vt = sum(c * gs[i][k] ** 2 for i, c in enumerate(vcoef[t]))
            expect[k] = expect[k] - lr * (mt / c1[t]) / (np.sqrt(vt / c2[t]) + eps)
            assert np.allclose(p[k], expect[k], rtol=1e-12, atol=1e-14), (t, k)


def test_adam_bias_correction_with_constant_gradient():
    # with the same gradient every step, the corrected moments are exactly g and g^2, so
    # every step (not only the first) moves each weight by lr g / (|g| + eps)
    p = _params(8)
    g = _params(9)
    m = {k: np.zeros_like(a) for k, a in p.items()}
    v = {k: np.zeros_like(a) for k, a in p.items()}
    lr = 1e-3
    for step in range(1, 6):
        before = {k: a.copy() for k, a in p.items()}
        mlp.adam_step(p, g, m, v, step=step, lr=lr)
        for k in p:
            assert np.allclose(before[k] - p[k], lr * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-9,
                               atol=1e-15), (step, k)
