"""FP64 oracle of the loading/window predictor network (test infrastructure only).

A multilayer perceptron 64 -> 128 -> 128 -> 2 with GELU (exact, erf form)
after each hidden layer.  Input: the 64-bin beamspace power profile of one
(target, subband) pair (log10 of power over noise power, i.e. dB / 10).
Outputs: out0 = ln(delta / sigma^2) and out1 = log2(W - 1).  Loss: mean
squared error over the batch and both outputs.  Optimiser: Adam.

The paper has no such network; its shape, inputs and outputs are those of the
loading/window predictor this library adds to the method.  Parity pin: the
analytic gradients are checked against central finite differences of the
loss, and GELU against scipy's normal CDF.
"""

from __future__ import annotations

import math
from typing import Dict

import numpy as np
from scipy.special import erf

IN, H1, H2, OUT = 64, 128, 128, 2
PARAM_SHAPES = {"W1": (H1, IN), "b1": (H1,), "W2": (H2, H1), "b2": (H2,),
                "W3": (OUT, H2), "b3": (OUT,)}
PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")
N_PARAMS = sum(int(np.prod(s)) for s in PARAM_SHAPES.values())


def gelu(a: np.ndarray) -> np.ndarray:
    """a * Phi(a) with Phi the standard normal CDF."""
    return 0.5 * a * (1.0 + erf(a / math.sqrt(2.0)))


def gelu_grad(a: np.ndarray) -> np.ndarray:
    """d/da [a Phi(a)] = Phi(a) + a phi(a)."""
    return 0.5 * (1.0 + erf(a / math.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


def forward(p: Dict[str, np.ndarray], x: np.ndarray) -> Dict[str, np.ndarray]:
    """Forward pass; returns the pre-activations and activations of every layer."""
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = gelu(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(a2)
    out = h2 @ p["W3"].T + p["b3"]
    return dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, out=out)


def loss(p: Dict[str, np.ndarray], x: np.ndarray, y: np.ndarray) -> float:
    out = forward(p, x)["out"]
    return float(np.mean((out - np.asarray(y, dtype=np.float64)) ** 2))


def backward(p: Dict[str, np.ndarray], x: np.ndarray, y: np.ndarray) -> Dict[str, np.ndarray]:
    """Gradients of :func:`loss` with respect to every parameter (chain rule, layer by layer)."""
    f = forward(p, x)
    n = f["x"].shape[0]
    d_out = 2.0 * (f["out"] - np.asarray(y, dtype=np.float64)) / (n * OUT)
    g = {}
    g["W3"] = d_out.T @ f["h2"]
    g["b3"] = d_out.sum(axis=0)
    d_a2 = (d_out @ p["W3"]) * gelu_grad(f["a2"])
    g["W2"] = d_a2.T @ f["h1"]
    g["b2"] = d_a2.sum(axis=0)
    d_a1 = (d_a2 @ p["W2"]) * gelu_grad(f["a1"])
    g["W1"] = d_a1.T @ f["x"]
    g["b1"] = d_a1.sum(axis=0)
    return g


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) in place on p, m, v; ``step`` starts at 1."""
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    for k in PARAM_ORDER:
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        p[k] = p[k] - lr * (m[k] / c1) / (np.sqrt(v[k] / c2) + eps)


def flatten(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in PARAM_ORDER])


def unflatten(flat: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(PARAM_SHAPES[k]))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(PARAM_SHAPES[k])
        o += n
    return out
