"""Training and use of the loading / window predictor (an addition to the paper's method).

Every step runs in the library's kernels through the C ABI: the power profiles, the windowed
MVDR of every swept (loading, width), its SINR against the scene's exact interference
covariance, the label argmax, the network's forward / backward passes and the Adam update.
Python only sequences the calls and draws the random numbers (initial weights, minibatch
order) that are passed in.
"""

from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

from . import MLP_PARAMS, Mlp, Plan

SWEEP_DELTAS = tuple(10.0 ** (-1.0 + 0.5 * i) for i in range(11))   # loading / noise power
SWEEP_WIDTHS = (5, 9, 17, 33)
GATHER_WIDTH = 33


def init_params(seed: int) -> np.ndarray:
    """He-uniform initial weights, zero biases, flat in the C ABI's parameter order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, fan_out in ((64, 128), (128, 128), (128, 2)):
        lim = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=(fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == MLP_PARAMS
    return p


def label_sweep(plan: Plan, mlp: Mlp, x, az_rad: Sequence[float], jam_az: Sequence[float],
                jam_inr: Sequence[float], noise_power: float = 1.0,
                deltas: Sequence[float] = SWEEP_DELTAS,
                widths: Sequence[int] = SWEEP_WIDTHS) -> Dict[str, object]:
    """Features [T*K, 64] and labels [T*K, 2] of one scene, plus the SINR table
    [len(deltas)*len(widths), T*K] of the swept plain method (row = id * nw + iw)."""
    import torch
    T, K = len(az_rad), plan.K
    dev = plan.device
    feat = plan.profiles(x, az_rad, noise_power).reshape(T * K, 64)
    win = [GATHER_WIDTH] * T
    table = torch.empty((len(deltas) * len(widths), T * K), dtype=torch.float32, device=dev)
    pw = torch.empty((T, K), dtype=torch.int32, device=dev)
    pd = torch.empty((T, K), dtype=torch.float32, device=dev)
    for iw, W in enumerate(widths):
        pw.fill_(int(W))
        for idl, d in enumerate(deltas):
            pd.fill_(float(d * noise_power))
            res = plan.beamform_pairs(x, az_rad, win, pw, pd)
            s = plan.sinr(az_rad, win, res["weights"], res["starts"], jam_az, jam_inr,
                          noise_power, pair_win=pw)
            table[idl * len(widths) + iw] = s.reshape(-1)
    labels = mlp.sweep_labels(table, deltas, widths, noise_power)
    return dict(feat=feat, labels=labels, table=table)


def train(mlp: Mlp, params, feats, labels, *, epochs: int, batch: int, lr: float, seed: int,
          log=None) -> List[float]:
    """Adam on the mean squared error; minibatch order from a seeded device permutation."""
    import torch
    n = int(feats.shape[0])
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    gen = torch.Generator(device=params.device)
    gen.manual_seed(int(seed))
    step = 0
    hist = []
    grad = torch.empty_like(params)
    loss = torch.empty((1,), dtype=torch.float32, device=params.device)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen, device=params.device)
        tot, nb = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            mlp.grad(params, feats[idx].contiguous(), labels[idx].contiguous(), grad, loss)
            step += 1
            mlp.adam(params, m, v, grad, step, lr)
            if nb % 50 == 0:
                tot += float(loss.item())
            nb += 1
        hist.append(tot / max(1, (nb + 49) // 50))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.4f}")
    return hist


def save_params(path: str, params) -> None:
    np.savez(path, params=params.detach().cpu().numpy().astype(np.float32))


def load_params(path: str) -> np.ndarray:
    with np.load(path, allow_pickle=False) as f:
        p = np.asarray(f["params"], dtype=np.float32)
    if p.size != MLP_PARAMS:
        raise ValueError(f"{path}: expected {MLP_PARAMS} parameters, found {p.size}")
    return p
