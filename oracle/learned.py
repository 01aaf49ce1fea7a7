"""FP64 oracle of the loading / window predictor's data path (test infrastructure only).

The paper fixes the loading and the window; these definitions belong to the predictor added
on top of it: the network input (training power profile), the decision rule mapping network
outputs to (loading, window), the sweep that labels training samples by output SINR, and
BF16 rounding of the weights.
"""

from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np

from . import bmvdr

PROFILE_BINS = 64
SWEEP_DELTAS = tuple(10.0 ** (-1.0 + 0.5 * i) for i in range(11))    # delta / sigma^2
SWEEP_WIDTHS = (5, 9, 17, 33)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def beam_bin(u: float) -> int:
    """Beamspace bin nearest the target's fractional beam position u: floor(u + 1/2)."""
    return int(math.floor(u + 0.5))


def power_profile(Yk_train: np.ndarray, u: float, noise_var: float) -> np.ndarray:
    """log10(P_j / sigma^2 + 1e-30), P_j = mean over training snapshots of |Y[c - 32 + j]|^2.

    Yk_train [M, L] is the beamspace of one subband over its training snapshots.
    """
    M = Yk_train.shape[0]
    c = beam_bin(u)
    bins = (c - PROFILE_BINS // 2 + np.arange(PROFILE_BINS)) % M
    P = np.mean(np.abs(Yk_train[bins]) ** 2, axis=1)
    return np.log10(P / noise_var + 1e-30)


def decision(out0: float, out1: float, noise_var: float, fb_win: int = 9,
             fb_delta: float = 10.0):
    """Network outputs -> (W, delta): delta = sigma^2 exp(clamp(out0, ln 0.1, ln 1e4)),
    W = 2^clamp(rint(out1), 2, 5) + 1; non-finite outputs give the fallback (fixed method)."""
    if not (math.isfinite(out0) and math.isfinite(out1)):
        return fb_win, fb_delta
    ld = min(max(out0, math.log(0.1)), math.log(1e4))
    lw = min(max(float(np.rint(out1)), 2.0), 5.0)
    return int(2 ** int(lw) + 1), noise_var * math.exp(ld)


def sweep_label(sinr_table: np.ndarray, deltas: Sequence[float], widths: Sequence[int],
                noise_var: float):
    """Best (loading, width) of one pair from sinr_table[id, iw]; ties go to the smaller width,
    then to the larger loading.  Returns (ln(delta / sigma^2), log2(W - 1))."""
    best, arg = -np.inf, None
    for iw in range(len(widths)):
        for idl in reversed(range(len(deltas))):
            if sinr_table[idl, iw] > best:
                best, arg = sinr_table[idl, iw], (idl, iw)
    idl, iw = arg
    return math.log(deltas[idl] / noise_var), math.log2(widths[iw] - 1)


def pair_sinr(w: np.ndarray, a: np.ndarray, bins: Sequence[int], N: int, M: int,
              jam_sin: Sequence[float], jam_inr: Sequence[float], ratio: float, dl: float,
              noise_var: float) -> float:
    """Output SINR of windowed weights w against the exact noise + jammer covariance."""
    R = bmvdr.interference_covariance(N, jam_sin, jam_inr, ratio, dl, noise_var)
    D = np.exp(-2j * np.pi * np.outer(np.asarray(bins, dtype=np.float64), np.arange(N)) / M)
    D /= math.sqrt(M)
    return bmvdr.sinr(w, a, D @ R @ D.conj().T)


def sweep(x: np.ndarray, *, M: int, K: int, L: int, Lt: int, sin_az: Sequence[float],
          jam_sin: Sequence[float], jam_inr: Sequence[float], noise_var: float = 1.0,
          beta: float = 0.2, dl: float = 0.5, subbands=None,
          deltas: Sequence[float] = SWEEP_DELTAS,
          widths: Sequence[int] = SWEEP_WIDTHS) -> Dict[str, np.ndarray]:
    """Features and labels of every (target, subband) pair by the plain method swept over
    loadings and widths (each run is :func:`bmvdr.windowed_mvdr`)."""
    N = x.shape[0]
    T = len(sin_az)
    ks = list(range(K)) if subbands is None else list(subbands)
    X = bmvdr.channelize(x, K) if subbands is None else bmvdr.channelize_bins(x, K, ks)
    ratio = bmvdr.subband_freq_ratio(K, beta)
    feat = np.zeros((T, len(ks), PROFILE_BINS))
    table = np.zeros((T, len(ks), len(deltas), len(widths)))
    for ik, k in enumerate(ks):
        col = k if subbands is None else ik
        Yk = bmvdr.beamspace(X[:, :L, col][:, :, None], M)[:, :, 0]
        for t in range(T):
            u = bmvdr.beam_position(float(sin_az[t]), float(ratio[k]), M, dl)
            feat[t, ik] = power_profile(Yk, u, noise_var)
    for iw, W in enumerate(widths):
        for idl, d in enumerate(deltas):
            res = bmvdr.windowed_mvdr(x, M=M, K=K, L=L, Lt=Lt, sin_az=sin_az, win=[W] * T,
                                      delta=d * noise_var, beta=beta, dl=dl,
                                      subbands=None if subbands is None else ks, X=None)
            for ik, k in enumerate(ks):
                for t in range(T):
                    bins = bmvdr.window_bins(int(res["start"][t, ik]), W, M)
                    table[t, ik, idl, iw] = pair_sinr(res["w"][t, ik, :W], res["a"][t, ik, :W],
                                                      bins, N, M, jam_sin, jam_inr, ratio[k], dl,
                                                      noise_var)
    labels = np.zeros((T, len(ks), 2))
    for t in range(T):
        for ik in range(len(ks)):
            labels[t, ik] = sweep_label(table[t, ik], deltas, widths, noise_var)
    return dict(feat=feat, table=table, labels=labels, subbands=np.asarray(ks))
