"""Scene synthesis (see the package docstring for the signal model)."""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from .configs import SceneConfig


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def subband_freq_ratio_gen(K: int, beta: float, half_bin: bool) -> np.ndarray:
    """f_k / f_c for every FFT bin k (Eq. 1 with half_bin, plain bins otherwise).

    Bin k stands for the signed frequency index ks = k (k < K/2) or k - K.
    """
    k = np.arange(K)
    ks = np.where(k < K // 2, k, k - K).astype(np.float64)
    off = 0.5 if half_bin else 0.0
    return 1.0 + beta * (ks + off) / K


@dataclasses.dataclass
class Scene:
    cfg: SceneConfig
    seed: int
    x: np.ndarray               # [N, S] element time samples, S = (L + Lt) * K
    target_az: np.ndarray       # [T] radians from broadside
    target_snr: np.ndarray      # [T] linear, per element
    target_delay: np.ndarray    # [T] samples
    jammer_az: np.ndarray       # [J] radians
    jammer_inr: np.ndarray      # [J] linear, per element
    win: np.ndarray             # [T] int32 window widths

    @property
    def sin_az(self) -> np.ndarray:
        return np.array([math.sin(a) for a in self.target_az], dtype=np.float64)


def _draw_geometry(cfg: SceneConfig, seed: int):
    rng = _rng(seed, 0)
    T, J = cfg.T, cfg.n_jammers
    lo, hi = cfg.az_range_deg
    if cfg.target_az_deg is not None:
        taz = np.asarray(cfg.target_az_deg, dtype=np.float64)
    else:
        taz = rng.uniform(lo, hi, size=T)
    if cfg.target_snr_db is not None:
        tsnr = np.asarray(cfg.target_snr_db, dtype=np.float64)
    else:
        tsnr = rng.uniform(*cfg.snr_range_db, size=T)
    tsin = np.sin(np.deg2rad(taz))
    if cfg.jammer_az_deg is not None:
        jaz = np.asarray(cfg.jammer_az_deg, dtype=np.float64)
    else:
        jaz = np.empty(J)
        for j in range(J):
            while True:
                a = rng.uniform(lo, hi)
                if np.all(np.abs(math.sin(math.radians(a)) - tsin) >= 2.0 / cfg.N):
                    jaz[j] = a
                    break
    if cfg.jammer_inr_db is not None:
        jinr = np.asarray(cfg.jammer_inr_db, dtype=np.float64)
    else:
        jinr = rng.uniform(*cfg.inr_range_db, size=J)
    if cfg.W is not None:
        win = np.full(T, cfg.W, dtype=np.int32)
    else:
        win = rng.choice(np.asarray(cfg.W_choices, dtype=np.int32), size=T).astype(np.int32)
    P = 4 * cfg.K
    delay = rng.integers(0, P, size=T)
    return taz, tsnr, jaz, jinr, win, delay


def _lfm_block_spectra(cfg: SceneConfig, delay: int) -> np.ndarray:
    """Unit-power baseband LFM, delayed, cut into blocks, unitary DFT per block -> [B, K]."""
    P = 4 * cfg.K
    t = (np.arange(cfg.S, dtype=np.int64) - int(delay)) % P
    tf = t.astype(np.float64)
    p = np.exp(1j * np.pi * (tf * tf / P - tf))
    return np.fft.fft(p.reshape(cfg.B, cfg.K), axis=1, norm="ortho")


def make_scene(cfg: SceneConfig, seed: Optional[int] = None,
               complex128: Optional[bool] = None, chunk_bytes: int = 256 << 20) -> Scene:
    """Build one seeded scene for ``cfg`` (``seed`` overrides ``cfg.seed``)."""
    seed = cfg.seed if seed is None else int(seed)
    c128 = cfg.complex128 if complex128 is None else complex128
    N, K, B = cfg.N, cfg.K, cfg.B
    taz, tsnr_db, jaz, jinr_db, win, delay = _draw_geometry(cfg, seed)
    tsnr = 10.0 ** (tsnr_db / 10.0)
    jinr = 10.0 ** (jinr_db / 10.0)

    # Source waveforms in the block/subband domain: G[src, b, k].
    srng = _rng(seed, 2)
    n_src = cfg.T + cfg.n_jammers
    G = np.empty((n_src, B, K), dtype=np.complex128)
    for t in range(cfg.T):
        alpha = np.exp(1j * srng.uniform(0.0, 2.0 * np.pi))
        G[t] = math.sqrt(tsnr[t]) * alpha * _lfm_block_spectra(cfg, int(delay[t]))
    for j in range(cfg.n_jammers):
        g = srng.standard_normal((B, K, 2))
        G[cfg.T + j] = (g[..., 0] + 1j * g[..., 1]) * math.sqrt(jinr[j] / 2.0)
    Gk = np.ascontiguousarray(G.transpose(2, 0, 1))          # [K, src, B]

    ratio = subband_freq_ratio_gen(K, cfg.beta, cfg.half_bin)      # [K]
    src_sin = np.concatenate([np.sin(np.deg2rad(taz)), np.sin(np.deg2rad(jaz))])
    e_idx = np.arange(N, dtype=np.float64)

    out_dtype = np.complex128 if c128 else np.complex64
    x = np.empty((N, cfg.S), dtype=out_dtype)
    per_elem = B * K * 16
    ec = max(1, min(N, chunk_bytes // per_elem))
    half_tw = np.exp(1j * np.pi * np.arange(K) / K) if cfg.half_bin else None
    nstd = math.sqrt(cfg.noise_var / 2.0)
    for e0 in range(0, N, ec):
        e1 = min(N, e0 + ec)
        # steering of every source at every subband for these elements: [K, ec, src]
        ph = 2.0 * np.pi * cfg.dl * (ratio[:, None, None] * e_idx[None, e0:e1, None]) * src_sin[None, None, :]
        A = np.exp(1j * ph)
        Xc = np.matmul(A, Gk)                                   # [K, ec, B]
        Xc = np.ascontiguousarray(Xc.transpose(1, 2, 0))        # [ec, B, K]
        for e in range(e0, e1):
            nz = _rng(seed, 1, e).standard_normal((B, K, 2))
            Xc[e - e0] += (nz[..., 0] + 1j * nz[..., 1]) * nstd
        xc = np.fft.ifft(Xc, axis=2, norm="ortho")
        if half_tw is not None:
            xc *= half_tw[None, None, :]
        x[e0:e1] = xc.reshape(e1 - e0, cfg.S)
    return Scene(cfg=cfg, seed=seed, x=x,
                 target_az=np.deg2rad(taz), target_snr=tsnr, target_delay=delay,
                 jammer_az=np.deg2rad(jaz), jammer_inr=jinr, win=win)
