"""Seeded scenes for a uniform planar array (UPA), the two-dimensional geometry of Sec. II-A.

Inputs only, like :mod:`scenes.generate`: element-space IQ samples, no beamformer arithmetic.
The array has Nz rows (vertical, z) and Nx columns (horizontal, x) at spacing d; element
(iz, ix) is row n = ix * Nz + iz of the sample matrix (the vectorisation of Eq. 6, where the
z index runs fastest).  A source at azimuth az and elevation el (both from broadside, Sec.
II-A) adds, in subband k,

    X[n, b, k] += exp(j 2 pi (d/lambda_c) (f_k/f_c) (ix cos(el) sin(az) + iz sin(el))) g[b, k]

with the same waveforms as the linear-array scenes: LFM returns for targets, wideband white
Gaussian jammers, CN(0, sigma^2) receiver noise, and time samples obtained by the inverse
unitary K-point DFT of every block.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

from .generate import _lfm_block_spectra, _rng, subband_freq_ratio_gen


@dataclasses.dataclass(frozen=True)
class UpaSceneConfig:
    name: str
    Nz: int                     # vertical elements
    Nx: int                     # horizontal elements
    Mz: int                     # vertical spatial FFT size (power of two, >= Nz)
    Mx: int                     # horizontal spatial FFT size (power of two, >= Nx)
    K: int                      # subbands
    L: int
    Lt: int
    T: int
    windows: Tuple[Tuple[int, int], ...] = ((2, 4), (4, 4), (4, 8))   # (Wz, Wx) choices
    beta: float = 0.2
    dl: float = 0.5
    half_bin: bool = False
    noise_var: float = 1.0
    loading_factor: float = 10.0
    n_jammers: int = 0
    target_dir_deg: Optional[Sequence[Tuple[float, float]]] = None   # fixed (az, el) per target
    target_snr_db: Optional[Sequence[float]] = None
    jammer_dir_deg: Optional[Sequence[Tuple[float, float]]] = None
    jammer_inr_db: Optional[Sequence[float]] = None
    target_az_deg: Tuple[float, float] = (-60.0, 60.0)
    target_el_deg: Tuple[float, float] = (0.0, 30.0)
    jammer_az_deg: Tuple[float, float] = (-60.0, 60.0)
    jammer_el_deg: Tuple[float, float] = (-30.0, -2.0)
    snr_range_db: Tuple[float, float] = (-10.0, 10.0)
    inr_range_db: Tuple[float, float] = (20.0, 50.0)
    seed: int = 0
    complex128: bool = False

    @property
    def N(self) -> int:
        return self.Nz * self.Nx

    @property
    def M(self) -> int:
        return self.Mz * self.Mx

    @property
    def B(self) -> int:
        return self.L + self.Lt

    @property
    def S(self) -> int:
        return self.B * self.K

    @property
    def delta(self) -> float:
        return self.loading_factor * self.noise_var

    @property
    def wmax(self) -> int:
        return max(wz * wx for wz, wx in self.windows)

    def replace(self, **kw) -> "UpaSceneConfig":
        return dataclasses.replace(self, **kw)


# The array of the paper's evaluation (4 x 32 elements, 128 subbands, 20 targets) with its
# largest beamspace grid (8 x 64) and its three window shapes.
UPA = UpaSceneConfig(name="upa", Nz=4, Nx=32, Mz=8, Mx=64, K=128, L=256, Lt=256, T=20,
                     n_jammers=6, seed=6)
UPA_SMALL = UpaSceneConfig(name="upa_small", Nz=2, Nx=8, Mz=4, Mx=16, K=8, L=48, Lt=16, T=2,
                           windows=((2, 3), (1, 5)), n_jammers=1, seed=7, complex128=True)
UPA_CONFIGS = {c.name: c for c in (UPA, UPA_SMALL)}


@dataclasses.dataclass
class UpaScene:
    cfg: UpaSceneConfig
    seed: int
    x: np.ndarray               # [N, S], row n = ix * Nz + iz
    target_az: np.ndarray       # [T] radians
    target_el: np.ndarray       # [T] radians
    target_snr: np.ndarray      # [T] linear
    jammer_az: np.ndarray
    jammer_el: np.ndarray
    jammer_inr: np.ndarray
    win_z: np.ndarray           # [T] int32
    win_x: np.ndarray           # [T] int32


def make_upa_scene(cfg: UpaSceneConfig, seed: Optional[int] = None) -> UpaScene:
    seed = cfg.seed if seed is None else int(seed)
    rng = _rng(seed, 10)
    T, J = cfg.T, cfg.n_jammers
    if cfg.target_dir_deg is not None:
        tdir = np.asarray(cfg.target_dir_deg, dtype=np.float64).reshape(T, 2)
    else:
        tdir = np.stack([rng.uniform(*cfg.target_az_deg, size=T),
                         rng.uniform(*cfg.target_el_deg, size=T)], axis=1)
    tsnr_db = (np.asarray(cfg.target_snr_db, dtype=np.float64) if cfg.target_snr_db is not None
               else rng.uniform(*cfg.snr_range_db, size=T))
    if cfg.jammer_dir_deg is not None:
        jdir = np.asarray(cfg.jammer_dir_deg, dtype=np.float64).reshape(J, 2)
    else:
        jdir = np.stack([rng.uniform(*cfg.jammer_az_deg, size=J),
                         rng.uniform(*cfg.jammer_el_deg, size=J)], axis=1)
    jinr_db = (np.asarray(cfg.jammer_inr_db, dtype=np.float64) if cfg.jammer_inr_db is not None
               else rng.uniform(*cfg.inr_range_db, size=J))
    pick = rng.integers(0, len(cfg.windows), size=T)
    win_z = np.array([cfg.windows[i][0] for i in pick], dtype=np.int32)
    win_x = np.array([cfg.windows[i][1] for i in pick], dtype=np.int32)
    delay = rng.integers(0, 4 * cfg.K, size=T)

    tsnr = 10.0 ** (tsnr_db / 10.0)
    jinr = 10.0 ** (jinr_db / 10.0)
    N, K, B = cfg.N, cfg.K, cfg.B
    srng = _rng(seed, 12)
    n_src = T + J
    G = np.empty((n_src, B, K), dtype=np.complex128)
    for t in range(T):
        alpha = np.exp(1j * srng.uniform(0.0, 2.0 * np.pi))
        G[t] = math.sqrt(tsnr[t]) * alpha * _lfm_block_spectra(cfg, int(delay[t]))
    for j in range(J):
        g = srng.standard_normal((B, K, 2))
        G[T + j] = (g[..., 0] + 1j * g[..., 1]) * math.sqrt(jinr[j] / 2.0)
    Gk = np.ascontiguousarray(G.transpose(2, 0, 1))                 # [K, src, B]

    az = np.deg2rad(np.concatenate([tdir[:, 0], jdir[:, 0]]))
    el = np.deg2rad(np.concatenate([tdir[:, 1], jdir[:, 1]]))
    cx = np.cos(el) * np.sin(az)                                    # direction cosine along x
    cz = np.sin(el)                                                 # along z
    n = np.arange(N)
    ix, iz = (n // cfg.Nz).astype(np.float64), (n % cfg.Nz).astype(np.float64)
    pos = ix[:, None] * cx[None, :] + iz[:, None] * cz[None, :]     # [N, src]
    ratio = subband_freq_ratio_gen(K, cfg.beta, cfg.half_bin)
    A = np.exp(1j * 2.0 * np.pi * cfg.dl * ratio[:, None, None] * pos[None, :, :])   # [K, N, src]
    X = np.ascontiguousarray(np.matmul(A, Gk).transpose(1, 2, 0))   # [N, B, K]
    nstd = math.sqrt(cfg.noise_var / 2.0)
    for e in range(N):
        nz = _rng(seed, 11, e).standard_normal((B, K, 2))
        X[e] += (nz[..., 0] + 1j * nz[..., 1]) * nstd
    xt = np.fft.ifft(X, axis=2, norm="ortho")
    if cfg.half_bin:
        xt *= np.exp(1j * np.pi * np.arange(K) / K)[None, None, :]
    x = xt.reshape(N, cfg.S).astype(np.complex128 if cfg.complex128 else np.complex64)
    return UpaScene(cfg=cfg, seed=seed, x=x, target_az=np.deg2rad(tdir[:, 0]),
                    target_el=np.deg2rad(tdir[:, 1]), target_snr=tsnr,
                    jammer_az=np.deg2rad(jdir[:, 0]), jammer_el=np.deg2rad(jdir[:, 1]),
                    jammer_inr=jinr, win_z=win_z, win_x=win_x)
