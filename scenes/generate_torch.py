"""Scene synthesis on the GPU with torch (for bulk training data of the loading/window predictor).

Same signal model as :mod:`scenes.generate` (per-subband Eq. 9 synthesis, inverse channelised
to time samples) and the same seeded geometry draws, but the waveforms and receiver noise come
from torch's device RNG seeded per scene, and everything runs in complex64 on the device.  It
holds none of the beamformer's arithmetic.
"""

from __future__ import annotations

import math

import numpy as np

from .configs import SceneConfig
from .generate import Scene, _draw_geometry, _lfm_block_spectra, subband_freq_ratio_gen


def make_scene_torch(cfg: SceneConfig, seed: int, device="cuda"):
    """Returns (Scene with x=None, x tensor [N, S] complex64 on ``device``)."""
    import torch

    taz, tsnr_db, jaz, jinr_db, win, delay = _draw_geometry(cfg, seed)
    tsnr = 10.0 ** (tsnr_db / 10.0)
    jinr = 10.0 ** (jinr_db / 10.0)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 7919 + 17)
    N, K, B = cfg.N, cfg.K, cfg.B
    n_src = cfg.T + cfg.n_jammers
    srng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 2])))
    G = torch.empty((n_src, B, K), dtype=torch.complex64, device=device)
    for t in range(cfg.T):
        alpha = np.exp(1j * srng.uniform(0.0, 2.0 * np.pi))
        spec = math.sqrt(tsnr[t]) * alpha * _lfm_block_spectra(cfg, int(delay[t]))
        G[t] = torch.from_numpy(spec.astype(np.complex64)).to(device)
    for j in range(cfg.n_jammers):
        g = torch.randn((B, K, 2), generator=gen, device=device) * math.sqrt(jinr[j] / 2.0)
        G[cfg.T + j] = torch.complex(g[..., 0], g[..., 1])
    ratio = torch.from_numpy(subband_freq_ratio_gen(K, cfg.beta, cfg.half_bin)).to(device)
    src_sin = torch.from_numpy(np.concatenate([np.sin(np.deg2rad(taz)),
                                               np.sin(np.deg2rad(jaz))])).to(device)
    Gk = G.permute(2, 0, 1).contiguous()                                  # [K, src, B]
    del G
    x = torch.empty((N, cfg.S), dtype=torch.complex64, device=device)
    tw = None
    if cfg.half_bin:
        tw = torch.polar(torch.ones(K, dtype=torch.float64, device=device),
                         math.pi * torch.arange(K, dtype=torch.float64, device=device) / K)
        tw = tw.to(torch.complex64)
    # element chunks of at most 2^27 complex samples bound the temporaries
    ec = max(1, min(N, (1 << 27) // (B * K)))
    for e0 in range(0, N, ec):
        e1 = min(N, e0 + ec)
        e_idx = torch.arange(e0, e1, dtype=torch.float64, device=device)
        ph = 2.0 * math.pi * cfg.dl * (ratio[:, None, None] * e_idx[None, :, None]) * src_sin[None, None, :]
        A = torch.polar(torch.ones_like(ph), ph).to(torch.complex64)        # [K, ec, src]
        Xc = torch.matmul(A, Gk).permute(1, 2, 0).contiguous()            # [ec, B, K]
        del A
        nz = torch.randn((e1 - e0, B, K, 2), generator=gen, device=device)
        nz *= math.sqrt(cfg.noise_var / 2.0)
        Xc += torch.view_as_complex(nz)
        del nz
        xc = torch.fft.ifft(Xc, dim=2, norm="ortho")
        del Xc
        if tw is not None:
            xc *= tw
        x[e0:e1] = xc.reshape(e1 - e0, cfg.S)
        del xc
    sc = Scene(cfg=cfg, seed=seed, x=None, target_az=np.deg2rad(taz), target_snr=tsnr,
               target_delay=delay, jammer_az=np.deg2rad(jaz), jammer_inr=jinr, win=win)
    return sc, x
