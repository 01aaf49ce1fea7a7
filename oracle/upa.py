"""Windowed beamspace MVDR on a uniform planar array -- FP64 oracle, TEST INFRASTRUCTURE ONLY.

The paper's own geometry (Sec. II-A, Sec. III-B): Nz x Nx elements, a zero-padded Mz x Mx
spatial DFT and a Wz x Wx window around the target's beam.  Everything else (channelizer,
covariance with loading, MVDR correlator, output) is the one-dimensional oracle's.

Vectorisation, as the Kronecker products of the paper fix it:
* element (iz, ix) is entry n = ix * Nz + iz of y (a = a_x kron a_z, Eq. 6);
* beam (mz, mx) is entry m = mx * Mz + mz of D y (D = D_h^T kron D_v, Eq. 16);
* window cell (iz_w, ix_w) is entry i = ix_w * Wz + iz_w of the windowed vector (Eq. 18).

Readings (also listed in the design notes):
* Eq. 18 writes the selector as S_h^T kron S_v with S_h of size Wx x Mx, which would not be
  W x M; it is read, like D_h (defined Nx x Mx and used transposed), as the Wx x Mx selector
  of the horizontal bins, so S selects the Wz x Wx block of beams with z fastest.
* Per axis the window is placed as on the linear array: u_z = Mz (d/lambda_c) sin(el) f_k/f_c,
  u_x = Mx (d/lambda_c) cos(el) sin(az) f_k/f_c (the beam positions of the spatial
  frequencies of Eq. 2-5), start s = floor(u - (W-1)/2 + 1/2), bins taken modulo the axis'
  FFT size.  The direction cosines are evaluated as cos(el) * sin(az) and sin(el) in float64.
"""

from __future__ import annotations

import math
from typing import Dict, Optional, Sequence

import numpy as np

from .bmvdr import (beam_output, channelize, channelize_bins, mvdr_weights, sample_covariance,
                    subband_freq_ratio, window_start)

__all__ = ["upa_direction_cosines", "upa_spatial_frequencies", "upa_steering",
           "upa_dft_matrix", "upa_beamspace", "upa_beam_position", "upa_window_rows",
           "upa_lift_correlator", "upa_beam_pattern", "upa_windowed_mvdr", "upa_full_mvdr"]


def upa_direction_cosines(az: float, el: float):
    """(cos(el) sin(az), sin(el)): the x and z components of the arrival direction (Sec. II-A)."""
    return math.cos(el) * math.sin(az), math.sin(el)


def upa_spatial_frequencies(az: float, el: float, ratio: float, dl: float = 0.5):
    """(Omega_z, Omega_x) at a subband: Eq. 2-5 with pi -> 2 pi d/lambda_c (pi at d = lambda/2)."""
    cx, cz = upa_direction_cosines(az, el)
    return 2.0 * math.pi * dl * cz * ratio, 2.0 * math.pi * dl * cx * ratio


def upa_steering(Nz: int, Nx: int, omega_z: float, omega_x: float) -> np.ndarray:
    """a = a_x(Omega_x) kron a_z(Omega_z)  (Eq. 6-8)."""
    az_ = np.exp(1j * omega_z * np.arange(Nz, dtype=np.float64))
    ax_ = np.exp(1j * omega_x * np.arange(Nx, dtype=np.float64))
    return np.kron(ax_, az_)


def upa_dft_matrix(Nz: int, Nx: int, Mz: int, Mx: int) -> np.ndarray:
    """D = D_h^T kron D_v  (Eq. 14-16), with D_v [Mz x Nz] and D_h [Nx x Mx] entry by entry."""
    Dv = np.exp(-2j * np.pi * np.outer(np.arange(Mz), np.arange(Nz)) / Mz) / math.sqrt(Mz)
    Dh = np.exp(-2j * np.pi * np.outer(np.arange(Nx), np.arange(Mx)) / Mx) / math.sqrt(Mx)
    return np.kron(Dh.T, Dv)


def upa_beamspace(X: np.ndarray, Nz: int, Mz: int, Mx: int) -> np.ndarray:
    """y^ = D y (Eq. 17) for every column: X[N, ...] -> Y[Mz*Mx, ...].

    Computed as the two zero-padded one-dimensional DFTs the Kronecker product factors into:
    along x (length Mx) and along z (length Mz), unitary scale.
    """
    N = X.shape[0]
    Nx = N // Nz
    assert Nz * Nx == N and Mz >= Nz and Mx >= Nx
    rest = X.shape[1:]
    Xr = np.asarray(X, dtype=np.complex128).reshape(Nx, Nz, *rest)       # [ix, iz, ...]
    Yr = np.fft.fft(np.fft.fft(Xr, n=Mx, axis=0), n=Mz, axis=1) / math.sqrt(Mx * Mz)
    return Yr.reshape(Mx * Mz, *rest)                                    # m = mx * Mz + mz


def upa_beam_position(az: float, el: float, ratio: float, Mz: int, Mx: int, dl: float = 0.5):
    """Fractional beam position (u_z, u_x) on the Mz x Mx grid, in the evaluation order
    ``((M * dl) * c) * ratio`` of the linear array."""
    cx, cz = upa_direction_cosines(az, el)
    return ((float(Mz) * dl) * cz) * ratio, ((float(Mx) * dl) * cx) * ratio


def upa_window_rows(sz: int, sx: int, Wz: int, Wx: int, Mz: int, Mx: int) -> np.ndarray:
    """Beam indices selected by S (Eq. 18-19): entry i = ix_w * Wz + iz_w is beam
    ((sx + ix_w) mod Mx) * Mz + (sz + iz_w) mod Mz."""
    iz = np.arange(Wz)
    ix = np.arange(Wx)
    return (((sx + ix[:, None]) % Mx) * Mz + (sz + iz[None, :]) % Mz).reshape(-1)


def upa_lift_correlator(w: np.ndarray, rows: Sequence[int], Nz: int, Nx: int, Mz: int,
                        Mx: int) -> np.ndarray:
    """Antenna-space equivalent correlator c^ = D^H S^T c~  (Eq. 21)."""
    D = upa_dft_matrix(Nz, Nx, Mz, Mx)
    return D[np.asarray(rows)].conj().T @ w


def upa_beam_pattern(c: np.ndarray, Nz: int, omegas) -> np.ndarray:
    """Cosine similarity |<c, a(Omega_z, Omega_x)>| / (||c|| ||a||) over (Omega_z, Omega_x)
    pairs (Eq. 22 with the planar steering vector of Eq. 6), one value per pair."""
    N = c.shape[0]
    Nx = N // Nz
    out = np.empty(len(omegas))
    for q, (omz, omx) in enumerate(omegas):
        a = upa_steering(Nz, Nx, float(omz), float(omx))
        out[q] = abs(np.vdot(c, a)) / (np.linalg.norm(c) * np.linalg.norm(a))
    return out


def upa_windowed_mvdr(x: np.ndarray, *, Nz: int, Mz: int, Mx: int, K: int, L: int, Lt: int,
                      az: Sequence[float], el: Sequence[float], win_z: Sequence[int],
                      win_x: Sequence[int], delta: float, beta: float = 0.2, dl: float = 0.5,
                      half_bin: bool = False, subbands: Optional[Sequence[int]] = None,
                      return_windows: bool = False) -> Dict[str, np.ndarray]:
    """Windowed beamspace MVDR on the planar array for every (target, subband) pair.

    Per subband: channelize (Sec. III-A) -> 2-D beamspace (Eq. 16-17) -> Wz x Wx window
    (Eq. 18-19) -> loaded covariance of the first L snapshots (Eq. 11) -> correlator (Eq. 20)
    with a~ = S D a (a of Eq. 6) -> output on the next Lt snapshots.

    Returns ``start`` [T, nk, 2] (s_z, s_x), ``u`` [T, nk, 2], ``rows`` (list of lists),
    ``w`` and ``a`` [T, nk, Wmax] zero padded, ``z`` [T, nk, Lt], and with ``return_windows``
    the loaded covariances ``R`` and windowed snapshots ``Yw`` [W, L + Lt] (lists of lists).
    """
    N = x.shape[0]
    Nx = N // Nz
    T = len(az)
    wz = [int(v) for v in win_z]
    wx = [int(v) for v in win_x]
    Wmax = max(a * b for a, b in zip(wz, wx))
    ks = list(range(K)) if subbands is None else [int(k) for k in subbands]
    X = channelize(x, K, half_bin) if subbands is None else channelize_bins(x, K, ks, half_bin)
    kcol = {k: (k if subbands is None else i) for i, k in enumerate(ks)}
    ratio = subband_freq_ratio(K, beta, half_bin)
    nk = len(ks)
    start = np.zeros((T, nk, 2), dtype=np.int64)
    upos = np.zeros((T, nk, 2))
    w_out = np.zeros((T, nk, Wmax), dtype=np.complex128)
    a_out = np.zeros((T, nk, Wmax), dtype=np.complex128)
    z_out = np.zeros((T, nk, Lt), dtype=np.complex128)
    rows_out = [[None] * nk for _ in range(T)]
    R_out = [[None] * nk for _ in range(T)]
    Yw_out = [[None] * nk for _ in range(T)]
    for ik, k in enumerate(ks):
        Yk = upa_beamspace(X[:, :L + Lt, kcol[k]], Nz, Mz, Mx)            # [M, B]
        for t in range(T):
            uz, ux = upa_beam_position(float(az[t]), float(el[t]), float(ratio[k]), Mz, Mx, dl)
            sz, sx = window_start(uz, wz[t]), window_start(ux, wx[t])
            rows = upa_window_rows(sz, sx, wz[t], wx[t], Mz, Mx)
            Yw = Yk[rows]
            om_z, om_x = upa_spatial_frequencies(float(az[t]), float(el[t]), float(ratio[k]), dl)
            a = upa_beamspace(upa_steering(Nz, Nx, om_z, om_x)[:, None], Nz, Mz, Mx)[rows, 0]
            R = sample_covariance(Yw[:, :L], delta)
            w = mvdr_weights(R, a)
            W = wz[t] * wx[t]
            start[t, ik] = (sz, sx)
            upos[t, ik] = (uz, ux)
            w_out[t, ik, :W] = w
            a_out[t, ik, :W] = a
            z_out[t, ik] = beam_output(w, Yw[:, L:L + Lt])
            rows_out[t][ik] = rows
            if return_windows:
                R_out[t][ik], Yw_out[t][ik] = R, Yw
    out = dict(start=start, u=upos, w=w_out, a=a_out, z=z_out, rows=rows_out,
               subbands=np.asarray(ks))
    if return_windows:
        out.update(R=R_out, Yw=Yw_out)
    return out


def upa_full_mvdr(x: np.ndarray, *, Nz: int, K: int, L: int, Lt: int, az: Sequence[float],
                  el: Sequence[float], delta: float, beta: float = 0.2, dl: float = 0.5,
                  half_bin: bool = False, subbands: Optional[Sequence[int]] = None
                  ) -> Dict[str, np.ndarray]:
    """Full-dimensional element-space MVDR on the planar array (Sec. II-B, Eq. 11-13) with the
    steering vector of Eq. 6.  Returns ``w`` [T, nk, N] and ``z`` [T, nk, Lt]."""
    N = x.shape[0]
    Nx = N // Nz
    T = len(az)
    ks = list(range(K)) if subbands is None else [int(k) for k in subbands]
    X = channelize(x, K, half_bin)
    ratio = subband_freq_ratio(K, beta, half_bin)
    w_out = np.zeros((T, len(ks), N), dtype=np.complex128)
    z_out = np.zeros((T, len(ks), Lt), dtype=np.complex128)
    for ik, k in enumerate(ks):
        Xk = X[:, :L + Lt, k]
        R = sample_covariance(Xk[:, :L], delta)
        for t in range(T):
            om_z, om_x = upa_spatial_frequencies(float(az[t]), float(el[t]), float(ratio[k]), dl)
            w = mvdr_weights(R, upa_steering(Nz, Nx, om_z, om_x))
            w_out[t, ik] = w
            z_out[t, ik] = beam_output(w, Xk[:, L:L + Lt])
    return dict(w=w_out, z=z_out, subbands=np.asarray(ks))
