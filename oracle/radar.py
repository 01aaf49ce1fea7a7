"""FP64 range-Doppler processing and 1-D CFAR detection of a beamformed pulse train (test
infrastructure only).

The paper names these steps (the synthesized wideband beam output goes through standard
range-Doppler processing; a 1-D CFAR with a threshold 10 dB above the estimated noise floor
runs across the velocity bins of the range-Doppler map, Sec. II and IV) without fixing their
parameters.  Readings, also listed in the design notes of the repository:
* the beam output z (one target) is a train of P pulses of R samples each (z_p[n] =
  z[p R + n]); the transmitted pulse is a unit-magnitude baseband LFM chirp of Lp <= R samples,
  c[m] = exp(j pi m^2 / Lp - j pi m), sweeping the band once;
* range compression is the matched filter within each pulse (linear correlation, samples past
  the pulse are zero): r[p, d] = sum_{m < Lp, d + m < R} conj(c[m]) z_p[d + m], d < R;
* Doppler processing is a unitary P-point DFT across pulses (rectangular window):
  RD[d, v] = P^-1/2 sum_p r[p, d] exp(-j 2 pi p v / P);
* CFAR is cell averaging along range, run for every velocity bin: the noise estimate of cell
  (d, v) is the mean power of the cells d' with guard < |d' - d| <= guard + train inside
  [0, R); the cell is a detection when its power exceeds 10^(threshold_db / 10) times it.
"""

from __future__ import annotations

import numpy as np

__all__ = ["lfm_chirp", "range_compress", "doppler", "cfar_1d", "range_doppler"]


def lfm_chirp(Lp: int) -> np.ndarray:
    """Unit-magnitude baseband LFM pulse c[m] = exp(j pi m^2 / Lp - j pi m), m < Lp."""
    m = np.arange(Lp, dtype=np.float64)
    return np.exp(1j * np.pi * m * m / Lp - 1j * np.pi * m)


def range_compress(z: np.ndarray, chirp: np.ndarray, R: int, P: int) -> np.ndarray:
    """Matched filter within each pulse: z[P*R] -> r[P, R] (see the module notes)."""
    zp = np.asarray(z, dtype=np.complex128)[:P * R].reshape(P, R)
    Lp = len(chirp)
    r = np.zeros((P, R), dtype=np.complex128)
    cc = np.conj(np.asarray(chirp, dtype=np.complex128))
    for d in range(R):
        m = min(Lp, R - d)
        r[:, d] = zp[:, d:d + m] @ cc[:m]
    return r


def doppler(r: np.ndarray) -> np.ndarray:
    """Unitary DFT across pulses: r[P, R] -> RD[R, P]."""
    return np.fft.fft(np.asarray(r, dtype=np.complex128), axis=0, norm="ortho").T


def cfar_1d(power: np.ndarray, guard: int, train: int, threshold_db: float):
    """Cell-averaging CFAR along range for every velocity bin: power[R, V] -> (noise[R, V],
    detections bool[R, V]).  Cells with no training cell get noise = inf (no detection)."""
    R, V = power.shape
    noise = np.full((R, V), np.inf)
    for d in range(R):
        idx = [dd for dd in range(R) if guard < abs(dd - d) <= guard + train]
        if idx:
            noise[d] = power[idx].mean(axis=0)
    return noise, power > (10.0 ** (threshold_db / 10.0)) * noise


def range_doppler(z: np.ndarray, chirp: np.ndarray, R: int, P: int, guard: int, train: int,
                  threshold_db: float = 10.0):
    """z[>= P R] -> (power[R, P] = |RD|^2, noise[R, P], detections bool[R, P])."""
    rd = doppler(range_compress(z, chirp, R, P))
    power = np.abs(rd) ** 2
    noise, det = cfar_1d(power, guard, train, threshold_db)
    return power, noise, det
