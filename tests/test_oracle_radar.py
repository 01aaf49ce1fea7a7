"""Pins of the oracle's range-Doppler and CFAR steps: closed forms for a delayed pulse (the
matched-filter peak equals the pulse energy at the true delay), a Doppler tone (the DFT peak
is sqrt(P) at its bin and zero elsewhere), a constructed CFAR map, brute force on a tiny train,
and an end-to-end point target."""

import cmath
import math

import numpy as np
import pytest

from oracle import radar


def _rand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def test_chirp_has_unit_magnitude_and_sweeps_the_band():
    c = radar.lfm_chirp(64)
    assert np.allclose(np.abs(c), 1.0, atol=1e-15)
    # instantaneous frequency (phase increment / 2 pi) rises by 1/Lp per sample across the
    # band, from -1/2 + 1/(2 Lp)
    f = np.angle(c[1:] / c[:-1]) / (2 * math.pi)
    assert np.allclose(np.diff(f), 1 / 64, atol=1e-12)
    assert abs(f[0] - (-0.5 + 1 / 128)) < 1e-12 and abs(f[-1] - 0.5) < 2 / 64


@pytest.mark.parametrize("d0", [0, 5, 17])
def test_matched_filter_peaks_at_the_delay_with_the_pulse_energy(d0):
    R, P, Lp, A = 40, 3, 16, 0.5 - 2j
    c = radar.lfm_chirp(Lp)
    z = np.zeros(P * R, dtype=np.complex128)
    for p in range(P):
        z[p * R + d0:p * R + d0 + Lp] = A * c
    r = radar.range_compress(z, c, R, P)
    assert np.allclose(r[:, d0], A * Lp, atol=1e-12)
    assert np.all(np.abs(r) <= abs(A) * Lp + 1e-12)
    assert np.argmax(np.abs(r[0])) == d0


def test_range_compression_brute_force_tiny():
    R, P, Lp = 7, 2, 3
    z = _rand((P * R + 4,), 1)
    c = _rand((Lp,), 2)
    r = radar.range_compress(z, c, R, P)
    for p in range(P):
        for d in range(R):
            acc = 0j
            for m in range(Lp):
                if d + m < R:
                    acc += c[m].conjugate() * z[p * R + d + m]
            assert abs(r[p, d] - acc) < 1e-13


def test_doppler_tone_peaks_at_its_bin():
    P, R, v0 = 16, 5, 3
    r = np.zeros((P, R), dtype=np.complex128)
    for p in range(P):
        r[p] = cmath.exp(2j * math.pi * v0 * p / P)
    rd = radar.doppler(r)
    assert rd.shape == (R, P)
    assert np.allclose(rd[:, v0], math.sqrt(P), atol=1e-12)
    rest = np.delete(rd, v0, axis=1)
    assert np.max(np.abs(rest)) < 1e-12


def test_cfar_on_a_constructed_map():
    R, V, g, n = 40, 4, 2, 6
    pw = np.ones((R, V))
    pw[10, 0] = 10 ** 1.1      # 11 dB above a floor of 1: detected
    pw[25, 1] = 10 ** 0.9      # 9 dB: not detected
    pw[26, 1] = 10 ** 0.95     # inside the first cell's guard band: does not raise its floor
    noise, det = radar.cfar_1d(pw, g, n, 10.0)
    assert det[10, 0] and not det[25, 1] and not det[26, 1]
    assert noise[10, 0] == 1.0 and noise[25, 1] == 1.0
    assert int(det.sum()) == 1
    # training cells straddle the target: the neighbour's estimate includes it
    assert noise[10 + g + 1, 0] > 1.0


def test_point_target_end_to_end():
    R, P, Lp, d0, v0, A = 64, 16, 16, 20, 5, 2.0
    c = radar.lfm_chirp(Lp)
    z = np.zeros(P * R, dtype=np.complex128)
    for p in range(P):
        z[p * R + d0:p * R + d0 + Lp] = A * c * cmath.exp(2j * math.pi * v0 * p / P)
    z += 1e-3 * _rand(z.shape, 3)
    power, noise, det = radar.range_doppler(z, c, R, P, guard=2, train=8)
    assert det[d0, v0]
    assert abs(power[d0, v0] - (A * Lp * math.sqrt(P)) ** 2) < 1e-3 * power[d0, v0]
    assert np.unravel_index(np.argmax(power), power.shape) == (d0, v0)
