"""Pins of the window selection (Eq. 18-19) and the windowed steering vector."""

import cmath
import math

import numpy as np
import pytest

import oracle


def _dirichlet_closed_form(N, M, omega, m):
    """M^-1/2 sum_{e<N} e^{j psi e} = M^-1/2 e^{j psi (N-1)/2} sin(N psi/2)/sin(psi/2), psi = Omega - 2 pi m / M."""
    psi = omega - 2.0 * math.pi * m / M
    if abs(math.sin(psi / 2)) < 1e-14:
        return N / math.sqrt(M)          # psi = 2 pi q: every term is 1
    return cmath.exp(1j * psi * (N - 1) / 2) * math.sin(N * psi / 2) / math.sin(psi / 2) / math.sqrt(M)


@pytest.mark.parametrize("N,M", [(16, 32), (16, 16), (256, 512), (33, 128)])
def test_windowed_steering_is_dirichlet(N, M):
    rng = np.random.default_rng(0)
    for _ in range(20):
        om = rng.uniform(-math.pi, math.pi) * 1.1
        bins = rng.integers(0, M, size=7)
        a = oracle.beamspace_steering(N, M, om, bins)
        ref = np.array([_dirichlet_closed_form(N, M, om, int(m)) for m in bins])
        assert np.max(np.abs(a - ref)) < 1e-11 * max(1.0, N / math.sqrt(M))


@pytest.mark.parametrize("N,M", [(16, 32), (256, 512), (1024, 2048), (64, 64)])
def test_odd_window_centre_is_peak_bin(N, M):
    # For odd W the window centre s + (W-1)/2 is the beamspace bin of largest |D a| (brute force).
    rng = np.random.default_rng(1)
    beta = 0.2
    for _ in range(25):
        s_az = math.sin(math.radians(rng.uniform(-60, 60)))
        ratio = float(rng.choice(oracle.subband_freq_ratio(16, beta)))
        om = oracle.spatial_frequency(s_az, ratio)
        Da = oracle.beamspace_rows(oracle.steering(N, om)[:, None], M, np.arange(M))[:, 0]
        peak = int(np.argmax(np.abs(Da)))
        for W in (1, 5, 9, 33):
            u = oracle.beam_position(s_az, ratio, M)
            s = oracle.window_start(u, W)
            assert (s + (W - 1) // 2) % M == peak


def test_window_start_brute_force_and_ties():
    # s minimises |s + (W-1)/2 - u| over integers; exact ties pick the larger s.
    rng = np.random.default_rng(2)
    us = list(rng.uniform(-300, 300, size=200)) + [0.0, 0.5, -0.5, 1.5, -2.5, 3.0]
    for u in us:
        for W in (1, 2, 4, 5, 8, 9, 17, 32, 33, 64):
            cands = range(int(math.floor(u)) - W - 2, int(math.ceil(u)) + 3)
            best = min(cands, key=lambda s: (abs(s + (W - 1) / 2 - u), -s))
            assert oracle.window_start(u, W) == best, (u, W)
    assert oracle.window_start(0.0, 4) == -1      # broadside, even W: centre -1.5 + 1/2 rounds up
    assert oracle.window_start(0.0, 5) == -2


def test_window_bins_wrap():
    assert list(oracle.window_bins(-2, 5, 32)) == [30, 31, 0, 1, 2]
    assert list(oracle.window_bins(30, 4, 32)) == [30, 31, 0, 1]


def test_beam_position_matches_spatial_frequency():
    for s_az in (-0.8, -0.1, 0.0, 0.3, 0.86):
        for ratio in (0.9, 1.0, 1.1):
            u = oracle.beam_position(s_az, ratio, 512)
            om = oracle.spatial_frequency(s_az, ratio)
            assert abs(2 * math.pi * u / 512 - om) < 1e-14
