"""Pins of the oracle's channelizer and beamspace transform against the paper's
definitions written out as explicit matrices (brute force on tiny inputs)."""

import cmath
import math

import numpy as np
import pytest

import oracle
import scenes


def _dft_matrix_eq14(M, N):
    """[D]_{m,n} = M^-1/2 exp(-j 2 pi (m-1)(n-1) / M), m = 1..M, n = 1..N  (Eq. 14/15), by loops."""
    D = np.zeros((M, N), dtype=np.complex128)
    for m in range(1, M + 1):
        for n in range(1, N + 1):
            D[m - 1, n - 1] = cmath.exp(-2j * math.pi * (m - 1) * (n - 1) / M) / math.sqrt(M)
    return D


def _rand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.mark.parametrize("N,M", [(4, 4), (5, 8), (8, 16), (16, 32), (7, 64)])
def test_beamspace_matches_eq14_matrix(N, M):
    X = _rand((N, 3, 2), 1)
    D = _dft_matrix_eq14(M, N)
    Y = oracle.beamspace(X, M)
    ref = np.einsum("mn,nbk->mbk", D, X)
    assert np.max(np.abs(Y - ref)) < 1e-12


@pytest.mark.parametrize("N,M", [(4, 8), (16, 32), (9, 64)])
def test_beamspace_rows_match_matrix(N, M):
    Xk = _rand((N, 5), 2)
    D = _dft_matrix_eq14(M, N)
    bins = [M - 1, 0, 3, M // 2]
    assert np.max(np.abs(oracle.beamspace_rows(Xk, M, bins) - D[bins] @ Xk)) < 1e-12


@pytest.mark.parametrize("N,M", [(4, 4), (8, 16), (16, 32), (12, 64)])
def test_dft_isometry_and_parseval(N, M):
    D = _dft_matrix_eq14(M, N)
    assert np.max(np.abs(D.conj().T @ D - np.eye(N))) < 1e-12      # D^H D = I_N for M >= N
    X = _rand((N, 4, 3), 3)
    Y = oracle.beamspace(X, M)
    assert np.allclose(np.sum(np.abs(Y) ** 2, axis=0), np.sum(np.abs(X) ** 2, axis=0), rtol=1e-12)


@pytest.mark.parametrize("K", [4, 8, 16])
@pytest.mark.parametrize("half_bin", [False, True])
def test_channelizer_matches_direct_sum(K, half_bin):
    N, B = 3, 5
    x = _rand((N, B * K), 4)
    X = oracle.channelize(x, K, half_bin)
    ref = np.zeros((N, B, K), dtype=np.complex128)
    for e in range(N):
        for b in range(B):
            for k in range(K):
                acc = 0j
                for tau in range(K):
                    h = cmath.exp(-1j * math.pi * tau / K) if half_bin else 1.0
                    acc += x[e, b * K + tau] * h * cmath.exp(-2j * math.pi * tau * k / K)
                ref[e, b, k] = acc / math.sqrt(K)
    assert np.max(np.abs(X - ref)) < 1e-12
    Xb = oracle.channelize_bins(x, K, [K - 1, 0, 2], half_bin)
    assert np.max(np.abs(Xb - ref[:, :, [K - 1, 0, 2]])) < 1e-12


def test_channelize_beamspace_commute():
    # Both transforms are linear maps on different axes: either order gives the same Y (Sec. I).
    N, M, K, B = 6, 16, 8, 4
    x = _rand((N, B * K), 5)
    Y1 = oracle.beamspace(oracle.channelize(x, K), M)                  # time first
    xs = oracle.beamspace(x.reshape(N, B * K, 1), M)[:, :, 0]          # space first, per time sample
    Y2 = oracle.channelize(xs, K)
    assert np.max(np.abs(Y1 - Y2)) < 1e-12


@pytest.mark.parametrize("K", [4, 16, 128])
def test_subband_ratio_half_bin_is_eq1(K):
    beta = 0.2
    r = oracle.subband_freq_ratio(K, beta, half_bin=True)
    # Eq. 1: centres f_c + ((l - 1/2)/K) f_s for l = -K/2+1 .. K/2
    eq1 = sorted(1.0 + ((l - 0.5) / K) * beta for l in range(-K // 2 + 1, K // 2 + 1))
    assert np.allclose(sorted(r), eq1, rtol=0, atol=1e-15)
    plain = oracle.subband_freq_ratio(K, beta, half_bin=False)
    assert plain[0] == 1.0 and abs(plain[K // 2] - (1.0 - beta / 2)) < 1e-15
    assert np.allclose(r - plain, beta / (2 * K), atol=1e-15)


@pytest.mark.parametrize("K", [8, 32])
@pytest.mark.parametrize("half_bin", [False, True])
def test_subband_centre_is_the_frequency_of_a_tone_in_that_bin(K, half_bin):
    # Sampling physics, not the oracle's formula: the complex baseband tone exp(j 2 pi nu n)
    # with nu = (ks + off) / K cycles per sample (ks the bin's signed index, k - K above K/2
    # with the Nyquist bin at -1/2; off = 1/2 for the half-bin centres of Eq. 1) is the RF
    # frequency f_c + nu f_s, so a plane wave at that frequency advances by
    # Omega = 2 pi (d / lambda_c) sin(az) (1 + beta nu) per element.  DFT orthogonality puts it
    # wholly into bin k with value K^(1/2) exp(j Omega e); the oracle's steering at its subband
    # ratio for bin k must carry the same phase progression.  Block b starts at sample bK, where
    # the tone's phase is 2 pi nu K b (a multiple of pi: half-bin tones flip sign every block).
    N, B, beta, dl, az = 6, 3, 0.2, 0.5, math.radians(25.0)
    off = 0.5 if half_bin else 0.0
    ratio = oracle.subband_freq_ratio(K, beta, half_bin)
    n = np.arange(B * K)
    for k in range(K):
        ks = k if k < K // 2 else k - K
        nu = (ks + off) / K
        omega = 2.0 * math.pi * dl * math.sin(az) * (1.0 + beta * nu)
        x = np.exp(1j * omega * np.arange(N))[:, None] * np.exp(2j * math.pi * nu * n)[None, :]
        X = oracle.channelize(x, K, half_bin)
        others = np.delete(X, k, axis=2)
        assert np.max(np.abs(others)) < 1e-11
        exact = math.sqrt(K) * np.exp(1j * omega * np.arange(N))
        for b in range(B):
            block = np.exp(2j * math.pi * nu * K * b)
            assert np.max(np.abs(X[:, b, k] - block * exact)) < 1e-11
        a = oracle.steering(N, oracle.spatial_frequency(math.sin(az), ratio[k], dl))
        assert np.max(np.abs(math.sqrt(K) * a - exact)) < 1e-11


@pytest.mark.parametrize("half_bin", [False, True])
def test_generator_tone_lands_in_its_subband(half_bin):
    # A single noiseless source: channelized element 0 equals the generator's per-bin source
    # waveform up to the steering phase, and element e carries exp(j Omega_k e).
    cfg = scenes.SceneConfig(name="t", N=4, M=8, K=8, L=3, Lt=1, T=1, W=3, noise_var=0.0,
                             target_az_deg=(20.0,), target_snr_db=(0.0,), half_bin=half_bin, seed=9,
                             complex128=True)
    sc = scenes.make_scene(cfg)
    X = oracle.channelize(sc.x, cfg.K, half_bin)
    ratio = oracle.subband_freq_ratio(cfg.K, cfg.beta, half_bin)
    for k in range(cfg.K):
        om = oracle.spatial_frequency(math.sin(sc.target_az[0]), ratio[k], cfg.dl)
        a = oracle.steering(cfg.N, om)
        g = X[0, :, k]
        assert np.max(np.abs(X[:, :, k] - np.outer(a, g))) < 1e-12
