"""Pins of the oracle's covariance, MVDR solve, output, lifting and beam pattern
against closed forms, optimality conditions and the W = M = N reduction identity."""

import math

import numpy as np
import pytest

import oracle
import scenes


def _rand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def _exact_cov_snapshots(R, L):
    """Snapshots Y (W x L) whose sample covariance (1/L) Y Y^H equals R exactly.

    Y = sqrt(L) R^1/2 Q with Q the first W rows of the unitary L-point DFT (Q Q^H = I)."""
    W = R.shape[0]
    evals, evecs = np.linalg.eigh(R)
    Rh = (evecs * np.sqrt(np.maximum(evals, 0))) @ evecs.conj().T
    n = np.arange(L)
    Q = np.exp(-2j * np.pi * np.outer(np.arange(W), n) / L) / math.sqrt(L)
    return math.sqrt(L) * Rh @ Q


def test_sample_covariance_properties():
    Y = _rand((7, 40), 0)
    d = 0.37
    R = oracle.sample_covariance(Y, d)
    assert np.allclose(R, R.conj().T, atol=1e-14)
    assert np.min(np.linalg.eigvalsh(R)) >= d - 1e-12
    assert abs(np.trace(R).real - (np.mean(np.sum(np.abs(Y) ** 2, axis=0)) + 7 * d)) < 1e-10
    # entry-wise definition of Eq. 11 by loops
    i, j = 2, 5
    ref = sum(Y[i, n] * np.conj(Y[j, n]) for n in range(40)) / 40
    assert abs(R[i, j] - ref) < 1e-13


@pytest.mark.parametrize("W", [1, 2, 5, 8])
def test_mvdr_matches_explicit_inverse_and_kkt(W):
    Y = _rand((W, 3 * W + 2), W)
    R = oracle.sample_covariance(Y, 0.5)
    a = _rand((W,), 10 + W)
    w = oracle.mvdr_weights(R, a)
    Ri = np.linalg.inv(R)
    ref = Ri @ a / (a.conj() @ Ri @ a)
    assert np.max(np.abs(w - ref)) < 1e-12 * np.max(np.abs(ref))
    assert abs(np.vdot(w, a) - 1.0) < 1e-12              # distortionless c^H a = 1 (Eq. 12)
    q = 1.0 / (a.conj() @ Ri @ a).real
    assert np.max(np.abs(R @ w - q * a)) < 1e-11 * np.max(np.abs(a))


def test_mvdr_is_the_constrained_minimiser():
    W = 6
    R = oracle.sample_covariance(_rand((W, 20), 3), 0.1)
    a = _rand((W,), 4)
    w = oracle.mvdr_weights(R, a)
    p0 = np.vdot(w, R @ w).real
    rng = np.random.default_rng(5)
    for _ in range(50):
        d = rng.standard_normal(W) + 1j * rng.standard_normal(W)
        d -= a * np.vdot(a, d) / np.vdot(a, a)           # keep (w + d)^H a = 1
        assert np.vdot(w + d, R @ (w + d)).real >= p0 - 1e-12


@pytest.mark.parametrize("N,rho_db,offset", [(16, 30.0, 1.3), (32, 20.0, 0.6), (64, 40.0, 2.7)])
def test_single_interferer_null_depth_closed_form(N, rho_db, offset):
    # R = s'^2 I + p a_J a_J^H: |w^H a_J| = |beta| s'^2 / (N (s'^2 + p N) - p |beta|^2), beta = a_J^H a_s.
    sigma2, delta = 1.0, 10.0
    p = 10 ** (rho_db / 10)
    om_s = 0.4
    om_j = om_s + offset * 2 * math.pi / N
    a_s, a_j = oracle.steering(N, om_s), oracle.steering(N, om_j)
    R0 = sigma2 * np.eye(N) + p * np.outer(a_j, a_j.conj())
    Y = _exact_cov_snapshots(R0, L=4 * N)
    R = oracle.sample_covariance(Y, delta)
    assert np.max(np.abs(R - (R0 + delta * np.eye(N)))) < 1e-8 * p
    w = oracle.mvdr_weights(R, a_s)
    beta = np.vdot(a_j, a_s)
    s2 = sigma2 + delta
    ref = abs(beta) * s2 / (N * (s2 + p * N) - p * abs(beta) ** 2)
    assert abs(abs(np.vdot(w, a_j)) - ref) < 1e-9 * max(ref, 1e-12) + 1e-14


@pytest.mark.parametrize("N,rho_db", [(16, 25.0), (40, 35.0)])
def test_optimum_sinr_single_jammer(N, rho_db):
    # With R = R_in (no loading, no target): SINR = a^H R_in^-1 a = (N (s^2 + pN) - p|beta|^2) / (s^2 (s^2 + pN)).
    p = 10 ** (rho_db / 10)
    s_sin, j_sin = 0.2, 0.2 + 1.7 / N
    R_in = oracle.interference_covariance(N, [j_sin], [p], 1.0)
    a = oracle.steering(N, oracle.spatial_frequency(s_sin, 1.0))
    aj = oracle.steering(N, oracle.spatial_frequency(j_sin, 1.0))
    w = oracle.mvdr_weights(R_in, a)
    beta2 = abs(np.vdot(aj, a)) ** 2
    ref = (N * (1 + p * N) - p * beta2) / (1 + p * N)
    assert abs(oracle.sinr(w, a, R_in) / ref - 1) < 1e-10


def test_beam_output_is_linear_correlation():
    w = _rand((5,), 1)
    Y = _rand((5, 9), 2)
    z = oracle.beam_output(w, Y)
    for n in range(9):
        assert abs(z[n] - sum(np.conj(w[i]) * Y[i, n] for i in range(5))) < 1e-13


@pytest.mark.parametrize("half_bin", [False, True])
def test_reduction_identity_W_eq_M_eq_N(half_bin):
    # With M = N (unitary D) and W = M the window is a cyclic permutation, so windowed beamspace
    # MVDR equals element-space MVDR (Eq. 13 vs Eq. 20-21), loading included.
    cfg = scenes.SMALL.replace(M=16, W=16, half_bin=half_bin)
    sc = scenes.make_scene(cfg)
    kw = dict(K=cfg.K, L=cfg.L, Lt=cfg.Lt, sin_az=sc.sin_az, delta=cfg.delta, half_bin=half_bin)
    bm = oracle.windowed_mvdr(sc.x, M=cfg.M, win=sc.win, **kw)
    fm = oracle.full_mvdr(sc.x, **kw)
    assert np.max(np.abs(bm["z"] - fm["z"])) < 1e-10 * np.max(np.abs(fm["z"]))
    for k in range(cfg.K):
        bins = oracle.window_bins(int(bm["start"][0, k]), cfg.N, cfg.M)
        c_hat = oracle.lift_correlator(bm["w"][0, k], bins, cfg.M, cfg.N)        # Eq. 21
        assert np.max(np.abs(c_hat - fm["w"][0, k])) < 1e-10 * np.max(np.abs(fm["w"][0, k]))


def test_beam_pattern_of_matched_filter_is_normalised_dirichlet():
    N = 24
    om0 = 0.7
    c = oracle.steering(N, om0)
    oms = np.linspace(-math.pi, math.pi, 31)
    B = oracle.beam_pattern(c, oms)
    for om, b in zip(oms, B):
        psi = om - om0
        ref = 1.0 if abs(math.sin(psi / 2)) < 1e-12 else abs(math.sin(N * psi / 2) / math.sin(psi / 2)) / N
        assert abs(b - ref) < 1e-12


def test_small_scene_beamformer_nulls_jammer_and_keeps_target():
    cfg = scenes.SMALL
    sc = scenes.make_scene(cfg)
    res = oracle.windowed_mvdr(sc.x, M=cfg.M, K=cfg.K, L=cfg.L, Lt=cfg.Lt, sin_az=sc.sin_az,
                               win=sc.win, delta=cfg.delta)
    ratio = oracle.subband_freq_ratio(cfg.K, cfg.beta)
    for k in range(cfg.K):
        bins = oracle.window_bins(int(res["start"][0, k]), cfg.W, cfg.M)
        w = res["w"][0, k, :cfg.W]
        a = res["a"][0, k, :cfg.W]
        assert abs(np.vdot(w, a) - 1) < 1e-10
        aj = oracle.beamspace_steering(cfg.N, cfg.M, oracle.spatial_frequency(
            math.sin(sc.jammer_az[0]), ratio[k]), bins)
        # the jammer (30 dB) is pushed at least 25 dB below the distortionless target response
        assert 20 * math.log10(abs(np.vdot(w, aj)) + 1e-30) < -25
