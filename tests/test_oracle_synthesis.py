"""Pins of the oracle's subband synthesis and lifted-correlator outputs: the synthesis inverts
the (separately pinned) channelizer and keeps energy; a single subband sample comes back as one
block of a tone; lifting is the adjoint of windowed beamspace projection (Eq. 21), so lifted
correlators applied in element space give the windowed beam outputs."""

import cmath
import math

import numpy as np
import pytest

import oracle
import scenes


def _rand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.mark.parametrize("K", [4, 16, 128])
@pytest.mark.parametrize("half_bin", [False, True])
def test_synthesis_inverts_channelizer(K, half_bin):
    T, B = 3, 6
    x = _rand((T, B * K), 11)
    X = oracle.channelize(x, K, half_bin)                       # [T, B, K]
    z = oracle.synthesize(np.swapaxes(X, 1, 2), K, half_bin)    # Z[T, K, B] -> [T, B*K]
    assert np.max(np.abs(z - x)) < 1e-12 * np.max(np.abs(x))


@pytest.mark.parametrize("half_bin", [False, True])
def test_synthesis_keeps_energy(half_bin):
    K, B = 32, 5
    Z = _rand((2, K, B), 12)
    z = oracle.synthesize(Z, K, half_bin)
    assert np.allclose(np.sum(np.abs(z) ** 2, axis=1), np.sum(np.abs(Z) ** 2, axis=(1, 2)),
                       rtol=1e-12)


@pytest.mark.parametrize("half_bin", [False, True])
def test_one_subband_sample_is_one_block_of_a_tone(half_bin):
    K, B, k0, b0 = 16, 4, 5, 2
    Z = np.zeros((K, B), dtype=np.complex128)
    Z[k0, b0] = 1.0
    z = oracle.synthesize(Z, K, half_bin)
    assert np.all(z[:b0 * K] == 0) and np.all(z[(b0 + 1) * K:] == 0)
    blk = z[b0 * K:(b0 + 1) * K]
    assert np.allclose(np.abs(blk), 1 / math.sqrt(K), rtol=1e-12)
    step = cmath.exp(2j * math.pi * (k0 + (0.5 if half_bin else 0.0)) / K)   # per-sample rotation
    assert np.max(np.abs(blk[1:] / blk[:-1] - step)) < 1e-12
    assert abs(blk[0] - 1 / math.sqrt(K)) < 1e-15


@pytest.mark.parametrize("N,M", [(8, 16), (16, 32), (13, 64)])
def test_lifting_is_the_adjoint_of_windowed_projection(N, M):
    # <c^, x> = <c~, S D x> for any c~, x and window (wrapping windows included)  (Eq. 21)
    for seed, start, W in [(1, 3, 5), (2, M - 2, 4), (3, -1, 3)]:
        c = _rand((W,), seed)
        x = _rand((N,), seed + 10)
        bins = oracle.window_bins(start, W, M)
        lhs = np.vdot(oracle.lift_correlator(c, bins, M, N), x)
        rhs = np.vdot(c, oracle.beamspace_rows(x[:, None], M, bins)[:, 0])
        assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(rhs))


@pytest.mark.parametrize("half_bin", [False, True])
def test_lifted_outputs_equal_windowed_beam_outputs(half_bin):
    cfg = scenes.SMALL.replace(half_bin=half_bin)
    sc = scenes.make_scene(cfg)
    bm = oracle.windowed_mvdr(sc.x, M=cfg.M, K=cfg.K, L=cfg.L, Lt=cfg.Lt, sin_az=sc.sin_az,
                              win=sc.win, delta=cfg.delta, half_bin=half_bin)
    T = len(sc.win)
    c_hat = np.empty((T, cfg.K, cfg.N), dtype=np.complex128)
    for t in range(T):
        for k in range(cfg.K):
            bins = oracle.window_bins(int(bm["start"][t, k]), int(sc.win[t]), cfg.M)
            c_hat[t, k] = oracle.lift_correlator(bm["w"][t, k], bins, cfg.M, cfg.N)
    z = oracle.lifted_outputs(sc.x, c_hat, K=cfg.K, L=cfg.L, Lt=cfg.Lt, half_bin=half_bin)
    assert np.max(np.abs(z - bm["z"])) < 1e-10 * np.max(np.abs(bm["z"]))
