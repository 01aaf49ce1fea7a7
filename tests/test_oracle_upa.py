"""Pins of the planar-array oracle (oracle.upa) against things other than itself: the linear
array oracle (already pinned) in the degenerate one-row and one-column arrays, the separable
structure of the two-dimensional DFT, Dirichlet closed forms per axis, isometry of D, the
brute-force beam peak, the W = M = N identity with element-space MVDR and the KKT conditions
on a seeded planar-array scene."""

import cmath
import math

import numpy as np
import pytest

import oracle
import scenes
from oracle import upa


def _rand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def _dirichlet(N, M, omega, m):
    psi = omega - 2.0 * math.pi * m / M
    if abs(math.sin(psi / 2)) < 1e-14:
        return N / math.sqrt(M)
    return cmath.exp(1j * psi * (N - 1) / 2) * math.sin(N * psi / 2) / math.sin(psi / 2) / math.sqrt(M)


@pytest.mark.parametrize("Nz,Nx,Mz,Mx", [(2, 3, 2, 4), (4, 8, 8, 16), (3, 5, 4, 8), (1, 6, 1, 8)])
def test_beamspace_is_the_2d_dft_by_direct_sum(Nz, Nx, Mz, Mx):
    # y^[mx Mz + mz] = (Mz Mx)^-1/2 sum_{ix, iz} y[ix Nz + iz] e^{-j 2 pi (mz iz / Mz + mx ix / Mx)}
    X = _rand((Nz * Nx, 3), 1)
    ref = np.zeros((Mz * Mx, 3), dtype=np.complex128)
    for mx in range(Mx):
        for mz in range(Mz):
            for ix in range(Nx):
                for iz in range(Nz):
                    ph = cmath.exp(-2j * math.pi * (mz * iz / Mz + mx * ix / Mx))
                    ref[mx * Mz + mz] += X[ix * Nz + iz] * ph
    ref /= math.sqrt(Mz * Mx)
    assert np.max(np.abs(upa.upa_beamspace(X, Nz, Mz, Mx) - ref)) < 1e-12
    assert np.max(np.abs(upa.upa_dft_matrix(Nz, Nx, Mz, Mx) @ X - ref)) < 1e-12


@pytest.mark.parametrize("Nz,Nx,Mz,Mx", [(4, 32, 8, 64), (2, 8, 4, 16), (4, 4, 4, 4)])
def test_dft_is_an_isometry(Nz, Nx, Mz, Mx):
    D = upa.upa_dft_matrix(Nz, Nx, Mz, Mx)
    assert np.max(np.abs(D.conj().T @ D - np.eye(Nz * Nx))) < 1e-12


def test_separable_input_gives_kronecker_of_1d_transforms():
    # D (u kron v) = (D_x u) kron (D_z v), the one-dimensional transforms of the linear-array oracle
    Nz, Nx, Mz, Mx = 4, 8, 8, 32
    u, v = _rand((Nx, 1), 2), _rand((Nz, 1), 3)
    Y = upa.upa_beamspace(np.kron(u, v), Nz, Mz, Mx)
    ref = np.kron(oracle.beamspace(u[:, :, None], Mx)[:, :, 0], oracle.beamspace(v[:, :, None], Mz)[:, :, 0])
    assert np.max(np.abs(Y - ref)) < 1e-12


def test_windowed_steering_is_product_of_dirichlets():
    Nz, Nx, Mz, Mx = 4, 32, 8, 64
    rng = np.random.default_rng(4)
    for _ in range(10):
        omz, omx = rng.uniform(-math.pi, math.pi, size=2)
        a = upa.upa_beamspace(upa.upa_steering(Nz, Nx, omz, omx)[:, None], Nz, Mz, Mx)[:, 0]
        for m in rng.integers(0, Mz * Mx, size=12):
            mx, mz = divmod(int(m), Mz)
            ref = _dirichlet(Nx, Mx, omx, mx) * _dirichlet(Nz, Mz, omz, mz)
            assert abs(a[m] - ref) < 1e-11


def test_steering_phase_of_every_element():
    # element (iz, ix) sees e^{j (Omega_z iz + Omega_x ix)} at index ix Nz + iz
    a = upa.upa_steering(3, 5, 0.7, -1.3)
    for ix in range(5):
        for iz in range(3):
            assert abs(a[ix * 3 + iz] - cmath.exp(1j * (0.7 * iz - 1.3 * ix))) < 1e-15


@pytest.mark.parametrize("Wz,Wx", [(1, 3), (3, 5), (5, 1)])
def test_odd_window_centre_is_peak_beam(Wz, Wx):
    # brute force over the grid: the window centre is the beam of largest |D a|
    Nz, Nx, Mz, Mx = 4, 32, 8, 64
    rng = np.random.default_rng(5)
    for _ in range(30):
        az, el = math.radians(rng.uniform(-60, 60)), math.radians(rng.uniform(-40, 40))
        ratio = 1.0 + 0.2 * rng.uniform(-0.5, 0.5)
        uz, ux = upa.upa_beam_position(az, el, ratio, Mz, Mx)
        if min(abs(uz - math.floor(uz) - 0.5), abs(ux - math.floor(ux) - 0.5)) < 1e-6:
            continue
        sz, sx = oracle.window_start(uz, Wz), oracle.window_start(ux, Wx)
        omz, omx = upa.upa_spatial_frequencies(az, el, ratio)
        mag = np.abs(upa.upa_beamspace(upa.upa_steering(Nz, Nx, omz, omx)[:, None], Nz, Mz, Mx)[:, 0])
        mx, mz = divmod(int(np.argmax(mag)), Mz)
        assert mz == (sz + (Wz - 1) // 2) % Mz and mx == (sx + (Wx - 1) // 2) % Mx


def test_window_rows_order_and_wrap():
    rows = upa.upa_window_rows(7, 62, 2, 4, 8, 64)
    # z fastest: (mz, mx) = (7, 62), (0, 62), (7, 63), (0, 63), (7, 0), (0, 0), (7, 1), (0, 1)
    assert list(rows) == [62 * 8 + 7, 62 * 8 + 0, 63 * 8 + 7, 63 * 8 + 0, 7, 0, 8 + 7, 8]


@pytest.mark.parametrize("half_bin", [False, True])
def test_one_row_array_is_the_linear_array(half_bin):
    # Nz = Mz = Wz = 1 at elevation 0: the linear-array oracle with N = Nx, M = Mx
    cfg = scenes.UPA_SMALL.replace(Nz=1, Mz=1, windows=((1, 5), (1, 3)), half_bin=half_bin,
                                   target_dir_deg=((14.0, 0.0), (-31.0, 0.0)),
                                   jammer_dir_deg=((40.0, 0.0),))
    sc = scenes.make_upa_scene(cfg)
    r2 = upa.upa_windowed_mvdr(sc.x, Nz=1, Mz=1, Mx=cfg.Mx, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                               az=sc.target_az, el=sc.target_el, win_z=sc.win_z, win_x=sc.win_x,
                               delta=cfg.delta, half_bin=half_bin)
    r1 = oracle.windowed_mvdr(sc.x, M=cfg.Mx, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                              sin_az=[math.sin(a) for a in sc.target_az], win=sc.win_x,
                              delta=cfg.delta, half_bin=half_bin)
    assert np.array_equal(r2["start"][:, :, 1], r1["start"])
    assert np.max(np.abs(r2["w"] - r1["w"])) < 1e-12 * np.max(np.abs(r1["w"]))
    assert np.max(np.abs(r2["z"] - r1["z"])) < 1e-12 * np.max(np.abs(r1["z"]))


def test_one_column_array_is_a_vertical_linear_array():
    # Nx = Mx = Wx = 1 at azimuth 0: the linear-array oracle with sin(az) -> sin(el)
    cfg = scenes.UPA_SMALL.replace(Nz=8, Nx=1, Mz=16, Mx=1, windows=((3, 1), (4, 1)),
                                   target_dir_deg=((0.0, 22.0), (0.0, -9.0)),
                                   jammer_dir_deg=((0.0, -45.0),))
    sc = scenes.make_upa_scene(cfg)
    r2 = upa.upa_windowed_mvdr(sc.x, Nz=8, Mz=16, Mx=1, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                               az=sc.target_az, el=sc.target_el, win_z=sc.win_z, win_x=sc.win_x,
                               delta=cfg.delta)
    r1 = oracle.windowed_mvdr(sc.x, M=16, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                              sin_az=[math.sin(e) for e in sc.target_el], win=sc.win_z,
                              delta=cfg.delta)
    assert np.array_equal(r2["start"][:, :, 0], r1["start"])
    assert np.max(np.abs(r2["z"] - r1["z"])) < 1e-12 * np.max(np.abs(r1["z"]))


def test_full_window_equals_element_space_mvdr():
    # Wz = Mz = Nz, Wx = Mx = Nx: D is unitary and S a permutation, so the beamspace MVDR output
    # equals the element-space one and the lifted correlator (Eq. 21) equals its weights
    cfg = scenes.UPA_SMALL.replace(Nz=2, Nx=4, Mz=2, Mx=4, windows=((2, 4),))
    sc = scenes.make_upa_scene(cfg)
    kw = dict(K=cfg.K, L=cfg.L, Lt=cfg.Lt, az=sc.target_az, el=sc.target_el, delta=cfg.delta)
    rb = upa.upa_windowed_mvdr(sc.x, Nz=2, Mz=2, Mx=4, win_z=sc.win_z, win_x=sc.win_x, **kw)
    rf = upa.upa_full_mvdr(sc.x, Nz=2, **kw)
    assert np.max(np.abs(rb["z"] - rf["z"])) < 1e-10 * np.max(np.abs(rf["z"]))
    for t in range(cfg.T):
        for k in range(cfg.K):
            c = upa.upa_lift_correlator(rb["w"][t, k], rb["rows"][t][k], 2, 4, 2, 4)
            assert np.max(np.abs(c - rf["w"][t, k])) < 1e-10 * np.max(np.abs(rf["w"][t, k]))


def test_kkt_on_a_planar_scene():
    cfg = scenes.UPA_SMALL
    sc = scenes.make_upa_scene(cfg)
    X = oracle.channelize(sc.x, cfg.K)
    r = upa.upa_windowed_mvdr(sc.x, Nz=cfg.Nz, Mz=cfg.Mz, Mx=cfg.Mx, K=cfg.K, L=cfg.L,
                              Lt=cfg.Lt, az=sc.target_az, el=sc.target_el, win_z=sc.win_z,
                              win_x=sc.win_x, delta=cfg.delta)
    for t in range(cfg.T):
        W = int(sc.win_z[t] * sc.win_x[t])
        for k in range(cfg.K):
            Yk = upa.upa_beamspace(X[:, :, k], cfg.Nz, cfg.Mz, cfg.Mx)
            Yw = Yk[r["rows"][t][k]]
            R = Yw[:, :cfg.L] @ Yw[:, :cfg.L].conj().T / cfg.L + cfg.delta * np.eye(W)
            w, a = r["w"][t, k, :W], r["a"][t, k, :W]
            assert abs(np.vdot(w, a) - 1.0) < 1e-12                   # w^H a = 1
            lam = R @ w
            q = 1.0 / np.vdot(a, np.linalg.solve(R, a)).real
            assert np.max(np.abs(lam - q * a)) < 1e-10 * np.max(np.abs(lam))   # R w = q a


def test_jammer_pushed_to_the_noise_floor():
    # a 40 dB jammer off the target's beam: at the output of the windowed MVDR its power is at
    # most about the noise power (jammer-to-noise ratio INR |w^H a_j|^2 / ||w||^2 below 2), while
    # the conventional window beam a~ / ||a~||^2 passes it far above the noise wherever it is
    # not already in a null of that beam
    cfg = scenes.UPA_SMALL.replace(Nz=4, Nx=16, Mz=8, Mx=32, windows=((3, 5),), T=1,
                                   target_dir_deg=((10.0, 12.0),), target_snr_db=(0.0,),
                                   jammer_dir_deg=((25.0, -6.0),), jammer_inr_db=(40.0,), L=128)
    sc = scenes.make_upa_scene(cfg)
    r = upa.upa_windowed_mvdr(sc.x, Nz=4, Mz=8, Mx=32, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                              az=sc.target_az, el=sc.target_el, win_z=sc.win_z, win_x=sc.win_x,
                              delta=cfg.delta)
    ratio = oracle.subband_freq_ratio(cfg.K, cfg.beta)
    inr = 1e4
    for k in range(cfg.K):
        rows = r["rows"][0][k]
        w, a = r["w"][0, k, :15], r["a"][0, k, :15]
        omz, omx = upa.upa_spatial_frequencies(sc.jammer_az[0], sc.jammer_el[0], ratio[k])
        aj = upa.upa_beamspace(upa.upa_steering(4, 16, omz, omx)[:, None], 4, 8, 32)[rows, 0]
        wc = a / np.vdot(a, a)
        jnr = inr * abs(np.vdot(w, aj)) ** 2 / np.vdot(w, w).real
        jnr_conv = inr * abs(np.vdot(wc, aj)) ** 2 / np.vdot(wc, wc).real
        assert abs(np.vdot(w, a) - 1.0) < 1e-12
        assert jnr < 2.0
        if jnr_conv > 10.0:
            assert jnr < jnr_conv / 100.0


def test_lift_of_separable_window_weights_is_kronecker_of_1d_lifts():
    # c~ = u kron v over (ix_w, iz_w) lifts to (lift_x u) kron (lift_z v), the 1-D lifts of Eq. 21
    Nz, Nx, Mz, Mx, Wz, Wx, sz, sx = 4, 16, 8, 32, 3, 5, 6, 29
    u, v = _rand((Wx,), 8), _rand((Wz,), 9)
    rows = upa.upa_window_rows(sz, sx, Wz, Wx, Mz, Mx)
    c = upa.upa_lift_correlator(np.kron(u, v), rows, Nz, Nx, Mz, Mx)
    cx = oracle.lift_correlator(u, oracle.window_bins(sx, Wx, Mx), Mx, Nx)
    cz = oracle.lift_correlator(v, oracle.window_bins(sz, Wz, Mz), Mz, Nz)
    assert np.max(np.abs(c - np.kron(cx, cz))) < 1e-12


def test_planar_beam_pattern_of_kronecker_correlator_is_product_of_1d_patterns():
    # |<cx kron cz, ax kron az>| = |<cx, ax>| |<cz, az>| and the norms multiply
    Nz, Nx = 4, 12
    cx, cz = _rand((Nx,), 10), _rand((Nz,), 11)
    rng = np.random.default_rng(12)
    om = rng.uniform(-math.pi, math.pi, size=(20, 2))
    B2 = upa.upa_beam_pattern(np.kron(cx, cz), Nz, om)
    Bx = oracle.beam_pattern(cx, om[:, 1])
    Bz = oracle.beam_pattern(cz, om[:, 0])
    assert np.max(np.abs(B2 - Bx * Bz)) < 1e-12


def test_planar_matched_filter_pattern_peaks_at_its_direction():
    Nz, Nx = 4, 32
    a0 = upa.upa_steering(Nz, Nx, 0.7, -1.1)
    B = upa.upa_beam_pattern(a0, Nz, [(0.7, -1.1), (0.7 + 2 * math.pi / Nz, -1.1),
                                      (0.7, -1.1 + 2 * math.pi / Nx)])
    assert abs(B[0] - 1.0) < 1e-12 and B[1] < 1e-12 and B[2] < 1e-12   # first nulls
