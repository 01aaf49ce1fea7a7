"""Pins of the predictor data path: profile by direct DFT rows, BF16 rounding on known values,
decision rule, label tie rules by brute force."""

import math

import numpy as np

import oracle
from oracle import learned


def test_bf16_round_known_values():
    one = 1.0
    ulp = 2.0 ** -7                       # bf16 spacing at 1.0
    vals = np.array([1.0, 1.0 + ulp / 2, 1.0 + 3 * ulp / 2, 1.0 + ulp / 4, -2.5, 3.0e-3, 65504.0],
                    dtype=np.float32)
    r = learned.bf16_round(vals)
    assert r[0] == one
    assert r[1] == one                      # tie -> even mantissa
    assert r[2] == 1.0 + 2 * ulp            # tie -> even (rounds up)
    assert r[3] == one
    assert r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    assert r[6] == 65536.0 or r[6] == 65280.0


def test_power_profile_matches_direct_dft_rows():
    rng = np.random.default_rng(0)
    N, M, L = 12, 32, 20
    Xk = rng.standard_normal((N, L)) + 1j * rng.standard_normal((N, L))
    Y = oracle.beamspace(Xk[:, :, None], M)[:, :, 0]
    u = 7.4
    f = learned.power_profile(Y, u, 2.0)
    c = 7
    for j in (0, 5, 31, 32, 63):
        m = (c - 32 + j) % M
        row = oracle.beamspace_rows(Xk, M, [m])[0]
        assert abs(f[j] - math.log10(np.mean(np.abs(row) ** 2) / 2.0 + 1e-30)) < 1e-12


def test_decision_rule():
    assert learned.decision(math.log(10.0), 3.0, 1.0) == (9, 10.0 * 1.0) or \
        abs(learned.decision(math.log(10.0), 3.0, 1.0)[1] - 10.0) < 1e-12
    W, d = learned.decision(50.0, 9.7, 2.0)
    assert W == 33 and abs(d - 2.0 * 1e4) < 1e-6
    W, d = learned.decision(-50.0, -3.0, 1.0)
    assert W == 5 and abs(d - 0.1) < 1e-12
    W, d = learned.decision(0.0, 3.5, 1.0)      # rint half to even -> 4 -> W = 17
    assert W == 17
    assert learned.decision(float("nan"), 1.0, 1.0, fb_win=9, fb_delta=10.0) == (9, 10.0)


def test_sweep_label_ties_and_argmax():
    deltas = learned.SWEEP_DELTAS
    widths = learned.SWEEP_WIDTHS
    rng = np.random.default_rng(1)
    for _ in range(50):
        tab = rng.integers(0, 4, size=(len(deltas), len(widths))).astype(float)
        ld, lw = learned.sweep_label(tab, deltas, widths, 1.0)
        best = tab.max()
        cands = [(iw, -idl) for iw in range(len(widths)) for idl in range(len(deltas))
                 if tab[idl, iw] == best]
        iw, midl = min(cands)
        assert abs(ld - math.log(deltas[-midl])) < 1e-12
        assert abs(lw - math.log2(widths[iw] - 1)) < 1e-12
