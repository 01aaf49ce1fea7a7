"""GPU parity of range-Doppler processing and 1-D CFAR against the FP64 oracle, on seeded
pulse trains with point targets in noise.

Bound (u = 2^-24): each compressed sample comes from two FP32 F-point FFTs of a zero-padded
pulse times the chirp spectrum, the Doppler value from one more P-point FFT, so an RD value is
off by at most about (2 log2 F + log2 P + 4) u sqrt(P) ||c|| max_p ||z_p||; the test allows
four times that (E), |power error| <= 2 sqrt(power) E + E^2, and compares CFAR decisions on
every cell whose margin |power - alpha noise| exceeds the error bound of both terms (cells
closer to the threshold may go either way); the true targets must be detected."""

import cmath
import math

import numpy as np
import pytest

from oracle import radar
from gpu_helpers import log

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    _t.cuda.set_device(0)
    return _t


@pytest.fixture(scope="module")
def wb():
    import paper_2508_11790_amd as _wb
    return _wb


def _train(T, R, P, Lp, stride, targets, noise, seed):
    c = radar.lfm_chirp(Lp)
    r = np.random.default_rng(seed)
    z = noise * (r.standard_normal((T, stride)) + 1j * r.standard_normal((T, stride))) / math.sqrt(2)
    for t, d0, v0, A in targets:
        for p in range(P):
            m = min(Lp, R - d0)
            z[t, p * R + d0:p * R + d0 + m] += A * c[:m] * cmath.exp(2j * math.pi * v0 * p / P)
    return z.astype(np.complex64), c.astype(np.complex64)


CASES = [
    dict(R=200, P=32, Lp=40, stride=32 * 200 + 7, guard=2, train=8,
         targets=[(0, 30, 5, 1.0), (0, 120, 20, 0.3), (1, 75, 31, 2.0)]),
    dict(R=5, P=2, Lp=5, stride=10, guard=0, train=1, targets=[(0, 0, 1, 3.0)]),
    dict(R=4096, P=64, Lp=512, stride=64 * 4096, guard=4, train=16,
         targets=[(0, 1000, 10, 0.5)]),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"R{c['R']}P{c['P']}Lp{c['Lp']}")
def test_range_doppler_and_cfar_match_oracle(torch, wb, case):
    R, P, Lp, stride = case["R"], case["P"], case["Lp"], case["stride"]
    T = 1 + max(t for t, *_ in case["targets"])
    log(f"range-Doppler {case}")
    z, c = _train(T, R, P, Lp, stride, case["targets"], 0.1, 31)
    plan = wb.Plan(16, 32, 4, 4, 4, 1, 5)
    power, det = plan.range_doppler(torch.from_numpy(z).cuda(), torch.from_numpy(c).cuda(), R, P,
                                    case["guard"], case["train"], 10.0)
    torch.cuda.synchronize()
    pg, dg = power.cpu().numpy().astype(np.float64), det.cpu().numpy()
    alpha = 10.0
    F = 1 << max(1, (R + Lp - 2).bit_length())
    compared = total = 0
    for t in range(T):
        pr, nr, dr = radar.range_doppler(z[t].astype(np.complex128), c.astype(np.complex128), R, P,
                                         case["guard"], case["train"], 10.0)
        zmax = max(np.linalg.norm(z[t, p * R:(p + 1) * R].astype(np.complex128)) for p in range(P))
        E = 4 * (2 * math.log2(F) + math.log2(P) + 4) * U * math.sqrt(P) * np.linalg.norm(c) * zmax
        tolp = 2 * np.sqrt(pr) * E + E * E
        assert np.all(np.abs(pg[t] - pr) <= tolp), t
        # CFAR decisions away from the threshold must agree exactly
        tn = np.zeros_like(nr)
        for d in range(R):
            idx = [dd for dd in range(R) if case["guard"] < abs(dd - d) <= case["guard"] + case["train"]]
            if idx:
                tn[d] = tolp[idx].mean(axis=0)
        margin = np.abs(pr - alpha * nr)
        sure = np.isfinite(nr) & (margin > tolp + alpha * tn)
        assert np.array_equal(dg[t][sure].astype(bool), dr[sure]), t
        compared += int(sure.sum())
        total += sure.size
        for tt, d0, v0, A in case["targets"]:
            if tt == t:
                assert dr[d0, v0] and dg[t, d0, v0] == 1, (d0, v0)
    log(f"  decisions compared on {compared} of {total} cells")
    assert compared >= 0.9 * total
    plan.close()


def test_range_doppler_rejects_bad_sizes(torch, wb):
    plan = wb.Plan(16, 32, 4, 4, 4, 1, 5)
    z = torch.zeros((1, 64), dtype=torch.complex64, device="cuda")
    c = torch.zeros((8,), dtype=torch.complex64, device="cuda")
    with pytest.raises(wb.WbmError):
        plan.range_doppler(z, c, 16, 3)          # P not a power of two
    with pytest.raises(wb.WbmError):
        plan.range_doppler(z, c, 4, 2)           # Lp > R
    with pytest.raises(wb.WbmError):
        plan.range_doppler(z, c, 16, 8)          # P R > z stride
    plan.close()
