"""GPU parity of the steps beside the beamformer: subband synthesis (inverse channelizer per
test block), lifted correlators (Eq. 21) and their use in element space, against the FP64
oracle on the same seeded complex64 inputs.

Bounds (u = 2^-24, FP32 unit roundoff):
* synthesis: a radix-8/4/2 FFT of K points in FP32 is off by at most about log2(K) u times the
  block's 2-norm per output (unitary transform); the test allows 4 log2(K) u ||Z[t, :, b]||.
* lift: W products of FP32 weights with FP32-rounded table twiddles, summed in FP64: at most
  2 u sum|w| / sqrt(M); allowed 4 u sum|w| / sqrt(M).
* element-space apply: an N-term FP32 dot product is off by at most (N + 2) u sum|c||X|; the
  FP32 channelizer adds at most about log2(K) u ||x block||_2 per X entry; allowed
  2 (N + 2) u sum|c||X| + 4 log2(K) u sum_n |c_n| ||x_{n,b}||_2.
"""

import math

import numpy as np
import pytest

import oracle
import scenes
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


def _crand(shape, seed):
    r = np.random.default_rng(seed)
    return (r.standard_normal(shape) + 1j * r.standard_normal(shape)).astype(np.complex64)


SHAPES = [
    dict(N=16, M=32, K=16, L=64, Lt=64, T=2),      # small
    dict(N=256, M=512, K=128, L=256, Lt=256, T=8),  # gpu workload
    dict(N=20, M=64, K=32, L=9, Lt=37, T=3),        # ragged test blocks (37 = 2 tiles + 5)
    dict(N=5, M=8, K=2, L=3, Lt=5, T=1),            # two subbands
    dict(N=33, M=128, K=512, L=2, Lt=3, T=2),       # K = 512, fewer blocks than one tile
]


@pytest.mark.parametrize("half_bin", [False, True])
@pytest.mark.parametrize("sh", SHAPES, ids=lambda d: f"N{d['N']}K{d['K']}Lt{d['Lt']}")
def test_synthesis_matches_oracle(torch, wb, sh, half_bin):
    log(f"synthesis {sh} half_bin={half_bin}")
    plan = wb.Plan(sh["N"], sh["M"], sh["K"], sh["L"], sh["Lt"], sh["T"], 4, half_bin=half_bin)
    T, K, Lt = sh["T"], sh["K"], sh["Lt"]
    Z = _crand((T, K, Lt), 21)
    z = plan.synthesize(torch.from_numpy(Z).cuda())
    torch.cuda.synchronize()
    zg = z.cpu().numpy().astype(np.complex128)
    ref = oracle.synthesize(Z.astype(np.complex128), K, half_bin)
    blk = np.linalg.norm(Z.astype(np.complex128), axis=1)            # [T, Lt]
    tol = 4 * max(1, math.log2(K)) * U * np.repeat(blk, K, axis=1) + U * np.abs(ref)
    err = np.abs(zg - ref)
    log(f"  max err / tol {np.max(err / tol):.3f}")
    assert np.all(err <= tol)
    plan.close()


@pytest.mark.parametrize("sh", SHAPES[:3], ids=lambda d: f"N{d['N']}M{d['M']}")
def test_lift_matches_oracle(torch, wb, sh):
    N, M, K, T, wmax = sh["N"], sh["M"], sh["K"], sh["T"], 9
    plan = wb.Plan(N, M, K, sh["L"], sh["Lt"], T, wmax)
    w = _crand((T, K, wmax), 22)
    r = np.random.default_rng(23)
    starts = r.integers(-wmax, M, size=(T, K)).astype(np.int32)    # negative and wrapping starts
    c = plan.lift(torch.from_numpy(w).cuda(), torch.from_numpy(starts).cuda())
    torch.cuda.synchronize()
    cg = c.cpu().numpy().astype(np.complex128)
    for t in range(T):
        for k in range(K):
            bins = oracle.window_bins(int(starts[t, k]), wmax, M)
            ref = oracle.lift_correlator(w[t, k].astype(np.complex128), bins, M, N)
            tol = 4 * U * np.sum(np.abs(w[t, k])) / math.sqrt(M)
            assert np.max(np.abs(cg[t, k] - ref)) <= tol, (t, k)
    plan.close()


APPLY_SHAPES = SHAPES[:3] + [
    dict(N=100, M=128, K=16, L=8, Lt=150, T=40),   # T > 8: matrix-core product, ragged tiles
]


@pytest.mark.parametrize("half_bin", [False, True])
@pytest.mark.parametrize("sh", APPLY_SHAPES, ids=lambda d: f"N{d['N']}K{d['K']}Lt{d['Lt']}T{d['T']}")
def test_apply_lifted_matches_oracle(torch, wb, sh, half_bin):
    N, K, L, Lt, T = sh["N"], sh["K"], sh["L"], sh["Lt"], sh["T"]
    log(f"element-space apply {sh} half_bin={half_bin}")
    plan = wb.Plan(N, sh["M"], K, L, Lt, T, 4, half_bin=half_bin)
    x = _crand((N, (L + Lt) * K), 24)
    c = _crand((T, K, N), 25)
    out = plan.apply_lifted(torch.from_numpy(x).cuda(), torch.from_numpy(c).cuda())
    torch.cuda.synchronize()
    og = out.cpu().numpy().astype(np.complex128)
    x64, c64 = x.astype(np.complex128), c.astype(np.complex128)
    ref = oracle.lifted_outputs(x64, c64, K=K, L=L, Lt=Lt, half_bin=half_bin)
    X = oracle.channelize(x64, K, half_bin)                               # [N, B, K]
    xblk = np.linalg.norm(x64.reshape(N, L + Lt, K), axis=2)             # [N, B]
    worst = 0.0
    for t in range(T):
        for k in range(K):
            Xt = np.abs(X[:, L:L + Lt, k])                                 # [N, Lt]
            ac = np.abs(c64[t, k])
            tol = (2 * (N + 2) * U * (ac @ Xt)
                   + 4 * max(1, math.log2(K)) * U * (ac @ xblk[:, L:L + Lt]))
            err = np.abs(og[t, k] - ref[t, k])
            worst = max(worst, float(np.max(err / tol)))
            assert np.all(err <= tol), (t, k)
    log(f"  max err / tol {worst:.3f}")
    plan.close()


def test_lifted_path_reproduces_windowed_outputs(torch, wb):
    # beamform -> lift -> element-space apply gives the beamformer's own outputs (Eq. 21)
    cfg = scenes.GPU
    sc = scenes.make_scene(cfg)
    x = torch.from_numpy(sc.x.astype(np.complex64)).cuda()
    plan = wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, cfg.T, int(max(sc.win)), beta=cfg.beta,
                   d_over_lambda=cfg.dl)
    res = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form="fused")
    c = plan.lift(res["weights"], res["starts"])
    z = plan.apply_lifted(x, c)
    torch.cuda.synchronize()
    a, b = z.cpu().numpy(), res["out"].cpu().numpy()
    rel = np.max(np.abs(a - b)) / np.max(np.abs(b))
    log(f"  lifted vs windowed outputs: max rel diff {rel:.2e}")
    assert rel < 2e-5
    # and the synthesized wideband outputs of both agree
    za = plan.synthesize(z).cpu().numpy()
    zb = plan.synthesize(res["out"]).cpu().numpy()
    assert np.max(np.abs(za - zb)) / np.max(np.abs(zb)) < 2e-5
    plan.close()


def test_synthesis_and_lift_reject_bad_arguments(torch, wb):
    plan = wb.Plan(16, 32, 16, 8, 8, 2, 5)
    with pytest.raises(wb.WbmError):
        plan.synthesize(torch.zeros((3, 16, 8), dtype=torch.complex64, device="cuda"))  # T > max
    with pytest.raises(ValueError):
        plan.synthesize(torch.zeros((2, 16, 7), dtype=torch.complex64, device="cuda"))   # shape
    plan.close()


@pytest.mark.parametrize("N", [24, 256])
def test_beam_pattern_matches_oracle(torch, wb, N):
    # FP64 sums and phase recurrence on the GPU; the FP32 result is within 1e-6 of the oracle
    plan = wb.Plan(N, 1 << (2 * N - 1).bit_length(), 4, 4, 4, 2, 5)
    c = _crand((2, 3, N), 26)
    omegas = np.concatenate([np.linspace(-math.pi, math.pi, 181), [0.0, 0.7, 3 * math.pi]])
    pat = plan.beam_pattern(torch.from_numpy(c).cuda(), torch.from_numpy(omegas).cuda())
    torch.cuda.synchronize()
    pg = pat.cpu().numpy()
    for i in range(2):
        for j in range(3):
            ref = oracle.beam_pattern(c[i, j].astype(np.complex128), omegas)
            assert np.max(np.abs(pg[i, j] - ref)) < 1e-6
    # a matched filter is a normalised Dirichlet kernel with its peak of 1 at its own angle
    a = np.exp(1j * 0.7 * np.arange(N)).astype(np.complex64)
    pk = plan.beam_pattern(torch.from_numpy(a).cuda(), torch.tensor([0.7], dtype=torch.float64,
                                                                   device="cuda"))
    assert abs(float(pk.cpu()[0]) - 1.0) < 1e-6
    plan.close()
