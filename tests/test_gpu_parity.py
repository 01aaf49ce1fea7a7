"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle on the same
seeded complex64 inputs -- stage by stage, end to end, and on edge cases."""

import math

import numpy as np
import pytest

import oracle
import scenes
from gpu_helpers import (compare_beamform, log, loss_by_pivot_ratio, snapshot_dynamic_range,
                         weight_tol)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    _t.cuda.set_device(0)
    return _t


@pytest.fixture(scope="module")
def wb():
    import paper_2508_11790_amd as _wb
    return _wb


def _plan(wb, cfg, scene):
    return wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, len(scene.win), int(max(scene.win)),
                   beta=cfg.beta, d_over_lambda=cfg.dl, half_bin=cfg.half_bin)


def _x32(scene):
    return scene.x.astype(np.complex64)


def _oracle(scene, x32, subbands=None, windows=True):
    cfg = scene.cfg
    return oracle.windowed_mvdr(x32.astype(np.complex128), M=cfg.M, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                                sin_az=[math.sin(a) for a in scene.target_az], win=scene.win,
                                delta=cfg.delta, beta=cfg.beta, dl=cfg.dl, half_bin=cfg.half_bin,
                                subbands=subbands, return_windows=windows)


# ----------------------------------------------------------------------------- stages

@pytest.mark.parametrize("half_bin", [False, True])
@pytest.mark.parametrize("shape", [(16, 32, 16, 64, 64), (20, 32, 8, 37, 11), (256, 512, 128, 256, 256),
                                   (4, 4, 2, 3, 1),
                                   # N = M/2 with 301 snapshots: whole tiles and a ragged last one
                                   # at every tile size
                                   (16, 32, 4, 200, 101)])
def test_channelizer_and_beamspace_stages(torch, wb, shape, half_bin):
    N, M, K, L, Lt = shape
    log(f"stage case N={N} M={M} K={K} L={L} Lt={Lt} half_bin={half_bin}")
    rng = np.random.default_rng(N + K)
    B = L + Lt
    x = (rng.standard_normal((N, B * K)) + 1j * rng.standard_normal((N, B * K))).astype(np.complex64)
    plan = wb.Plan(N, M, K, L, Lt, 1, 1, half_bin=half_bin)
    X_g = plan.channelize(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    X_o = oracle.channelize(x.astype(np.complex128), K, half_bin)            # [N, B, K]
    d = np.max(np.abs(X_g.cpu().numpy().transpose(2, 1, 0) - X_o)) / np.max(np.abs(X_o))
    assert d < 2e-6, d
    # beamspace fed with the oracle's X rounded to complex64
    X32 = X_o.astype(np.complex64)
    Y_g = plan.beamspace(torch.from_numpy(np.ascontiguousarray(X32.transpose(2, 1, 0))).cuda())
    torch.cuda.synchronize()
    Y_o = oracle.beamspace(X32.astype(np.complex128), M)                   # [M, B, K]
    d = np.max(np.abs(Y_g.cpu().numpy().transpose(1, 2, 0) - Y_o)) / np.max(np.abs(Y_o))
    assert d < 2e-6, d
    plan.close()


@pytest.mark.parametrize("half_bin", [False, True])
@pytest.mark.parametrize("N,M,K,wmax", [(16, 32, 16, 5), (256, 512, 128, 9), (1024, 2048, 256, 33),
                                        (4096, 8192, 512, 64), (7, 8, 4, 8)])
def test_window_starts_bit_exact_and_steering(torch, wb, N, M, K, wmax, half_bin):
    log(f"steer case N={N} M={M} K={K} wmax={wmax}")
    rng = np.random.default_rng(N)
    T = 48
    az = np.deg2rad(rng.uniform(-89, 89, size=T))
    az[:6] = np.deg2rad([0.0, 30.0, -30.0, 90.0, -90.0, 10.0])
    win = rng.integers(1, wmax + 1, size=T).astype(np.int32)
    win[:4] = [wmax, 1, 2, min(4, wmax)]
    plan = wb.Plan(N, M, K, 1, 1, T, wmax, half_bin=half_bin)
    starts, abar = plan.steer(az, win)
    torch.cuda.synchronize()
    starts = starts.cpu().numpy()
    abar = abar.cpu().numpy()
    ratio = oracle.subband_freq_ratio(K, 0.2, half_bin)
    for t in range(T):
        s_az = math.sin(az[t])
        for k in range(K):
            u = oracle.beam_position(s_az, ratio[k], M, 0.5)
            s = oracle.window_start(u, int(win[t]))
            assert starts[t, k] == s, (t, k, u)
        for k in (0, K // 2, K - 1, 1):
            bins = oracle.window_bins(int(starts[t, k]), int(win[t]), M)
            a = oracle.beamspace_steering(N, M, oracle.spatial_frequency(s_az, ratio[k], 0.5), bins)
            assert np.max(np.abs(abar[t, k, :win[t]] - a)) < 1e-11 * max(1.0, N / math.sqrt(M))
            assert np.all(abar[t, k, win[t]:] == 0)
    plan.close()


# ----------------------------------------------------------------------------- end to end

EXT_FORMS = ("fused", "graph")   # extended-precision transforms: held to 1e-5 and 0.1 dB


@pytest.mark.parametrize("form", ["plain", "fused", "graph", "fused_f32", "graph_f32"])
@pytest.mark.parametrize("half_bin", [False, True])
def test_small_config_end_to_end(torch, wb, form, half_bin):
    cfg = scenes.SMALL.replace(half_bin=half_bin)
    log(f"small end-to-end form={form} half_bin={half_bin}")
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    res = plan.beamform(torch.from_numpy(x32).cuda(), sc.target_az, sc.win, cfg.delta, form=form)
    torch.cuda.synchronize()
    st = compare_beamform(sc, ref, res, plain=(form == "plain"), ext=form in EXT_FORMS)
    log(f"  {st}")
    assert st["max_weight_err"] < 1e-5
    plan.close()


@pytest.mark.parametrize("form", ["plain", "fused", "graph", "fused_f32"])
def test_gpu_config_all_pairs(torch, wb, form):
    cfg = scenes.GPU
    log(f"gpu config (N=256 M=512 K=128 W=9 L=256) all 1024 pairs form={form}")
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    res = plan.beamform(torch.from_numpy(x32).cuda(), sc.target_az, sc.win, cfg.delta, form=form)
    torch.cuda.synchronize()
    st = compare_beamform(sc, ref, res, plain=(form == "plain"), ext=form in EXT_FORMS)
    log(f"  {st}")
    assert st["max_weight_err"] < 1e-5       # seeded scene: every window is well conditioned
    plan.close()


def test_batch_config_full_size_sampled_subbands(torch, wb):
    """Batching workload at full size (N=1024, M=2048, K=256, L=Lt=512, 64 targets, W in
    {5, 9, 17, 33}, 6 jammers up to 50 dB): fused and graph forms within 1e-5 / 0.1 dB of the
    oracle on six subbands (every target); the FP32-transform form within its derived bound."""
    cfg = scenes.BATCH
    log("batch config (N=1024 M=2048 K=256 L=512, W in {5,9,17,33}, 64 targets): generating")
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    plan = _plan(wb, cfg, sc)
    xd = torch.from_numpy(x32).cuda()
    ks = [0, 1, 77, 128, 200, 255]
    log("  oracle on sampled subbands")
    ref = _oracle(sc, x32, subbands=ks)
    for form in ("fused", "graph", "fused_f32", "mixed", "mixed_bf16"):
        res = dict(plan.beamform(xd, sc.target_az, sc.win, cfg.delta, form=form))
        torch.cuda.synchronize()
        mixed = form.startswith("mixed")
        if mixed:
            info = res["info"].cpu().numpy()
            assert np.all((info & ~wb.INFO_ROUTED) == 0), "Cholesky failures"
            log(f"  {form}: routed to FP64: {int(((info & wb.INFO_ROUTED) != 0).sum())}")
            res["info"] = torch.zeros_like(res["info"])
        st = compare_beamform(sc, ref, res, subbands=ks, ext=form in EXT_FORMS,
                              tol_scale=None if mixed else 1.0,
                              pairs=True)
        pp = st.pop("per_pair")
        log(f"  {form}: {st}")
        if mixed:
            log(f"    by pivot ratio (oracle LDL^H): {loss_by_pivot_ratio(pp)}")
    del xd
    plan.close()


def _host_channelize_bins(x, K, ks, half_bin, chunk=64):
    """Oracle channelizer (direct DFT at the listed bins) of a device-resident x, copied to the
    host in chunks of elements: [N, B, len(ks)] complex128."""
    parts = []
    for e0 in range(0, x.shape[0], chunk):
        parts.append(oracle.channelize_bins(x[e0:e0 + chunk].cpu().numpy(), K, ks, half_bin))
        if (e0 // chunk) % 16 == 15:
            log(f"    elements {e0 + chunk}/{x.shape[0]}")
    return np.concatenate(parts, axis=0)


@pytest.mark.timeout(1200)
def test_precision_config_full_size_sampled_subbands(torch, wb):
    """Precision workload at full size (N=4096, M=8192, K=512, L=Lt=1024, W=64, 32 targets,
    8 jammers of 20-60 dB; 34 GB of samples generated on the device): on four subbands, every
    target, against the FP64 oracle on the same complex64 samples -- the fused and graph forms
    within 1e-5 relative weight error and 0.1 dB SINR loss; the mixed forms (BF16 covariance)
    and the FP32-transform form within 0.1 dB, their weight errors stated."""
    cfg = scenes.PRECISION
    log("precision config (N=4096 M=8192 K=512 L=Lt=1024 W=64, 32 targets): generating")
    sc, x = scenes.make_scene_torch(cfg, cfg.seed)
    torch.cuda.synchronize()
    ks = [0, 129, 256, 511]
    log(f"  oracle channelizer on subbands {ks} (host)")
    X = _host_channelize_bins(x, cfg.K, ks, cfg.half_bin)
    ref = oracle.windowed_mvdr(None, X=X, M=cfg.M, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                               sin_az=[math.sin(a) for a in sc.target_az], win=sc.win,
                               delta=cfg.delta, beta=cfg.beta, dl=cfg.dl, half_bin=cfg.half_bin,
                               subbands=ks, return_windows=True)
    del X
    plan = _plan(wb, cfg, sc)
    for form in ("fused", "graph", "fused_f32", "mixed", "mixed_bf16"):
        log(f"  form {form}")
        res = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form)
        torch.cuda.synchronize()
        res = dict(res)
        if form.startswith("mixed"):
            info = res["info"].cpu().numpy()
            assert np.all((info & ~wb.INFO_ROUTED) == 0), "Cholesky failures"
            log(f"    routed to FP64: {int(((info & wb.INFO_ROUTED) != 0).sum())}")
            res["info"] = torch.zeros_like(res["info"])
        st = compare_beamform(sc, ref, res, subbands=ks, ext=form in EXT_FORMS,
                              tol_scale=1.0 if form in EXT_FORMS else None, pairs=True)
        pp = st.pop("per_pair")
        log(f"    {st}")
        if form.startswith("mixed"):
            log(f"    by pivot ratio (oracle LDL^H): {loss_by_pivot_ratio(pp)}")
    del x
    plan.close()


@pytest.mark.timeout(900)
def test_precision_config_every_jammer_at_60db(torch, wb):
    """The precision workload's array and targets with all eight jammers at the workload's
    largest INR (60 dB): the extended-precision forms still within 1e-5 relative weight error
    and 0.1 dB SINR loss on three subbands (every target); the FP32-transform error logged."""
    cfg = scenes.PRECISION.replace(name="precision_60dB", inr_range_db=(60.0, 60.0), seed=777)
    log("precision config with 8 jammers at 60 dB: generating")
    sc, x = scenes.make_scene_torch(cfg, cfg.seed)
    torch.cuda.synchronize()
    ks = [0, 200, 400]
    X = _host_channelize_bins(x, cfg.K, ks, cfg.half_bin)
    ref = oracle.windowed_mvdr(None, X=X, M=cfg.M, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                               sin_az=[math.sin(a) for a in sc.target_az], win=sc.win,
                               delta=cfg.delta, beta=cfg.beta, dl=cfg.dl, half_bin=cfg.half_bin,
                               subbands=ks, return_windows=True)
    del X
    plan = _plan(wb, cfg, sc)
    for form in ("graph", "graph_f32"):
        res = dict(plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form))
        torch.cuda.synchronize()
        ext = form == "graph"
        st = compare_beamform(sc, ref, res, subbands=ks, ext=ext,
                              tol_scale=1.0 if ext else None)
        log(f"  {form}: {st}")
    del x
    plan.close()


def _pin(plan, pair, overlap=1, precision="ext"):
    chan, beam, _, _ = plan.get_tuning(precision)
    plan.set_tuning(chan, beam, pair, overlap, precision=precision)
    assert plan.get_tuning(precision)[2:] == (pair, overlap)


# pair kernels each precision of the fused sequence runs: the extended-precision windows are
# staged as FP64 by the vector kernels; the FP64 matrix-core and LDS-resident kernels read FP32
PAIR_FORMS = [("fused", "ext", "wave"), ("fused", "ext", "block"),
              ("fused_f32", "f32", "mfma"), ("fused_f32", "f32", "wave"),
              ("fused_f32", "f32", "block"), ("fused_f32", "f32", "resident")]


@pytest.mark.parametrize("form,precision,pair", PAIR_FORMS)
@pytest.mark.parametrize("name", ["small", "gpu"])
def test_pair_kernels_match_oracle(torch, wb, name, form, precision, pair):
    cfg = scenes.config_by_name(name)
    log(f"pair kernel {pair} ({form}) on the {name} config, all pairs")
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    _pin(plan, pair, precision=precision)
    res = plan.beamform(torch.from_numpy(x32).cuda(), sc.target_az, sc.win, cfg.delta, form=form)
    torch.cuda.synchronize()
    st = compare_beamform(sc, ref, res, ext=form in EXT_FORMS)
    log(f"  {st}")
    assert st["max_weight_err"] < 1e-5
    plan.close()


@pytest.mark.parametrize("form", ["fused", "graph"])
@pytest.mark.parametrize("overlap", [2, 4])
def test_overlapped_subband_chunks_match_oracle(torch, wb, overlap, form):
    # spatial DFT and pair kernel overlapped over subband chunks on two streams (graph: fork/join)
    cfg = scenes.GPU
    log(f"overlap {overlap} chunks, form {form}, gpu config all pairs")
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    _pin(plan, "block", overlap)
    x = torch.from_numpy(x32).cuda()
    res = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form)
    torch.cuda.synchronize()
    st = compare_beamform(sc, ref, res, ext=True)
    log(f"  {st}")
    assert st["max_weight_err"] < 1e-5
    # same results as the unchunked sequence, every replay
    _pin(plan, "block", 1)
    one = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form="fused")
    _pin(plan, "block", overlap)
    for rep in range(3):
        again = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form)
        torch.cuda.synchronize()
        assert torch.equal(again["out"], one["out"]), rep
        assert torch.equal(again["weights"], one["weights"]), rep
    plan.close()


@pytest.mark.parametrize("form,precision,pair", [("fused_f32", "f32", "mfma"),
                                                  ("fused_f32", "f32", "block"),
                                                  ("fused", "ext", "wave")])
def test_pair_kernels_batch_config_sampled_subbands(torch, wb, form, precision, pair):
    cfg = scenes.BATCH
    log(f"pair kernel {pair} ({form}), batch config (W in {{5,9,17,33}}, 64 targets), "
        f"sampled subbands")
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    plan = _plan(wb, cfg, sc)
    _pin(plan, pair, precision=precision)
    xd = torch.from_numpy(x32).cuda()
    res = plan.beamform(xd, sc.target_az, sc.win, cfg.delta, form=form)
    torch.cuda.synchronize()
    ks = [0, 3, 130, 255]
    ref = _oracle(sc, x32, subbands=ks)
    st = compare_beamform(sc, ref, res, subbands=ks, ext=form in EXT_FORMS)
    log(f"  {st}")
    del xd
    plan.close()


def test_graph_replays_match_eager(torch, wb):
    cfg = scenes.GPU
    sc = scenes.make_scene(cfg)
    x = torch.from_numpy(_x32(sc)).cuda()
    plan = _plan(wb, cfg, sc)
    eager = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form="fused")
    e_out = eager["out"].clone()
    e_w = eager["weights"].clone()
    out = torch.empty_like(e_out)
    w = torch.empty_like(e_w)
    for rep in range(4):
        out.zero_()
        w.zero_()
        plan.beamform(x, sc.target_az, sc.win, cfg.delta, form="graph", out=out, weights=w)
        torch.cuda.synchronize()
        assert torch.equal(out, e_out), rep
        assert torch.equal(w, e_w), rep
        # eager work between replays
        plan.beamform(x, sc.target_az, sc.win, cfg.delta, form="fused")
        torch.cuda.synchronize()
    plan.close()


# ----------------------------------------------------------------------------- edge cases

@pytest.mark.parametrize("case", [
    dict(N=20, M=32, K=8, L=37, Lt=11, W=(4, 1, 32, 7)),       # ragged snapshots, even W, W = M
    dict(N=5, M=8, K=2, L=9, Lt=3, W=(8, 3)),                   # tiny, full window
    dict(N=33, M=64, K=4, L=70, Lt=0, W=(5, 6)),                # no test snapshots
    dict(N=16, M=16, K=16, L=40, Lt=40, W=(16,)),               # M = N (unitary D)
    dict(N=16, M=32, K=4, L=200, Lt=101, W=(5, 3)),             # N = M/2: whole and ragged tiles
])
def test_edge_shapes(torch, wb, case):
    W = case["W"]
    T = len(W)
    log(f"edge case {case}")
    cfg = scenes.SceneConfig(name="edge", N=case["N"], M=case["M"], K=case["K"], L=case["L"],
                             Lt=case["Lt"], T=T, W=None, W_choices=(1,), n_jammers=1,
                             target_az_deg=tuple(np.linspace(-40, 50, T)),
                             target_snr_db=(0.0,) * T, jammer_az_deg=(-70.0,),
                             jammer_inr_db=(25.0,), seed=11)
    sc = scenes.make_scene(cfg)
    sc.win = np.asarray(W, dtype=np.int32)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    runs = [("plain", None, None), ("fused", "block", "ext"), ("fused_f32", "mfma", "f32"),
            ("fused_f32", "block", "f32"), ("fused_f32", "resident", "f32")]
    if max(W) <= 40:
        runs += [("fused", "wave", "ext"), ("fused_f32", "wave", "f32")]
    for form, pair, precision in runs:
        if pair:
            _pin(plan, pair, precision=precision)
        res = plan.beamform(torch.from_numpy(x32).cuda(), sc.target_az, sc.win, cfg.delta, form=form)
        torch.cuda.synchronize()
        compare_beamform(sc, ref, res, plain=(form == "plain"), ext=form in EXT_FORMS)
    plan.close()


@pytest.mark.parametrize("beam_tile", [12, 13])
def test_extended_precision_spatial_dft_at_8192_bins(torch, wb, beam_tile):
    """M = 8192 with N <= 4096: the extended-precision spatial DFT splits every row into its
    even- and odd-bin 4096-point halves (tile 2^13: the radix-16 engine, 256 threads; below:
    the radix-8 engine, 512 threads); windows of 64, 5 and 33 bins, one next to the wrap, the
    others at the band centre and edge; N not a multiple of the thread count."""
    cfg = scenes.SceneConfig(name="m8192", N=300, M=8192, K=4, L=50, Lt=10, T=3, W=None,
                             W_choices=(1,), n_jammers=1, target_az_deg=(-89.0, 0.0, 55.0),
                             target_snr_db=(5.0, 0.0, 10.0), jammer_az_deg=(20.0,),
                             jammer_inr_db=(40.0,), seed=31)
    sc = scenes.make_scene(cfg)
    sc.win = np.asarray((64, 5, 33), dtype=np.int32)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    plan.set_tuning(11, beam_tile, "block", 1, precision="ext")
    x = torch.from_numpy(x32).cuda()
    for form in ("fused", "graph"):
        res = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form)
        torch.cuda.synchronize()
        st = compare_beamform(sc, ref, res, ext=True)
        log(f"  tile {beam_tile} {form}: {st}")
    # per-pair sub-windows of the gathered ones (the learned form's path): rows 16..47 of the
    # 64-bin window, 1..3 of the 5-bin one, 8..24 of the 33-bin one -- the oracle at those widths
    sub = np.asarray((32, 3, 17), dtype=np.int32)
    pw = torch.from_numpy(np.repeat(sub[:, None], cfg.K, axis=1)).cuda()
    pd = torch.full((cfg.T, cfg.K), cfg.delta, dtype=torch.float32, device="cuda")
    res = plan.beamform_pairs(x, sc.target_az, sc.win, pw, pd)
    torch.cuda.synchronize()
    sc_sub = scenes.make_scene(cfg)
    sc_sub.win = sub
    st = compare_beamform(sc_sub, _oracle(sc_sub, x32), res, ext=True)
    log(f"  tile {beam_tile} sub-windows: {st}")
    plan.close()


@pytest.mark.parametrize("beam_tile,form", [(13, "fused"), (13, "graph"), (12, "graph")])
def test_overlapped_chunks_at_8192_bins(torch, wb, beam_tile, form):
    """Two overlapped subband chunks at M = 8192 with N <= 4096: the split-half spatial DFTs
    (tile 2^13: radix-16, 2^12: radix-8) start each chunk at its first subband and the pair
    kernel of one chunk runs beside the transform of the next; every pair against the oracle,
    and the same outputs as the unchunked sequence bit for bit."""
    cfg = scenes.SceneConfig(name="m8192k16", N=300, M=8192, K=16, L=40, Lt=8, T=3, W=None,
                             W_choices=(1,), n_jammers=1, target_az_deg=(-60.0, 0.0, 35.0),
                             target_snr_db=(5.0, 0.0, 10.0), jammer_az_deg=(20.0,),
                             jammer_inr_db=(40.0,), seed=43)
    sc = scenes.make_scene(cfg)
    sc.win = np.asarray((64, 9, 33), dtype=np.int32)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    plan.set_tuning(11, beam_tile, "block", 1, precision="ext")
    x = torch.from_numpy(x32).cuda()
    one = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form="fused")
    plan.set_tuning(11, beam_tile, "block", 2, precision="ext")
    for rep in range(2):
        res = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form)
        torch.cuda.synchronize()
        st = compare_beamform(sc, ref, res, ext=True)
        log(f"  tile {beam_tile} {form} two chunks, call {rep}: {st}")
        assert torch.equal(res["out"], one["out"]), rep
        assert torch.equal(res["weights"], one["weights"]), rep
    plan.close()


def test_windows_of_61_to_64_bins(torch, wb):
    """Windows of 61, 62, 63 and 64 bins, where the pair kernels' Gram works on 16 block rows
    of 4 (the last one partly past W for 61..63): the four-wave vector kernel on extended
    windows (fused and graph forms) and on FP32 windows, and the FP64 matrix-core kernel on FP32
    windows, each against the oracle.  On FP32 windows the two pair kernels may return the same
    weights bit for bit: both sum exact products in FP64, and the rounding to FP32 hides the
    different summation orders."""
    cfg = scenes.SceneConfig(name="w61", N=64, M=128, K=4, L=192, Lt=8, T=4, W=None,
                             W_choices=(1,), n_jammers=2, target_az_deg=(-40.0, -5.0, 20.0, 55.0),
                             target_snr_db=(0.0, 5.0, -5.0, 10.0), jammer_az_deg=(30.0, -20.0),
                             jammer_inr_db=(35.0, 45.0), seed=61)
    sc = scenes.make_scene(cfg)
    sc.win = np.asarray((61, 62, 63, 64), dtype=np.int32)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    x = torch.from_numpy(x32).cuda()
    for form, pk, prec in (("fused", "block", "ext"), ("graph", "block", "ext"),
                           ("fused_f32", "block", "f32"), ("fused_f32", "mfma", "f32")):
        _pin(plan, pk, precision=prec)
        res = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form)
        torch.cuda.synchronize()
        st = compare_beamform(sc, ref, res, ext=form in EXT_FORMS)
        log(f"  {form} ({pk}): {st}")
    plan.close()


def test_window_rows_beyond_the_pinned_tile(torch, wb):
    """320 targets of 64 bins at M = 2048 (20480 window rows): the extended spatial DFT's 2^13
    tile (128 KiB of LDS) cannot hold their row table beside it, so a call with that tile pinned
    runs at, and moves the plan to, 2^12, with the pair kernels following the smaller tile's
    window layout; every target's weights on two subbands still match the oracle (fused, graph,
    fused_f32 and mixed forms).  The FP32 2^13 tile (64 KiB) holds the table and stays."""
    # jammer directions fixed: 320 targets leave no sin-space gap the random draw accepts
    cfg = scenes.SceneConfig(name="rows", N=64, M=2048, K=4, L=160, Lt=16, T=320, W=64,
                             n_jammers=2, jammer_az_deg=(20.0, -35.0),
                             jammer_inr_db=(30.0, 40.0), seed=41)
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    ks = [0, 3]
    ref = _oracle(sc, x32, subbands=ks)
    plan = _plan(wb, cfg, sc)
    plan.set_tuning(12, 13, "block", 1, precision="ext")
    plan.set_tuning(12, 13, "block", 1, precision="f32")
    x = torch.from_numpy(x32).cuda()
    for form in ("fused", "graph", "fused_f32", "mixed"):
        res = dict(plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form))
        torch.cuda.synchronize()
        if form == "mixed":
            info = res["info"].cpu().numpy()
            assert np.all((info & ~wb.INFO_ROUTED) == 0), "Cholesky failures"
            res["info"] = torch.zeros_like(res["info"])
        st = compare_beamform(sc, ref, res, subbands=ks, ext=form in EXT_FORMS,
                              tol_scale=None if form == "mixed" else 1.0)
        log(f"  {form}: {st}")
    assert plan.get_tuning("ext")[1] == 12
    assert plan.get_tuning("f32")[1] == 13
    plan.close()


def test_identity_windowed_equals_full_dimensional(torch, wb):
    # W = M = N: the windowed beamspace MVDR equals element-space MVDR (Eq. 13 vs Eq. 20-21)
    cfg = scenes.SMALL.replace(M=16, W=16)
    sc = scenes.make_scene(cfg)
    x = torch.from_numpy(_x32(sc)).cuda()
    plan = _plan(wb, cfg, sc)
    bm = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form="fused")
    fm = plan.full_mvdr(x, sc.target_az, cfg.delta)
    torch.cuda.synchronize()
    zb, zf = bm["out"].cpu().numpy(), fm["out"].cpu().numpy()
    assert np.max(np.abs(zb - zf)) < 1e-4 * np.max(np.abs(zf))
    assert int(fm["info"].abs().sum()) == 0
    plan.close()


def test_rejects_bad_targets(torch, wb):
    plan = wb.Plan(16, 32, 16, 64, 64, 2, 5)
    x = torch.zeros((16, 128 * 16), dtype=torch.complex64, device="cuda")
    with pytest.raises(wb.WbmError):
        plan.beamform(x, [0.1, 0.2, 0.3], [5, 5, 5], 10.0)          # T > max_targets
    with pytest.raises(wb.WbmError):
        plan.beamform(x, [0.1], [6], 10.0)                           # W > w_max
    with pytest.raises(wb.WbmError):
        plan.beamform(x, [float("nan")], [5], 10.0)
    with pytest.raises(wb.WbmError):
        plan.beamform(x, [0.1], [5], -1.0)
    plan.close()


@pytest.mark.parametrize("form", ["plain", "fused_f32-mfma", "fused-block", "fused-wave",
                                  "fused_f32-block", "fused_f32-wave", "fused_f32-resident"])
def test_zero_loading_singular_reports_info(torch, wb, form):
    # silent input and no loading: the window covariance is 0, the first pivot fails (info = 1)
    plan = wb.Plan(16, 32, 4, 3, 2, 1, 9)
    if form.startswith("fused"):
        form, pair = form.split("-")
        _pin(plan, pair, precision="f32" if form.endswith("f32") else "ext")
    x = torch.zeros((16, 5 * 4), dtype=torch.complex64, device="cuda")
    res = plan.beamform(x, [0.2], [9], 0.0, form=form)
    torch.cuda.synchronize()
    assert np.all(res["info"].cpu().numpy() == 1)
    assert np.all(res["out"].cpu().numpy() == 0)
    assert np.all(res["weights"].cpu().numpy() == 0)
    plan.close()


def test_target_changes_between_calls(torch, wb):
    # an unchanged target list is not uploaded again; a changed one must be
    cfg = scenes.SMALL
    sc = scenes.make_scene(cfg)
    x = torch.from_numpy(_x32(sc)).cuda()

    def new_plan():
        return wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, 3, 5, beta=cfg.beta,
                       d_over_lambda=cfg.dl, half_bin=cfg.half_bin)

    plan = new_plan()
    az_a, win_a = [0.1, -0.3, 0.5], [5, 3, 5]
    az_b, win_b = [0.2, 0.4], [3, 5]
    a1 = plan.beamform(x, az_a, win_a, cfg.delta, form="fused")
    a2 = plan.beamform(x, az_a, win_a, cfg.delta, form="fused")
    b1 = plan.beamform(x, az_b, win_b, cfg.delta, form="fused")
    a3 = plan.beamform(x, az_a, win_a, cfg.delta, form="graph")
    torch.cuda.synchronize()
    fresh = new_plan()
    fresh.set_tuning(*plan.tuning)
    b2 = fresh.beamform(x, az_b, win_b, cfg.delta, form="fused")
    torch.cuda.synchronize()
    for key in ("out", "weights", "starts"):
        assert torch.equal(a1[key], a2[key]), key
        assert torch.equal(a1[key], a3[key]), key
        assert torch.equal(b1[key], b2[key]), key
    plan.close()
    fresh.close()


def test_pair_kernel_limits_rejected(torch, wb):
    # the one-wave kernel needs w_max <= 40; the resident kernel w_max L, w_max Lt <= 2304
    plan = wb.Plan(64, 128, 8, 512, 512, 2, 41)
    chan, beam, _, _ = plan.tuning
    for pair in ("wave", "resident"):
        with pytest.raises(wb.WbmError):
            plan.set_tuning(chan, beam, pair)
    plan.set_tuning(chan, beam, "block")
    plan.close()


# N = 200: the blocked Cholesky's 64-column panels end in a ragged one of 8 columns
FULL_RAGGED = scenes.GPU.replace(name="full_ragged", N=200, K=16, L=256, Lt=32, T=4,
                                 seed=4242)


@pytest.mark.parametrize("name,subbands", [("small", None), ("gpu", [0, 5, 64, 127]),
                                           ("full_ragged", [0, 3, 15]), ("batch", [0, 100])])
def test_full_dimensional_mvdr_matches_oracle(torch, wb, name, subbands):
    cfg = FULL_RAGGED if name == "full_ragged" else scenes.config_by_name(name)
    log(f"full-dimensional MVDR, {name} config (N={cfg.N})")
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    plan = _plan(wb, cfg, sc)
    ks = list(range(cfg.K)) if subbands is None else subbands
    # N = 1024: 16 Cholesky panels; only the sampled subbands are solved there
    rng_ = (ks[0], ks[-1] - ks[0] + 1) if cfg.N >= 1024 else None
    res = plan.full_mvdr(torch.from_numpy(x32).cuda(), sc.target_az, cfg.delta, subbands=rng_)
    torch.cuda.synchronize()
    assert int(res["info"][ks].abs().sum()) == 0
    X = oracle.channelize_bins(x32, cfg.K, ks, cfg.half_bin)
    ref = oracle.full_mvdr(x32, K=cfg.K, L=cfg.L, Lt=cfg.Lt, sin_az=[math.sin(a) for a in sc.target_az],
                           delta=cfg.delta, beta=cfg.beta, dl=cfg.dl, half_bin=cfg.half_bin,
                           subbands=ks, X=None)
    w_g = res["weights"].cpu().numpy().astype(np.complex128)
    z_g = res["out"].cpu().numpy().astype(np.complex128)
    worst = 0.0
    for ik, k in enumerate(ks):
        R = oracle.sample_covariance(X[:, :cfg.L, ik], cfg.delta)
        kappa = float(np.linalg.cond(R))
        for t in range(cfg.T):
            err = oracle.rel_weight_error(w_g[t, k], ref["w"][t, ik])
            tol = weight_tol(kappa, False, snapshot_dynamic_range(sc))
            assert err <= tol, (t, k, err, tol, kappa)
            worst = max(worst, err)
            zc = w_g[t, k].conj() @ X[:, cfg.L:, ik]
            scale = np.linalg.norm(w_g[t, k]) * np.max(np.linalg.norm(X[:, cfg.L:, ik], axis=0))
            assert np.max(np.abs(z_g[t, k] - zc)) <= 1e-5 * scale
    log(f"  max weight error {worst:.3e}")
    plan.close()


# ----------------------------------------------------------------------------- mixed precision

@pytest.mark.parametrize("form", ["mixed", "mixed_bf16"])
def test_mixed_forms_route_ill_conditioned_windows_to_fp64(torch, wb, form):
    """A 60 dB jammer inside a target's window drives its covariance past the routing threshold
    (condition estimate 1e4): those windows must be flagged (info bit 30) and solved by the exact
    FP64 kernel (bit-identical to the fused_f32 form on the same vector kernel, both reading the
    FP32 transforms' windows); the others stay on
    the mixed path within its bound."""
    cfg = scenes.SceneConfig(name="route", N=32, M=64, K=16, L=64, Lt=32, T=4, W=9,
                             W_choices=(9,), n_jammers=2,
                             target_az_deg=(0.0, -25.0, 20.0, 45.0), target_snr_db=(0.0,) * 4,
                             jammer_az_deg=(1.5, -55.0), jammer_inr_db=(60.0, 30.0), seed=21)
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    _pin(plan, "block", precision="f32")
    x = torch.from_numpy(x32).cuda()
    exact = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form="fused_f32")
    res = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form)
    torch.cuda.synchronize()
    info = res["info"].cpu().numpy()
    routed = (info & wb.INFO_ROUTED) != 0
    log(f"  {form}: routed {int(routed.sum())}/{routed.size}")
    assert routed.sum() > 0 and not routed.all()
    assert np.all((info & ~wb.INFO_ROUTED) == 0)
    w_m = res["weights"].cpu().numpy()
    w_e = exact["weights"].cpu().numpy()
    o_m = res["out"].cpu().numpy()
    o_e = exact["out"].cpu().numpy()
    assert np.array_equal(w_m[routed], w_e[routed])
    assert np.array_equal(o_m[routed], o_e[routed])
    res = dict(res)
    res["info"] = torch.zeros_like(res["info"])
    unit = 2.0 ** -16 if form == "mixed" else 2.0 ** -8
    # bar: a tenth of the derived 4 u kappa bound (measured at most 0.007 of the full bound).
    # One BF16 product keeps 8 significant bits of every snapshot; no routing threshold bounds
    # its SINR loss in general (the one window of this 60 dB scene it keeps on the BF16 path
    # loses 0.17 dB), so here it is reported; the workload tests hold it to 0.1 dB.
    st = compare_beamform(sc, ref, res, plain=True, unit=unit, tol_scale=0.1,
                          sinr_bar_db=0.1 if form == "mixed" else None)
    log(f"  {st}")
    plan.close()


@pytest.mark.parametrize("name", ["small", "gpu"])
def test_mixed_precision_forms(torch, wb, name):
    """MFMA BF16 covariance forms: weights within the bound of each form's product precision
    (2^-16 split hi/lo, 2^-8 single BF16), SINR loss <= 0.1 dB, every result's error logged."""
    cfg = scenes.config_by_name(name)
    sc = scenes.make_scene(cfg)
    x32 = _x32(sc)
    ref = _oracle(sc, x32)
    plan = _plan(wb, cfg, sc)
    x = torch.from_numpy(x32).cuda()
    for form in ("mixed", "mixed_bf16"):
        res = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form=form)
        torch.cuda.synchronize()
        info = res["info"].cpu().numpy()
        routed = (info & wb.INFO_ROUTED) != 0
        assert np.all((info & ~wb.INFO_ROUTED) == 0), "Cholesky failures"
        res = dict(res)
        res["info"] = torch.zeros_like(res["info"])
        unit = 2.0 ** -16 if form == "mixed" else 2.0 ** -8
        # bar: a tenth of the derived 4 u kappa bound (measured at most 0.028 of the full bound)
        st = compare_beamform(sc, ref, res, plain=True, sinr_bar_db=0.1, unit=unit,
                              tol_scale=0.1)
        log(f"  {name} {form}: routed {int(routed.sum())}/{routed.size} {st}")
    plan.close()
