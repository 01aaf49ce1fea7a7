"""GPU parity of the loading / window predictor path against the FP64 oracle, and a test of
what the trained network gains over the fixed method."""

import math

import numpy as np
import pytest

import oracle
import scenes
from gpu_helpers import log, snapshot_dynamic_range, weight_tol
from oracle import learned as olearned
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

SMALL_MULTI = scenes.SceneConfig(
    name="small_multi", N=24, M=64, K=8, L=48, Lt=16, T=3, W=9, n_jammers=2,
    target_az_deg=(-20.0, 5.0, 33.0), target_snr_db=(5.0, -3.0, 12.0),
    jammer_az_deg=(-10.0, 48.0), jammer_inr_db=(32.0, 26.0), seed=21)


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    _t.cuda.set_device(0)
    return _t


@pytest.fixture(scope="module")
def wb():
    import paper_2508_11790_amd as _wb
    return _wb


def _plan(wb, cfg, wmax=33):
    return wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, cfg.T, wmax, beta=cfg.beta,
                   d_over_lambda=cfg.dl)


def _sin(sc):
    return [math.sin(a) for a in sc.target_az]


def test_profiles_match_oracle(torch, wb):
    cfg = SMALL_MULTI
    sc = scenes.make_scene(cfg)
    x32 = sc.x.astype(np.complex64)
    plan = _plan(wb, cfg)
    feat = plan.profiles(torch.from_numpy(x32).cuda(), sc.target_az, 1.0).cpu().numpy()
    X = oracle.channelize(x32.astype(np.complex128), cfg.K)
    ratio = oracle.subband_freq_ratio(cfg.K, cfg.beta)
    for k in range(cfg.K):
        Yk = oracle.beamspace(X[:, :cfg.L, k][:, :, None], cfg.M)[:, :, 0]
        for t in range(cfg.T):
            u = oracle.beam_position(_sin(sc)[t], ratio[k], cfg.M, cfg.dl)
            ref = olearned.power_profile(Yk, u, 1.0)
            assert np.max(np.abs(feat[t, k] - ref)) < 2e-4, (t, k)
    plan.close()


@pytest.mark.parametrize("beam_tile", [13, 12])
def test_profiles_at_8192_bins_match_oracle(torch, wb, beam_tile):
    """Training power profiles at M = 8192 with N <= 4096, where the extended-precision spatial
    DFT computes each row's even and odd bins as two 4096-point transforms (tile 2^13: the
    radix-16 kernel; 2^12: the radix-8 split-half kernel) and accumulates each parity's profile
    bins in its own half: every profile against the oracle's, one target next to the wrap, N not
    a multiple of the thread count."""
    cfg = scenes.SceneConfig(name="prof8192", N=300, M=8192, K=4, L=40, Lt=8, T=3, W=9,
                             n_jammers=2, target_az_deg=(-89.0, 3.0, 41.0),
                             target_snr_db=(5.0, 0.0, 10.0), jammer_az_deg=(-30.0, 20.0),
                             jammer_inr_db=(40.0, 30.0), seed=37)
    sc = scenes.make_scene(cfg)
    x32 = sc.x.astype(np.complex64)
    plan = _plan(wb, cfg)
    chan = plan.get_tuning("ext")[0]
    plan.set_tuning(chan, beam_tile, "block", 1, precision="ext")
    feat = plan.profiles(torch.from_numpy(x32).cuda(), sc.target_az, 1.0).cpu().numpy()
    X = oracle.channelize(x32.astype(np.complex128), cfg.K)
    ratio = oracle.subband_freq_ratio(cfg.K, cfg.beta)
    worst = 0.0
    for k in range(cfg.K):
        Yk = oracle.beamspace(X[:, :cfg.L, k][:, :, None], cfg.M)[:, :, 0]
        for t in range(cfg.T):
            u = oracle.beam_position(_sin(sc)[t], ratio[k], cfg.M, cfg.dl)
            ref = olearned.power_profile(Yk, u, 1.0)
            err = float(np.max(np.abs(feat[t, k] - ref)))
            assert err < 2e-4, (t, k, err)
            worst = max(worst, err)
    log(f"  tile {beam_tile}: worst profile error {worst:.2e} (log10 units)")
    plan.close()


def _pair_oracle(x128, cfg, s_az, k, W, d):
    return oracle.windowed_mvdr(x128, M=cfg.M, K=cfg.K, L=cfg.L, Lt=cfg.Lt, sin_az=[s_az], win=[W],
                                delta=d, beta=cfg.beta, dl=cfg.dl, subbands=[k])


def test_pair_windows_and_loadings_match_oracle(torch, wb):
    cfg = SMALL_MULTI
    sc = scenes.make_scene(cfg)
    x32 = sc.x.astype(np.complex64)
    x128 = x32.astype(np.complex128)
    rng = np.random.default_rng(4)
    pw = rng.choice([5, 9, 17, 33], size=(cfg.T, cfg.K)).astype(np.int32)
    pd = rng.choice(olearned.SWEEP_DELTAS, size=(cfg.T, cfg.K)).astype(np.float32)
    plan = _plan(wb, cfg)
    res = plan.beamform_pairs(torch.from_numpy(x32).cuda(), sc.target_az, [33] * cfg.T,
                              torch.from_numpy(pw).cuda(), torch.from_numpy(pd).cuda())
    sinr = plan.sinr(sc.target_az, [33] * cfg.T, res["weights"], res["starts"], sc.jammer_az,
                     sc.jammer_inr, 1.0, pair_win=torch.from_numpy(pw).cuda()).cpu().numpy()
    w = res["weights"].cpu().numpy().astype(np.complex128)
    starts = res["starts"].cpu().numpy()
    assert int(res["info"].abs().sum()) == 0
    ratio = oracle.subband_freq_ratio(cfg.K, cfg.beta)
    for t in range(cfg.T):
        for k in range(cfg.K):
            W, d = int(pw[t, k]), float(pd[t, k])
            ref = _pair_oracle(x128, cfg, _sin(sc)[t], k, W, d)
            assert starts[t, k] == ref["start"][0, 0]
            err = oracle.rel_weight_error(w[t, k, :W], ref["w"][0, 0, :W])
            kappa = float(np.linalg.cond(ref["R"][0][0]))
            tol = weight_tol(kappa, False, snapshot_dynamic_range(sc))
            assert err <= tol, (t, k, W, d, err, tol)
            assert np.all(w[t, k, W:] == 0)
            bins = oracle.window_bins(int(starts[t, k]), W, cfg.M)
            s_ref = olearned.pair_sinr(w[t, k, :W], ref["a"][0, 0, :W], bins, cfg.N, cfg.M,
                                       np.sin(sc.jammer_az), sc.jammer_inr, ratio[k], cfg.dl, 1.0)
            assert abs(sinr[t, k] / s_ref - 1) < 1e-5, (t, k, sinr[t, k], s_ref)
    plan.close()


def test_rejected_pair_widths_solve_the_full_window(torch, wb):
    cfg = SMALL_MULTI
    sc = scenes.make_scene(cfg)
    x = torch.from_numpy(sc.x.astype(np.complex64)).cuda()
    rng = np.random.default_rng(11)
    pw = rng.choice([5, 9, 17, 33], size=(cfg.T, cfg.K)).astype(np.int32)
    pd = np.full((cfg.T, cfg.K), 10.0, dtype=np.float32)
    bad = {(0, 0): 8, (1, 2): 35, (2, 3): 0, (2, 7): -5}     # other parity, too wide, < 1
    fixed = pw.copy()
    for (t, k), v in bad.items():
        pw[t, k] = v
        fixed[t, k] = 33
    plan = _plan(wb, cfg)
    win = [33] * cfg.T
    r_bad = plan.beamform_pairs(x, sc.target_az, win, torch.from_numpy(pw).cuda(),
                                torch.from_numpy(pd).cuda())
    r_fix = plan.beamform_pairs(x, sc.target_az, win, torch.from_numpy(fixed).cuda(),
                                torch.from_numpy(pd).cuda())
    info = r_bad["info"].cpu().numpy()
    for t in range(cfg.T):
        for k in range(cfg.K):
            assert info[t, k] == (wb.INFO_WIDTH if (t, k) in bad else 0), (t, k, info[t, k])
    assert int(r_fix["info"].abs().sum()) == 0
    assert torch.equal(r_bad["weights"], r_fix["weights"])
    assert torch.equal(r_bad["starts"], r_fix["starts"])
    s_bad = plan.sinr(sc.target_az, win, r_bad["weights"], r_bad["starts"], sc.jammer_az,
                      sc.jammer_inr, 1.0, pair_win=torch.from_numpy(pw).cuda())
    s_fix = plan.sinr(sc.target_az, win, r_fix["weights"], r_fix["starts"], sc.jammer_az,
                      sc.jammer_inr, 1.0, pair_win=torch.from_numpy(fixed).cuda())
    assert torch.equal(s_bad, s_fix)
    plan.close()


def test_sweep_labels_match_oracle(torch, wb):
    from paper_2508_11790_amd import learned
    cfg = SMALL_MULTI
    sc = scenes.make_scene(cfg)
    x32 = sc.x.astype(np.complex64)
    plan = _plan(wb, cfg)
    mlp = wb.Mlp(256)
    r = learned.label_sweep(plan, mlp, torch.from_numpy(x32).cuda(), sc.target_az, sc.jammer_az,
                            sc.jammer_inr)
    g_lab = r["labels"].cpu().numpy().reshape(cfg.T, cfg.K, 2)
    g_tab = r["table"].cpu().numpy()
    log("  oracle sweep (44 runs)")
    ref = olearned.sweep(x32.astype(np.complex128), M=cfg.M, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                         sin_az=_sin(sc), jam_sin=np.sin(sc.jammer_az), jam_inr=sc.jammer_inr)
    nd, nw = len(olearned.SWEEP_DELTAS), len(olearned.SWEEP_WIDTHS)
    for t in range(cfg.T):
        for k in range(cfg.K):
            tab = g_tab[:, t * cfg.K + k].reshape(nd, nw)
            assert np.allclose(tab, ref["table"][t, k], rtol=1e-4), (t, k)
            # the GPU's choice is optimal for the oracle's table (ties and near-ties may differ)
            ld, lw = g_lab[t, k]
            idl = int(np.argmin([abs(math.log(d) - ld) for d in olearned.SWEEP_DELTAS]))
            iw = int(np.argmin([abs(math.log2(w - 1) - lw) for w in olearned.SWEEP_WIDTHS]))
            best = ref["table"][t, k].max()
            assert ref["table"][t, k][idl, iw] >= best * (1 - 1e-4)
            if np.sort(ref["table"][t, k].ravel())[-2] < best * (1 - 1e-3):
                assert abs(ld - ref["labels"][t, k, 0]) < 1e-5 and abs(lw - ref["labels"][t, k, 1]) < 1e-5
    feat = r["feat"].cpu().numpy().reshape(cfg.T, cfg.K, 64)
    assert np.max(np.abs(feat - ref["feat"])) < 2e-4
    plan.close()
    mlp.close()


def _rand_params(seed, scale=0.2):
    r = np.random.default_rng(seed)
    return (r.standard_normal(omlp.N_PARAMS) * scale).astype(np.float32)


def test_mlp_forward_gradients_and_adam_match_oracle(torch, wb):
    flat = _rand_params(0)
    r = np.random.default_rng(1)
    n = 37
    x = (r.standard_normal((n, 64)) * 2).astype(np.float32)
    y = r.standard_normal((n, 2)).astype(np.float32)
    mlp = wb.Mlp(64)
    P = torch.from_numpy(flat).cuda()
    out = mlp.forward(P, torch.from_numpy(x).cuda()).cpu().numpy()
    grad, loss = mlp.grad(P, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    grad = grad.cpu().numpy()
    pr = omlp.unflatten(olearned.bf16_round(flat))              # the weights the GPU uses
    ref_out = omlp.forward(pr, x.astype(np.float64))["out"]
    assert np.max(np.abs(out - ref_out)) < 1e-4 * max(1.0, np.max(np.abs(ref_out)))
    ref_g = omlp.flatten(omlp.backward(pr, x.astype(np.float64), y.astype(np.float64)))
    scale = np.max(np.abs(ref_g))
    assert np.max(np.abs(grad - ref_g)) < 1e-4 * scale
    assert abs(float(loss.item()) - omlp.loss(pr, x, y)) < 1e-4 * omlp.loss(pr, x, y)
    # three Adam steps (bias correction past the first step) against the oracle's
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    P2 = P.clone()
    pp = omlp.unflatten(flat.astype(np.float64))
    mm = {k2: np.zeros_like(a) for k2, a in pp.items()}
    vv = {k2: np.zeros_like(a) for k2, a in pp.items()}
    for step in (1, 2, 3):
        g_np = (ref_g * (1.0 + 0.5 * step) + r.standard_normal(ref_g.size) * scale).astype(np.float32)
        mlp.adam(P2, m, v, torch.from_numpy(g_np).cuda(), step, 1e-3)
        omlp.adam_step(pp, omlp.unflatten(g_np.astype(np.float64)), mm, vv, step, 1e-3)
        assert np.max(np.abs(P2.cpu().numpy() - omlp.flatten(pp))) < 1e-6 * step, step
    mlp.close()


def test_learned_form_follows_network_and_falls_back(torch, wb):
    cfg = SMALL_MULTI
    sc = scenes.make_scene(cfg)
    x = torch.from_numpy(sc.x.astype(np.complex64)).cuda()
    plan = _plan(wb, cfg)
    mlp = wb.Mlp(64)
    flat = _rand_params(3, 0.05)
    flat[-2:] = [math.log(10.0), 3.2]                 # biases: loading ~10, W ~ 9
    P = torch.from_numpy(flat).cuda()
    lr = plan.beamform_learned(x, sc.target_az, P, 1.0, 9, 10.0)
    feat = plan.profiles(x, sc.target_az, 1.0).reshape(-1, 64)
    out = mlp.forward(P, feat).cpu().numpy()
    pw = lr["pair_win"].cpu().numpy().reshape(-1)
    pd = lr["pair_loading"].cpu().numpy().reshape(-1)
    for i in range(out.shape[0]):
        W, d = olearned.decision(float(out[i, 0]), float(out[i, 1]), 1.0)
        assert pw[i] == W and abs(pd[i] / d - 1) < 1e-5
    assert int(lr["fallback"].sum()) == 0
    again = plan.beamform_pairs(x, sc.target_az, [33] * cfg.T, lr["pair_win"], lr["pair_loading"])
    assert torch.equal(again["weights"], lr["weights"]) and torch.equal(again["out"], lr["out"])
    # non-finite network -> every pair uses the fixed method (W = 9, loading 10)
    bad = P.clone()
    bad[-1] = float("nan")
    fb = plan.beamform_learned(x, sc.target_az, bad, 1.0, 9, 10.0)
    assert int(fb["fallback"].sum()) == cfg.T * cfg.K
    fixed = plan.beamform(x, sc.target_az, [9] * cfg.T, 10.0, form="fused")
    assert torch.allclose(fb["weights"][:, :, :9], fixed["weights"][:, :, :9], rtol=0, atol=1e-6)
    plan.close()
    mlp.close()


def test_trained_network_gains_over_fixed_method(torch, wb):
    from paper_2508_11790_amd import learned
    from paper_2508_11790_amd.train_predictor import evaluate
    cfg = scenes.SceneConfig(name="learn_small", N=64, M=128, K=32, L=96, Lt=32, T=8, W=9,
                             n_jammers=3, inr_range_db=(20.0, 45.0), seed=7000)
    plan = _plan(wb, cfg)
    mlp = wb.Mlp(1024)
    feats, labels = [], []
    for i in range(48):
        sc, x = scenes.make_scene_torch(cfg, 7000 + i)
        r = learned.label_sweep(plan, mlp, x, sc.target_az, sc.jammer_az, sc.jammer_inr)
        feats.append(r["feat"])
        labels.append(r["labels"])
    feats, labels = torch.cat(feats), torch.cat(labels)
    log(f"  {feats.shape[0]} training samples labelled")
    P = torch.from_numpy(learned.init_params(5)).cuda()
    hist = learned.train(mlp, P, feats, labels, epochs=40, batch=512, lr=2e-3, seed=6)
    log(f"  loss {hist[0]:.3f} -> {hist[-1]:.3f}")
    assert hist[-1] < 0.5 * hist[0]
    ev = evaluate(wb, learned, scenes, cfg, 6, 9000, P, with_ceiling=True)
    log(f"  {ev}")
    assert ev["fallback_pairs"] == 0
    assert ev["gain_db"] > 0.0
    assert ev["learned_mean_sinr_db"] <= ev["best_mean_sinr_db"] + 1e-3
    plan.close()
    mlp.close()


def test_learned_form_at_evaluation_shape(torch, wb):
    """The committed network at its evaluation shape (batch-sized array: N = 1024, M = 2048,
    K = 256, 64 targets, L = Lt = 512): per-pair profiles, network outputs and (W, delta)
    decisions, then the resulting weights, against the oracle on sampled subbands; and the
    held-out SINR gain over the fixed method."""
    import os
    from paper_2508_11790_amd import learned
    from paper_2508_11790_amd.train_predictor import evaluate
    cfg = scenes.LEARNED_EVAL
    path = os.path.join(os.path.dirname(learned.__file__), "predictor_params.npz")
    flat = learned.load_params(path)
    P = torch.from_numpy(flat).cuda()
    sc, x = scenes.make_scene_torch(cfg, cfg.seed + 77)
    plan = wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, cfg.T, 33, beta=cfg.beta,
                   d_over_lambda=cfg.dl)
    mlp = wb.Mlp(cfg.T * cfg.K)
    lr = plan.beamform_learned(x, sc.target_az, P, cfg.noise_var, 9, cfg.delta)
    feat = plan.profiles(x, sc.target_az, cfg.noise_var)
    out = mlp.forward(P, feat.reshape(-1, 64)).reshape(cfg.T, cfg.K, 2).cpu().numpy()
    feat = feat.cpu().numpy()
    pw = lr["pair_win"].cpu().numpy()
    pd = lr["pair_loading"].cpu().numpy()
    w = lr["weights"].cpu().numpy().astype(np.complex128)
    starts = lr["starts"].cpu().numpy()
    assert int(lr["fallback"].sum()) == 0 and int(lr["info"].abs().sum()) == 0
    x128 = x.cpu().numpy().astype(np.complex128)
    del x
    torch.cuda.empty_cache()
    ks = [0, 101, 255]
    log(f"  oracle on subbands {ks}, all {cfg.T} targets")
    Xs = oracle.channelize_bins(x128, cfg.K, ks)                     # [N, B, len(ks)]
    del x128
    ratio = oracle.subband_freq_ratio(cfg.K, cfg.beta)
    pr = omlp.unflatten(olearned.bf16_round(flat))
    n_boundary, err_max, loss_max = 0, 0.0, 0.0
    for ik, k in enumerate(ks):
        Yk = oracle.beamspace(Xs[:, :cfg.L, ik], cfg.M)               # training beamspace [M, L]
        for t in range(cfg.T):
            u = oracle.beam_position(_sin(sc)[t], ratio[k], cfg.M, cfg.dl)
            f_ref = olearned.power_profile(Yk, u, cfg.noise_var)
            assert np.max(np.abs(feat[t, k] - f_ref)) < 2e-4, (t, k)
            o_ref = omlp.forward(pr, f_ref[None, :])["out"][0]
            assert np.max(np.abs(out[t, k] - o_ref)) < 1e-3, (t, k, out[t, k], o_ref)
            W_ref, d_ref = olearned.decision(float(o_ref[0]), float(o_ref[1]), cfg.noise_var)
            assert abs(pd[t, k] / d_ref - 1) < 1e-3, (t, k, pd[t, k], d_ref)
            # a width decided within the two networks' rounding of a rint() boundary may
            # differ; every other decision is the oracle's
            frac = abs(float(o_ref[1]) - math.floor(float(o_ref[1])) - 0.5)
            if frac < 1e-3 and 2.0 < o_ref[1] < 5.0:
                n_boundary += 1
                assert pw[t, k] in (W_ref, 2 * W_ref - 1, (W_ref + 1) // 2)
            else:
                assert pw[t, k] == W_ref, (t, k, pw[t, k], W_ref, o_ref)
            # weights of the GPU's decision against the oracle's MVDR with that (W, delta)
            W, d = int(pw[t, k]), float(pd[t, k])
            ref = oracle.windowed_mvdr(None, X=Xs[:, :, ik:ik + 1], M=cfg.M, K=cfg.K, L=cfg.L,
                                       Lt=cfg.Lt, sin_az=[_sin(sc)[t]], win=[W], delta=d,
                                       beta=cfg.beta, dl=cfg.dl, subbands=[k])
            assert starts[t, k] == ref["start"][0, 0]
            err = oracle.rel_weight_error(w[t, k, :W], ref["w"][0, 0, :W])
            bins = oracle.window_bins(int(starts[t, k]), W, cfg.M)
            s_g = olearned.pair_sinr(w[t, k, :W], ref["a"][0, 0, :W], bins, cfg.N, cfg.M,
                                     np.sin(sc.jammer_az), sc.jammer_inr, ratio[k], cfg.dl,
                                     cfg.noise_var)
            s_o = olearned.pair_sinr(ref["w"][0, 0, :W], ref["a"][0, 0, :W], bins, cfg.N, cfg.M,
                                     np.sin(sc.jammer_az), sc.jammer_inr, ratio[k], cfg.dl,
                                     cfg.noise_var)
            err_max = max(err_max, err)
            loss_max = max(loss_max, abs(10 * math.log10(s_o / s_g)))
    log(f"  max weight error {err_max:.3g}, max SINR loss {loss_max:.3g} dB, "
        f"{n_boundary} width decisions at a rounding boundary")
    assert err_max <= 1e-5 and loss_max <= 0.1
    plan.close()
    mlp.close()
    ev = evaluate(wb, learned, scenes, cfg, 2, cfg.seed + 500, P, with_ceiling=False)
    log(f"  held-out: {ev}")
    assert ev["fallback_pairs"] == 0
    assert ev["gain_db"] > 0.0
