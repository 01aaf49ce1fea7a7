#!/usr/bin/env python3
"""Throughput of windowed beamspace MVDR on one MI355X: (target, subband) beams per second.

A step is one pass of the whole path over one batch of synthetic array data already resident
in HBM: window placement and steering, FFT channelizer, zero-padded spatial FFT with the
window gather, and per-pair covariance / LDL^H / solve / apply.  The chosen form (fused kernels
with extended-precision transforms, replayed from a HIP graph) is timed and reported beside the
same sequence with FP32 transforms, the plain per-stage FP32 form, the mixed-precision (BF16
MFMA covariance) forms, the learned loading/window form, full-dimensional element-space MVDR
on the same GPU, and the FP64 CPU oracle on the host's cores.

Workload (default): the precision configuration -- N=4096 elements, M=8192-point spatial FFT,
K=512 subbands, W=64, L=1024 training and Lt=1024 test snapshots, 32 targets, 8 wideband
jammers of 20-60 dB, seeded and generated on the device (34 GB of samples).  The batching
(N=1024) and GPU-scale (N=256) configurations run as extra legs.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "(target,subband) MVDR beams/s at ≤0.1 dB SINR loss vs FP64; chosen vs plain"
HBM_PEAK_GBS = 8000.0
TRAFFIC_DIR = os.path.join(ROOT, "profiles")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hashes() -> dict:
    """SHA-256 of each kernel source file and header of the library."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2508_11790_amd", "csrc")
    out = {}
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                out[f] = hashlib.sha256(fh.read()).hexdigest()
    return out


def kernel_source_file(name: str) -> str:
    """The source file that defines a kernel of the fused sequence."""
    return "mvdr_kernels.hip" if name.startswith("k_mvdr") else "fft_kernels.hip"


def kernel_source_deps(fname: str) -> list:
    """The source file and the library headers it includes, directly or through others."""
    import re
    csrc = os.path.join(ROOT, "paper_2508_11790_amd", "csrc")
    seen, todo = [], [fname]
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(os.path.join(csrc, f)):
            continue
        seen.append(f)
        with open(os.path.join(csrc, f)) as fh:
            todo += re.findall(r'^\s*#\s*include\s+"([^"]+)"', fh.read(), re.M)
    return seen


def dispatch_name(stage: str, cfg, tuning, wmax: int, ext: bool) -> str:
    """Kernel name (as the profiler lists it, without arguments) a stage of the fused sequence
    launches for the plan's tuning."""
    lk, lm = int(math.log2(cfg.K)), int(math.log2(cfg.M))
    if stage == "channelize":
        return f"k_channelize{'_x' if ext else ''}<{lk}, {max(tuning[0], lk)}>"
    if stage == "beamspace":
        zh = 2 * cfg.N <= cfg.M
        if ext and zh and lm >= 13:
            # split-half forms: the radix-16 engine at tile 2^13 and M = 8192, else radix 8
            return ("k_beamspace_x16" if lm == 13 and tuning[1] == 13
                    else f"k_beamspace_x2<{lm - 1}>")
        return f"k_beamspace{'_x' if ext else ''}<{lm}, {max(tuning[1], lm)}, " \
               f"{'true' if zh else 'false'}>"
    pair = tuning[2]
    if pair == "resident":
        return "k_mvdr_res"
    if pair == "mfma":
        return f"k_mvdr_xm<{40 if wmax <= 40 else 64}>"
    name = ("k_mvdr_xw40" if pair == "wave" else
            "k_mvdr_xv16" if wmax <= 16 else "k_mvdr_xv40" if wmax <= 40 else "k_mvdr_xv64")
    return f"{name}<{'true' if ext else 'false'}>"


def counter_traffic(workload: str, name: str):
    """HBM bytes per launch of the named kernel from the committed FETCH_SIZE / WRITE_SIZE
    record of this workload, or None when there is none, the kernel is not in it, or the
    kernel's source file or a header it includes changed since the counters were taken."""
    path = os.path.join(TRAFFIC_DIR, f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("dispatches", {}).get(name)
    if k is None:
        return None
    now, then = kernel_source_hashes(), rec.get("sources", {})
    if any(then.get(f) != now.get(f) for f in kernel_source_deps(kernel_source_file(name))):
        return None
    return k["hbm_bytes"]


def timed_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


# ------------------------------------------------------------------------------ host side

def host_cpu():
    """(model name, physical cores, logical CPUs available to this process)."""
    model, cores = "unknown", set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name" and model == "unknown":
                    model = val
                elif key == "physical id":
                    phys = val
                elif key == "core id":
                    core = val
                elif not key and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, len(cores) or None, avail


def oracle_subbands(cfg):
    """Subbands the CPU oracle and the validity check cover: all of them up to 128, else eight
    fixed ones spread over the band (both band edges included)."""
    if cfg.K <= 128:
        return list(range(cfg.K))
    return sorted({int(round(v)) for v in np.linspace(0, cfg.K - 1, 8)})


def host_copy(torch, x, chunk_bytes=1 << 30):
    """Device [N, S] complex64 -> host numpy, element chunks at a time."""
    N = x.shape[0]
    out = np.empty(tuple(x.shape), dtype=np.complex64)
    per = max(1, chunk_bytes // (x.shape[1] * 8))
    for e0 in range(0, N, per):
        out[e0:e0 + per] = x[e0:e0 + per].cpu().numpy()
    return out


def cpu_baseline_leg(scene, x_host, ks, budget_s=10.0):
    """Time the FP64 oracle on the listed subbands of the workload (every target) on the host's
    cores, repeated until about budget_s of work; also returns its result for the validity
    check."""
    import oracle
    from threadpoolctl import threadpool_limits
    cfg = scene.cfg
    model, phys, avail = host_cpu()
    threads = min(avail, int(os.environ.get("OMP_NUM_THREADS", avail)))
    sin_az = [math.sin(a) for a in scene.target_az]
    passes, t_total, ref = 0, 0.0, None
    with threadpool_limits(limits=threads):
        while passes == 0 or t_total < budget_s:
            t0 = time.perf_counter()
            ref = oracle.windowed_mvdr(x_host, M=cfg.M, K=cfg.K, L=cfg.L, Lt=cfg.Lt,
                                       sin_az=sin_az, win=scene.win, delta=cfg.delta,
                                       beta=cfg.beta, dl=cfg.dl, half_bin=cfg.half_bin,
                                       subbands=None if len(ks) == cfg.K else ks)
            t_total += time.perf_counter() - t0
            passes += 1
    beams = cfg.T * len(ks)
    sample = (f"{len(ks)} of {cfg.K} subbands ({ks}), all {cfg.T} targets: {beams} pairs "
              f"from the complex64 samples (channelizer at those bins, spatial FFT, windows, "
              f"covariance, Cholesky, apply), {passes} pass(es), {t_total:.1f} s; "
              f"numpy/scipy complex128, BLAS on {threads} threads; host {model}, "
              f"{phys} physical cores, {avail} CPUs available")
    if len(ks) < cfg.K:
        sample += (f"; the whole workload is {cfg.K // len(ks)}x this sample "
                   f"(every subband costs the same): beams/s carries over, the time does not")
    res = dict(value=beams * passes / t_total, unit="beams/s", cores=threads, kind="oracle",
               sample=sample)
    return res, ref


def windowed_interference(cfg, scene, bins, ratio):
    """S D R_in D^H S^T of one window, as sigma^2 (S D)(S D)^H + sum_j INR_j (S D a_j)(..)^H."""
    import oracle
    D = np.exp(-2j * np.pi * np.outer(np.asarray(bins, dtype=np.float64), np.arange(cfg.N)) / cfg.M)
    D /= math.sqrt(cfg.M)
    R = cfg.noise_var * (D @ D.conj().T)
    for s, p in zip(np.sin(scene.jammer_az), scene.jammer_inr):
        a = D @ oracle.steering(cfg.N, oracle.spatial_frequency(float(s), ratio, cfg.dl))
        R += p * np.outer(a, a.conj())
    return R


def validity(scene, ref, ks, weights_by_form, info_by_form):
    """Every pair of the oracle's subbands: maximum SINR loss and relative weight error of each
    form's weights against the FP64 oracle, over the pairs the form solved; pairs whose
    factorisation failed (info pivot, outputs zero) or whose weights are not finite are
    counted apart."""
    import oracle
    cfg = scene.cfg
    ratio = oracle.subband_freq_ratio(cfg.K, cfg.beta, cfg.half_bin)
    rins = {}
    out = {}
    for form, w in weights_by_form.items():
        loss_max, err_max, failed, nonfinite = 0.0, 0.0, 0, 0
        pivots = info_by_form[form] & ((1 << 29) - 1)   # bits 29, 30: width / FP64-route flags
        for ik, k in enumerate(ks):
            for t in range(cfg.T):
                W = int(scene.win[t])
                wg = w[t, ik, :W]
                if pivots[t, ik] != 0:
                    failed += 1
                    continue
                if not np.all(np.isfinite(wg)):
                    nonfinite += 1
                    continue
                bins = oracle.window_bins(int(ref["start"][t, ik]), W, cfg.M)
                key = (t, k)
                if key not in rins:
                    rins[key] = windowed_interference(cfg, scene, bins, ratio[k])
                wo = ref["w"][t, ik, :W]
                loss = abs(oracle.sinr_loss_db(wg, wo, ref["a"][t, ik, :W], rins[key]))
                err = oracle.rel_weight_error(wg, wo)
                loss_max = loss_max if loss <= loss_max else loss     # NaN propagates
                err_max = err_max if err <= err_max else err
        out[form] = {"max_sinr_loss_db": loss_max, "max_rel_weight_err": err_max,
                     "failed_pairs": failed, "nonfinite_pairs": nonfinite,
                     "pairs": cfg.T * len(ks)}
    return out


# ------------------------------------------------------------------------------ legs

def beside_legs(torch, plan, cfg, sc, x, steps, warmup):
    """Beside the path: lifted correlators in element space (Eq. 21), beam patterns (Eq. 22),
    subband synthesis and range-Doppler + CFAR of the synthesized outputs."""
    T, K = cfg.T, cfg.K
    az, win, delta = sc.target_az, sc.win, cfg.delta
    fres = plan.beamform(x, az, win, delta, form="fused")
    ms_lift = timed_steps(torch, lambda: plan.lift(fres["weights"], fres["starts"]), steps, warmup)
    c_hat = plan.lift(fres["weights"], fres["starts"])
    out_l = torch.empty_like(fres["out"])
    ms_applied = timed_steps(torch, lambda: plan.apply_lifted(x, c_hat, out=out_l), steps, warmup)
    lift_diff = float((out_l - fres["out"]).abs().max() / fres["out"].abs().max())
    omega = torch.linspace(-math.pi, math.pi, 512, dtype=torch.float64, device=x.device)
    pat = torch.empty((T, K, 512), dtype=torch.float32, device=x.device)
    ms_pattern = timed_steps(torch, lambda: plan.beam_pattern(c_hat, omega, pattern=pat),
                             max(2, steps // 10), 1)
    del c_hat, out_l, pat, omega
    zbuf = torch.empty((T, cfg.Lt * K), dtype=torch.complex64, device=x.device)
    ms_synth = timed_steps(torch, lambda: plan.synthesize(fres["out"], z=zbuf), steps, warmup)
    synth_bytes = 2.0 * T * K * cfg.Lt * 8
    # the targets' LFM repeats every 4K samples (the scene's pulse), so the test snapshots hold
    # Lt / 4 pulses of R = 4K samples
    R_rd = 4 * K
    P_rd = 1 << ((cfg.Lt * K // R_rd).bit_length() - 1)
    m = np.arange(R_rd, dtype=np.float64)
    chirp = torch.from_numpy(np.exp(1j * np.pi * (m * m / R_rd - m)).astype(np.complex64)).to(
        x.device)
    ms_rd = timed_steps(torch, lambda: plan.range_doppler(zbuf, chirp, R_rd, P_rd, 2, 8, 10.0),
                        max(2, steps // 10), 1)
    _, det = plan.range_doppler(zbuf, chirp, R_rd, P_rd, 2, 8, 10.0)
    det_np = det.cpu().numpy()
    found = int(sum(det_np[t, int(sc.target_delay[t]) % R_rd, 0] for t in range(T)))
    del zbuf, det, fres
    return {
        "lifted": {"value": T * K / (ms_applied * 1e-3), "ms_per_step": ms_applied,
                   "form": "channelize + c^H X on the test snapshots (no spatial DFT, no window "
                           "gather)", "lift_ms": ms_lift,
                   "max_rel_diff_vs_fused_outputs": lift_diff, "beam_pattern_ms": ms_pattern,
                   "beam_pattern": "Eq. 22, every pair's lifted correlator at 512 angles"},
        "synthesis": {"ms_per_call": ms_synth, "gbs": synth_bytes / (ms_synth * 1e-3) / 1e9,
                      "bytes": synth_bytes},
        "range_doppler": {"ms_per_call": ms_rd, "pulses": P_rd, "range_bins": R_rd,
                          "targets_detected_at_their_delay": found, "targets": T,
                          "cfar": "cell averaging along range, guard 2, 8 training cells a "
                                  "side, 10 dB"},
    }


def upa_leg(torch, wb, scenes, steps, warmup):
    """The paper's planar geometry (Sec. IV): 4 x 32 array, 8 x 64 beam grid, 128 subbands,
    20 targets with 2x4 / 4x4 / 4x8 windows; fused, mixed and plain forms timed per step, and
    the fused weights against the planar oracle on three subbands."""
    import oracle.upa as oupa
    cfg = scenes.UPA
    sc = scenes.make_upa_scene(cfg)
    x32 = sc.x.astype(np.complex64)
    x = torch.from_numpy(x32).cuda()
    wmax = int(np.max(sc.win_z * sc.win_x))
    plan = wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, cfg.T, wmax, beta=cfg.beta,
                   d_over_lambda=cfg.dl)
    out = torch.empty((cfg.T, cfg.K, cfg.Lt), dtype=torch.complex64, device=x.device)
    wts = torch.empty((cfg.T, cfg.K, wmax), dtype=torch.complex64, device=x.device)
    info = torch.empty((cfg.T, cfg.K), dtype=torch.int32, device=x.device)
    args = (x, cfg.Nz, cfg.Mz, sc.target_az, sc.target_el, sc.win_z, sc.win_x, cfg.delta)
    res = {}

    def step(form):
        return lambda: plan.beamform_upa(*args, form=form, out=out, weights=wts, info=info,
                                         want_starts=False)
    ms = timed_steps(torch, step("fused"), steps, warmup)
    assert int(info.abs().sum()) == 0
    res["fused"] = {"value": cfg.T * cfg.K / (ms * 1e-3), "ms_per_step": ms}
    w_fused = wts.cpu().numpy().astype(np.complex128)
    fres = plan.beamform_upa(*args, form="fused")
    starts = fres["starts"].cpu().numpy()
    ms_lift = timed_steps(torch, lambda: plan.lift_upa(fres["weights"], fres["starts"], cfg.Nz,
                                                       cfg.Mz, sc.win_z), steps, warmup)
    c_hat = plan.lift_upa(fres["weights"], fres["starts"], cfg.Nz, cfg.Mz, sc.win_z)
    out_l = torch.empty_like(out)
    ms_applied = timed_steps(torch, lambda: plan.apply_lifted(x, c_hat, out=out_l), steps, warmup)
    lift_diff = float((out_l - fres["out"]).abs().max() / fres["out"].abs().max())
    g = torch.linspace(-math.pi, math.pi, 32, dtype=torch.float64, device=x.device)
    omega = torch.stack(torch.meshgrid(g, g, indexing="ij"), dim=-1).reshape(-1, 2).contiguous()
    pat = torch.empty((cfg.T, cfg.K, omega.shape[0]), dtype=torch.float32, device=x.device)
    ms_pattern = timed_steps(torch, lambda: plan.beam_pattern_upa(c_hat, cfg.Nz, omega,
                                                                  pattern=pat),
                             max(2, steps // 10), 1)
    res["lifted"] = {"value": cfg.T * cfg.K / (ms_applied * 1e-3), "ms_per_step": ms_applied,
                     "lift_ms": ms_lift, "max_rel_diff_vs_fused_outputs": lift_diff,
                     "beam_pattern_ms": ms_pattern,
                     "beam_pattern": "Eq. 22 over a 32 x 32 (Omega_z, Omega_x) grid, every pair"}
    del c_hat, out_l, pat, omega
    for form in ("mixed", "mixed_bf16"):
        ms = timed_steps(torch, step(form), steps, warmup)
        res[form] = {"value": cfg.T * cfg.K / (ms * 1e-3), "ms_per_step": ms,
                     "routed_pairs": int(((info.cpu().numpy() & wb.INFO_ROUTED) != 0).sum())}
    ms = timed_steps(torch, step("plain"), steps, warmup)
    res["plain"] = {"value": cfg.T * cfg.K / (ms * 1e-3), "ms_per_step": ms,
                    "form": "per-stage FP32 kernels, full planar beamspace in HBM"}
    plan.close()
    sumW = int(np.sum(sc.win_z * sc.win_x))
    subbands = [0, 64, 127]
    ref = oupa.upa_windowed_mvdr(x32.astype(np.complex128), Nz=cfg.Nz, Mz=cfg.Mz, Mx=cfg.Mx,
                                 K=cfg.K, L=cfg.L, Lt=cfg.Lt, az=sc.target_az, el=sc.target_el,
                                 win_z=sc.win_z, win_x=sc.win_x, delta=cfg.delta,
                                 subbands=subbands)
    err = 0.0
    for ik, k in enumerate(subbands):
        for t in range(cfg.T):
            W = int(sc.win_z[t] * sc.win_x[t])
            wo, wg = ref["w"][t, ik, :W], w_fused[t, k, :W]
            err = max(err, float(np.linalg.norm(wg - wo) / np.linalg.norm(wo)))
    res.update({"workload": f"UPA {cfg.Nz}x{cfg.Nx}, beams {cfg.Mz}x{cfg.Mx}, K={cfg.K}, "
                            f"L={cfg.L}, Lt={cfg.Lt}, T={cfg.T}, windows "
                            f"{sorted({f'{a}x{b}' for a, b in zip(sc.win_z, sc.win_x)})}, "
                            f"{cfg.n_jammers} jammers",
                "window_rows_per_subband": sumW,
                "validity": {"subbands": subbands,
                             "starts_equal": bool(np.array_equal(starts[:, subbands],
                                                                 ref["start"])),
                             "max_rel_weight_err": err}})
    return res


def extra_leg(torch, wb, scenes, name, steps, warmup):
    """Another configuration at full size: the chosen form, the FP32-transform form, the mixed
    forms (with their routed pairs) and the plain form, and the per-stage times of both
    transform precisions."""
    cfg = scenes.config_by_name(name)
    if cfg.N >= 1024:
        sc, x = scenes.make_scene_torch(cfg, cfg.seed)
    else:
        sc = scenes.make_scene(cfg)
        x = torch.from_numpy(sc.x.astype(np.complex64)).cuda()
    wmax = int(sc.win.max())
    plan = wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, cfg.T, wmax, beta=cfg.beta,
                   d_over_lambda=cfg.dl, half_bin=cfg.half_bin)
    out = torch.empty((cfg.T, cfg.K, cfg.Lt), dtype=torch.complex64, device=x.device)
    wts = torch.empty((cfg.T, cfg.K, wmax), dtype=torch.complex64, device=x.device)
    info = torch.empty((cfg.T, cfg.K), dtype=torch.int32, device=x.device)
    res = {"workload": f"{cfg.name}: ULA N={cfg.N}, M={cfg.M}, K={cfg.K}, W<={wmax}, L={cfg.L}, "
                       f"Lt={cfg.Lt}, T={cfg.T}, {cfg.n_jammers} jammers"}
    for form in ("graph", "graph_f32", "mixed", "mixed_bf16", "plain"):
        ms = timed_steps(torch, lambda: plan.beamform(x, sc.target_az, sc.win, cfg.delta,
                                                      form=form, out=out, weights=wts,
                                                      info=info, want_starts=False),
                         steps, warmup)
        inf = info.cpu().numpy()
        res[form] = {"value": cfg.T * cfg.K / (ms * 1e-3), "ms_per_step": ms}
        if form.startswith("mixed"):
            res[form]["routed_pairs"] = int(((inf & wb.INFO_ROUTED) != 0).sum())
        failed = int(((inf & ((1 << 29) - 1)) != 0).sum())
        if form.startswith("graph"):
            assert failed == 0
        else:
            res[form]["failed_pairs"] = failed
    for prec in ("ext", "f32"):
        st = plan.stage_times(x, sc.target_az, sc.win, cfg.delta, reps=20, precision=prec)
        res["stage_ms_" + prec] = {k: round(v, 5) for k, v in st.items()}
    plan.close()
    del x
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="precision",
                    help="scene config name (default: precision)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle and validity")
    ap.add_argument("--no-full", action="store_true", help="skip full-dimensional MVDR")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision forms")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-stage form")
    ap.add_argument("--no-upa", action="store_true", help="skip the planar-array leg")
    ap.add_argument("--no-beside", action="store_true",
                    help="skip lifted correlators, beam patterns, synthesis, range-Doppler")
    ap.add_argument("--extra", default="gpu,batch",
                    help="other configurations timed after the main one ('' for none)")
    ap.add_argument("--predictor", default=os.path.join(ROOT, "paper_2508_11790_amd",
                                                        "predictor_params.npz"),
                    help="trained loading/window predictor for the learned form ('' to skip)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="also run 5 plain device copies of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the path is measured on one GPU's share of the "
              f"work (--gpus {args.gpus} requested)", file=sys.stderr)
        return 2

    import torch
    import scenes
    import paper_2508_11790_amd as wb

    torch.cuda.set_device(0)
    cfg = scenes.config_by_name(args.workload)
    log(f"workload {cfg.name}: generating scene")
    if cfg.N >= 1024:
        sc, x = scenes.make_scene_torch(cfg, cfg.seed)       # seeded, generated on the GPU
    else:
        sc = scenes.make_scene(cfg)
        x = torch.from_numpy(sc.x.astype(np.complex64)).cuda()
        sc.x = None
    torch.cuda.synchronize()
    T, K = cfg.T, cfg.K
    wmax = int(sc.win.max())
    ks = oracle_subbands(cfg)
    plan = wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, T, wmax, beta=cfg.beta,
                   d_over_lambda=cfg.dl, half_bin=cfg.half_bin)
    dev = x.device
    out = torch.empty((T, K, cfg.Lt), dtype=torch.complex64, device=dev)
    wts = torch.empty((T, K, wmax), dtype=torch.complex64, device=dev)
    info = torch.empty((T, K), dtype=torch.int32, device=dev)
    az, win, delta = sc.target_az, sc.win, cfg.delta
    weights, infos = {}, {}

    def step(form):
        return lambda: plan.beamform(x, az, win, delta, form=form, out=out, weights=wts,
                                     info=info, want_starts=False)

    def keep(form):
        weights[form] = wts[:, ks, :].cpu().numpy().astype(np.complex128)
        infos[form] = info[:, ks].cpu().numpy()

    log("timing chosen form (fused kernels, extended-precision transforms, HIP graph replay)")
    ms_chosen = timed_steps(torch, step("graph"), args.steps, args.warmup)
    assert int(info.abs().sum()) == 0
    keep("graph")
    log("timing the same sequence with FP32 transforms (graph_f32)")
    ms_f32 = timed_steps(torch, step("graph_f32"), args.steps, args.warmup)
    assert int(info.abs().sum()) == 0
    keep("graph_f32")
    mixed = {}
    if not args.no_mixed:
        for form in ("mixed", "mixed_bf16"):
            log(f"timing {form} form")
            ms = timed_steps(torch, step(form), args.steps, args.warmup)
            routed = int(((info.cpu().numpy() & wb.INFO_ROUTED) != 0).sum())
            mixed[form] = {"value": T * K / (ms * 1e-3), "ms_per_step": ms,
                           "routed_pairs": routed}
            keep(form)

    log("per-kernel times (HIP events)")
    st = plan.stage_times(x, az, win, delta, reps=max(10, args.steps // 2), precision="ext")
    st32 = plan.stage_times(x, az, win, delta, reps=max(10, args.steps // 2), precision="f32")
    sumW = int(np.sum(win))
    B, S = cfg.B, cfg.B * cfg.K
    # algorithmic bytes per launch: complex64 = 8 B, extended precision = 8 B + a 4 B remainder
    bytes_ext = {
        "channelize": 8.0 * cfg.N * S + 12.0 * cfg.N * S,
        "beamspace": 12.0 * cfg.N * S + 12.0 * K * B * sumW,
        "mvdr": 12.0 * K * B * sumW + 8.0 * T * K * cfg.Lt + 8.0 * T * K * wmax,
    }
    bytes_f32 = {
        "channelize": 16.0 * cfg.N * S,
        "beamspace": 8.0 * cfg.N * S + 8.0 * K * B * sumW,
        "mvdr": 8.0 * K * B * sumW + 8.0 * T * K * cfg.Lt + 8.0 * T * K * wmax,
    }
    tun = plan.get_tuning("ext")
    kern = max(bytes_ext, key=lambda n: st[n])
    achieved = bytes_ext[kern] / (st[kern] * 1e-3) / 1e9
    dname = dispatch_name(kern, cfg, tun, wmax, True)
    roofline = dict(bound="hbm", kernel=kern, achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=counter_traffic(cfg.name, dname), dispatch=dname,
                    bytes_per_launch=bytes_ext[kern], ms_per_launch=st[kern],
                    stage_ms={k: round(v, 5) for k, v in st.items()},
                    stage_gbs={n: round(bytes_ext[n] / (st[n] * 1e-3) / 1e9, 1)
                               for n in bytes_ext},
                    stage_ms_f32={k: round(v, 5) for k, v in st32.items()},
                    stage_gbs_f32={n: round(bytes_f32[n] / (st32[n] * 1e-3) / 1e9, 1)
                                   for n in bytes_f32})

    # the covariance engines: BF16 MFMA utilisation of the mixed forms' pair stage (MFMA kernel
    # plus the FP64 re-solve of routed windows) against the 2.5 PFLOP/s dense BF16 peak, and
    # the exact path's FP64 vector Gram beside the FP64 matrix-core Gram on the same windows
    # algorithmic flops: the lower triangle (with the diagonal) of each pair's Hermitian W x W
    # covariance, W (W + 1) / 2 complex entries of L complex products (8 real flops each) --
    # what every engine forms (the matrix-core ones as lower tiles of the real 2W x 2W Gram)
    wv = np.asarray(win, dtype=np.float64)
    cov_flops = 4.0 * float(np.sum(wv * (wv + 1.0))) * cfg.L * K
    covariance = {"algorithmic_tflop_per_step": cov_flops / 1e12,
                  "flops_per_pair": "4 W (W + 1) L (lower triangle of the Hermitian covariance)"}
    if not args.no_mixed:
        for form, prods in (("mixed", 3), ("mixed_bf16", 1)):
            stm = plan.stage_times(x, az, win, delta, reps=max(5, args.steps // 4),
                                   precision=form)
            ms = stm["mvdr"]
            covariance[form] = {
                "pair_stage_ms": round(ms, 4), "mfma": "v_mfma_f32_32x32x16_bf16",
                "bf16_products_per_entry": prods, "peak_tflops": 2500.0,
                "achieved_tflops_algorithmic": round(cov_flops / (ms * 1e-3) / 1e12, 2),
                "frac_algorithmic": round(cov_flops / (ms * 1e-3) / 2.5e15, 5),
                "routed_pairs": mixed.get(form, {}).get("routed_pairs")}
    tun32 = plan.get_tuning("f32")
    for pair in ("block", "mfma"):
        plan.set_tuning(tun32[0], tun32[1], pair, 1, precision="f32")
        ms = plan.stage_times(x, az, win, delta, reps=max(5, args.steps // 4),
                              precision="f32")["mvdr"]
        covariance["fp64_" + ("vector" if pair == "block" else "mfma") + "_pair_kernel"] = {
            "ms": round(ms, 4), "achieved_tflops": round(cov_flops / (ms * 1e-3) / 1e12, 2),
            "peak_tflops": 78.6, "frac": round(cov_flops / (ms * 1e-3) / 78.6e12, 4)}
    plan.set_tuning(*tun32, precision="f32")

    learned_res = None
    if args.predictor and os.path.exists(args.predictor):
        from paper_2508_11790_amd import learned as wlearned
        log("timing learned form")
        params = torch.from_numpy(wlearned.load_params(args.predictor)).cuda()
        plan_l = wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, T, 33, beta=cfg.beta,
                         d_over_lambda=cfg.dl, half_bin=cfg.half_bin)
        lres = {}

        def lstep():
            lres.update(plan_l.beamform_learned(x, az, params, cfg.noise_var, 9, delta))
        ms_l = timed_steps(torch, lstep, args.steps, args.warmup)
        fx = plan.beamform(x, az, win, delta, form="fused")
        s_fixed = plan.sinr(az, win, fx["weights"], fx["starts"], sc.jammer_az, sc.jammer_inr,
                            cfg.noise_var)
        s_learn = plan_l.sinr(az, [33] * T, lres["weights"], lres["starts"], sc.jammer_az,
                              sc.jammer_inr, cfg.noise_var, pair_win=lres["pair_win"])
        gain = float((10 * torch.log10(s_learn)).mean() - (10 * torch.log10(s_fixed)).mean())
        learned_res = {"value": T * K / (ms_l * 1e-3), "ms_per_step": ms_l,
                       "mean_sinr_gain_db_vs_fixed": gain,
                       "fallback_pairs": int(lres["fallback"].sum()),
                       "form": "profiles -> MLP (BF16 weights) -> per-pair loading and window"}
        plan_l.close()
        del lres, fx, params
        torch.cuda.empty_cache()

    beside = {}
    if not args.no_beside:
        log("timing lifted correlators, beam patterns, subband synthesis and range-Doppler")
        beside = beside_legs(torch, plan, cfg, sc, x, args.steps, args.warmup)

    ms_plain = None
    if not args.no_plain:
        log("timing plain per-stage FP32 form")
        ms_plain = timed_steps(torch, step("plain"), args.steps, args.warmup)
        keep("plain")

    ms_full = None
    if not args.no_full:
        # element-space N x N MVDR per subband over the whole workload: 4 N (N + 1) L flops of
        # covariance (its lower triangle) and 4 N^3 / 3 of Cholesky per subband (82 TFLOP per
        # step at N = 4096), so few steps at large N
        full_sub = None
        nfs = max(2, min(args.steps // 20, 20))
        full_k = cfg.K
        if cfg.N >= 2048:
            nfs = 2
        log(f"timing full-dimensional element-space MVDR on {full_k} subbands ({nfs} step(s))")
        ms_full = timed_steps(torch, lambda: plan.full_mvdr(x, az, delta, want_weights=False,
                                                            subbands=full_sub), nfs, 1)

    upa_res = None
    if not args.no_upa:
        log("timing the planar-array leg (4 x 32 array, 8 x 64 beams)")
        upa_res = upa_leg(torch, wb, scenes, args.steps, args.warmup)

    if args.copy_calib:
        src = torch.empty(args.copy_calib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 copies of {args.copy_calib} MiB")
        del src, dst

    beams = T * K
    result = {
        "metric": METRIC,
        "value": beams / (ms_chosen * 1e-3),
        "unit": "beams/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_chosen,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: ULA N={cfg.N}, M={cfg.M}, K={cfg.K}, W={wmax}, "
                               f"L={cfg.L}, Lt={cfg.Lt}, T={T}, {cfg.n_jammers} jammers "
                               f"(INR {cfg.inr_range_db[0]:.0f}-{cfg.inr_range_db[1]:.0f} dB)",
                   "form": "fused + HIP graph, extended-precision transforms",
                   "precision": "FP64 transforms, covariance, LDL^H and normalisation; X and "
                                "the windows stored as FP32 + BF16 remainder",
                   "pairs_per_step": beams,
                   "tuning": dict(zip(("chan_logtile", "beam_logtile", "pair_kernel",
                                       "overlap_chunks"), tun)),
                   "tuning_f32": dict(zip(("chan_logtile", "beam_logtile", "pair_kernel",
                                           "overlap_chunks"), plan.get_tuning("f32")))},
        "graph_f32": {"value": beams / (ms_f32 * 1e-3), "ms_per_step": ms_f32,
                      "form": "the chosen sequence with FP32 transforms and FP32 X / windows"},
        "plain": (None if ms_plain is None else
                  {"value": beams / (ms_plain * 1e-3), "ms_per_step": ms_plain,
                   "form": "per-stage FP32 kernels, full beamspace in HBM, no graph"}),
        "mixed": mixed,
        "learned": learned_res,
        "full_dim": (None if ms_full is None else
                     {"value": T * full_k / (ms_full * 1e-3), "ms_per_step": ms_full,
                      "subbands_per_step": full_k,
                      "form": f"element-space {cfg.N}x{cfg.N} MVDR per subband, FP64 "
                              f"(covariance, blocked Cholesky, blocked solves, apply; "
                              f"{full_k} of {K} subbands per step)"}),
        **beside,
        "upa": upa_res,
        "roofline": roofline,
        "covariance": covariance,
    }
    plan.close()
    del out, wts, info
    torch.cuda.empty_cache()

    extras = {}
    for name in [n for n in args.extra.split(",") if n and n != cfg.name]:
        log(f"extra leg: {name}")
        extras[name] = extra_leg(torch, wb, scenes, name, args.steps, args.warmup)
    result["extra_legs"] = extras

    if not args.no_cpu:
        log(f"CPU oracle leg on subbands {ks}")
        x_host = host_copy(torch, x) if cfg.N >= 1024 else sc_host_x(scenes, cfg)
        del x
        torch.cuda.empty_cache()
        cpu, ref = cpu_baseline_leg(sc, x_host, ks)
        result["cpu_baseline"] = cpu
        log("validity of every pair on those subbands")
        val = validity(sc, ref, ks, weights, infos)
        val["subbands"] = ks
        val["bar_db"] = 0.1
        g = val["graph"]
        val["valid"] = bool(g["max_sinr_loss_db"] <= 0.1 and g["max_rel_weight_err"] <= 1e-5
                            and g["failed_pairs"] == 0 and g["nonfinite_pairs"] == 0)
        result["validity"] = val
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)
    return 0


def sc_host_x(scenes, cfg):
    """The small workloads' samples on the host (the same seeded scene the GPU ran)."""
    return scenes.make_scene(cfg).x.astype(np.complex64)


if __name__ == "__main__":
    sys.exit(main())
