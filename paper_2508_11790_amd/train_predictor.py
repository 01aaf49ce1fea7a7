"""Train the loading / window predictor on the GPU and measure what it gains.

    python -m paper_2508_11790_amd.train_predictor --train-scenes 2048 --eval-scenes 4 \\
        --epochs 20 --out predictor.npz --summary predictor.json

Training data: seeded synthetic scenes of the N=256, M=512, K=128, L=256 shape (8 targets,
3 wideband jammers at 20-40 dB INR), every (target, subband) pair one sample (1024 per
scene); labels from the plain method swept over 11 loadings x 4 window widths and scored by
output SINR against the scene's exact interference covariance.  Evaluation: held-out scenes
of the N=1024, M=2048, K=256, L=512 shape (64 targets with windows drawn from {5, 9, 17, 33},
6 jammers at 20-50 dB): mean output SINR of the learned form against the fixed method
(loading 10 sigma^2, each target's own window), with the sweep's best as the ceiling.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, flush=True)


def build_dataset(wb, learned, scenes, cfg, n_scenes, seed0, plan, mlp):
    import torch
    feats, labels = [], []
    t0 = time.time()
    for i in range(n_scenes):
        sc, x = scenes.make_scene_torch(cfg, seed0 + i)
        r = learned.label_sweep(plan, mlp, x, sc.target_az, sc.jammer_az, sc.jammer_inr)
        feats.append(r["feat"])
        labels.append(r["labels"])
        del x
        if (i + 1) % 64 == 0 or i + 1 == n_scenes:
            torch.cuda.synchronize()
            log(f"  scenes {i + 1}/{n_scenes} labelled ({time.time() - t0:.1f} s)")
    return torch.cat(feats), torch.cat(labels)


def evaluate(wb, learned, scenes, cfg, n_scenes, seed0, params, with_ceiling=True):
    """Mean output SINR (dB) per pair: fixed method, learned form, sweep best."""
    import torch
    res = dict(fixed=[], learned=[], best=[], fallback=0, pairs=0, wins=[])
    plan = wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, cfg.T, 33, beta=cfg.beta,
                   d_over_lambda=cfg.dl)
    mlp = wb.Mlp(4096)
    for i in range(n_scenes):
        sc, x = scenes.make_scene_torch(cfg, seed0 + i)
        fx = plan.beamform(x, sc.target_az, sc.win, cfg.delta, form="fused")
        s_fixed = plan.sinr(sc.target_az, sc.win, fx["weights"], fx["starts"], sc.jammer_az,
                            sc.jammer_inr)
        lr = plan.beamform_learned(x, sc.target_az, params, 1.0, 9, cfg.delta)
        win33 = [33] * cfg.T
        s_learn = plan.sinr(sc.target_az, win33, lr["weights"], lr["starts"], sc.jammer_az,
                            sc.jammer_inr, pair_win=lr["pair_win"])
        res["fixed"].append(10 * torch.log10(s_fixed).reshape(-1))
        res["learned"].append(10 * torch.log10(s_learn).reshape(-1))
        res["fallback"] += int(lr["fallback"].sum())
        res["pairs"] += cfg.T * cfg.K
        res["wins"].append(torch.bincount(lr["pair_win"].reshape(-1).long(), minlength=34)[[5, 9, 17, 33]])
        if with_ceiling:
            r = learned.label_sweep(plan, mlp, x, sc.target_az, sc.jammer_az, sc.jammer_inr)
            res["best"].append(10 * torch.log10(r["table"].max(dim=0).values))
        del x
        torch.cuda.synchronize()
        log(f"  eval scene {i + 1}/{n_scenes}")
    out = {}
    for key in ("fixed", "learned", "best"):
        if res[key]:
            v = torch.cat(res[key])
            out[key + "_mean_sinr_db"] = float(v.mean())
    fx_all, ln_all = torch.cat(res["fixed"]), torch.cat(res["learned"])
    out["gain_db"] = out["learned_mean_sinr_db"] - out["fixed_mean_sinr_db"]
    out["pairs_improved"] = float((ln_all > fx_all).float().mean())
    out["fallback_pairs"] = res["fallback"]
    out["pairs"] = res["pairs"]
    out["chosen_widths_5_9_17_33"] = [int(v) for v in torch.stack(res["wins"]).sum(0).tolist()]
    plan.close()
    mlp.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--train-scenes", type=int, default=2048)
    ap.add_argument("--eval-scenes", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--eval-config", default="learned_eval")
    ap.add_argument("--out", default="predictor.npz")
    ap.add_argument("--summary", default=None)
    args = ap.parse_args(argv)

    import torch
    import scenes
    import paper_2508_11790_amd as wb
    from paper_2508_11790_amd import learned

    torch.cuda.set_device(0)
    cfg = scenes.LEARNED_TRAIN
    plan = wb.Plan(cfg.N, cfg.M, cfg.K, cfg.L, cfg.Lt, cfg.T, 33, beta=cfg.beta,
                   d_over_lambda=cfg.dl)
    mlp = wb.Mlp(args.batch)
    log(f"labelling {args.train_scenes} training scenes ({args.train_scenes * cfg.T * cfg.K} samples)")
    t0 = time.time()
    feats, labels = build_dataset(wb, learned, scenes, cfg, args.train_scenes, cfg.seed, plan, mlp)
    t_label = time.time() - t0
    params = torch.from_numpy(learned.init_params(args.seed)).cuda()
    log(f"training: {feats.shape[0]} samples, {args.epochs} epochs, batch {args.batch}")
    t0 = time.time()
    hist = learned.train(mlp, params, feats, labels, epochs=args.epochs, batch=args.batch,
                         lr=args.lr, seed=args.seed + 1, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    learned.save_params(args.out, params)
    ecfg = scenes.config_by_name(args.eval_config)
    log(f"evaluating on {args.eval_scenes} {ecfg.name} scenes")
    ev = evaluate(wb, learned, scenes, ecfg, args.eval_scenes, ecfg.seed, params)
    summary = dict(train_samples=int(feats.shape[0]), label_seconds=t_label, train_seconds=t_train,
                   epochs=args.epochs, loss_history=hist, eval=ev, eval_config=ecfg.name)
    log(json.dumps(summary))
    if args.summary:
        with open(args.summary, "w") as f:
            json.dump(summary, f, indent=1)
    plan.close()
    mlp.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
