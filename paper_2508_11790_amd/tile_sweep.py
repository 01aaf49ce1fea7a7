"""Per-stage kernel times of the fused sequence for every FFT tile, in both transform
precisions, at one workload shape.

Usage: ``python -m paper_2508_11790_amd.tile_sweep [--workload precision] [--half-bin]``

For each precision ("ext": FP64 transforms with FP32 + BF16-remainder storage; "f32") and each
channelizer tile it pins the launch configuration (``Plan.set_tuning``) and prints the average
milliseconds per launch of every stage from ``Plan.stage_times``: one untimed and ``--reps``
timed launches.  The samples are random complex Gaussian numbers of the workload's shape (the
kernels' times do not depend on the values); targets are spread over [-50, 43] degrees.
"""

from __future__ import annotations

import argparse
import math


SHAPES = {   # name: (N, M, K, L, Lt, targets, window)
    "gpu": (256, 512, 128, 256, 256, 8, 9),
    "batch": (1024, 2048, 256, 512, 512, 64, 33),
    "precision": (4096, 8192, 512, 1024, 1024, 32, 64),
}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="precision", choices=sorted(SHAPES))
    ap.add_argument("--half-bin", action="store_true", help="subband centres of Eq. 1")
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args(argv)
    import torch
    import paper_2508_11790_amd as wb
    N, M, K, L, Lt, T, W = SHAPES[args.workload]
    torch.cuda.set_device(0)
    gen = torch.Generator(device="cuda").manual_seed(1)
    x = torch.randn((N, (L + Lt) * K), dtype=torch.complex64, device="cuda", generator=gen)
    az = [math.radians(-50.0 + 93.0 * t / max(1, T - 1)) for t in range(T)]
    plan = wb.Plan(N, M, K, L, Lt, T, W, beta=0.2, d_over_lambda=0.5, half_bin=args.half_bin)
    lm = int(math.log2(M))
    for prec, tiles in (("f32", (11, 12, 13)), ("ext", (10, 11, 12, 13))):
        beam = max(min(13, lm), tiles[0])       # spatial DFT at its largest tile
        for tile in tiles:
            plan.set_tuning(tile, beam, "block", 1, precision=prec)
            st = plan.stage_times(x, az, [W] * T, 10.0, reps=args.reps, precision=prec)
            print(f"{prec} chan_logtile {tile} beam_logtile {beam}: "
                  + ", ".join(f"{k} {v:.3f} ms" for k, v in st.items()), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
