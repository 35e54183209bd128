"""Train the warm-start surrogate on solver-generated steady states and
measure what it gains over the plain solver.

    python -m paper_1804_02418_amd.train_surrogate --train 512 --heldout 64 \
        --epochs 30 --out weights.npz --report report.json

1. Steady states (FP64, residual < 1e-8 over 100 steps) of `train` samples
   of the uneven-sample generator at a fixed size, and of `heldout` samples
   with disjoint seeds; the held-out cold runs are the baseline.
2. Adam on the BF16 U-Net (mean squared error of the linear-response
   targets).
3. Warm start of every held-out sample from the network's prediction
   (falling back to a cold start if the prediction is unusable), run to the
   same tolerance; steps and wall time (network inference included) are
   compared with the cold runs.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=512)
    ap.add_argument("--heldout", type=int, default=64)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--max-steps", type=int, default=300_000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--out", default="")
    ap.add_argument("--report", default="")
    args = ap.parse_args(argv)

    import torch

    from . import _binding as B
    from . import surrogate as S
    from . import workloads

    def log(msg):
        print(msg, flush=True)

    t_all = time.perf_counter()
    Xtr, Ytr, info_tr = S.generate(args.train, args.size, 0, args.max_steps, args.tol, log=log)
    Xte, Yte, info_te = S.generate(args.heldout, args.size, args.train, args.max_steps, args.tol, log=log)
    held = workloads.batch_samples(args.train + args.heldout, fixed_size=(args.size, args.size))[args.train:]
    keep = np.array([i["residual"] < args.tol for i in info_tr])
    log(f"training on {keep.sum()} converged samples of {len(info_tr)}")

    net = B.UNet(16, S.CIN, S.COUT, args.size, args.size, max_batch=args.batch, seed=1)
    scale = S.channel_scales(Ytr[keep])
    log(f"target scales {scale}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    curve = S.train(net, Xtr[keep], Ytr[keep] / scale, args.epochs, args.batch, args.lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    preds = S.predict(net, Xte, args.batch) * scale
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    err = np.sqrt(((preds - Yte) ** 2).mean(axis=(1, 2, 3)) / (Yte ** 2).mean(axis=(1, 2, 3)))
    inits = S.warm_start_inits(held, preds)
    fallbacks = sum(1 for i in inits if i is None)
    _, steps_w, r_w, t_warm = S.solve_batch(held, args.max_steps, tol=args.tol, init=inits)
    steps_c = np.array([i["steps"] for i in info_te])
    # per-sample cold wall time is not separable inside a batch: time a cold batch again
    _, steps_c2, r_c2, t_cold = S.solve_batch(held, args.max_steps, tol=args.tol)
    report = {
        "samples": {"train": int(keep.sum()), "heldout": args.heldout, "size": args.size},
        "train": {"epochs": args.epochs, "batch": args.batch, "lr": args.lr, "seconds": round(t_train, 2),
                  "loss_first": curve[0], "loss_last": curve[-1], "params": net.nparam,
                  "target_scales": [float(v) for v in scale]},
        "heldout_prediction_rel_rms_error": {"median": float(np.median(err)), "max": float(err.max())},
        "cold": {"steps_median": float(np.median(steps_c2)), "steps_mean": float(steps_c2.mean()),
                 "seconds_batch": round(t_cold, 2), "converged": int((r_c2 < args.tol).sum())},
        "warm": {"steps_median": float(np.median(steps_w)), "steps_mean": float(steps_w.mean()),
                 "seconds_batch_plus_inference": round(t_warm + t_infer, 2), "inference_seconds": round(t_infer, 3),
                 "converged": int((r_w < args.tol).sum()), "fallbacks": fallbacks},
        "step_ratio_median": float(np.median(steps_w / np.maximum(steps_c2, 1))),
        "total_seconds": round(time.perf_counter() - t_all, 1),
    }
    log(json.dumps(report))
    if args.out:
        np.savez(args.out, theta=net.get_params(), scale=scale, base=16, cin=S.CIN, cout=S.COUT, size=args.size,
                 loss=np.array(curve))
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
