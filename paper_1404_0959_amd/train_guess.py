"""Train the learned pressure guess and measure what it gains.

    python -m paper_1404_0959_amd.train_guess [--epochs 20] [--out weights/guess.npy]
        [--loss residual|mse] [--init weights/guess_hit32.npy]

(the committed weights/guess_hit32_residual.npy: the defaults; the earlier
weights/guess_hit32.npy: --loss mse --epochs 30 --out weights/guess_hit32.npy)

Data: 20 seeded 32^3 decaying-HIT runs (Mach 0.2, Stokes 0.1, pressure
tolerance 1e-8), 100 steps each, first-corrector systems -> 2000 snapshots.
Training on the GPU with the project's kernels.  Evaluation on unseen seeds:
CG iterations per step and wall time with and without the guess, at
residual 1e-6, FP64 and FP32 modes, at 32^3, 128^3 and 256^3.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import learn


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seeds", type=int, default=20)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "weights",
                                                  "guess_hit32_residual.npy"))
    ap.add_argument("--eval-sizes", default="32,128,256")
    ap.add_argument("--loss", default="residual", choices=["mse", "residual"],
                    help="mse: against the solution p'/s1; residual: the relative residual "
                         "|b - alpha M g|^2/|b|^2 the solve would start from")
    ap.add_argument("--init", default=None, help="start from these weights (.npy)")
    ap.add_argument("--report", default=None)
    ap.add_argument("--extra", default="",
                    help="extra training data at other sizes, e.g. 64:4:25,128:2:12 "
                         "(size:seeds:steps, seeds taken after the 32^3 ones)")
    args = ap.parse_args()

    def log(m):
        print(m, file=sys.stderr, flush=True)
    import torch
    from . import pisoc as P
    t0 = time.time()
    res = args.loss == "residual"
    xs, ts, sys_ = [], [], []
    sets = [(32, range(args.seeds), args.steps)]
    for spec in [e for e in args.extra.split(",") if e]:
        n_e, s_e, st_e = (int(v) for v in spec.split(":"))
        sets.append((n_e, range(100, 100 + s_e), st_e))
    for n_e, seeds, steps in sets:
        out = learn.generate(seeds, steps, n=n_e, log=log, systems=res)
        xs.append(out[0])
        ts.append(out[1])
        if res:
            sys_.append(out[2])
    nsnap = sum(x.shape[0] for x in xs)
    log(f"{nsnap} snapshots in {time.time() - t0:.1f}s")
    t1 = time.time()
    w0 = np.load(args.init, allow_pickle=False) if args.init else None
    w, hist = learn.train(xs, ts, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log,
                          w0=w0, systems=sys_ if res else None)
    log(f"trained in {time.time() - t1:.1f}s, loss {hist[0]:.4e} -> {hist[-1]:.4e}")
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, w.cpu().numpy())
    del xs, ts, sys_
    torch.cuda.empty_cache()
    report = dict(snapshots=nsnap, extra=args.extra, epochs=args.epochs, loss=args.loss,
                  init=args.init, loss_history=hist,
                  weights=os.path.basename(args.out), eval={})
    for n in [int(v) for v in args.eval_sizes.split(",")]:
        seeds = (20, 21, 22, 23, 24) if n <= 32 else ((20,) if n >= 256 else (20, 21))
        steps = 20 if n <= 128 else 10
        for mode, prec in (("fp64", P.FP64), ("fp32", P.FP32_REFINED)):
            r = learn.evaluate(w, n, seeds, steps, precision=prec)
            report["eval"][f"{n}_{mode}"] = r
            log(f"n={n} {mode}: {json.dumps(r)}")
    print(json.dumps(report))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
