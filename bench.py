#!/usr/bin/env python3
"""Throughput of the PISO + Equilibrium-Eulerian dust step on one MI355X.

Workload: seeded synthetic decaying homogeneous isotropic turbulence on the
periodic 256^3 cube (r.m.s. Mach 0.2, one dust class at Stokes 0.2, CFL 0.5,
two PISO correctors, pressure residual 1e-6), the paper's 256^3 DNS setting
with a synthetic initial field.  A "step" is one full time step: dt, density
predictor, momentum predictor, two correctors with their pressure solves, flux
and velocity correction and dust transport.

Prints one JSON line: cell-steps/s, the roofline figures of the dominant
kernel (HIP events around every launch in the timed region, algorithmic bytes
per launch counted by the library) and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PISO cell-steps/s at 256^3: plain FP64 vs FP32+learned guess, resid 1e-6"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--mode", default="both", choices=["fp64", "fp32", "both"],
                    help="both: time plain FP64 and the FP32 mode; the FP32 run is the headline")
    ap.add_argument("--inner-tol", type=float, default=1e-6)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--p-tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target CPU time of the oracle sample")
    return ap.parse_args()


def cpu_baseline(case, p_tol, target_s):
    """Time the FP64 oracle on the host on whole steps of the same workload."""
    import oracle
    oracle.build(force=False)
    o = oracle.Oracle.from_case(case, p_tol=p_tol)
    n3 = case.n ** 3
    t0 = time.perf_counter()
    st, _ = o.step(1)              # first step (includes first touch of the work arrays)
    t1 = time.perf_counter()
    first = t1 - t0
    steps, elapsed = 0, 0.0
    if first < target_s / 2:
        while elapsed < target_s and steps < 10:
            t2 = time.perf_counter()
            o.step(1)
            elapsed += time.perf_counter() - t2
            steps += 1
        sample = f"{steps} step(s) of the {case.n}^3 workload after 1 untimed step"
    else:
        steps, elapsed = 1, first
        sample = f"1 step of the {case.n}^3 workload (first step, cold work arrays)"
    return dict(value=n3 * steps / elapsed, unit="cell-steps/s", cores=oracle.num_threads(),
                kind="oracle", sample=sample, seconds=round(elapsed, 3))


def timed_run(P, torch, case, prec, args, guess=None):
    """Warm up, then time exactly args.steps steps with per-kernel events on."""
    kw = dict(p_tol=args.p_tol, cfl=0.5, n_corr=2, n_mom_sweeps=4, n_dust_sweeps=4)
    if guess is not None:
        kw.update(guess=P.GUESS_LEARNED, guess_weights=guess)
    s = P.Solver.from_case(case, precision=prec, inner_tol=args.inner_tol, **kw)
    st, _ = s.step(args.warmup)
    torch.cuda.synchronize()
    s.profile(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    st, info = s.step(args.steps)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    prof = s.profile_read()
    s.profile(False)
    s.close()
    return t_end - t_start, info, prof


def roofline(prof):
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    per_launch = dom["bytes"] / dom["launches"]
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    kernels = {k: dict(launches=v["launches"], avg_us=round(1e3 * v["ms"] / v["launches"], 2),
                       share=round(v["ms"] / sum(x["ms"] for x in prof.values()), 4),
                       gbs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1))
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
    roof = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None, "avg_launch_us": round(avg_ms * 1e3, 2),
            "bytes_per_launch": per_launch}
    return roof, kernels


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        log("bench.py: one GPU only (the multi-GPU decomposition is a design note, not built)")
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1404_0959_amd.pisoc as P
    from paper_1404_0959_amd.inputs import make_hit_case

    if not torch.cuda.is_available():
        log("bench.py needs the GPU")
        sys.exit(1)
    t0 = time.time()
    case = make_hit_case(args.n, args.seed, mach=0.2, stokes=(0.2,))
    log(f"inputs {case.name} ready in {time.time() - t0:.1f}s")
    n3 = args.n ** 3

    runs = {}
    modes = ["fp64", "fp32"] if args.mode == "both" else [args.mode]
    for m in modes:
        prec = P.FP64 if m == "fp64" else P.FP32_REFINED
        el, info, prof = timed_run(P, torch, case, prec, args)
        iters = [i["pcg_iters"] for i in info]
        runs[m] = dict(elapsed=el, info=info, prof=prof, value=n3 * args.steps / el,
                       iters=float(np.mean([sum(i) / len(i) for i in iters])))
        log(f"{m}: {el * 1e3 / args.steps:.3f} ms/step, {n3 * args.steps / el:.4e} cell-steps/s, "
            f"mean CG iterations per solve {runs[m]['iters']:.2f}")
    head = "fp32" if "fp32" in runs else modes[0]
    H = runs[head]
    roof, kernels = roofline(H["prof"])
    log(json.dumps(kernels))

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        cpu = cpu_baseline(case, args.p_tol, args.cpu_seconds)
        log(f"oracle: {cpu}")

    out = {
        "metric": METRIC,
        "value": H["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": H["elapsed"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"decaying HIT {args.n}^3, Mach 0.2, 1 dust class St 0.2, "
                               f"CFL 0.5, 2 PISO correctors, Jacobi-PCG rel. residual "
                               f"{args.p_tol:g}, seed {args.seed}",
                   "grid": args.n, "mode": head, "guess": "zero"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "pcg_iters_mean": H["iters"],
        "modes": {m: {"value": r["value"], "ms_per_step": r["elapsed"] * 1e3 / args.steps,
                      "pcg_iters_mean": r["iters"]} for m, r in runs.items()},
        "kernels": kernels,
    }
    if "fp64" in runs and "fp32" in runs:
        out["speedup_vs_fp64"] = runs["fp32"]["value"] / runs["fp64"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
