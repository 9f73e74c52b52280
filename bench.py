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
per launch counted by the library), beside them the practical ceiling of the
same read/write mixes measured by the library's streaming probe, and the FP64
CPU oracle timed on a bounded sample of the same workload on the host cores.
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
    ap.add_argument("--mode", default="all", choices=["fp64", "fp32", "fp32_learned", "all"],
                    help="all: time plain FP64, FP32 and FP32 + learned guess; the last is the "
                         "headline")
    ap.add_argument("--guess-audit", type=int, default=16,
                    help="learned guess: audit period in steps (0: apply to every solve)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the runs, copy a buffer of this size a few times (a plain copy "
                         "kernel of known traffic for scaling HBM byte counters)")
    ap.add_argument("--inner-tol", type=float, default=1e-6)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--p-tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the 64-member mixed-size ensemble measurement")
    ap.add_argument("--ens-members", type=int, default=64)
    ap.add_argument("--ens-steps", type=int, default=20)
    ap.add_argument("--ens-seq-steps", type=int, default=3,
                    help="timed steps per member of the sequential single-grid runs")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the two-way coupling and diagnostics measurements")
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
    """Warm up, time exactly args.steps steps (the value), then as many more with
    per-kernel HIP events on the library's stream (the per-kernel times of the
    roofline: recording an event pair around every launch adds a gap before
    each kernel, so those steps are not the ones the value is taken from)."""
    kw = dict(p_tol=args.p_tol, cfl=0.5, n_corr=2, n_mom_sweeps=4, n_dust_sweeps=4)
    if guess is not None:
        kw.update(guess=P.GUESS_LEARNED, guess_weights=guess.data_ptr(),
                  guess_audit=args.guess_audit)
    s = P.Solver.from_case(case, precision=prec, inner_tol=args.inner_tol, **kw)
    st, _ = s.step(args.warmup)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    st, info = s.step(args.steps)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    s.profile(True)
    torch.cuda.synchronize()
    t_prof = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    t_prof_end = time.perf_counter()
    prof = s.profile_read()
    s.profile(False)
    s.close()
    return t_end - t_start, info, prof, t_prof_end - t_prof


def ensemble_run(P, torch, args, weights):
    """The mixed-size ensemble (32^3, 48^3, 64^3 in the ratio 2:1:1, Mach from
    {0.2, 0.5}, Stokes U[0.05, 0.5]; FP32 + learned guess under the audit, whose
    verdict per size class the captured step keeps) stepped by replaying one
    captured graph per step after the launch-shape autotuner, against the same
    members stepped one after another as single grids."""
    import tempfile

    import numpy as np

    from paper_1404_0959_amd.inputs import ensemble_cases
    cases = ensemble_cases(args.ens_members, seed=args.seed)
    cells = sum(c.n ** 3 for c in cases)
    common = dict(p_tol=args.p_tol, cfl=0.5, n_corr=2, n_mom_sweeps=4, n_dust_sweeps=4)
    fast = dict(precision=P.FP32_REFINED, inner_tol=args.inner_tol, guess=P.GUESS_LEARNED,
                guess_weights=weights.data_ptr(), guess_audit=args.guess_audit, **common)
    out = {"members": len(cases), "cells": cells,
           "sizes": {str(n): sum(1 for c in cases if c.n == n) for n in sorted({c.n for c in cases})}}

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    E = P.Ensemble(cases, **fast)
    E.step(1, mode=P.ENS_EAGER)
    cache = os.path.join(tempfile.gettempdir(), "pisoc_tune.json")
    t0 = time.perf_counter()
    E.autotune(cache, force=True)
    out["autotune_s"] = round(time.perf_counter() - t0, 3)
    st_holder = {}

    def graph_steps(mode):
        def run(k):
            st_holder["st"], st_holder["info"] = E.step(k, mode=mode)
        return run
    # one graph per size class, replayed on the class streams
    E.step(args.warmup, mode=P.ENS_GRAPH)
    el = timed(graph_steps(P.ENS_GRAPH), args.ens_steps)
    out["per_class_graphs"] = dict(value=cells * args.ens_steps / el,
                                   ms_per_step=el * 1e3 / args.ens_steps)
    log(f"ensemble, one graph per class: {el * 1e3 / args.ens_steps:.3f} ms/step")
    # one graph for the whole ensemble: one launch per step (the value)
    E.step(args.warmup, mode=P.ENS_GRAPH_ONE)
    el = timed(graph_steps(P.ENS_GRAPH_ONE), args.ens_steps)
    out["mode"] = "one graph launch per step (every size class a branch)"
    out["value"] = cells * args.ens_steps / el
    out["unit"] = "cell-steps/s"
    out["ms_per_step"] = el * 1e3 / args.ens_steps
    out["status"] = st_holder["st"]
    out["max_relres"] = max(max(i["pcg_relres"]) for i in st_holder["info"])
    out["pcg_iters_mean"] = float(np.mean([np.mean(i["pcg_iters"]) for i in st_holder["info"]]))
    out["classes"] = [{k: c[k] for k in ("n", "members", "block", "cells_z", "cg_cells_z",
                                         "tiled_cells_z", "caps", "rounds", "guess_mask")}
                      for c in E.classes()]
    log(f"ensemble, one graph per step: {out['ms_per_step']:.3f} ms/step, "
        f"{out['value']:.4e} cell-steps/s")

    def eager_steps(k):
        E.step(k, mode=P.ENS_EAGER)
    el = timed(eager_steps, max(2, args.ens_steps // 4))
    out["eager_batched"] = cells * max(2, args.ens_steps // 4) / el
    E.close()
    del E

    def sequential(kw, k):
        total = 0.0
        for c in cases:
            s = P.Solver.from_case(c, **kw)
            s.step(1)
            torch.cuda.synchronize()
            total += timed(lambda j: s.step(j), k) / k
            s.close()
        return cells / total
    out["sequential_plain_fp64"] = sequential(dict(precision=P.FP64, **common), args.ens_seq_steps)
    out["sequential_fp32_learned"] = sequential(fast, args.ens_seq_steps)
    out["vs_sequential_plain"] = out["value"] / out["sequential_plain_fp64"]
    out["vs_sequential_same_method"] = out["value"] / out["sequential_fp32_learned"]
    log(f"ensemble: {json.dumps(out)}")
    return out


def extras_run(P, torch, case, args):
    """The other rows of the step at the benchmark's size: the two-way coupled
    mixture with gravity settling (FP32 refined, same workload, dust loading
    raised to 0.2), the FP64 variants (Fourier closure, BDF2, momentum
    predictor solved by BiCGStab), the flow diagnostics on the velocity field,
    each with its algorithmic bytes (words each kernel must read or write
    once), and the guess network alone."""
    import numpy as np
    out = {}
    n3 = args.n ** 3
    kw = dict(p_tol=args.p_tol, cfl=0.5, n_corr=2, n_mom_sweeps=4, n_dust_sweeps=4,
              precision=P.FP32_REFINED, inner_tol=args.inner_tol, two_way=True,
              gravity=(0.0, 0.0, -1.0))
    s = P.Solver(case.n, case.rho, case.u, case.rho_p * 200.0, gamma=case.gamma, C_=case.C,
                 mu=case.mu, tau_p=case.tau_p, **kw)
    s.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = s.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["two_way_fp32"] = dict(value=n3 * args.steps / el, unit="cell-steps/s",
                               ms_per_step=el * 1e3 / args.steps, status=st,
                               pcg_iters_mean=float(np.mean([np.mean(i["pcg_iters"]) for i in info])))
    log(f"two-way FP32: {el * 1e3 / args.steps:.3f} ms/step")
    u = s.get(P.FIELD_U)
    s.close()
    del s
    # variants of the FP64 step, all on the gathered field kernels: the Fourier
    # closure (ideal gas with R = 1, c_v = 2.5, so c_p/c_v = 1.4, T0 = C so
    # that the sound speed matches the barotropic gas), BDF2, and the momentum
    # predictor solved to 1e-8 by BiCGStab
    fz = dict(R=1.0, cv=2.5, kappa=1e-3, T0=case.C)
    base = dict(p_tol=args.p_tol, cfl=0.5, n_corr=2, n_mom_sweeps=4, n_dust_sweeps=4)
    for name, extra in (("fourier_fp64", dict(fourier=fz)), ("bdf2_fp64", dict(bdf2=True)),
                        ("mom_bicgstab_fp64", dict(mom_tol=1e-8))):
        s = P.Solver(case.n, case.rho, case.u, case.rho_p, gamma=case.gamma, C_=case.C,
                     mu=case.mu, tau_p=case.tau_p, **base, **extra)
        s.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = s.step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = dict(value=n3 * args.steps / el, unit="cell-steps/s",
                         ms_per_step=el * 1e3 / args.steps, status=st,
                         pcg_iters_mean=float(np.mean([np.mean(i["pcg_iters"]) for i in info])))
        if "mom_tol" in extra:
            out[name]["mom_iters_mean"] = float(np.mean([i["mom_iters"] for i in info]))
        log(f"{name}: {el * 1e3 / args.steps:.3f} ms/step")
        s.close()
        del s

    def time_it(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps
    diag = {}
    # bytes per cell: spectrum, per component: the real field read (8), three
    # FFT passes reading and writing the complex field (3 x 32), the shell
    # binning reading it (16); Q: 3 velocity words read, Q written; filtered
    # statistics: u read (24) and nine filtered fields written (72), then read
    # back (72)
    for name, fn, bpc in (("spectrum", lambda: P.spectrum(u), 3 * (8 + 96 + 16)),
                          ("qcriterion", lambda: P.qcriterion(u), 32),
                          ("filtered_stats", lambda: P.sgs_stats(u), 168)):
        t = time_it(fn)
        diag[name] = dict(ms=round(t * 1e3, 3), gbs=round(bpc * n3 / t / 1e9, 1),
                          bytes_per_cell=bpc)
        log(f"{name}: {t * 1e3:.3f} ms, {bpc * n3 / t / 1e9:.1f} GB/s")
    E, lam, D = P.spectrum(u)
    diag["taylor_microscale"] = lam
    out["diagnostics"] = diag
    del u
    # the learned guess's network alone on one n^3 input (seeded normal):
    # forward (30,240 BF16 flops per cell; 204 bytes per cell of activations
    # read and written once, layer by layer) and one training gradient
    from paper_1404_0959_amd.learn import load_weights
    w = load_weights()
    g = torch.Generator(device="cuda").manual_seed(args.seed)
    x = torch.randn(1, n3, 2, generator=g, device="cuda")
    net = P.Net(args.n, 1)
    t_fwd = time_it(lambda: net.forward(w, x))
    flop, bpc = 30240 * n3, 204
    out["net"] = dict(forward_ms=round(t_fwd * 1e3, 3), forward_tflops=round(flop / t_fwd / 1e12, 1),
                      forward_frac_bf16_peak=round(flop / t_fwd / 2.5e15, 4),
                      forward_gbs=round(bpc * n3 / t_fwd / 1e9, 1),
                      forward_frac_hbm=round(bpc * n3 / t_fwd / 8e12, 4))
    t_grad = time_it(lambda: net.grad(w, x, x[..., 0].contiguous()))
    out["net"]["grad_ms"] = round(t_grad * 1e3, 3)
    log(f"network forward: {t_fwd * 1e3:.3f} ms ({flop / t_fwd / 1e12:.0f} TFLOP/s), "
        f"gradient {t_grad * 1e3:.3f} ms")
    return out


KERNEL_SOURCES = ("kernels.hip", "device.hpp", "launch.hpp", "net.hip")
# dominant kernel class -> the 256^3 kernels whose HBM bytes the committed
# counter summary holds (template instances of one kernel class are averaged
# over their working launches)
TRAFFIC_NAME = {("k_pcg_spmv", "f32+f64"): tuple(f"k_pcg_spmv_rows<float, 4, 1, {m}, true>"
                                                  for m in range(3)),
                ("k_pcg_spmv", "f64"): tuple(f"k_pcg_spmv_rows<double, 2, 2, {m}, false>"
                                             for m in range(3))}


def measured_traffic(kernel, dtype, n):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel
    calibration), or None when it does not cover this kernel and size or the
    kernel sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_256.json")
    if n != 256 or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1404_0959_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    recs = [rec["kernels"].get(name) for name in TRAFFIC_NAME.get((kernel, dtype), ())]
    if not recs or any(r is None for r in recs):
        return None
    launches = sum(r["launches"] for r in recs)
    if launches == 0:
        return None
    return sum((r["fetch_bytes"] + r["write_bytes"]) * r["launches"] for r in recs) / launches


STREAM_MIXES = ((1, 1), (3, 2), (5, 3), (7, 4))
# FP32 words per cell each field kernel class reads and writes (the writes as
# the WRITE_SIZE counter measures them, the reads the rest of the kernel's
# algorithmic words); k_refine's mix depends on the round and is left out
FIELD_MIXES = {"k_predict": (7, 4), "k_mom_source": (5, 3), "k_mom_sweep": (11, 3),
               "k_hbya": (11, 5), "k_corr_rhs": (7, 7), "k_corr_update": (11, 7),
               "k_dudt": (6, 3), "k_dust_flux": (9, 4), "k_dust_sweep": (6, 1),
               "k_dust_finish": (5, 1)}


def stream_ceiling(P, torch, n, mixes=STREAM_MIXES, reps=20):
    """Practical HBM ceiling of read/write mixes: the library's plain streaming
    probe over n^3 FP32 fields, GB/s per mix (reads + writes), timed with HIP
    events on the stream it runs on.  The CG moves 3 reads + 2 writes per cell
    at k = 0, 5 + 3 at odd k, 7 + 4 at even k."""
    count = n ** 3 // 4 * 4
    rmax, wmax = max(r for r, _ in mixes), max(w for _, w in mixes)
    bufs = [torch.ones(count, dtype=torch.float32, device="cuda") for _ in range(rmax + wmax)]
    out = {}
    for r, w in mixes:
        ins, outs = bufs[:r], bufs[rmax:rmax + w]
        for _ in range(3):
            P.stream_probe(ins, outs)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            P.stream_probe(ins, outs)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / reps
        out[f"{r}r{w}w"] = round(4.0 * count * (r + w) / sec / 1e9, 1)
    del bufs
    torch.cuda.empty_cache()
    return out


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

    if args.calib_copy_mib > 0:
        a = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.calib_copy_mib} MiB")
        del a, b

    from paper_1404_0959_amd.learn import load_weights
    weights = load_weights()
    runs = {}
    modes = ["fp64", "fp32", "fp32_learned"] if args.mode == "all" else [args.mode]
    for m in modes:
        prec = P.FP64 if m == "fp64" else P.FP32_REFINED
        el, info, prof, el_prof = timed_run(P, torch, case, prec, args,
                                            guess=weights if m == "fp32_learned" else None)
        iters = [i["pcg_iters"] for i in info]
        runs[m] = dict(elapsed=el, elapsed_events=el_prof, info=info, prof=prof,
                       value=n3 * args.steps / el,
                       iters=float(np.mean([sum(i) / len(i) for i in iters])),
                       guess_steps=sum(1 for i in info if not i["flags"] & P.FLAG_GUESS_SKIPPED))
        log(f"{m}: {el * 1e3 / args.steps:.3f} ms/step, {n3 * args.steps / el:.4e} cell-steps/s, "
            f"mean CG iterations per solve {runs[m]['iters']:.2f} "
            f"({el_prof * 1e3 / args.steps:.3f} ms/step with per-kernel events)")
    head = modes[-1]
    H = runs[head]
    roof, kernels = roofline(H["prof"])
    roof["traffic"] = measured_traffic(roof["kernel"], "f64" if head == "fp64" else "f32+f64",
                                       args.n)
    f32 = head != "fp64"
    mixes = sorted(set(STREAM_MIXES) | (set(FIELD_MIXES.values()) if f32 else set()))
    gbs = stream_ceiling(P, torch, args.n, mixes)
    if f32:   # each FP32 field kernel against the stream of its own mix
        for k, rec in kernels.items():
            if k in FIELD_MIXES:
                r, w = FIELD_MIXES[k]
                rec["ceiling_gbs"] = gbs[f"{r}r{w}w"]
                rec["of_ceiling"] = round(rec["gbs"] / gbs[f"{r}r{w}w"], 3)
    # odd and even CG iterations alternate: 8 and 11 words per cell, bytes-weighted
    mix = 19.0 / (8.0 / gbs["5r3w"] + 11.0 / gbs["7r4w"])
    roof["ceiling"] = {"kind": "streaming probe (k_stream), same read/write mixes, n^3 FP32 fields",
                       "gbs": gbs, "cg_mix_gbs": round(mix, 1),
                       "frac": round(roof["achieved"] / mix, 4)
                       if roof["kernel"] == "k_pcg_spmv" else None}
    log(f"streaming ceiling: {gbs}; CG mix {mix:.1f} GB/s")
    log(json.dumps(kernels))

    ens = None
    if not args.no_ensemble:
        ens = ensemble_run(P, torch, args, weights)
    extras = None
    if not args.no_extras:
        extras = extras_run(P, torch, case, args)

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
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"decaying HIT {args.n}^3, Mach 0.2, 1 dust class St 0.2, "
                               f"CFL 0.5, 2 PISO correctors, Jacobi-PCG rel. residual "
                               f"{args.p_tol:g}, seed {args.seed}",
                   "grid": args.n, "mode": head,
                   "guess": (f"learned, audited (trial of the rejected choice after {args.guess_audit} "
                             f"steps, the interval doubling up to {16 * args.guess_audit}; no trial "
                             f"of a guess that costs the whole zero-start solve or more)"
                             if head == "fp32_learned" else "zero")},
        "roofline": roof,
        "cpu_baseline": cpu,
        "pcg_iters_mean": H["iters"],
        "modes": {m: {"value": r["value"], "ms_per_step": r["elapsed"] * 1e3 / args.steps,
                      "ms_per_step_with_kernel_events": r["elapsed_events"] * 1e3 / args.steps,
                      "pcg_iters_mean": r["iters"], "steps_with_guess": r["guess_steps"]
                      if m == "fp32_learned" else 0} for m, r in runs.items()},
        "kernels": kernels,
        "ensemble": ens,
        "extras": extras,
    }
    if "fp64" in runs and head != "fp64":
        out["speedup_vs_fp64"] = runs[head]["value"] / runs["fp64"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
