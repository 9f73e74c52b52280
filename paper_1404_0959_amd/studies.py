"""Long runs of the step that report physics rather than throughput.

    python -m paper_1404_0959_amd.studies precision [--n 256] [--steps 200]
    python -m paper_1404_0959_amd.studies stats [--n 128] [--steps 500]
    python -m paper_1404_0959_amd.studies stokes [--n 128] [--steps 500] [--mach 0.5]
    python -m paper_1404_0959_amd.studies rivals [--steps 4]

precision: the FP32 mode (FP32 fields and inner CG, FP64 residual
refinement, reductions and mass budget) against plain FP64 on the same seeded
decaying-HIT case (Mach 0.2, one dust class at Stokes 0.2, pressure residual
1e-6).  Every `every` steps the kinetic energy, enstrophy and particle
concentration variance of both runs are compared.  Instantaneous fields of a
turbulent flow decorrelate, so the differences are set beside the spread of a
second FP64 run whose initial velocity is perturbed by 1e-7 (relative): the
FP32 error is acceptable where it stays within a small multiple of that
chaotic spread, with floors of 1e-5 (energy), 1e-4 (enstrophy) and 1e-3
(concentration variance) relative.

stats: the plain FP64 method at 128^3, Mach 0.5, three dust classes (Stokes
0.05, 0.2, 0.5), adaptive dt at CFL 0.5, statistics every 10 steps: energy,
enstrophy, density and Mach r.m.s., concentration variance per class and the
gas and dust mass budgets.

stokes: one run per Stokes number at 128^3 (default Mach 0.5): when the dust
flags first rise (negative bulk density, non-positive implicit diagonal, the
dust's Courant number past the transport update's stability bound),
the concentration variance over time and the smallest relative dust density,
which bound the Stokes range where the transport reading stays usable.

rivals: the learned guess against the Chebyshev-polynomial preconditioner on
the same captured pressure systems at 32^3, 128^3 and 256^3 (iterations and
time per solve, and the network's time per application).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import pisoc as P
from .inputs import make_hit_case

FLOORS = {"ke": 1e-5, "enstrophy": 1e-4, "conc_var": 1e-3}


def _series(solver, steps, every):
    out = [dict(step=0, t=solver.t, **solver.stats())]
    done = 0
    while done < steps:
        k = min(every, steps - done)
        st, info = solver.step(k)
        if st < 0:
            raise P.PisocError(st, solver.last_error())
        done += k
        out.append(dict(step=done, t=solver.t, iters=[i["pcg_iters"] for i in info], **solver.stats()))
    return out


def precision(n=256, steps=200, every=10, seed=0, p_tol=1e-6, inner_tol=1e-7, log=print):
    case = make_hit_case(n, seed, mach=0.2, stokes=(0.2,))
    kw = dict(p_tol=p_tol, cfl=0.5)
    runs = {}
    t0 = time.time()
    runs["fp64"] = _series(P.Solver.from_case(case, **kw), steps, every)
    log(f"fp64 done {time.time() - t0:.1f}s")
    pert = make_hit_case(n, seed, mach=0.2, stokes=(0.2,))
    rng = np.random.default_rng(seed + 1000)
    pert.u = pert.u * (1.0 + 1e-7 * rng.standard_normal(pert.u.shape))
    runs["fp64_perturbed"] = _series(P.Solver.from_case(pert, **kw), steps, every)
    log(f"perturbed done {time.time() - t0:.1f}s")
    runs["fp32"] = _series(P.Solver.from_case(case, precision=P.FP32_REFINED,
                                              inner_tol=inner_tol, **kw), steps, every)
    log(f"fp32 done {time.time() - t0:.1f}s")

    def rel(a, b):
        return abs(a - b) / abs(b) if b != 0 else abs(a - b)
    rows = []
    worst = {k: 0.0 for k in FLOORS}
    for a, b, c in zip(runs["fp32"], runs["fp64"], runs["fp64_perturbed"]):
        row = dict(step=b["step"], t=b["t"])
        for key in FLOORS:
            va = a[key][0] if key == "conc_var" else a[key]
            vb = b[key][0] if key == "conc_var" else b[key]
            vc = c[key][0] if key == "conc_var" else c[key]
            err, spread = rel(va, vb), rel(vc, vb)
            bound = max(3.0 * spread, FLOORS[key])
            row[key] = dict(fp64=vb, fp32_rel_err=err, chaotic_spread=spread, bound=bound)
            # step 0 is the shared initial state (the uniform dust's variance there
            # is rounding noise of a constant field), so it is not scored
            if b["step"] > 0:
                worst[key] = max(worst[key], err / bound)
        rows.append(row)
    mass = [abs(r["mass_gas"] - runs["fp32"][0]["mass_gas"]) / runs["fp32"][0]["mass_gas"]
            for r in runs["fp32"]]
    return dict(n=n, steps=steps, every=every, seed=seed, p_tol=p_tol, rows=rows,
                worst_err_over_bound=worst, fp32_gas_mass_drift_max=max(mass),
                t_end=runs["fp64"][-1]["t"])


def stats_run(n=128, steps=500, every=10, seed=0, p_tol=1e-8, mach=0.5,
              stokes=(0.05, 0.2, 0.5), log=print):
    case = make_hit_case(n, seed, mach=mach, stokes=stokes)
    s = P.Solver.from_case(case, p_tol=p_tol, cfl=0.5)
    t0 = time.time()
    series = _series(s, steps, every)
    log(f"{steps} steps in {time.time() - t0:.1f}s")
    m0 = series[0]["mass_gas"]
    mp0 = series[0]["mass_p"]
    drift = max(abs(r["mass_gas"] - m0) / m0 for r in series)
    pdrift = max(abs(r["mass_p"][c] - mp0[c]) / mp0[c] for r in series for c in range(len(mp0)))
    return dict(n=n, steps=steps, every=every, mach=mach, stokes=list(stokes), p_tol=p_tol,
                series=[{k: v for k, v in r.items() if k != "iters"} for r in series],
                mean_pcg_iters=float(np.mean([np.mean(i) for r in series[1:] for i in r["iters"]])),
                gas_mass_drift_max=drift, dust_mass_drift_max=pdrift)


def stokes_range(n=128, steps=500, every=10, seed=0, p_tol=1e-8, mach=0.5,
                 stokes=(0.025, 0.05, 0.1, 0.2, 0.3, 0.5), log=print):
    """One run per Stokes number (one dust class each): the first steps at which
    the dust flags are raised (a negative bulk density; a non-positive diagonal
    of the implicit transport equation), the concentration variance every
    `every` steps and the smallest relative bulk density at the end."""
    out = []
    for st_num in stokes:
        case = make_hit_case(n, seed, mach=mach, stokes=(st_num,))
        s = P.Solver.from_case(case, p_tol=p_tol, cfl=0.5)
        first_neg = first_diag = first_courant = None
        cmax = 0.0
        var = [s.stats()["conc_var"][0]]
        done, status = 0, 0
        t0 = time.time()
        while done < steps:
            k = min(every, steps - done)
            st, info = s.step(k, raise_on_error=False)
            for j, i in enumerate(info):
                if first_neg is None and i["flags"] & P.FLAG_DUST_NEG:
                    first_neg = done + j + 1
                if first_diag is None and i["flags"] & P.FLAG_DUST_DIAG:
                    first_diag = done + j + 1
                if first_courant is None and i["flags"] & P.FLAG_DUST_COURANT:
                    first_courant = done + j + 1
                cmax = max(cmax, i["courant_dust"])
            if st < 0:
                status = st
                break
            done += k
            var.append(s.stats()["conc_var"][0])
        rp = s.get(P.FIELD_RHO_P).cpu().numpy()[0]
        row = dict(stokes=st_num, tau_p=case.tau_p[0], steps=done, status=status,
                   first_negative_step=first_neg, first_diagonal_step=first_diag,
                   first_dust_courant_step=first_courant, dust_courant_max=cmax,
                   conc_var_every=var, conc_var_max=float(np.max(var)),
                   min_rel_density=float(rp.min() / rp.mean()))
        log(f"St {st_num}: {done} steps in {time.time() - t0:.1f}s, first negative "
            f"{first_neg}, first diagonal {first_diag}, first dust Courant >= 0.638 "
            f"{first_courant} (max {cmax:.3f}), variance max {row['conc_var_max']:.3g}, "
            f"min rho_j/<rho_j> {row['min_rel_density']:.3g}")
        out.append(row)
        s.close()
    return dict(n=n, steps=steps, every=every, mach=mach, seed=seed, runs=out)


def rivals(sizes=(32, 128, 256), steps=4, seed=20, p_tol=1e-6, reps=3, log=print):
    """The learned guess against a non-learned rival on the same systems: the
    first corrector's pressure system of step `steps` of a run with the
    learned guess (FP64, Mach 0.2, Stokes 0.2) is solved again stand-alone to
    the same residual with Jacobi-PCG and with the Chebyshev-polynomial
    preconditioner, each from zero and from the learned guess's start x0:
    iterations and wall time per solve (best of reps), beside the time of one
    network application on a grid of that size."""
    import math

    import torch

    from .learn import load_weights
    wts = load_weights()
    out = []
    for n in sizes:
        case = make_hit_case(n, seed, mach=0.2, stokes=(0.2,))
        s = P.Solver.from_case(case, p_tol=p_tol, capture=True, guess=P.GUESS_LEARNED,
                               guess_weights=wts.data_ptr())
        st, info = s.step(steps)
        f = s.fields(P.FIELD_PSOLVE_B | P.FIELD_PSOLVE_PSIDT | P.FIELD_PSOLVE_W |
                     P.FIELD_GUESS_X0)
        s.close()
        b, psidt, w = f[P.FIELD_PSOLVE_B], f[P.FIELD_PSOLVE_PSIDT], f[P.FIELD_PSOLVE_W]
        x0 = f[P.FIELD_GUESS_X0]
        row = dict(n=n, step=steps, fallback=bool(float(x0.abs().max()) == 0.0),
                   in_step_iters=info[-1]["pcg_iters"][0])
        for name, pc in (("jacobi", P.PRECOND_JACOBI), ("cheb", P.PRECOND_CHEB)):
            for start, xs in (("zero", None), ("learned", x0)):
                best, it = math.inf, None
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, it, rel, stt = P.helm_solve(psidt, w, b, x0=xs, tol=p_tol, maxit=1000,
                                                   precond=pc)
                    torch.cuda.synchronize()
                    best = min(best, time.perf_counter() - t0)
                row[f"{name}_{start}"] = dict(iters=it, ms=round(best * 1e3, 3))
        net = P.Net(n, 1)
        xin = torch.zeros(1, n ** 3, 2, dtype=torch.float32, device="cuda")
        best = math.inf
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            net.forward(wts, xin)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        row["network_ms"] = round(best * 1e3, 3)
        log(json.dumps(row))
        out.append(row)
    return dict(seed=seed, p_tol=p_tol, runs=out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["precision", "stats", "stokes", "rivals"])
    ap.add_argument("--mach", type=float, default=0.5)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()

    def log(m):
        print(m, file=sys.stderr, flush=True)
    if args.what == "precision":
        r = precision(n=args.n or 256, steps=args.steps or 200, every=args.every, log=log)
    elif args.what == "rivals":
        r = rivals(steps=args.steps or 4, log=log)
    elif args.what == "stokes":
        r = stokes_range(n=args.n or 128, steps=args.steps or 500, every=args.every,
                         mach=args.mach, log=log)
    else:
        r = stats_run(n=args.n or 128, steps=args.steps or 500, every=args.every, log=log)
    text = json.dumps(r)
    print(text)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main()
