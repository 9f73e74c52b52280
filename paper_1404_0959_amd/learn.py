"""Training and evaluation of the learned pressure-guess network.

Data: the solver itself, run on seeded decaying-HIT cases (the 32^3, Mach
0.2, Stokes 0.1, tolerance 1e-8 configuration), captures the pressure system
of its first corrector after every step; the library turns each capture into
the network's normalised inputs and target p'/s1.  Training: mini-batch Adam
on the mean squared error, or on the relative residual the solve would start
from (the measure its stopping rule applies), with the project's own forward,
backward and Adam kernels.  This module only orchestrates those calls (and holds the data
tensors); every arithmetic step runs in the HIP library.
"""
from __future__ import annotations

import math
import os
import time

import numpy as np

from . import pisoc as P
from .inputs import make_hit_case


# trained on the relative residual the solve starts from (20 epochs from He
# initialisation); guess_hit32.npy holds the earlier network trained on the
# mean squared error against the solution (30 epochs), kept for comparison
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                            "guess_hit32_residual.npy")


def load_weights(path: str = WEIGHTS_PATH, device="cuda:0"):
    """The trained FP32 weights as a device tensor (numpy load, no pickle)."""
    import torch
    w = np.load(path, allow_pickle=False).astype(np.float32)
    assert w.shape == (P.NET_NWEIGHTS,), w.shape
    return torch.as_tensor(w, device=device).contiguous()


def init_weights(seed: int = 0):
    """He-normal initial weights, FP32 numpy vector of PISOC_NET_NWEIGHTS."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(4):
        cin, cout = P.NET_CH[l], P.NET_CH[l + 1]
        std = math.sqrt(2.0 / (27 * cin)) if l < 3 else math.sqrt(1.0 / (27 * cin))
        parts.append(rng.standard_normal(cout * cin * 27) * std)
    return np.concatenate(parts).astype(np.float32)


def generate(seeds, steps, n=32, mach=0.2, stokes=(0.1,), p_tol=1e-8, device="cuda:0", log=None,
             systems=False):
    """Snapshots (x [S, n^3, 2], t [S, n^3]) from the solver's first corrector;
    with systems, also the systems (b, diag, w) as FP64 [S, n^3] each."""
    import torch
    xs, ts, sy = [], [], []
    bits = P.FIELD_PSOLVE_B | P.FIELD_PSOLVE_DIAG | P.FIELD_P_PREV | P.FIELD_PSOLVE_X
    if systems:
        bits |= P.FIELD_PSOLVE_W
    for seed in seeds:
        case = make_hit_case(n, seed, mach=mach, stokes=stokes)
        s = P.Solver.from_case(case, p_tol=p_tol, capture=True, device=device)
        for _ in range(steps):
            st, _ = s.step(1)
            if st < 0:
                break
            f = s.fields(bits)
            x, t, _ = P.net_inputs(f[P.FIELD_PSOLVE_B], f[P.FIELD_PSOLVE_DIAG],
                                   f[P.FIELD_P_PREV], f[P.FIELD_PSOLVE_X])
            xs.append(x)
            ts.append(t)
            if systems:
                sy.append(tuple(f[k].reshape(-1).clone() for k in
                                (P.FIELD_PSOLVE_B, P.FIELD_PSOLVE_DIAG, P.FIELD_PSOLVE_W)))
        s.close()
        if log:
            log(f"seed {seed}: {len(xs)} snapshots")
    if systems:
        return torch.stack(xs), torch.stack(ts), tuple(torch.stack(c) for c in zip(*sy))
    return torch.stack(xs), torch.stack(ts)


def train(x, t, epochs=20, batch=16, lr=2e-3, seed=0, w0=None, log=None, systems=None):
    """Adam on the MSE against t, or with systems on the relative residual
    |b - alpha M g|^2 / |b|^2 the solve would start from; returns (weights
    FP32 device tensor, loss history).

    x, t: one dataset (tensors [S, n^3, 2], [S, n^3]) or a list of datasets of
    different grid sizes; systems: None or, per dataset, the (b, diag, w) FP64
    tensors [S, n^3] of generate(systems=True).  Mini-batches never mix sizes
    and each epoch visits every batch of every size once, in a seeded random
    order."""
    import torch
    sets = list(zip(x, t)) if isinstance(x, (list, tuple)) else [(x, t)]
    if systems is not None and not isinstance(x, (list, tuple)):
        systems = [systems]
    dev = sets[0][0].device
    w = torch.as_tensor(init_weights(seed) if w0 is None else w0, device=dev).float().contiguous()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    g = torch.empty_like(w)
    nets = []
    for xs, _ in sets:
        n = round(xs.shape[1] ** (1 / 3))
        nets.append(P.Net(n, min(batch, xs.shape[0]), device=dev))
    rng = np.random.default_rng(seed + 1)
    hist = []
    step = 0
    for ep in range(epochs):
        jobs = []
        for si, (xs, _) in enumerate(sets):
            bsz = min(batch, xs.shape[0])
            perm = rng.permutation(xs.shape[0])
            jobs += [(si, perm[i:i + bsz]) for i in range(0, xs.shape[0] - bsz + 1, bsz)]
        order = rng.permutation(len(jobs))
        losses = []
        for o in order:
            si, idx = jobs[o]
            xs, ts = sets[si]
            ix = torch.as_tensor(idx, device=dev)
            xb = xs.index_select(0, ix).contiguous()
            if systems is None:
                tb = ts.index_select(0, ix).contiguous()
                loss, _ = nets[si].grad(w, xb, tb, out=g)
            else:
                b, d, wk = (c.index_select(0, ix).contiguous() for c in systems[si])
                loss, _ = nets[si].grad_residual(w, xb, b, d, wk, out=g)
            step += 1
            nets[si].adam(w, g, m, v, step, lr=lr)
            losses.append(loss)
        hist.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    return w, hist


def evaluate(w, n, seeds, steps, mach=0.2, stokes=(0.2,), p_tol=1e-6, precision=P.FP64,
             device="cuda:0"):
    """CG iterations and wall time with and without the learned guess."""
    import torch
    out = {}
    for name, kw in (("zero", {}), ("learned", dict(guess=P.GUESS_LEARNED,
                                                   guess_weights=w.data_ptr()))):
        its, fb, el = [], 0, 0.0
        for seed in seeds:
            case = make_hit_case(n, seed, mach=mach, stokes=stokes)
            s = P.Solver.from_case(case, p_tol=p_tol, precision=precision, device=device, **kw)
            s.step(1)                   # warm-up step (first-step prediction)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, info = s.step(steps)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            for i in info:
                its.append(sum(i["pcg_iters"]))
                fb += 1 if i["flags"] & P.FLAG_GUESS_FALLBACK else 0
                assert max(i["pcg_relres"]) <= p_tol
            s.close()
        out[name] = dict(iters_per_step=float(np.mean(its)), fallbacks=fb,
                         ms_per_step=1e3 * el / (len(seeds) * steps))
    return out
