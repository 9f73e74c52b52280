"""The batched ensemble (members of mixed grid sizes stepped together) through
the C ABI.

Bars: in eager mode every member's fields are bitwise identical to the same
case run alone (members of one size class share each launch, but every
reduction runs over the member's own blocks in the same order); a member agrees
with the FP64 oracle to the whole-step parity bar; the captured-graph mode
reproduces eager mode (FP64: identical solves while the iteration caps hold;
FP32 + learned guess: within the pressure tolerance, each solve at
||r|| <= p_tol ||b||, the gas and dust mass conserved to round-off, an audited
guess applied per its captured verdict); the autotuner's cache round-trips.
"""
import json

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import ensemble_cases, make_hit_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1404_0959_amd.pisoc as P
    P.lib()
    return P


def cases():
    # interleaved sizes: member -> class mapping is not the identity
    return [make_hit_case(32, 11, mach=0.2, stokes=(0.1,)),
            make_hit_case(48, 12, mach=0.5, stokes=(0.3,)),
            make_hit_case(32, 13, mach=0.5, stokes=(0.05,))]


BITS = None


def fields(P, get):
    bits = P.FIELD_RHO | P.FIELD_U | P.FIELD_PHI | P.FIELD_RHO_P | P.FIELD_P
    return {k: v.cpu().numpy() for k, v in get(bits).items()}


def test_eager_members_equal_single_runs(P):
    cs = cases()
    kw = dict(p_tol=1e-9, cfl=0.5)
    ens = P.Ensemble(cs, **kw)
    singles = [P.Solver.from_case(c, **kw) for c in cs]
    assert [c["n"] for c in ens.classes()] == [32, 48]
    assert [c["members"] for c in ens.classes()] == [2, 1]
    for step in range(3):
        st, infos = ens.step(1, mode=P.ENS_EAGER)
        assert st in (P.OK, P.WARN_DUST)
        for m, s in enumerate(singles):
            st1, (i1,) = s.step(1)
            assert st1 in (P.OK, P.WARN_DUST)
            assert infos[m]["flags"] == i1["flags"], (step, m)
            assert infos[m]["pcg_iters"] == i1["pcg_iters"], (step, m)
            assert infos[m]["dt"] == i1["dt"] and infos[m]["t"] == i1["t"]
            assert infos[m]["mass_gas"] == i1["mass_gas"]
    for m, s in enumerate(singles):
        a = fields(P, lambda b: ens.fields(m, b))
        b = fields(P, lambda b: s.fields(b))
        for k in a:
            assert np.array_equal(a[k], b[k]), (m, k)
    st = ens.stats()
    for m, s in enumerate(singles):
        assert st[m] == s.stats()
    t = ens.times()
    assert t == [s.t for s in singles]


def test_member_matches_oracle(P, ora):
    from test_gpu_parity import compare_state
    cs = cases()
    kw = dict(p_tol=1e-8)
    ens = P.Ensemble(cs, **kw)
    o = ora.Oracle.from_case(cs[1], **kw)
    st, infos = ens.step(2, mode=P.ENS_EAGER)
    st_o, info_o = o.step(2)
    assert st == st_o and st in (P.OK, P.WARN_DUST)
    assert infos[1]["pcg_iters"] == info_o[-1]["pcg_iters"]

    class View:
        def fields(self, bits):
            return ens.fields(1, bits)
    compare_state(P, ora, View(), o)


def test_graph_reproduces_eager_fp64(P):
    cs = cases()
    kw = dict(p_tol=1e-9)
    a = P.Ensemble(cs, **kw)
    b = P.Ensemble(cs, **kw)
    for _ in range(4):
        sa, ia = a.step(1, mode=P.ENS_EAGER)
    sb, ib = b.step(4, mode=P.ENS_GRAPH)
    assert sa == sb and sa in (P.OK, P.WARN_DUST)
    assert b.steps_done == 4
    for cl in b.classes():
        assert all(cap > 0 for cap in cl["caps"][:2])
    for m in range(len(cs)):
        assert ia[m]["pcg_iters"] == ib[m]["pcg_iters"], m
        assert ia[m]["t"] == ib[m]["t"]
        fa = fields(P, lambda bits: a.fields(m, bits))
        fb = fields(P, lambda bits: b.fields(m, bits))
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), (m, k)
    # further captured steps replay the two parity graphs
    sb, ib = b.step(3, mode=P.ENS_GRAPH)
    sa, ia = a.step(3, mode=P.ENS_EAGER)
    for m in range(len(cs)):
        assert ia[m]["t"] == ib[m]["t"]
        fa = fields(P, lambda bits: a.fields(m, bits))
        fb = fields(P, lambda bits: b.fields(m, bits))
        assert np.array_equal(fa[P.FIELD_U], fb[P.FIELD_U]), m


def test_graph_fp32_learned(P):
    from paper_1404_0959_amd.learn import load_weights
    w = load_weights()
    cs = ensemble_cases(8, seed=3)
    assert sorted({c.n for c in cs}) == [32, 48, 64]
    kw = dict(p_tol=1e-6, precision=P.FP32_REFINED, inner_tol=1e-3, guess=P.GUESS_LEARNED,
              guess_weights=w.data_ptr())
    a = P.Ensemble(cs, **kw)
    b = P.Ensemble(cs, **kw)
    m0 = [s["mass_gas"] for s in b.stats()]
    p0 = [s["mass_p"][0] for s in b.stats()]
    sa, ia = a.step(6, mode=P.ENS_EAGER)
    sb, ib = b.step(6, mode=P.ENS_GRAPH)
    print("classes", b.classes())
    for m in range(len(cs)):
        print(m, cs[m].n, "eager", ia[m]["pcg_iters"], ia[m]["refinements"], "graph",
              ib[m]["pcg_iters"], ib[m]["refinements"], ib[m]["pcg_relres"], ib[m]["flags"])
    assert sa in (P.OK, P.WARN_GUESS_FALLBACK, P.WARN_DUST) and sb in (P.OK, P.WARN_GUESS_FALLBACK, P.WARN_DUST)
    sb_stats = b.stats()
    for m in range(len(cs)):
        assert max(ib[m]["pcg_relres"]) <= 1e-6, ib[m]
        assert not ib[m]["flags"] & P.FLAG_PCG_MAXIT
        assert abs(sb_stats[m]["mass_gas"] - m0[m]) <= 1e-10 * m0[m]
        assert abs(sb_stats[m]["mass_p"][0] - p0[m]) <= 1e-7 * p0[m]
        ua = a.get(m, P.FIELD_U).cpu().numpy()
        ub = b.get(m, P.FIELD_U).cpu().numpy()
        assert np.max(np.abs(ua - ub)) <= 1e-4 * np.max(np.abs(ua)), m


def test_graph_keeps_audit_verdict(P):
    """Audited learned guess in captured mode: the first captured call is too
    short to capture (the audit has measured only the guess), the second
    measures the zero guess and captures; the captured steps then apply each
    class's verdict (PISOC_FLAG_GUESS_SKIPPED exactly where a corrector goes
    without the guess), meet the tolerance, conserve mass and stay within the
    solver tolerance of the audited eager run."""
    from paper_1404_0959_amd.learn import load_weights
    w = load_weights()
    cs = cases()
    kw = dict(p_tol=1e-6, precision=P.FP32_REFINED, inner_tol=1e-3, guess=P.GUESS_LEARNED,
              guess_weights=w.data_ptr(), guess_audit=8)
    a = P.Ensemble(cs, **kw)
    b = P.Ensemble(cs, **kw)
    m0 = [s["mass_gas"] for s in b.stats()]
    sb, ib = b.step(1, mode=P.ENS_GRAPH)
    assert b.steps_done == 1
    assert all(not i["flags"] & P.FLAG_GUESS_SKIPPED for i in ib)
    sb, ib = b.step(1, mode=P.ENS_GRAPH)
    assert b.steps_done == 2
    assert all(i["flags"] & P.FLAG_GUESS_SKIPPED for i in ib)
    sb, ib = b.step(3, mode=P.ENS_GRAPH)
    assert b.steps_done == 5
    sa, ia = a.step(5, mode=P.ENS_EAGER)
    assert sa in (P.OK, P.WARN_GUESS_FALLBACK, P.WARN_DUST) and sb in (P.OK, P.WARN_GUESS_FALLBACK, P.WARN_DUST)
    full = (1 << b.prms[0].n_corr) - 1
    mask = {}
    for cl in b.classes():
        assert 0 <= cl["guess_mask"] <= full
        mask[cl["n"]] = cl["guess_mask"]
    print("verdicts", mask)
    st = b.stats()
    for m, c in enumerate(cs):
        assert bool(ib[m]["flags"] & P.FLAG_GUESS_SKIPPED) == (mask[c.n] != full), (m, ib[m])
        assert max(ib[m]["pcg_relres"]) <= 1e-6, ib[m]
        assert not ib[m]["flags"] & P.FLAG_PCG_MAXIT
        assert abs(st[m]["mass_gas"] - m0[m]) <= 1e-10 * m0[m]
        ua = a.get(m, P.FIELD_U).cpu().numpy()
        ub = b.get(m, P.FIELD_U).cpu().numpy()
        assert np.max(np.abs(ua - ub)) <= 1e-4 * np.max(np.abs(ua)), m


def test_bench_ensemble_configuration(P, tmp_path):
    """The ensemble the benchmark times, at its full size: 64 members (32 x
    32^3, 16 x 48^3, 16 x 64^3), FP32 + learned guess under the audit,
    autotuned, captured steps.  Every solve meets the tolerance, gas and dust
    mass are conserved, and the first member of each size class agrees with
    the same case stepped alone to 1e-5 of max |u| (in practice bitwise: a
    member's reductions do not depend on the other members).  Regression: a
    member converged in an eager step's first FP32 round, in a class where
    another member needed a second round, once took a stale solution copy."""
    from paper_1404_0959_amd.learn import load_weights
    w = load_weights()
    cs = ensemble_cases(64, seed=0)
    assert [sum(1 for c in cs if c.n == n) for n in (32, 48, 64)] == [32, 16, 16]
    kw = dict(p_tol=1e-6, cfl=0.5, n_corr=2, n_mom_sweeps=4, n_dust_sweeps=4,
              precision=P.FP32_REFINED, inner_tol=1e-6, guess=P.GUESS_LEARNED,
              guess_weights=w.data_ptr(), guess_audit=16)
    E = P.Ensemble(cs, **kw)
    m0 = [s["mass_gas"] for s in E.stats()]
    p0 = [s["mass_p"][0] for s in E.stats()]
    st, info = E.step(1, mode=P.ENS_EAGER)
    assert st in (P.OK, P.WARN_GUESS_FALLBACK, P.WARN_DUST)
    E.autotune(str(tmp_path / "tune.json"), force=True)
    for c in E.classes():
        assert c["cg_cells_z"] > 0      # every class runs the tiled CG kernel
    st, info = E.step(6, mode=P.ENS_GRAPH)
    assert st in (P.OK, P.WARN_GUESS_FALLBACK, P.WARN_DUST), st
    assert E.steps_done == 7
    stats = E.stats()
    for m in range(len(cs)):
        assert max(info[m]["pcg_relres"]) <= 1e-6, (m, info[m])
        assert not info[m]["flags"] & P.FLAG_PCG_MAXIT
        assert abs(stats[m]["mass_gas"] - m0[m]) <= 1e-10 * m0[m]
        assert abs(stats[m]["mass_p"][0] - p0[m]) <= 1e-7 * p0[m]
    firsts = [min(m for m, c in enumerate(cs) if c.n == n) for n in (32, 48, 64)]
    for m in firsts:
        s = P.Solver.from_case(cs[m], **kw)
        st1, _ = s.step(7)
        assert st1 in (P.OK, P.WARN_GUESS_FALLBACK, P.WARN_DUST)
        assert abs(s.t - E.times()[m]) <= 1e-4 * s.t
        ua = s.get(P.FIELD_U).cpu().numpy()
        ub = E.get(m, P.FIELD_U).cpu().numpy()
        assert np.max(np.abs(ua - ub)) <= 1e-5 * np.max(np.abs(ua)), m
        s.close()
    E.close()


def test_graph_caps_follow_iterations(P):
    """Captured FP32 steps over a decaying flow: the CG iterations grow from
    step to step, and the graphs are captured again before a solve reaches
    the caps they hold, so no call in 120 steps reports a solve stopped at a
    cap (PISOC_FLAG_PCG_MAXIT) and every solve meets the tolerance."""
    cs = [make_hit_case(32, 31, mach=0.2, stokes=(0.2,)),
          make_hit_case(32, 32, mach=0.5, stokes=(0.4,)),
          make_hit_case(48, 33, mach=0.2, stokes=(0.1,))]
    kw = dict(p_tol=1e-6, precision=P.FP32_REFINED, inner_tol=1e-6)
    E = P.Ensemble(cs, **kw)
    first_caps = None
    for call in range(12):
        st, info = E.step(10, mode=P.ENS_GRAPH)
        assert st in (P.OK, P.WARN_DUST), (call, st, [i["flags"] for i in info])
        for m, i in enumerate(info):
            assert max(i["pcg_relres"]) <= 1e-6, (call, m, i)
            assert not i["flags"] & P.FLAG_PCG_MAXIT, (call, m, i)
        caps = [c["caps"][:2] for c in E.classes()]
        first_caps = first_caps or caps
    assert E.steps_done == 120
    print("caps", first_caps, "->", caps)
    E.close()


def test_autotune_cache_round_trip(P, tmp_path):
    cs = cases()
    kw = dict(p_tol=1e-8)
    path = str(tmp_path / "tune.json")
    e = P.Ensemble(cs, **kw)
    with pytest.raises(P.PisocError):
        e.autotune(path)            # needs one completed step
    e.step(1, mode=P.ENS_EAGER)
    e.autotune(path)
    cache = json.load(open(path))
    cl = e.classes()
    assert len(cache) == 2
    for c in cl:
        key = [k for k in cache if k.startswith(f"n{c['n']}_b{c['members']}_fp64")]
        assert len(key) == 1
        assert cache[key[0]] == [c["block"][0], c["cells_z"], c["cg_cells_z"], c["tiled_cells_z"]]
    # tuned shapes still give converged, mass-conserving steps (graph mode)
    m0 = [s["mass_gas"] for s in e.stats()]
    st, info = e.step(3, mode=P.ENS_GRAPH)
    assert st in (P.OK, P.WARN_DUST)
    for m, i in enumerate(info):
        assert max(i["pcg_relres"]) <= 1e-8
        assert abs(i["mass_gas"] - m0[m]) <= 1e-12 * m0[m]
    # a second ensemble takes the cached shapes without timing
    e2 = P.Ensemble(cs, **kw)
    e2.step(1, mode=P.ENS_EAGER)
    e2.autotune(path)
    key_of = lambda c: (c["block"], c["cells_z"], c["cg_cells_z"], c["tiled_cells_z"])
    assert [key_of(c) for c in e2.classes()] == [key_of(c) for c in cl]
    assert json.load(open(path)) == cache


def test_graph_eager_graph_interleaved_fp64(P):
    """Captured and eager calls mixed on one ensemble (GRAPH 3, EAGER 1, GRAPH 2):
    the graphs, captured for a buffer rotation, stay in step with the eager
    step's rotation, so the six steps are bitwise the six steps of an ensemble
    run eagerly throughout."""
    cs = cases()
    kw = dict(p_tol=1e-9)
    a = P.Ensemble(cs, **kw)
    b = P.Ensemble(cs, **kw)
    for _ in range(6):
        sa, ia = a.step(1, mode=P.ENS_EAGER)
    for nst, mode in ((3, P.ENS_GRAPH), (1, P.ENS_EAGER), (2, P.ENS_GRAPH)):
        sb, ib = b.step(nst, mode=mode)
        assert sb in (P.OK, P.WARN_DUST)
    assert b.steps_done == 6
    for m in range(len(cs)):
        assert ia[m]["pcg_iters"] == ib[m]["pcg_iters"], m
        assert ia[m]["t"] == ib[m]["t"]
        fa = fields(P, lambda bits: a.fields(m, bits))
        fb = fields(P, lambda bits: b.fields(m, bits))
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), (m, k)


def test_graph_member_matches_oracle(P, ora):
    """A member stepped by captured graphs against the FP64 oracle directly (the
    graph's solves run to a fixed iteration cap, each member stopping at its
    own convergence, so the iterates are the oracle's)."""
    from test_gpu_parity import compare_state
    cs = cases()
    kw = dict(p_tol=1e-8)
    ens = P.Ensemble(cs, **kw)
    o = ora.Oracle.from_case(cs[2], **kw)
    st, infos = ens.step(4, mode=P.ENS_GRAPH)
    st_o, info_o = o.step(4)
    assert st in (P.OK, P.WARN_DUST) and st_o in (P.OK, P.WARN_DUST)
    assert infos[2]["pcg_iters"] == info_o[-1]["pcg_iters"]

    class View:
        def fields(self, bits):
            return ens.fields(2, bits)
    compare_state(P, ora, View(), o, label="graph member")


def test_captured_solve_at_cap_reports_its_residual(P, ora):
    """One long captured call on a decaying flow: the CG iterations a solve
    needs outgrow the caps the graph was built with (+25 % + 2 of the first
    step's), so the last steps stop their solves at the cap.  The launch at the
    cap brings x up to date, so the relative residual the step reports is that
    of the solution it applies: ||b - M x|| / ||b|| from the captured system,
    with M rebuilt from the captured w and diagonal."""
    import math
    case = make_hit_case(32, 41, mach=0.2, stokes=(0.1,))
    ens = P.Ensemble([case], p_tol=1e-10, capture=True)
    st, info = ens.step(1, mode=P.ENS_GRAPH)
    st, info = ens.step(150, mode=P.ENS_GRAPH)
    assert st >= 0
    hit = bool(info[0]["flags"] & P.FLAG_PCG_MAXIT)
    f = ens.fields(0, P.FIELD_PSOLVE_B | P.FIELD_PSOLVE_X | P.FIELD_PSOLVE_DIAG | P.FIELD_PSOLVE_W)
    b, x, diag, w = (f[k].cpu().numpy() for k in (P.FIELD_PSOLVE_B, P.FIELD_PSOLVE_X,
                                                   P.FIELD_PSOLVE_DIAG, P.FIELD_PSOLVE_W))
    n = case.n
    h = 2 * math.pi / n
    K = ora.kfaces(w)
    ksum = sum(K[d] + np.roll(K[d], 1, axis=2 - d) for d in range(3))
    psidt = diag - ksum / h ** 2
    r = b - ora.helm_apply(psidt, K, x)
    true_rel = np.linalg.norm(r) / np.linalg.norm(b)
    reported = info[0]["pcg_relres"][0]
    print(f"cap reached {hit}: corrector-1 relres reported {reported:.3e}, of x {true_rel:.3e}, "
          f"caps {[c['caps'][:2] for c in ens.classes()]}")
    assert hit, "the caps were not reached: the test does not exercise the cap"
    assert abs(true_rel / reported - 1) < 1e-2


def test_one_graph_per_step_fp64(P):
    """PISOC_ENS_GRAPH_ONE: the whole ensemble's step is one graph launch (each
    size class a branch); FP64 steps are bitwise those of the per-class graphs
    and of eager steps, and the captured modes may alternate on one ensemble."""
    cs = cases()
    kw = dict(p_tol=1e-9)
    a = P.Ensemble(cs, **kw)
    b = P.Ensemble(cs, **kw)
    c = P.Ensemble(cs, **kw)
    for _ in range(6):
        sa, ia = a.step(1, mode=P.ENS_EAGER)
    sb, ib = b.step(6, mode=P.ENS_GRAPH_ONE)
    for nst, mode in ((2, P.ENS_GRAPH_ONE), (2, P.ENS_GRAPH), (1, P.ENS_EAGER),
                      (1, P.ENS_GRAPH_ONE)):
        sc, ic = c.step(nst, mode=mode)
        assert sc in (P.OK, P.WARN_DUST)
    assert sa == sb and sa in (P.OK, P.WARN_DUST)
    assert b.steps_done == c.steps_done == 6
    for m in range(len(cs)):
        assert ia[m]["pcg_iters"] == ib[m]["pcg_iters"] == ic[m]["pcg_iters"], m
        fa = fields(P, lambda bits: a.fields(m, bits))
        fb = fields(P, lambda bits: b.fields(m, bits))
        fc = fields(P, lambda bits: c.fields(m, bits))
        for k in fa:
            assert np.array_equal(fa[k], fb[k]) and np.array_equal(fa[k], fc[k]), (m, k)


def test_one_graph_benchmark_ensemble(P):
    """The benchmark's 64 mixed members (FP32 + learned guess, audited) in
    one-graph mode: every solve meets the tolerance, gas mass is conserved."""
    from paper_1404_0959_amd.learn import load_weights
    w = load_weights()
    cs = ensemble_cases(64, seed=0)
    E = P.Ensemble(cs, p_tol=1e-6, precision=P.FP32_REFINED, inner_tol=1e-6,
                   guess=P.GUESS_LEARNED, guess_weights=w.data_ptr(), guess_audit=16)
    m0 = [s["mass_gas"] for s in E.stats()]
    E.step(1, mode=P.ENS_EAGER)
    E.autotune()
    st, info = E.step(10, mode=P.ENS_GRAPH_ONE)
    assert st in (P.OK, P.WARN_DUST, P.WARN_GUESS_FALLBACK)
    eps32 = float(np.finfo(np.float32).eps)
    for m, i in enumerate(info):
        assert max(i["pcg_relres"]) <= 1e-6, (m, i)
        # FP64 sums of FP32-stored densities: a random walk of FP32 roundings
        assert abs(i["mass_gas"] / m0[m] - 1) <= 8 * eps32 * np.sqrt(11 / cs[m].n ** 3)
