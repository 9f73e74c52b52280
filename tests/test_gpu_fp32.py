"""The FP32 mode (FP32 fields, stencils, transport and inner CG; FP64
continuity defect, residual refinement, reductions and mass budget) against
the FP64 oracle and the FP64 GPU path.

Tolerances: a field after a few steps carries the FP32 rounding of every
stage (unit round-off 6e-8, amplified by the step's stencils and the
solve): the bound is 5e-5 of the field's spread plus 16 FP32 unit round-offs
of its magnitude (a field that varies by 1e-7 of its size, like the dust
after one step, cannot be represented more closely in FP32).  The pressure solve itself must reach the requested FP64
relative residual.  Statistics follow the calibration rule: the difference to
the FP64 run must not exceed max(3 delta(t), floor), delta(t) the spread of
two FP64 runs whose initial velocity differs by 1e-7 relative.
"""
import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case

pytestmark = pytest.mark.gpu

FIELD_TOL = 5e-5


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1404_0959_amd.pisoc as P
    P.lib()
    return P


EPS32 = 2.0 ** -24


def dev_err(g, o):
    """Error relative to the bound FIELD_TOL * spread + 16 eps32 * magnitude,
    scaled so that 1.0 is the bound."""
    spread = np.max(np.abs(o - o.mean()))
    bound = FIELD_TOL * spread + 16 * EPS32 * np.max(np.abs(o))
    return float(np.max(np.abs(g - o)) / bound)


def check_fields(P, ora, s, o, tol):
    f = s.fields(P.FIELD_RHO | P.FIELD_U | P.FIELD_RHO_P | P.FIELD_PHI)
    errs = dict(rho=dev_err(f[P.FIELD_RHO].cpu().numpy(), o.get(ora.RHO)),
                u=dev_err(f[P.FIELD_U].cpu().numpy(), o.get(ora.U)),
                phi=dev_err(f[P.FIELD_PHI].cpu().numpy(), o.get(ora.PHI)),
                rho_p=dev_err(f[P.FIELD_RHO_P].cpu().numpy()[0], o.get(ora.RHO_P)[0]))
    assert all(v <= 1.0 for v in errs.values()), errs
    return errs


@pytest.mark.parametrize("n,steps", [(32, 1), (32, 20), (40, 3), (128, 1)])
def test_fp32_vs_oracle(P, ora, n, steps):
    case = make_hit_case(n, 0, mach=0.2, stokes=(0.1,))
    tol = 1e-6
    o = ora.Oracle.from_case(case, p_tol=tol)
    s = P.Solver.from_case(case, p_tol=tol, precision=P.FP32_REFINED, inner_tol=1e-7)
    o.step(steps)
    st, info = s.step(steps)
    assert st in (P.OK, P.WARN_DUST)
    for i in info:
        assert all(r <= tol for r in i["pcg_relres"]), i
        assert all(k >= 1 for k in i["refinements"]), i
    check_fields(P, ora, s, o, FIELD_TOL)


def test_fp32_bench_workload_vs_oracle(P, ora):
    """One step of the 256^3 benchmark workload in the benchmark's FP32 settings
    (inner tolerance 1e-6): the full-row CG kernel in FP32."""
    case = make_hit_case(256, 0, mach=0.2, stokes=(0.2,))
    tol = 1e-6
    o = ora.Oracle.from_case(case, p_tol=tol)
    s = P.Solver.from_case(case, p_tol=tol, precision=P.FP32_REFINED, inner_tol=1e-6)
    o.step(1)
    st, info = s.step(1)
    assert st in (P.OK, P.WARN_DUST)
    for i in info:
        assert all(r <= tol for r in i["pcg_relres"]), i
    check_fields(P, ora, s, o, FIELD_TOL)


def test_fp32_mass_budget(P):
    """FP64 reductions of FP32 fields: the face fluxes telescope, so total gas
    and dust mass only drift by the FP32 rounding of the per-cell updates, an
    unbiased random walk of relative size eps32 sqrt(steps / cells); bound 8x."""
    case = make_hit_case(48, 2, mach=0.5, stokes=(0.05, 0.5))
    s = P.Solver.from_case(case, p_tol=1e-6, precision=P.FP32_REFINED)
    m0 = s.stats()
    st, info = s.step(30)
    assert st in (P.OK, P.WARN_DUST)
    for k, i in enumerate(info, start=1):
        bound = 8 * EPS32 * np.sqrt(k / case.n ** 3)
        assert abs(i["mass_gas"] / m0["mass_gas"] - 1) < bound
        for c in range(2):
            assert abs(i["mass_p"][c] / m0["mass_p"][c] - 1) < bound


def test_fp32_statistics_within_calibrated_spread(P):
    """Energy, enstrophy and particle-concentration variance of the FP32 run
    against the FP64 run of the same seed, over 60 steps at 64^3, Mach 0.2,
    Stokes 0.2, residual 1e-6."""
    case = make_hit_case(64, 0, mach=0.2, stokes=(0.2,))
    kw = dict(gamma=case.gamma, C_=case.C, mu=case.mu, tau_p=case.tau_p, p_tol=1e-6)
    a = P.Solver(case.n, case.rho, case.u, case.rho_p, **kw)
    u_pert = case.u * (1 + 1e-7)
    b = P.Solver(case.n, case.rho, u_pert, case.rho_p, **kw)
    f = P.Solver(case.n, case.rho, case.u, case.rho_p, precision=P.FP32_REFINED, **kw)
    floors = dict(ke=1e-5, enstrophy=1e-4, conc=1e-3)
    worst = {}
    for _ in range(6):
        for s in (a, b, f):
            assert s.step(10)[0] in (P.OK, P.WARN_DUST)
        sa, sb, sf = a.stats(), b.stats(), f.stats()
        for key, ga, gb, gf in (("ke", sa["ke"], sb["ke"], sf["ke"]),
                                ("enstrophy", sa["enstrophy"], sb["enstrophy"], sf["enstrophy"]),
                                ("conc", sa["conc_var"][0], sb["conc_var"][0], sf["conc_var"][0])):
            delta = abs(gb - ga) / abs(ga)
            err = abs(gf - ga) / abs(ga)
            bound = max(3 * delta, floors[key])
            assert err <= bound, (key, err, delta)
            worst[key] = max(worst.get(key, 0.0), err / bound)
    print("worst error / bound:", worst)


def test_fp32_statistics_config3_256(P):
    """The precision configuration at size: 256^3, Mach 0.2, one class at Stokes
    0.2, residual 1e-6, 200 steps.  Energy, enstrophy and concentration
    variance of the FP32-refined run against the FP64 run of the same seed,
    every 20 steps, within max(3 x the chaotic spread of an FP64 run whose
    initial velocity is perturbed by 1e-7, the floors 1e-5 / 1e-4 / 1e-3); the
    errors per statistic are printed."""
    case = make_hit_case(256, 0, mach=0.2, stokes=(0.2,))
    kw = dict(gamma=case.gamma, C_=case.C, mu=case.mu, tau_p=case.tau_p, p_tol=1e-6)
    a = P.Solver(case.n, case.rho, case.u, case.rho_p, **kw)
    b = P.Solver(case.n, case.rho, case.u * (1 + 1e-7), case.rho_p, **kw)
    f = P.Solver(case.n, case.rho, case.u, case.rho_p, precision=P.FP32_REFINED, inner_tol=1e-6,
                 **kw)
    floors = dict(ke=1e-5, enstrophy=1e-4, conc=1e-3)
    worst = {}
    for k in range(10):
        for s in (a, b, f):
            st, info = s.step(20)
            assert st in (P.OK, P.WARN_DUST)
            assert all(max(i["pcg_relres"]) <= 1e-6 for i in info)
        sa, sb, sf = a.stats(), b.stats(), f.stats()
        line = []
        for key, ga, gb, gf in (("ke", sa["ke"], sb["ke"], sf["ke"]),
                                ("enstrophy", sa["enstrophy"], sb["enstrophy"], sf["enstrophy"]),
                                ("conc", sa["conc_var"][0], sb["conc_var"][0], sf["conc_var"][0])):
            delta = abs(gb - ga) / abs(ga)
            err = abs(gf - ga) / abs(ga)
            bound = max(3 * delta, floors[key])
            assert err <= bound, (k, key, err, delta)
            worst[key] = max(worst.get(key, 0.0), err / bound)
            line.append(f"{key} err {err:.2e} spread {delta:.2e}")
        print(f"256^3 step {20 * (k + 1)} t {a.t:.4f}: " + "; ".join(line), flush=True)
    print("256^3 worst error / bound:", worst)
