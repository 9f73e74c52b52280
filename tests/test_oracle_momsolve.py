"""Pins of the oracle's tolerance-solved momentum predictor (BiCGStab,
preconditioned by diag(a_P), on the three components stacked).

* the solution is the linear system's: it matches the fixed point of the
  Jacobi sweeps run to convergence (a different algorithm);
* the reported relative residual meets the tolerance and a tighter tolerance
  never takes fewer iterations;
* a shear wave u_x = U sin(y) at uniform density is an eigenvector of the
  preconditioned operator: one iteration solves it exactly (the second
  half-step finds s = 0 and takes omega = 0);
* the iteration cap raises its flag (1024) and the not-converged warning.
"""
import math

import numpy as np

from paper_1404_0959_amd.inputs import make_hit_case


def test_bicgstab_matches_converged_sweeps(ora):
    case = make_hit_case(16, 8, mach=0.3, stokes=(0.1,))
    a = ora.Oracle.from_case(case, p_tol=1e-10, capture=True, n_mom_sweeps=300)
    b = ora.Oracle.from_case(case, p_tol=1e-10, capture=True, mom_tol=1e-14)
    a.step(1)
    st, info = b.step(1)
    ua, ub = a.get(ora.SYS_USTAR), b.get(ora.SYS_USTAR)
    assert info[0]["mom_iters"] > 1 and info[0]["mom_relres"] <= 1e-14
    assert np.max(np.abs(ua - ub)) <= 1e-12 * np.max(np.abs(ua))


def test_bicgstab_tolerance_monotone(ora):
    case = make_hit_case(16, 9, mach=0.3, stokes=(0.1,))
    its = []
    for tol in (1e-3, 1e-6, 1e-9, 1e-12):
        o = ora.Oracle.from_case(case, p_tol=1e-10, mom_tol=tol)
        st, info = o.step(1)
        assert info[0]["mom_relres"] <= tol
        its.append(info[0]["mom_iters"])
    assert its == sorted(its) and its[0] >= 1


def test_bicgstab_shear_wave_one_iteration(ora):
    n, mu, dt = 16, 0.05, 0.05
    h = 2 * math.pi / n
    y = (np.arange(n) + 0.5) * h
    u = np.zeros((3, n, n, n))
    u[0] = 0.01 * np.sin(y)[None, :, None]
    o = ora.Oracle(n, np.ones((n, n, n)), u, gamma=1.4, C_=1e4, mu=mu, dt_fixed=dt,
                   p_tol=1e-12, mom_tol=1e-13, capture=True)
    st, info = o.step(1)
    assert st == ora.OK and info[0]["mom_iters"] == 1
    lam = (2 - 2 * math.cos(h)) / h ** 2
    want = 0.01 * np.sin(y) / (1 + dt * mu * lam)
    ux = o.get(ora.SYS_USTAR)[0]
    assert np.max(np.abs(ux - want[None, :, None])) <= 1e-15


def test_bicgstab_cap_flag(ora):
    case = make_hit_case(16, 10, mach=0.3, stokes=(0.1,))
    o = ora.Oracle.from_case(case, p_tol=1e-10, mom_tol=1e-14, mom_maxit=1)
    st, info = o.step(1)
    assert st == ora.WARN_NOT_CONVERGED
    assert info[0]["flags"] & ora.FLAG_MOM_MAXIT and info[0]["mom_iters"] == 1
