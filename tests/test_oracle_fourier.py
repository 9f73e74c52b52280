"""Pins of the oracle's Fourier (non-barotropic) closure: the ideal gas
p = rho R T with the internal-energy equation whose heat flux is
q = -kappa grad T (the paper's first footnote to the Results section).

* pure conduction: gas at rest with uniform density and a cosine temperature
  mode; the energy predictor's backward-Euler step divides the mode by
  1 + dt kappa lambda / (c_v rho), lambda the compact Laplacian's eigenvalue
  (converged Jacobi sweeps), and the step keeps T* as T^{n+1};
* conservation: summed over the periodic grid, convection and conduction
  cancel, so sum c_v (rho* T* - rho^n T^n) / dt = -sum p^n div u^n exactly
  (converged sweeps), whatever the flow;
* closure in the corrector: psi/dt = 1 / (R T* dt) and p0 = rho* R T*, with
  rho* = rho^n - dt div(phi^n).
"""
import math

import numpy as np

from paper_1404_0959_amd.inputs import make_hit_case

FOURIER = dict(R=1.0, cv=2.5, kappa=2e-2, T0=10.0)


def test_conduction_mode_decay(ora):
    n, kx, eps = 16, 2, 0.05
    h = 2 * math.pi / n
    x = (np.arange(n) + 0.5) * h
    T = FOURIER["T0"] * (1 + eps * np.cos(kx * x))[None, None, :] * np.ones((n, n, n))
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    kap, cv = FOURIER["kappa"], FOURIER["cv"]
    dt = cv / (6 * kap / h ** 2)            # Jacobi contraction 1/2
    o = ora.Oracle(n, rho, u, gamma=1.4, C_=10.0, mu=1e-3, dt_fixed=dt, p_tol=1e-12,
                   n_mom_sweeps=120, fourier=FOURIER, T=T)
    st, info = o.step(1)
    assert st == ora.OK
    lam = 2.0 / h ** 2 * (1 - math.cos(kx * h))
    want = FOURIER["T0"] * (1 + eps * np.cos(kx * x) / (1 + dt * kap * lam / cv))
    got = o.get(ora.T)
    assert np.max(np.abs(got - want[None, None, :])) <= 1e-12 * FOURIER["T0"]


def test_energy_budget(ora):
    case = make_hit_case(16, 3, mach=0.3, stokes=(0.1,))
    rng = np.random.default_rng(1)
    T = FOURIER["T0"] * (1 + 0.05 * rng.standard_normal((16, 16, 16)))
    o = ora.Oracle.from_case(case, p_tol=1e-12, n_mom_sweeps=200, capture=True, fourier=FOURIER,
                             T=T)
    o.step(1)
    rho_n, u_n, T_n = o.get(ora.RHO), o.get(ora.U), o.get(ora.T)
    p_n = o.get(ora.P)
    assert np.max(np.abs(p_n - rho_n * FOURIER["R"] * T_n)) <= 1e-13 * np.max(p_n)
    st, info = o.step(1)
    dt = info[0]["dt"]
    rho_star_T = o.get(ora.SYS_P0, 0) / FOURIER["R"]        # rho* T* of corrector 1
    lhs = FOURIER["cv"] * np.sum(rho_star_T - rho_n * T_n) / dt
    work = np.sum(p_n * ora.div_vel(u_n))
    assert abs(work) > 0
    assert abs(lhs + work) <= 1e-9 * np.sum(np.abs(p_n * ora.div_vel(u_n))), (lhs, -work)


def test_closure_in_corrector(ora):
    case = make_hit_case(16, 4, mach=0.2, stokes=(0.1,))
    o = ora.Oracle.from_case(case, p_tol=1e-10, capture=True, fourier=FOURIER)
    o.step(1)
    rho_n, phi_n = o.get(ora.RHO), o.get(ora.PHI)
    st, info = o.step(1)
    dt = info[0]["dt"]
    T1 = o.get(ora.T)
    rho_star = rho_n - dt * ora.div_flux(phi_n)
    assert np.max(np.abs(o.get(ora.SYS_PSIDT, 0) * (FOURIER["R"] * T1 * dt) - 1)) <= 1e-13
    p0 = o.get(ora.SYS_P0, 0)
    assert np.max(np.abs(p0 - rho_star * FOURIER["R"] * T1)) <= 1e-12 * np.max(p0)
    assert np.max(np.abs(o.get(ora.P) - o.get(ora.RHO) * FOURIER["R"] * T1)) <= 1e-13 * np.max(p0)
