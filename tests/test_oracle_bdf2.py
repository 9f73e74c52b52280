"""Pins of the oracle's variable-step BDF2 time scheme.

* a viscous shear wave u_x = U sin(y) at uniform density: every flux
  divergence vanishes exactly, so each step is the scalar recurrence of the
  scheme for du/dt = -(mu lambda / rho) u, lambda = (2 - 2 cos h)/h^2 the
  compact Laplacian's eigenvalue.  BDF2 reproduces it to round-off (first step
  BDF1), and its error against exp(-mu lambda t / rho) falls 4-fold per
  halving of dt, backward Euler's 2-fold;
* the first BDF2 step is the backward-Euler step, bit for bit;
* gas and dust masses stay conserved to round-off (c0 = c1 - c2);
* a variable step (adaptive dt) still integrates the shear wave to second
  order.
"""
import math

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case


def shear(n, U=0.01):
    h = 2 * math.pi / n
    y = (np.arange(n) + 0.5) * h
    u = np.zeros((3, n, n, n))
    u[0] = U * np.sin(y)[None, :, None]
    return u, y


def run_shear(ora, n, mu, dt, steps, bdf2, **kw):
    u, y = shear(n)
    o = ora.Oracle(n, np.ones((n, n, n)), u, gamma=1.4, C_=1e4, mu=mu, dt_fixed=dt,
                   p_tol=1e-12, n_mom_sweeps=60, bdf2=bdf2, **kw)
    st, info = o.step(steps)
    assert st == ora.OK
    ux = o.get(ora.U)[0]
    amp = ux[0, :, 0] / np.sin(y)
    assert np.max(np.abs(ux - ux[0:1, :, 0:1])) == 0.0      # still a pure y mode
    return float(np.mean(amp)) / 0.01, info


def test_shear_wave_recurrence(ora):
    n, mu, dt, steps = 16, 0.05, 0.05, 12
    h = 2 * math.pi / n
    a = mu * (2 - 2 * math.cos(h)) / h ** 2          # decay rate (rho = 1)
    amp, _ = run_shear(ora, n, mu, dt, steps, True)
    # BDF2 recurrence at w = 1 (c0, c1, c2 = 3/2, 2, 1/2) after a backward-Euler step
    x = [1.0, 1.0 / (1 + a * dt)]
    for _ in range(steps - 1):
        x.append((2 * x[-1] - 0.5 * x[-2]) / (1.5 + a * dt))
    assert abs(amp - x[-1]) <= 1e-12, (amp, x[-1])


@pytest.mark.parametrize("bdf2,rate", [(False, 2.0), (True, 4.0)])
def test_shear_wave_order(ora, bdf2, rate):
    n, mu, T = 16, 0.05, 2.0
    h = 2 * math.pi / n
    a = mu * (2 - 2 * math.cos(h)) / h ** 2
    errs = []
    for m in (20, 40, 80):
        amp, _ = run_shear(ora, n, mu, T / m, m, bdf2)
        errs.append(abs(amp - math.exp(-a * T)))
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(abs(r / rate - 1) < 0.1 for r in ratios), (errs, ratios)


def test_shear_wave_variable_step(ora):
    """Adaptive dt: with the Courant number fixed, dt = cfl h / max|u| grows as
    the wave decays (more than 2-fold over the run), so every step takes its own
    w = dt / dt_prev.  Over two halvings of cfl the BDF2 error falls more than
    8-fold (second order: 16; first order, as backward Euler measures here: 4),
    and it stays two orders of magnitude below backward Euler's."""
    n, mu, T = 16, 0.5, 2.0
    h = 2 * math.pi / n
    a = mu * (2 - 2 * math.cos(h)) / h ** 2

    def run(cfl, bdf2):
        u, y = shear(n)
        o = ora.Oracle(n, np.ones((n, n, n)), u, gamma=1.4, C_=1e4, mu=mu, cfl=cfl,
                       dt_growth=10.0, p_tol=1e-12, n_mom_sweeps=80, bdf2=bdf2)
        t, dts = 0.0, []
        while t < T:
            st, info = o.step(1)
            t = info[0]["t"]
            dts.append(info[0]["dt"])
        amp = float(np.mean(o.get(ora.U)[0][0, :, 0] / np.sin(y))) / 0.01
        return abs(amp - math.exp(-a * t)), dts[-1] / dts[0]
    e1, g1 = run(0.00125, True)
    e2, g2 = run(0.0003125, True)
    eb, _ = run(0.0003125, False)
    assert g1 > 2.0 and g2 > 2.0, (g1, g2)
    assert e1 / e2 > 8.0, (e1, e2)
    assert e2 < 0.01 * eb, (e2, eb)


def test_first_step_is_backward_euler(ora):
    case = make_hit_case(16, 5, mach=0.3, stokes=(0.1,))
    a = ora.Oracle.from_case(case, p_tol=1e-10)
    b = ora.Oracle.from_case(case, p_tol=1e-10, bdf2=True)
    a.step(1)
    b.step(1)
    for f in (ora.RHO, ora.U, ora.PHI, ora.RHO_P):
        assert np.array_equal(a.get(f), b.get(f)), f
    a.step(1)
    b.step(1)
    assert not np.array_equal(a.get(ora.U), b.get(ora.U))


def test_bdf2_conserves_mass(ora):
    case = make_hit_case(16, 6, mach=0.3, stokes=(0.1, 0.3))
    o = ora.Oracle.from_case(case, p_tol=1e-10, bdf2=True)
    m0 = o.stats()
    st, info = o.step(6)
    assert st in (ora.OK, ora.WARN_DUST)
    m1 = o.stats()
    assert abs(m1["mass_gas"] / m0["mass_gas"] - 1) <= 1e-13
    for c in range(2):
        assert abs(m1["mass_p"][c] / m0["mass_p"][c] - 1) <= 1e-12
