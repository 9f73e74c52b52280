"""Pins of the oracle's two-way coupling and gravity settling (the mixture of
gas and dust whose buoyancy motivates the paper: Introduction; Results, the
Equilibrium-Eulerian model and Marble's dusty gas of the third footnote).

* dusty-gas sound speed: with tau = 0 and a uniform dust loading Z = rho_d/rho
  the dust moves with the gas, the mixture's inertia is (1 + Z) times the
  gas's while the pressure is the gas's, so the acoustic period grows by
  sqrt(1 + Z) (Marble's equilibrium sound speed c / sqrt(1 + Z));
* buoyancy: gas at rest, dust rho_j = Y0 (1 + e sin kx), tau = 0, gravity
  along -z, mu = 0: the heavier columns sink with u_z = -g t (rho_m -
  <rho_m>)/rho_m exactly (no divergence, no pressure response, no convection);
* settling: gas at rest, one-way, tau > 0, gravity: the dust drifts at the
  uniform velocity tau g, and a Fourier mode of the dust moves by the closed
  form of the transport scheme (the uniform-flow dust pin with U = tau g);
* two-way coupling with zero dust density and no gravity is bitwise the
  one-way step (with gravity the gas's own density fluctuations are buoyant).
"""
import math

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case

GAMMA = 1.4


def grid(n):
    h = 2 * math.pi / n
    xc = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(xc, xc, xc, indexing="ij")
    return h, (x, y, z)


def period(ora, Z):
    n, e, dt = 16, 1e-4, 0.02
    h, (x, y, z) = grid(n)
    C = 1.0 / GAMMA
    rho = 1 + e * np.cos(x)
    u = np.zeros((3, n, n, n))
    rp = (Z * rho)[None]
    o = ora.Oracle(n, rho, u, rp, gamma=GAMMA, C_=C, mu=0.0, dt_fixed=dt, p_tol=1e-12,
                   tau_p=(0.0,), two_way=True)
    amps, ts = [], []
    for _ in range(int(7.0 * math.sqrt(1 + Z) / dt)):
        o.step(1)
        amps.append(np.mean((o.get(ora.RHO) - 1) * np.cos(x)) * 2 / e)
        ts.append(o.t)
    amps, ts = np.array(amps), np.array(ts)
    zc = [ts[i - 1] - amps[i - 1] * (ts[i] - ts[i - 1]) / (amps[i] - amps[i - 1])
          for i in range(1, len(amps)) if amps[i - 1] * amps[i] < 0]
    return 2 * np.mean(np.diff(zc))


def test_dusty_gas_sound_speed(ora):
    p0 = period(ora, 0.0)
    p1 = period(ora, 1.0)
    assert abs(p0 / (2 * math.pi) - 1) < 0.015, p0
    assert abs(p1 / p0 / math.sqrt(2.0) - 1) < 0.01, (p0, p1)


def test_buoyant_columns(ora):
    n, k, Y0, e, g0, dt = 16, 2, 0.5, 0.3, 9.8, 0.01
    h, (x, y, z) = grid(n)
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    rp = (Y0 * (1 + e * np.sin(k * x)))[None]
    o = ora.Oracle(n, rho, u, rp, gamma=GAMMA, C_=10.0, mu=0.0, dt_fixed=dt, p_tol=1e-12,
                   tau_p=(0.0,), two_way=True, gravity=(0.0, 0.0, -g0))
    rm = 1 + rp[0]
    for steps in (1, 3):
        o.step(steps if steps == 1 else 2)
        uu = o.get(ora.U)
        want = -g0 * steps * dt * (rm - rm.mean()) / rm
        assert np.max(np.abs(uu[2] - want)) < 1e-13 * np.max(np.abs(want)), steps
        assert np.max(np.abs(uu[0])) == 0.0 and np.max(np.abs(uu[1])) == 0.0
    assert np.max(np.abs(o.get(ora.RHO_P)[0] - rp[0])) < 1e-16
    # one-way: the gas does not feel the dust
    o1 = ora.Oracle(n, rho, u, rp, gamma=GAMMA, C_=10.0, mu=0.0, dt_fixed=dt, p_tol=1e-12,
                    tau_p=(0.0,), gravity=(0.0, 0.0, -g0))
    o1.step(2)
    assert np.max(np.abs(o1.get(ora.U))) == 0.0


@pytest.mark.parametrize("two_way", [False, True])
def test_settling_closed_form(ora, two_way):
    n, k, th, tau, g0, dt, Y0, e = 16, 2, 0.4, 0.05, 4.0, 0.1, 1e-3, 0.5
    h, (x, y, z) = grid(n)
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    rp = (Y0 * (1 + e * np.sin(k * z + th)))[None]
    o = ora.Oracle(n, rho, u, rp, gamma=GAMMA, C_=10.0, mu=1e-3, tau_p=(tau,), dt_fixed=dt,
                   n_dust_sweeps=4, p_tol=1e-12, gravity=(0.0, 0.0, -g0), two_way=two_way)
    W = -tau * g0
    zz = 1j * (W * dt / h) * (20 * math.sin(k * h) - 2 * math.sin(2 * k * h)) / 16
    A = sum((-zz) ** l for l in range(4 + 2))
    o.step(1)
    got = o.get(ora.RHO_P)[0]
    want = Y0 * (1 + e * np.imag(A * np.exp(1j * (k * z + th))))
    if not two_way:
        assert np.max(np.abs(got - want)) < 1e-15
        assert np.max(np.abs(o.get(ora.U))) == 0.0
    else:
        # the mixture's buoyancy now moves the gas too: the dust still settles,
        # departing from the one-way closed form only through the gas it drags
        assert np.max(np.abs(got - want)) < 1e-2 * Y0 * e
        assert np.max(np.abs(o.get(ora.U)[2])) > 0.0


def test_two_way_without_dust_mass_is_one_way(ora):
    case = make_hit_case(16, 2, mach=0.2, stokes=(0.1,))
    rp = np.zeros_like(case.rho_p)
    kw = dict(gamma=case.gamma, C_=case.C, mu=case.mu, tau_p=case.tau_p, p_tol=1e-10)
    a = ora.Oracle(case.n, case.rho, case.u, rp, **kw)
    b = ora.Oracle(case.n, case.rho, case.u, rp, two_way=True, **kw)
    a.step(3)
    b.step(3)
    for which in (ora.RHO, ora.U, ora.PHI):
        assert np.array_equal(a.get(which), b.get(which)), which
