"""The oracle's dust failure flags, each forced on purpose.

* negative density (64, warning): a dust front (a step in the mass ratio)
  carried by a uniform flow; the central fourth-order fluxes are not monotone,
  so the front undershoots below zero.  The flag is raised exactly when the
  returned field has a negative value, and a smooth mode raises nothing.
* non-finite density (128, error): a NaN in the dust input; the step is
  rejected and the state kept.
* non-positive implicit diagonal (256, warning): the Taylor-Green vortex, whose
  material acceleration (u.grad)u = (sin 2x, sin 2y, 0)/2 has divergence
  cos 2x + cos 2y.  With G = phi - tau I4(rho) I4(a) A the diagonal
  rho/dt + (9/16) div G falls to about 1/dt - (9/16) 2 tau at the vortex
  cores' saddle points, so it crosses zero near tau* = 8/(9 dt): the flag is
  off at 0.8 tau* and on at 1.25 tau*, which pins the 9/16 and the sign.
"""
import math

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import taylor_green_case

GAMMA = 1.4


def grid(n):
    h = 2 * math.pi / n
    xc = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(xc, xc, xc, indexing="ij")
    return h, (x, y, z)


def uniform_flow(n, U):
    rho = np.ones((n, n, n))
    u = np.stack([np.full((n, n, n), U), np.zeros((n, n, n)), np.zeros((n, n, n))])
    return rho, u


def test_negative_density_flag(ora):
    n = 16
    rho, u = uniform_flow(n, 0.5)
    h, (x, y, z) = grid(n)
    front = (1e-3 * (x < math.pi))[None]
    o = ora.Oracle(n, rho, u, front, gamma=GAMMA, C_=10.0, mu=1e-3, tau_p=(0.1,), dt_fixed=0.05,
                   p_tol=1e-12)
    st, info = o.step(1)
    rp = o.get(ora.RHO_P)[0]
    assert rp.min() < 0.0
    assert st == ora.WARN_DUST and info[0]["flags"] & ora.FLAG_DUST_NEG
    assert not info[0]["flags"] & (ora.FLAG_DUST_DIAG | ora.FLAG_DUST_NONFINITE)
    # the same flow with a smooth mode stays positive and raises nothing
    smooth = (1e-3 * (1 + 0.5 * np.sin(x)))[None]
    o = ora.Oracle(n, rho, u, smooth, gamma=GAMMA, C_=10.0, mu=1e-3, tau_p=(0.1,), dt_fixed=0.05,
                   p_tol=1e-12)
    st, info = o.step(3)
    assert st == ora.OK and all(i["flags"] == 0 for i in info)
    assert o.get(ora.RHO_P)[0].min() > 0.0


def test_nonfinite_density_flag(ora):
    n = 8
    rho, u = uniform_flow(n, 0.2)
    rp = np.full((2, n, n, n), 1e-3)
    rp[1, 2, 3, 4] = np.nan
    o = ora.Oracle(n, rho, u, rp, gamma=GAMMA, C_=10.0, mu=1e-3, tau_p=(0.0, 0.1),
                   dt_fixed=0.05, p_tol=1e-12)
    before = o.get(ora.RHO_P)
    st, info = o.step(1)
    assert st == ora.ERR_DIVERGED
    assert info[0]["flags"] & ora.FLAG_DUST_NONFINITE
    assert o.t == 0.0
    after = o.get(ora.RHO_P)
    assert np.array_equal(np.isnan(after), np.isnan(before))
    assert np.array_equal(np.nan_to_num(after), np.nan_to_num(before))


@pytest.mark.parametrize("factor,flagged", [(0.8, False), (1.25, True)])
def test_diagonal_flag_threshold(ora, factor, flagged):
    n, dt = 32, 0.01
    tau_star = 8.0 / (9.0 * dt)
    tg = taylor_green_case(n=n, mach=0.05, nu=1e-3)
    rp = (1e-3 * tg["rho"])[None]
    o = ora.Oracle(n, tg["rho"], tg["u"], rp, gamma=tg["gamma"], C_=tg["C"], mu=tg["mu"],
                   tau_p=(factor * tau_star,), dt_fixed=dt, p_tol=1e-12)
    st, info = o.step(1)
    assert bool(info[0]["flags"] & ora.FLAG_DUST_DIAG) == flagged, info[0]["flags"]
    if flagged:
        assert st == ora.WARN_DUST


def test_dust_courant_number_and_flag(ora):
    """Dust settling through gas at rest: G = -tau g rho A on every z-face, so
    the dust's Courant number sum_f |G_f| dt / (2 rho V) is tau g dt / h
    exactly.  Beyond 0.638 the transport's amplification of a uniform drift
    exceeds 1 for some Fourier mode (the root of (1 + y^6)^2 = 1 + y^2,
    y = 0.8130, over the symbol's maximum 1.2739): the flag (512, warning)
    rises there, and the settled dust mode grows instead of decaying."""
    n, dt, g0 = 16, 0.1, 1.0
    h = 2 * math.pi / n
    x, y, z = grid(n)[1]
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    k = 4      # near the symbol's maximum: (20 sin kh - 2 sin 2kh)/16 at kh = pi/2
    rp = (1e-3 * (1 + 0.01 * np.sin(k * z)))[None]
    amps = {}
    for c in (0.5, 0.7):
        tau = c * h / (g0 * dt)
        o = ora.Oracle(n, rho, u, rp, gamma=1.4, C_=10.0, mu=1e-3, tau_p=(tau,), dt_fixed=dt,
                       p_tol=1e-12, gravity=(0.0, 0.0, -g0))
        st, info = o.step(3)
        assert abs(info[0]["courant_dust"] - c) < 1e-12
        flagged = bool(info[0]["flags"] & ora.FLAG_DUST_COURANT)
        assert flagged == (c >= ora.DUST_COURANT_MAX)
        d = o.get(ora.RHO_P)[0] / 1e-3 - 1
        amps[c] = np.max(np.abs(d)) / 0.01
    assert amps[0.5] < 1.0 < amps[0.7], amps
