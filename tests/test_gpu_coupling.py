"""Two-way coupling (mixture momentum) and gravity settling on the GPU, through
the C ABI, against the oracle and its closed forms.

* parity: decaying HIT with two-way coupling and gravity, FP64, at 32^3 (the
  gathered kernels), a ragged 40^3 with two classes and 64^3 (the tiled
  kernels, whose fused dust finish accumulates the next step's dust flux),
  fields within the deviation-normalised bound, flags and CG counts equal;
  FP32 storage within the FP32 tests' bound;
* the oracle's closed forms repeated: buoyant columns, settling of a dust
  mode, the dusty-gas sound speed;
* captured ensemble steps with two-way coupling bitwise the eager ones (the
  dust-flux buffers rotate with the graphs' buffer parity).
"""
import math

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case

pytestmark = pytest.mark.gpu

G = (0.0, 0.0, -2.0)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1404_0959_amd.pisoc as P
    P.lib()
    return P


def grid(n):
    h = 2 * math.pi / n
    xc = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(xc, xc, xc, indexing="ij")
    return h, (x, y, z)


@pytest.mark.parametrize("n,stokes,steps", [(32, (0.1,), 6), (40, (0.05, 0.4), 3), (64, (0.2,), 2)])
def test_two_way_parity(P, ora, n, stokes, steps):
    from test_gpu_parity import SHARED_FLAGS, compare_state
    case = make_hit_case(n, 12, mach=0.2, stokes=stokes)
    # a heavy loading, so that the coupling moves the gas
    rp = case.rho_p * 200.0
    kw = dict(gamma=case.gamma, C_=case.C, mu=case.mu, tau_p=case.tau_p, p_tol=1e-9,
              two_way=True, gravity=G)
    o = ora.Oracle(n, case.rho, case.u, rp, **kw)
    s = P.Solver(n, case.rho, case.u, rp, **kw)
    sto, io = o.step(steps)
    stg, ig = s.step(steps)
    assert sto == stg and sto in (P.OK, P.WARN_DUST)
    for a, b in zip(io, ig):
        assert a["pcg_iters"] == b["pcg_iters"], (a, b)
        assert a["flags"] & SHARED_FLAGS == b["flags"] & SHARED_FLAGS
    compare_state(P, ora, s, o, label=f"two-way {n}^3", spread_tol=1e-9 if n == 64 else 1e-10)
    # the coupling matters: the one-way run differs
    o1 = ora.Oracle(n, case.rho, case.u, rp, **{**kw, "two_way": False})
    o1.step(steps)
    assert np.max(np.abs(o1.get(ora.U) - o.get(ora.U))) > 1e-6


def test_two_way_fp32(P, ora):
    from test_gpu_fp32 import check_fields, FIELD_TOL
    case = make_hit_case(32, 13, mach=0.2, stokes=(0.2,))
    rp = case.rho_p * 200.0
    kw = dict(gamma=case.gamma, C_=case.C, mu=case.mu, tau_p=case.tau_p, p_tol=1e-6,
              two_way=True, gravity=G)
    o = ora.Oracle(case.n, case.rho, case.u, rp, **kw)
    s = P.Solver(case.n, case.rho, case.u, rp, precision=P.FP32_REFINED, inner_tol=1e-7, **kw)
    o.step(5)
    st, info = s.step(5)
    assert st in (P.OK, P.WARN_DUST)
    check_fields(P, ora, s, o, FIELD_TOL)


def test_buoyant_columns(P):
    n, k, Y0, e, g0, dt = 16, 2, 0.5, 0.3, 9.8, 0.01
    h, (x, y, z) = grid(n)
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    rp = (Y0 * (1 + e * np.sin(k * x)))[None]
    s = P.Solver(n, rho, u, rp, gamma=1.4, C_=10.0, mu=0.0, dt_fixed=dt, p_tol=1e-12,
                 tau_p=(0.0,), two_way=True, gravity=(0.0, 0.0, -g0))
    s.step(3)
    uu = s.get(P.FIELD_U).cpu().numpy()
    rm = 1 + rp[0]
    want = -g0 * 3 * dt * (rm - rm.mean()) / rm
    assert np.max(np.abs(uu[2] - want)) < 1e-13 * np.max(np.abs(want))
    assert np.max(np.abs(uu[0])) == 0.0 and np.max(np.abs(uu[1])) == 0.0


def test_settling_closed_form(P):
    n, k, th, tau, g0, dt, Y0, e = 16, 2, 0.4, 0.05, 4.0, 0.1, 1e-3, 0.5
    h, (x, y, z) = grid(n)
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    rp = (Y0 * (1 + e * np.sin(k * z + th)))[None]
    s = P.Solver(n, rho, u, rp, gamma=1.4, C_=10.0, mu=1e-3, tau_p=(tau,), dt_fixed=dt,
                 n_dust_sweeps=4, p_tol=1e-12, gravity=(0.0, 0.0, -g0))
    W = -tau * g0
    zz = 1j * (W * dt / h) * (20 * math.sin(k * h) - 2 * math.sin(2 * k * h)) / 16
    A = sum((-zz) ** l for l in range(6))
    s.step(1)
    got = s.get(P.FIELD_RHO_P).cpu().numpy()[0]
    want = Y0 * (1 + e * np.imag(A * np.exp(1j * (k * z + th))))
    assert np.max(np.abs(got - want)) < 1e-15


def test_dusty_gas_sound_speed(P):
    def period(Z):
        n, eps, dt = 16, 1e-4, 0.02
        h, (x, y, z) = grid(n)
        rho = 1 + eps * np.cos(x)
        s = P.Solver(n, rho, np.zeros((3, n, n, n)), (Z * rho)[None], gamma=1.4, C_=1 / 1.4,
                     mu=0.0, dt_fixed=dt, p_tol=1e-12, tau_p=(0.0,), two_way=True)
        amps, ts = [], []
        for _ in range(int(7.0 * math.sqrt(1 + Z) / dt)):
            s.step(1)
            amps.append(np.mean((s.get(P.FIELD_RHO).cpu().numpy() - 1) * np.cos(x)) * 2 / eps)
            ts.append(s.t)
        zc = [ts[i - 1] - amps[i - 1] * (ts[i] - ts[i - 1]) / (amps[i] - amps[i - 1])
              for i in range(1, len(amps)) if amps[i - 1] * amps[i] < 0]
        return 2 * np.mean(np.diff(zc))
    p0, p1 = period(0.0), period(1.0)
    assert abs(p1 / p0 / math.sqrt(2.0) - 1) < 0.01, (p0, p1)


def test_two_way_ensemble_graph_is_eager(P):
    cs = [make_hit_case(32, 21, mach=0.2, stokes=(0.1,)),
          make_hit_case(64, 22, mach=0.5, stokes=(0.3,))]
    for c in cs:
        c.rho_p[:] *= 100.0
    kw = dict(p_tol=1e-9, two_way=True, gravity=G)
    a = P.Ensemble(cs, **kw)
    b = P.Ensemble(cs, **kw)
    for _ in range(5):
        a.step(1, mode=P.ENS_EAGER)
    b.step(5, mode=P.ENS_GRAPH_ONE)
    bits = P.FIELD_RHO | P.FIELD_U | P.FIELD_PHI | P.FIELD_RHO_P
    for m in range(len(cs)):
        fa = {k: v.cpu().numpy() for k, v in a.fields(m, bits).items()}
        fb = {k: v.cpu().numpy() for k, v in b.fields(m, bits).items()}
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), (m, k)
