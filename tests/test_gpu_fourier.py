"""The Fourier (non-barotropic) closure on the GPU against the FP64 oracle:
the ideal gas p = rho R T with the internal-energy predictor whose heat flux
is q = -kappa grad T (FP64; at 64^3 the tiled form of every field kernel
the closure leaves unchanged).

Bars as in the barotropic parity tests: every field within 1e-10 of its
magnitude and of its spread, the same CG iteration counts and dt; plus the
conduction closed form on the GPU and the captured system's closure.
"""
import math

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case

pytestmark = pytest.mark.gpu

TOL = 1e-10
FOURIER = dict(R=1.0, cv=2.5, kappa=2e-2, T0=10.0)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1404_0959_amd.pisoc as P
    P.lib()
    return P


def err(g, o):
    """(max|g - o| / max|o - <o>|, max|g - o| / max|o|)."""
    g, o = np.asarray(g), np.asarray(o)
    d = float(np.max(np.abs(g - o)))
    spread = float(np.max(np.abs(o - o.mean())))
    mag = float(np.max(np.abs(o)))
    return (d / spread if spread > 0 else (0.0 if d == 0 else np.inf),
            d / mag if mag > 0 else (0.0 if d == 0 else np.inf))


def case_and_T(n, seed, mach=0.3):
    case = make_hit_case(n, seed, mach=mach, stokes=(0.1,))
    rng = np.random.default_rng(seed + 7)
    x = (np.arange(n) + 0.5) * 2 * math.pi / n
    T = FOURIER["T0"] * (1 + 0.03 * np.sin(x)[None, None, :] * np.cos(x)[None, :, None]
                         + 0.01 * rng.standard_normal((n, n, n)))
    return case, T


@pytest.mark.parametrize("n,steps", [(16, 5), (32, 4), (40, 3), (64, 2)])
def test_fourier_step_parity(P, ora, n, steps):
    case, T = case_and_T(n, 11)
    o = ora.Oracle.from_case(case, p_tol=1e-10, fourier=FOURIER, T=T)
    s = P.Solver.from_case(case, p_tol=1e-10, fourier=FOURIER, T=T)
    for k in range(steps):
        so, io = o.step(1)
        sg, ig = s.step(1)
        assert so == sg, (k, so, sg)
        assert abs(ig[0]["dt"] / io[0]["dt"] - 1) <= 1e-12
        assert ig[0]["pcg_iters"] == io[0]["pcg_iters"], (k, ig[0]["pcg_iters"], io[0]["pcg_iters"])
    f = s.fields(P.FIELD_RHO | P.FIELD_U | P.FIELD_RHO_P | P.FIELD_P | P.FIELD_T)
    pairs = [(P.FIELD_RHO, ora.RHO), (P.FIELD_U, ora.U), (P.FIELD_RHO_P, ora.RHO_P),
             (P.FIELD_P, ora.P), (P.FIELD_T, ora.T)]
    for fb, ob in pairs:
        g = f[fb].cpu().numpy()
        want = o.get(ob)
        r_dev, r_mag = err(g, want)
        print(f"{n}^3 Fourier, field {fb}: dev {r_dev:.2e} mag {r_mag:.2e}")
        assert r_mag <= TOL and r_dev <= TOL, fb
    sg, so = s.stats(), o.stats()
    for key in ("ke", "enstrophy", "rho_rms", "mach_rms"):
        assert abs(sg[key] / so[key] - 1) <= 1e-10, (key, sg[key], so[key])


def test_fourier_conduction_mode(P):
    """Gas at rest, uniform density, a cosine temperature mode: after one step
    T is the backward-Euler decay of the mode (converged sweeps)."""
    n, kx, eps = 16, 2, 0.05
    h = 2 * math.pi / n
    x = (np.arange(n) + 0.5) * h
    T = FOURIER["T0"] * (1 + eps * np.cos(kx * x))[None, None, :] * np.ones((n, n, n))
    kap, cv = FOURIER["kappa"], FOURIER["cv"]
    dt = cv / (6 * kap / h ** 2)
    s = P.Solver(n, np.ones((n, n, n)), np.zeros((3, n, n, n)), gamma=1.4, C_=10.0, mu=1e-3,
                 dt_fixed=dt, p_tol=1e-12, n_mom_sweeps=120, fourier=FOURIER, T=T)
    st, _ = s.step(1)
    assert st == P.OK
    lam = 2.0 / h ** 2 * (1 - math.cos(kx * h))
    want = FOURIER["T0"] * (1 + eps * np.cos(kx * x) / (1 + dt * kap * lam / cv))
    got = s.get(P.FIELD_T).cpu().numpy()
    assert np.max(np.abs(got - want[None, None, :])) <= 1e-12 * FOURIER["T0"]


def test_fourier_captured_system(P, ora):
    """The corrector's system under the ideal gas: psi/dt = 1/(R T* dt) and p0
    against the oracle's, and b, diag within the parity bars."""
    case, T = case_and_T(32, 12, mach=0.2)
    o = ora.Oracle.from_case(case, p_tol=1e-10, capture=True, fourier=FOURIER, T=T)
    s = P.Solver.from_case(case, p_tol=1e-10, capture=True, fourier=FOURIER, T=T)
    o.step(2)
    st, info = s.step(2)
    f = s.fields(P.FIELD_PSOLVE_B | P.FIELD_PSOLVE_DIAG | P.FIELD_P_PREV | P.FIELD_PSOLVE_PSIDT |
                 P.FIELD_T)
    T1 = f[P.FIELD_T].cpu().numpy()
    psidt = f[P.FIELD_PSOLVE_PSIDT].cpu().numpy()
    assert np.max(np.abs(psidt * FOURIER["R"] * T1 * info[-1]["dt"] - 1)) <= 1e-12
    for fb, ob in ((P.FIELD_PSOLVE_B, ora.SYS_B), (P.FIELD_PSOLVE_DIAG, ora.SYS_DIAG),
                   (P.FIELD_P_PREV, ora.SYS_P0), (P.FIELD_PSOLVE_PSIDT, ora.SYS_PSIDT)):
        r_dev, r_mag = err(f[fb].cpu().numpy(), o.get(ob, 0))
        print(f"Fourier captured field {fb}: dev {r_dev:.2e} mag {r_mag:.2e}")
        assert r_mag <= TOL and r_dev <= TOL, fb


def test_fourier_rejections(P):
    import torch
    case, T = case_and_T(16, 1)
    with pytest.raises(P.PisocError):
        P.Solver.from_case(case, fourier=FOURIER, precision=P.FP32_REFINED, inner_tol=1e-6)
    s = P.Solver.from_case(case)
    with pytest.raises(P.PisocError):
        s.get(P.FIELD_T)
    assert P.lib().pisoc_set_temperature(s._h, torch.ones(16 ** 3, dtype=torch.float64,
                                                          device="cuda").data_ptr()) == P.ERR_INVALID
