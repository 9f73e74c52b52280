"""The variable-step BDF2 time scheme on the GPU (FP64; at 64^3 the tiled
form of every kernel BDF2 leaves unchanged) against the FP64 oracle: fields, dt and CG iterations over several steps of
decaying HIT with two dust classes (adaptive dt, so w = dt/dt_prev varies),
within the barotropic parity bars; and the viscous shear wave's BDF2
recurrence on the GPU to round-off."""
import math

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1404_0959_amd.pisoc as P
    P.lib()
    return P


def err(g, o):
    g, o = np.asarray(g), np.asarray(o)
    d = float(np.max(np.abs(g - o)))
    spread = float(np.max(np.abs(o - o.mean())))
    mag = float(np.max(np.abs(o)))
    return (d / spread if spread > 0 else (0.0 if d == 0 else np.inf),
            d / mag if mag > 0 else (0.0 if d == 0 else np.inf))


@pytest.mark.parametrize("n,steps", [(16, 6), (32, 5), (40, 4), (64, 3)])
def test_bdf2_step_parity(P, ora, n, steps):
    case = make_hit_case(n, 21, mach=0.3, stokes=(0.05, 0.3))
    o = ora.Oracle.from_case(case, p_tol=1e-10, bdf2=True)
    s = P.Solver.from_case(case, p_tol=1e-10, bdf2=True)
    dts = []
    for k in range(steps):
        so, io = o.step(1)
        sg, ig = s.step(1)
        assert so == sg, (k, so, sg)
        assert abs(ig[0]["dt"] / io[0]["dt"] - 1) <= 1e-12
        assert ig[0]["pcg_iters"] == io[0]["pcg_iters"], (k, ig[0]["pcg_iters"], io[0]["pcg_iters"])
        dts.append(io[0]["dt"])
    assert len({round(a / b, 12) for a, b in zip(dts[1:], dts[:-1])}) > 1   # w varies
    f = s.fields(P.FIELD_RHO | P.FIELD_U | P.FIELD_PHI | P.FIELD_RHO_P)
    for fb, ob in ((P.FIELD_RHO, ora.RHO), (P.FIELD_U, ora.U), (P.FIELD_PHI, ora.PHI),
                   (P.FIELD_RHO_P, ora.RHO_P)):
        r_dev, r_mag = err(f[fb].cpu().numpy(), o.get(ob))
        print(f"{n}^3 BDF2, field {fb}: dev {r_dev:.2e} mag {r_mag:.2e}")
        assert r_mag <= TOL and r_dev <= TOL, fb
    sg, so = s.stats(), o.stats()
    assert abs(sg["mass_gas"] / so["mass_gas"] - 1) <= 1e-13
    for c in range(2):
        assert abs(sg["mass_p"][c] / so["mass_p"][c] - 1) <= 1e-12


def test_bdf2_shear_wave_recurrence(P):
    n, mu, dt, steps = 16, 0.05, 0.05, 12
    h = 2 * math.pi / n
    y = (np.arange(n) + 0.5) * h
    u = np.zeros((3, n, n, n))
    u[0] = 0.01 * np.sin(y)[None, :, None]
    s = P.Solver(n, np.ones((n, n, n)), u, gamma=1.4, C_=1e4, mu=mu, dt_fixed=dt, p_tol=1e-12,
                 n_mom_sweeps=60, bdf2=True)
    st, _ = s.step(steps)
    assert st == P.OK
    ux = s.get(P.FIELD_U).cpu().numpy()[0]
    amp = float(np.mean(ux[0, :, 0] / np.sin(y))) / 0.01
    a = mu * (2 - 2 * math.cos(h)) / h ** 2
    x = [1.0, 1.0 / (1 + a * dt)]
    for _ in range(steps - 1):
        x.append((2 * x[-1] - 0.5 * x[-2]) / (1.5 + a * dt))
    assert abs(amp - x[-1]) <= 1e-12, (amp, x[-1])


def test_bdf2_rejected_in_fp32(P):
    case = make_hit_case(16, 1, mach=0.2, stokes=(0.1,))
    with pytest.raises(P.PisocError):
        P.Solver.from_case(case, bdf2=True, precision=P.FP32_REFINED, inner_tol=1e-6)
