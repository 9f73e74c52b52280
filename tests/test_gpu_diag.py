"""The flow diagnostics on the GPU (hand-written FFT, shell binning, Q kernel)
through the C ABI against the oracle's (numpy FFT, the oracle's Gauss-I4
gradient).

Bars: every shell within 1e-12 of the largest shell energy, the Taylor
micro-scale and D within 1e-12 relative; Q within 1e-12 of max|Q|; the
discrete identity <Q> = -<(div u)^2>/2 to rounding; bitwise repeatable.
"""
import math

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1404_0959_amd.pisoc as P
    P.lib()
    return P


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("n", [8, 32, 128, 256])
def test_spectrum_vs_oracle(P, ora, n):
    u = make_hit_case(n, 1, mach=0.2).u
    E, lam, D = P.spectrum(dev(u))
    Eo, lamo, Do = ora.spectrum(u)
    assert E.shape == Eo.shape
    err = np.max(np.abs(E - Eo)) / np.max(Eo)
    print(f"spectrum {n}^3: max shell error {err:.2e} of the peak; lambda {lam:.6f} vs {lamo:.6f}")
    assert err <= 1e-12
    assert abs(lam / lamo - 1) <= 1e-12 and abs(D / Do - 1) <= 1e-12
    E2, lam2, D2 = P.spectrum(dev(u))
    assert np.array_equal(E, E2) and lam == lam2


def test_spectrum_single_mode(P):
    n, A = 64, 0.5
    h = 2 * math.pi / n
    xc = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(xc, xc, xc, indexing="ij")
    u = np.stack([np.zeros_like(x), A * np.sin(2 * x + 3 * z + 0.1), np.zeros_like(x)])
    E, lam, D = P.spectrum(dev(u))
    s = int(math.floor(math.sqrt(13) + 0.5))
    assert abs(E[s] - A * A / 4) < 1e-14
    assert np.max(np.abs(np.delete(E, s))) < 1e-26
    assert abs(lam - math.sqrt(5 / 13)) < 1e-13


def test_spectrum_of_a_running_step(P, ora):
    """The spectrum of the solver's own velocity after a few steps (the field a
    user would hand to the diagnostic), against the oracle on the same field."""
    case = make_hit_case(64, 2, mach=0.2, stokes=(0.1,))
    s = P.Solver.from_case(case, p_tol=1e-8)
    s.step(3)
    u = s.get(P.FIELD_U)
    E, lam, D = P.spectrum(u)
    Eo, lamo, Do = ora.spectrum(u.cpu().numpy())
    assert np.max(np.abs(E - Eo)) <= 1e-12 * np.max(Eo)
    assert abs(lam / lamo - 1) <= 1e-12


@pytest.mark.parametrize("n", [16, 40, 64])
def test_qcriterion_vs_oracle(P, ora, n):
    u = make_hit_case(n, 4, mach=0.5).u
    u = u + 0.1 * np.random.default_rng(n).standard_normal(u.shape)   # a compressible part
    q, qmean, divsq = P.qcriterion(dev(u))
    qo = ora.qcriterion(u)
    err = float(np.max(np.abs(q.cpu().numpy() - qo)) / np.max(np.abs(qo)))
    print(f"Q {n}^3: max error {err:.2e} of max|Q|; <Q> {qmean:.6e}, -<div^2>/2 {-0.5 * divsq:.6e}")
    assert err <= 1e-12
    assert abs(qmean + 0.5 * divsq) <= 1e-12 * divsq
    assert abs(qmean - qo.mean()) <= 1e-12 * np.max(np.abs(qo))


def test_spectrum_rejects_unsupported_sizes(P):
    import torch
    u = torch.zeros((3, 40, 40, 40), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PisocError):
        P.spectrum(u)


@pytest.mark.parametrize("n", [16, 40, 64])
def test_sgs_stats_vs_oracle(P, ora, n):
    u = make_hit_case(n, 7, mach=0.5).u
    got = P.sgs_stats(dev(u))
    want, _, _ = ora.sgs_stats(u)
    print(f"filtered statistics {n}^3: gpu {got}, oracle {want}")
    for g, w in zip(got[:3], want[:3]):
        assert abs(g - w) <= 1e-12 * abs(w)
    # the backscatter fraction counts cells; a cell with Pi within rounding of
    # 0 could fall either side, so one cell's worth of slack
    assert abs(got[3] - want[3]) <= 1.0 / n ** 3 + 1e-15
