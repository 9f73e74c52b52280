"""Pins of the oracle's pressure (Helmholtz) operator and its Jacobi-PCG solver.

* constant coefficients: the operator is diagonalised by the discrete Fourier
  transform, so numpy's FFT gives an independent direct solve;
* variable coefficients (taken from a real corrector of a HIT step): the
  operator assembled column by column is exactly symmetric and positive
  definite, rows sum to psi/dt, and a dense LAPACK solve agrees with PCG.
"""
import math

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case


def fft_eigs(n, psidt, kappa):
    h = 2 * math.pi / n
    m = np.arange(n)
    lam1 = 2 - 2 * np.cos(2 * math.pi * m / n)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    return psidt + kappa / h ** 2 * lam


@pytest.mark.parametrize("n", [8, 12])
def test_helmholtz_constant_coeff_fft(ora, n):
    rng = np.random.default_rng(n)
    psidt, kappa = 3.7, 0.11
    P = np.full((n, n, n), psidt)
    K = [np.full((n, n, n), kappa) for _ in range(3)]
    x = rng.standard_normal((n, n, n))
    eig = fft_eigs(n, psidt, kappa)
    y_fft = np.real(np.fft.ifftn(eig * np.fft.fftn(x)))
    assert np.max(np.abs(ora.helm_apply(P, K, x) - y_fft)) < 1e-11 * np.max(np.abs(y_fft))
    b = rng.standard_normal((n, n, n))
    x_fft = np.real(np.fft.ifftn(np.fft.fftn(b) / eig))
    xs, it, rel = ora.pcg(P, K, b, tol=1e-13, maxit=500)
    assert it > 0 and rel <= 1e-13
    assert np.max(np.abs(xs - x_fft)) <= 1e-12 * np.max(np.abs(x_fft))


@pytest.fixture(scope="module")
def hit_system(ora):
    """The pressure system of corrector 1 of the first step of an 8^3 HIT case."""
    case = make_hit_case(8, 3, mach=0.2, stokes=(0.1,))
    o = ora.Oracle.from_case(case, p_tol=1e-12, capture=True)
    st, info = o.step(1)
    assert st == 0
    return dict(b=o.get(ora.SYS_B), psidt=o.get(ora.SYS_PSIDT), K=o.get(ora.SYS_K),
                x=o.get(ora.SYS_X), w=o.get(ora.SYS_W), diag=o.get(ora.SYS_DIAG), n=8)


def assemble(ora, psidt, K, n):
    N = n ** 3
    M = np.zeros((N, N))
    e = np.zeros(N)
    for c in range(N):
        e[:] = 0
        e[c] = 1
        M[:, c] = ora.helm_apply(psidt, K, e.reshape(n, n, n)).ravel()
    return M


def test_helmholtz_variable_coeff_dense(ora, hit_system):
    s = hit_system
    n = s["n"]
    M = assemble(ora, s["psidt"], s["K"], n)
    assert np.array_equal(M, M.T)                      # exactly symmetric
    assert np.linalg.eigvalsh(M).min() > 0             # positive definite
    # rows sum to psi/dt (the Laplacian part annihilates constants)
    assert np.max(np.abs(M.sum(axis=1) - s["psidt"].ravel())) < 1e-9 * np.abs(M).max()
    # the diagonal the preconditioner uses is M's diagonal
    assert np.max(np.abs(np.diag(M) - s["diag"].ravel())) <= 1e-15 * np.abs(M).max()
    x_dense = np.linalg.solve(M, s["b"].ravel()).reshape(n, n, n)
    scale = np.max(np.abs(x_dense))
    assert np.max(np.abs(s["x"] - x_dense)) <= 1e-10 * scale
    xs, it, rel = ora.pcg(s["psidt"], s["K"], s["b"], tol=1e-14, maxit=1000)
    assert np.max(np.abs(xs - x_dense)) <= 1e-12 * scale


def test_helmholtz_energy_form(ora, hit_system):
    """x^T M x = sum psi/dt x^2 + (1/h^2) sum over faces K_f (x_P - x_nb)^2,
    the face-by-face form of the same quadratic (each face once)."""
    s = hit_system
    n = s["n"]
    h = 2 * math.pi / n
    rng = np.random.default_rng(1)
    x = rng.standard_normal((n, n, n))
    q = np.sum(x * ora.helm_apply(s["psidt"], s["K"], x))
    # numpy axis for direction d: x -> axis 2, y -> axis 1, z -> axis 0
    face = sum(np.sum(s["K"][d] * (x - np.roll(x, -1, axis=2 - d)) ** 2) for d in range(3))
    want = np.sum(s["psidt"] * x * x) + face / h ** 2
    assert abs(q - want) <= 1e-12 * abs(want)


def test_pcg_stopping_rule(ora, hit_system):
    """Stopping is relative to ||b||: a start at the solution takes 0 iterations;
    b = 0 returns x = 0 with 0 iterations; maxit exhaustion is reported."""
    s = hit_system
    xs, it, rel = ora.pcg(s["psidt"], s["K"], s["b"], x0=s["x"], tol=1e-8)
    assert it == 0 and rel <= 1e-8
    z = np.zeros_like(s["b"])
    xs, it, rel = ora.pcg(s["psidt"], s["K"], z, tol=1e-8)
    assert it == 0 and np.all(xs == 0)
    xs, it, rel = ora.pcg(s["psidt"], s["K"], s["b"], tol=1e-14, maxit=2)
    assert it < 0 and rel > 1e-14
    # monotone: a tighter tolerance never needs fewer iterations
    its = [ora.pcg(s["psidt"], s["K"], s["b"], tol=t)[1] for t in (1e-4, 1e-6, 1e-8, 1e-10)]
    assert its == sorted(its) and its[0] >= 1


# ------------------------------------- Chebyshev polynomial preconditioner
def test_cheb_polynomial_is_the_minimax_one(ora, hit_system):
    """The residual polynomial 1 - lambda p(lambda) of the degree-1
    preconditioner equioscillates on [a, 2 - a] (+e at both ends, -e at the
    midpoint, e = its maximum modulus), which fixes the degree-2 minimax
    polynomial normalised at 0; a is min psi/dt / diag, and the dense spectrum
    of D^-1 M lies inside [a, 2 - a]."""
    s = hit_system
    c0, c1, a = ora.cheb_coef(s["psidt"], s["K"])
    assert a == np.min(s["psidt"] / s["diag"])
    b = 2.0 - a
    res = lambda lam: 1.0 - lam * (c0 + c1 * lam)
    e = res(a)
    assert 0 < e < 1 and abs(res(b) - e) <= 1e-14 and abs(res((a + b) / 2) + e) <= 1e-14
    lam = np.linspace(a, b, 1001)
    assert np.max(np.abs(res(lam))) <= e * (1 + 1e-12)
    M = assemble(ora, s["psidt"], s["K"], s["n"])
    d = s["diag"].ravel()
    ev = np.linalg.eigvalsh(M / np.sqrt(np.outer(d, d)))
    assert a - 1e-12 <= ev.min() and ev.max() <= b + 1e-12


@pytest.mark.parametrize("n", [8, 12])
def test_cheb_apply_on_fourier_modes(ora, n):
    """Constant coefficients: every Fourier mode is an eigenvector of D^-1 M
    (eigenvalue lambda = FFT eigenvalue / D), so the preconditioner maps a
    random field r to the inverse FFT of p(lambda) r_hat / D."""
    rng = np.random.default_rng(n + 1)
    psidt, kappa = 3.7, 0.11
    P = np.full((n, n, n), psidt)
    K = [np.full((n, n, n), kappa) for _ in range(3)]
    D = psidt + 6 * kappa / (2 * math.pi / n) ** 2
    c0, c1, a = ora.cheb_coef(P, K)
    assert abs(a - psidt / D) <= 1e-15
    lam = fft_eigs(n, psidt, kappa) / D
    r = rng.standard_normal((n, n, n))
    want = np.real(np.fft.ifftn((c0 + c1 * lam) * np.fft.fftn(r))) / D
    z = ora.cheb_apply(P, K, r)
    assert np.max(np.abs(z - want)) <= 1e-12 * np.max(np.abs(want))


def test_pcg_cheb_solves_and_stops_like_pcg(ora, hit_system):
    """Same solution as the dense solve; same stopping rule as Jacobi-PCG (a
    start at the solution takes 0 iterations, maxit exhaustion reported); on
    this system it needs no more iterations than Jacobi-PCG."""
    s = hit_system
    n = s["n"]
    M = assemble(ora, s["psidt"], s["K"], n)
    x_dense = np.linalg.solve(M, s["b"].ravel()).reshape(n, n, n)
    xs, it, rel = ora.pcg_cheb(s["psidt"], s["K"], s["b"], tol=1e-14, maxit=1000)
    assert it > 0 and np.max(np.abs(xs - x_dense)) <= 1e-12 * np.max(np.abs(x_dense))
    _, it0, _ = ora.pcg_cheb(s["psidt"], s["K"], s["b"], x0=x_dense, tol=1e-8)
    assert it0 == 0
    _, itm, rel = ora.pcg_cheb(s["psidt"], s["K"], s["b"], tol=1e-14, maxit=1)
    assert itm < 0
    for tol in (1e-6, 1e-10):
        assert ora.pcg_cheb(s["psidt"], s["K"], s["b"], tol=tol)[1] <= \
            ora.pcg(s["psidt"], s["K"], s["b"], tol=tol)[1]
