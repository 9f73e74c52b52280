"""Pins of the oracle's learned-guess inputs and solve start (oracle/guess.c).

The inputs are the Jacobi-scaled continuity defect and the pressure less its
mean, each divided by its r.m.s.; the pins are the invariants that definition
fixes (unit r.m.s., zero mean, reconstruction of b, invariance under scaling b
and shifting p0), so that a dropped mean, a variance in place of a standard
deviation or b in place of b/diag fails.

The start is x0 = alpha g with alpha = g.b / g.(M g), falling back to 0 when
||b - alpha M g|| >= ||b||.  Its pins: the exact solution (from a dense LAPACK
solve of the assembled operator) as the guess gives alpha = 1 and a zero
residual, any multiple c of it gives alpha = 1/c; alpha is the minimiser of
the energy E(a) = a^2 g.(Mg)/2 - a g.b found by a bounded scalar search on the
dense operator; the reported residual ratio is the dense one; g = 0 and a
guess built to raise the residual fall back.
"""
import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case


@pytest.fixture(scope="module")
def sys8(ora):
    case = make_hit_case(8, 5, mach=0.2, stokes=(0.1,))
    o = ora.Oracle.from_case(case, p_tol=1e-12, capture=True)
    st, _ = o.step(1)
    assert st == 0
    s = dict(b=o.get(ora.SYS_B), psidt=o.get(ora.SYS_PSIDT), K=o.get(ora.SYS_K),
             diag=o.get(ora.SYS_DIAG), p0=o.get(ora.SYS_P0), n=8)
    n = 8
    N = n ** 3
    M = np.zeros((N, N))
    e = np.zeros(N)
    for c in range(N):
        e[:] = 0
        e[c] = 1
        M[:, c] = ora.helm_apply(s["psidt"], s["K"], e.reshape(n, n, n)).ravel()
    s["M"] = M
    s["xstar"] = np.linalg.solve(M, s["b"].ravel()).reshape(n, n, n)
    return s


# ------------------------------------------------------------------ inputs
def test_net_inputs_invariants(ora, sys8):
    s = sys8
    x, (s1, s2) = ora.net_inputs(s["b"], s["diag"], s["p0"])
    c0, c1 = x[:, 0], x[:, 1]
    assert abs(np.sqrt(np.mean(c0 ** 2)) - 1) < 1e-14
    assert abs(np.mean(c1)) < 1e-14 and abs(np.sqrt(np.mean(c1 ** 2)) - 1) < 1e-14
    # channel 0 times s1 times diag is b (so it is b/diag, not b)
    b = s["b"].ravel()
    assert np.max(np.abs(c0 * s1 * s["diag"].ravel() - b)) <= 1e-14 * np.max(np.abs(b))
    # channel 1 times s2 is p0 less its mean (so s2 is a standard deviation)
    p = s["p0"].ravel()
    assert np.max(np.abs(c1 * s2 - (p - p.mean()))) <= 1e-12 * np.max(np.abs(p - p.mean()))


def test_net_inputs_scaling_and_shift(ora, sys8):
    s = sys8
    x, (s1, s2) = ora.net_inputs(s["b"], s["diag"], s["p0"])
    y, (t1, t2) = ora.net_inputs(-3.0 * s["b"], s["diag"], s["p0"] + 17.5)
    assert abs(t1 / s1 - 3.0) < 1e-14 and abs(t2 / s2 - 1) < 1e-9
    assert np.max(np.abs(y[:, 0] + x[:, 0])) < 1e-13
    assert np.max(np.abs(y[:, 1] - x[:, 1])) < 1e-8


def test_net_inputs_degenerate(ora, sys8):
    s = sys8
    z = np.zeros_like(s["b"])
    x, (s1, s2) = ora.net_inputs(z, s["diag"], np.full_like(s["p0"], 4.0))
    assert s1 == 0.0 and s2 == 0.0 and np.all(x == 0.0)


# ------------------------------------------------------------------ start
def test_exact_solution_as_guess(ora, sys8):
    s = sys8
    for c in (1.0, -2.5, 1e-3):
        x0, alpha, ratio, fell = ora.guess_start(s["psidt"], s["K"], s["b"], c * s["xstar"])
        assert not fell
        assert abs(alpha * c - 1) < 1e-10, (c, alpha)
        assert np.max(np.abs(x0 - s["xstar"])) <= 1e-10 * np.max(np.abs(s["xstar"]))
        assert ratio < 1e-9


def test_alpha_minimises_the_energy(ora, sys8):
    from scipy.optimize import minimize_scalar
    s = sys8
    rng = np.random.default_rng(7)
    g = s["xstar"] + 0.3 * np.max(np.abs(s["xstar"])) * rng.standard_normal(s["b"].shape)
    x0, alpha, ratio, fell = ora.guess_start(s["psidt"], s["K"], s["b"], g)
    gv, bv, M = g.ravel(), s["b"].ravel(), s["M"]
    energy = lambda a: 0.5 * a * a * (gv @ (M @ gv)) - a * (gv @ bv)
    best = minimize_scalar(energy, bounds=(-10 * abs(alpha) - 1, 10 * abs(alpha) + 1),
                           method="bounded", options=dict(xatol=1e-12))
    assert abs(best.x - alpha) <= 1e-6 * abs(alpha), (best.x, alpha)
    dense_ratio = np.linalg.norm(bv - alpha * (M @ gv)) / np.linalg.norm(bv)
    assert abs(ratio - dense_ratio) <= 1e-12
    assert fell == (dense_ratio >= 1.0)
    if not fell:
        assert np.max(np.abs(x0 - alpha * g)) == 0.0


def test_fallbacks(ora, sys8):
    s = sys8
    n = s["n"]
    # no guess: alpha = 0 and the residual is b itself, which is not below ||b||
    x0, alpha, ratio, fell = ora.guess_start(s["psidt"], s["K"], s["b"], np.zeros_like(s["b"]))
    assert fell and alpha == 0.0 and ratio == 1.0 and np.all(x0 == 0.0)
    # a one-cell guess against a right-hand side whose M-image is negative at
    # that cell: alpha > 0 but b.(M g) < 0, so the residual grows
    i = (3, 4, 5)
    b = np.zeros((n, n, n))
    b[i] = 1.0
    for ax in range(3):
        for sgn in (-1, 1):
            j = list(i)
            j[ax] = (j[ax] + sgn) % n
            b[tuple(j)] = 50.0
    g = np.zeros((n, n, n))
    g[i] = 1.0
    Mg = s["M"] @ g.ravel()
    assert b.ravel() @ Mg < 0.0
    x0, alpha, ratio, fell = ora.guess_start(s["psidt"], s["K"], b, g)
    assert alpha > 0 and fell and ratio > 1.0 and np.all(x0 == 0.0)
    dense_ratio = np.linalg.norm(b.ravel() - alpha * Mg) / np.linalg.norm(b)
    assert abs(ratio - dense_ratio) <= 1e-12


# ------------------------------------------------- the solve's own loss
def test_residual_loss_pins(ora, sys8):
    """L(g) = |b - alpha M g|^2 / |b|^2 with alpha = g.b / g.(M g), and its
    gradient: zero at the exact solution; invariant to the scale of g (the
    gradient then scales by 1/c); for a constant g under a uniform psi/dt
    (M 1 = psi/dt 1) the closed form 1 - (sum b)^2 / (N sum b^2); the gradient
    equals central differences along random directions."""
    b, psidt, K, xs = sys8["b"], sys8["psidt"], sys8["K"], sys8["xstar"]
    L, gr = ora.residual_loss(psidt, K, b, xs)
    assert L <= 1e-24, L
    rng = np.random.default_rng(9)
    g = xs + 0.3 * np.std(xs) * rng.standard_normal(xs.shape)
    L1, g1 = ora.residual_loss(psidt, K, b, g)
    L2, g2 = ora.residual_loss(psidt, K, b, 3.7 * g)
    assert 0.0 < L1 and abs(L2 - L1) <= 1e-13 * L1
    assert np.max(np.abs(3.7 * g2 - g1)) <= 1e-12 * np.max(np.abs(g1))
    flat = np.full_like(psidt, 2.5)
    Lc, _ = ora.residual_loss(flat, K, b, np.ones_like(b))
    want = 1.0 - b.sum() ** 2 / (b.size * np.sum(b * b))
    assert abs(Lc - want) <= 1e-13, (Lc, want)
    h = 1e-6 * np.std(g)
    for _ in range(4):
        v = rng.standard_normal(g.shape)
        fd = (ora.residual_loss(psidt, K, b, g + h * v)[0] -
              ora.residual_loss(psidt, K, b, g - h * v)[0]) / (2 * h)
        assert abs(fd - np.sum(g1 * v)) <= 1e-6 * abs(fd), (fd, np.sum(g1 * v))
