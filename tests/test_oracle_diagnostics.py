"""Pins of the oracle's flow diagnostics (energy spectrum, Taylor micro-scale,
second invariant Q).

* Parseval: the shells sum to <|u|^2>/2 for any field;
* single Fourier modes: all energy in the shell of |k| (axis-aligned and
  oblique modes, and modes on either side of a shell boundary), amplitude A^2/4
  per component mode, and lambda = sqrt(5)/|k| exactly;
* the synthetic initial field's spectrum peaks where E(k) = k^4 exp(-2 (k/4)^2)
  does (k = 4);
* Q of the Taylor-Green vortex (sin x cos y, -cos x sin y, 0): the Gauss-I4
  derivative of a k = 1 mode is the exact one times F = (20 sin h - 2 sin 2h)
  / (16 h), so Q = F^2 (sin^2 x sin^2 y - cos^2 x cos^2 y) to round-off;
* sum_P Q = -(1/2) sum_P (div u)^2 for any field (the difference operators are
  antisymmetric and commute), which fixes the sign and the index order.
"""
import math

import numpy as np
import pytest

from paper_1404_0959_amd.inputs import make_hit_case


def grid(n):
    h = 2 * math.pi / n
    xc = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(xc, xc, xc, indexing="ij")
    return h, (x, y, z)


def test_parseval(ora):
    u = make_hit_case(16, 3, mach=0.2).u
    E, lam, D = ora.spectrum(u)
    assert len(E) == ora.spectrum_bins(16) == 15
    assert abs(E.sum() / (0.5 * np.mean(np.sum(u * u, axis=0))) - 1) < 1e-13


@pytest.mark.parametrize("k", [(3, 0, 0), (0, 2, 0), (1, 2, 2), (1, 1, 0), (1, 1, 1), (0, 4, 3)])
def test_single_mode(ora, k):
    n, A, th = 16, 0.7, 0.3
    h, (x, y, z) = grid(n)
    kv = np.array(k, dtype=float)
    # a velocity perpendicular to k, so the field is a pure shear mode
    e = np.cross(kv, [0.3, 0.5, 0.7])
    e /= np.linalg.norm(e)
    ph = k[0] * x + k[1] * y + k[2] * z + th
    u = np.stack([A * e[d] * np.sin(ph) for d in range(3)])
    E, lam, D = ora.spectrum(u)
    kk = math.sqrt(sum(c * c for c in k))
    s = int(math.floor(kk + 0.5))
    assert abs(E[s] - A * A / 4) < 1e-14
    assert np.max(np.abs(np.delete(E, s))) < 1e-28
    assert abs(lam - math.sqrt(5) / kk) < 1e-13
    assert abs(D - kk * kk * A * A / 4) < 1e-12


def test_initial_spectrum_peak(ora):
    u = make_hit_case(32, 0, mach=0.2).u
    E, lam, D = ora.spectrum(u)
    assert int(np.argmax(E)) in (3, 4, 5)
    assert 0.0 < lam < 1.0


def test_q_taylor_green(ora):
    n = 32
    h, (x, y, z) = grid(n)
    u = np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y), np.zeros_like(x)])
    F = (20 * math.sin(h) - 2 * math.sin(2 * h)) / (16 * h)
    want = F * F * (np.sin(x) ** 2 * np.sin(y) ** 2 - np.cos(x) ** 2 * np.cos(y) ** 2)
    got = ora.qcriterion(u)
    assert np.max(np.abs(got - want)) < 1e-14


def test_q_sum_identity(ora):
    u = make_hit_case(16, 5, mach=0.5).u
    u = u + 0.3 * np.random.default_rng(1).standard_normal(u.shape)   # a compressible part
    Q = ora.qcriterion(u)
    div = ora.div_vel(u)
    assert abs(Q.sum() + 0.5 * np.sum(div * div)) < 1e-12 * np.sum(div * div)


# ------------------------------------------------------------ filtered statistics
def test_box_filter_transfer_function(ora):
    """A Fourier mode comes out of the filter multiplied by
    prod_d (1 + cos k_d h) / 2, which fixes the weights (1/4, 1/2, 1/4)."""
    n = 16
    h, (x, y, z) = grid(n)
    k = (1, 3, 2)
    q = np.cos(k[0] * x + k[1] * y + k[2] * z + 0.4)
    T = np.prod([(1 + math.cos(kd * h)) / 2 for kd in k])
    assert np.max(np.abs(ora.box_filter(q) - T * q)) < 1e-14
    assert np.max(np.abs(ora.box_filter(np.full((n, n, n), 2.5)) - 2.5)) < 1e-15


def test_sgs_galilean_and_positive(ora):
    """tau is unchanged by a uniform velocity added to the field, and k_sgs >= 0
    in every cell (the filter's weights are positive and sum to 1)."""
    u = make_hit_case(16, 6, mach=0.2).u
    (r1, k1, p1, f1), ks1, pi1 = ora.sgs_stats(u)
    shift = np.array([0.7, -1.2, 0.4])[:, None, None, None]
    (r2, k2, p2, f2), ks2, pi2 = ora.sgs_stats(u + shift)
    assert np.max(np.abs(ks1 - ks2)) < 1e-12 * np.max(ks1)
    assert np.max(np.abs(pi1 - pi2)) < 1e-11 * np.max(np.abs(pi1))
    assert ks1.min() >= -1e-15
    assert 0.0 < f1 < 1.0


def test_sgs_single_shear_mode(ora):
    """u = (0, A sin kx, 0): tau_yy = (A^2/2) [(1 - T1^2) - (T2 - T1^2) cos 2kx],
    T_m = (1 + cos m k h)/2, tau_xy = 0 and S_bar_yy = 0, so Pi = 0: a single
    shear mode transfers no energy."""
    n, A, k = 32, 0.8, 3
    h, (x, y, z) = grid(n)
    u = np.stack([np.zeros_like(x), A * np.sin(k * x), np.zeros_like(x)])
    (res, ks, pi, frac), ksf, pif = ora.sgs_stats(u)
    T1 = (1 + math.cos(k * h)) / 2
    T2 = (1 + math.cos(2 * k * h)) / 2
    want = 0.25 * A * A * ((1 - T1 * T1) - (T2 - T1 * T1) * np.cos(2 * k * x))
    assert np.max(np.abs(ksf - want)) < 1e-15
    assert np.max(np.abs(pif)) < 1e-15
    assert abs(res - 0.25 * A * A * T1 * T1) < 1e-15
