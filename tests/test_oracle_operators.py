"""Pins of the oracle's discrete operators against closed-form Fourier symbols.

Each operator is applied to a single Fourier mode; on a uniform periodic grid
a linear, translation-invariant stencil maps the mode to itself times its
symbol, which is written here from the stencil's weights by hand (not from the
oracle), so a wrong weight, sign, index or scale breaks the equality.
"""
import math

import numpy as np
import pytest


def grid(n):
    h = 2 * math.pi / n
    xc = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(xc, xc, xc, indexing="ij")
    return h, (x, y, z)


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("k", [1, 3])
def test_i4_symbol(ora, d, k):
    """I4 maps sin(k x_d + th) at centres to T(kh) sin(k x_face + th) at the
    faces P + 1/2, with T(h) = (9 cos(h/2) - cos(3h/2)) / 8 (Results: fourth-order
    central interpolation)."""
    n = 16
    h, X = grid(n)
    th = 0.3
    f = np.sin(k * X[d] + th)
    got = ora.i4(f, d)
    T = (9 * math.cos(k * h / 2) - math.cos(3 * k * h / 2)) / 8
    want = T * np.sin(k * (X[d] + h / 2) + th)
    assert np.max(np.abs(got - want)) < 1e-14


def test_i4_fourth_order(ora):
    """Interpolation error on a manufactured field falls as h^4: observed order
    >= 3.9 over n = 16..128 (the paper's fourth-order claim)."""
    errs = []
    ns = [16, 32, 64, 128]
    for n in ns:
        h = 2 * math.pi / n
        xc = (np.arange(n) + 0.5) * h
        # one x-line is enough: broadcast a 3D field that varies along x only
        f = np.broadcast_to(np.sin(2 * xc + 0.7) + 0.5 * np.cos(xc), (n, n, n)).copy()
        got = ora.i4(f, 0)[0, 0]
        xf = xc + h / 2
        want = np.sin(2 * xf + 0.7) + 0.5 * np.cos(xf)
        errs.append(np.max(np.abs(got - want)))
    orders = [math.log(errs[i] / errs[i + 1], 2) for i in range(len(errs) - 1)]
    assert min(orders) >= 3.9, orders


@pytest.mark.parametrize("d", [0, 1, 2])
def test_gauss_gradient_symbol(ora, d):
    """Gauss-I4 gradient of sin(k x_d + th): component d equals
    (20 sin kh - 2 sin 2kh)/(16 h) cos(k x_d + th); the other two vanish."""
    n = 16
    k = 2
    h, X = grid(n)
    f = np.sin(k * X[d] + 0.4)
    g = ora.grad(f)
    S = (20 * math.sin(k * h) - 2 * math.sin(2 * k * h)) / (16 * h)
    assert np.max(np.abs(g[d] - S * np.cos(k * X[d] + 0.4))) < 1e-13
    for e in range(3):
        if e != d:
            assert np.max(np.abs(g[e])) < 1e-13


def test_div_vel_symbol(ora):
    """Cell divergence of u = (sin kx, cos ky, sin kz): sum of the Gauss-I4 symbols."""
    n = 16
    k = 1
    h, (x, y, z) = grid(n)
    u = [np.sin(k * x), np.cos(k * y), np.sin(k * z)]
    S = (20 * math.sin(k * h) - 2 * math.sin(2 * k * h)) / (16 * h)
    want = S * (np.cos(k * x) - np.sin(k * y) + np.cos(k * z))
    assert np.max(np.abs(ora.div_vel(u) - want)) < 1e-13


def test_laplacian_symbol(ora):
    """Compact Laplacian: symbol -(2 - 2 cos kh)/h^2 per direction."""
    n = 16
    h, (x, y, z) = grid(n)
    f = np.sin(x + 2 * y + 3 * z)
    lam = sum((2 - 2 * math.cos(m * h)) / h ** 2 for m in (1, 2, 3))
    assert np.max(np.abs(ora.lap(f) + lam * f)) < 1e-11


@pytest.mark.parametrize("d", [0, 1, 2])
def test_sngrad_symbol(ora, d):
    """Compact face gradient of sin(k x + th) at P + 1/2: (2 sin(kh/2)/h) cos(k x_f + th)."""
    n = 12
    k = 2
    h, X = grid(n)
    got = ora.sngrad(np.sin(k * X[d] + 0.1), d)
    want = 2 * math.sin(k * h / 2) / h * np.cos(k * (X[d] + h / 2) + 0.1)
    assert np.max(np.abs(got - want)) < 1e-13


def test_div_flux_symbol_and_telescoping(ora):
    """Face-flux divergence: face fluxes F_d = cos(k x_d) sampled at the faces
    P + 1/2 give div = -(2 sin(kh/2)/V) sum_d sin(k x_d) at the centres; and
    sum_P div V vanishes to round-off for arbitrary fluxes (each face enters two
    cells with opposite signs)."""
    n = 10
    h, (x, y, z) = grid(n)
    V = h ** 3
    k = 1
    F = [np.cos(k * (x + h / 2)), np.cos(k * (y + h / 2)), np.zeros_like(x)]
    got = ora.div_flux(F)
    want = (-2 * math.sin(k * h / 2) / V) * (np.sin(k * x) + np.sin(k * y))
    assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))
    rng = np.random.default_rng(5)
    G = [rng.standard_normal((n, n, n)) for _ in range(3)]
    assert abs(np.sum(ora.div_flux(G)) * V) < 1e-12


def test_kfaces_is_i4(ora):
    """Face coefficients of the pressure operator are I4 of the cell field w:
    a constant w gives constant faces and a mode gets the I4 symbol."""
    n = 8
    h, (x, y, z) = grid(n)
    K = ora.kfaces(np.full((n, n, n), 0.25))
    for d in range(3):
        assert np.max(np.abs(K[d] - 0.25)) < 1e-16
    w = 1.0 + 0.1 * np.sin(y)
    K = ora.kfaces(w)
    T = (9 * math.cos(h / 2) - math.cos(3 * h / 2)) / 8
    assert np.max(np.abs(K[1] - (1.0 + 0.1 * T * np.sin(y + h / 2)))) < 1e-15
    assert np.max(np.abs(K[0] - w)) < 1e-15
