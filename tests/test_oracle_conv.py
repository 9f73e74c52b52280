"""Pins of the CPU oracle of the learned-guess network (periodic 3x3x3
convolutions 2 -> 16 -> 16 -> 16 -> 1, ReLU, no biases)."""
import numpy as np
import pytest


def zero_w(ora):
    return np.zeros(ora.conv_nweights())


def tap(dz, dy, dx):
    return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)


def set_w(ora, w, layer, co, ci, t, v):
    cin = ora.NET_CH[layer]
    w[ora.conv_layer_slices()[layer].start + (co * cin + ci) * 27 + t] = v


def test_weight_count(ora):
    assert ora.conv_nweights() == 27 * (2 * 16 + 16 * 16 + 16 * 16 + 16 * 1) == 15120


@pytest.mark.parametrize("d", [(0, 0, 1), (0, -1, 0), (1, 1, -1)])
def test_impulse_response_fixes_tap_convention(ora, d):
    """Identity centre taps in layers 1-3 and a single tap d in layer 4:
    an impulse at x0 appears at x0 - d (cross-correlation, periodic wrap)."""
    n = 6
    w = zero_w(ora)
    for l in range(3):
        set_w(ora, w, l, 0, 0, tap(0, 0, 0), 1.0)
    set_w(ora, w, 3, 0, 0, tap(*d), 2.5)
    x = np.zeros((1, n, n, n, 2))
    x0 = (1, 2, 3)           # (k, j, i)
    x[0, x0[0], x0[1], x0[2], 0] = 1.0
    y = ora.conv_forward(w, x)[0]
    dz, dy, dx = d
    want = np.zeros((n, n, n))
    want[(x0[0] - dz) % n, (x0[1] - dy) % n, (x0[2] - dx) % n] = 2.5
    assert np.array_equal(y, want)


def test_constant_input_closed_form(ora):
    """A constant input gives a constant output equal to the weight sums pushed
    through the ReLUs layer by layer."""
    rng = np.random.default_rng(0)
    w = rng.standard_normal(ora.conv_nweights())
    n = 4
    c = np.array([0.7, -1.3])
    x = np.broadcast_to(c, (1, n, n, n, 2)).copy()
    y = ora.conv_forward(w, x)[0]
    v = c
    for l, sl in enumerate(ora.conv_layer_slices()):
        W = w[sl].reshape(ora.NET_CH[l + 1], ora.NET_CH[l], 27).sum(axis=2)
        v = W @ v
        if l < 3:
            v = np.maximum(v, 0.0)
    assert np.max(np.abs(y - v[0])) < 1e-12 * max(1.0, abs(v[0]))


def test_translation_equivariance(ora):
    rng = np.random.default_rng(1)
    w = rng.standard_normal(ora.conv_nweights()) * 0.2
    x = rng.standard_normal((1, 6, 6, 6, 2))
    y = ora.conv_forward(w, x)[0]
    xs = np.roll(x, shift=(1, -2, 3), axis=(1, 2, 3))
    ys = ora.conv_forward(w, xs)[0]
    assert np.max(np.abs(np.roll(y, shift=(1, -2, 3), axis=(0, 1, 2)) - ys)) < 1e-12


def test_gradient_matches_central_differences(ora):
    """Backward pass vs central differences of the forward loss, h = 1e-6,
    relative error <= 1e-6 on a sample of weights in every layer."""
    rng = np.random.default_rng(2)
    n, batch = 4, 2
    w = rng.standard_normal(ora.conv_nweights()) * 0.3
    x = rng.standard_normal((batch, n, n, n, 2))
    t = rng.standard_normal((batch, n, n, n))
    loss, g = ora.conv_backward(w, x, t)
    y = ora.conv_forward(w, x)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-12 * loss

    def L(wv):
        return np.mean((ora.conv_forward(wv, x) - t) ** 2)
    h = 1e-6
    idx = []
    for sl in ora.conv_layer_slices():
        idx += list(rng.choice(np.arange(sl.start, sl.stop), 8, replace=False))
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (L(wp) - L(wm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(g))), (i, fd, g[i])


def test_backward_from_output_gradient(ora):
    """Back-propagation of a given output gradient dy: with dy = 2 (y - t) /
    (batch n^3) it is the mean-squared-error gradient of the separate MSE pass;
    along random weight directions v it is the central difference of
    sum dy * net(x)."""
    rng = np.random.default_rng(4)
    n, batch = 4, 2
    w = rng.standard_normal(ora.conv_nweights()) * 0.3
    x = rng.standard_normal((batch, n, n, n, 2))
    t = rng.standard_normal((batch, n, n, n))
    y = ora.conv_forward(w, x)
    _, g_mse = ora.conv_backward(w, x, t)
    g = ora.conv_backward_dy(w, x, 2 * (y - t) / (batch * n ** 3))
    assert np.max(np.abs(g - g_mse)) <= 1e-12 * np.max(np.abs(g_mse))
    dy = rng.standard_normal((batch, n, n, n))
    g = ora.conv_backward_dy(w, x, dy)
    h = 1e-6
    for _ in range(4):
        v = rng.standard_normal(w.shape)
        fd = (np.sum(dy * ora.conv_forward(w + h * v, x)) -
              np.sum(dy * ora.conv_forward(w - h * v, x))) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * abs(fd), (fd, g @ v)
