"""Pins of the learned-smoother oracle (oracle/nn.py): convolution against a
brute-force definition, lattice-translation equivariance, gradients against
central finite differences, Adam's first step, positive homogeneity."""
import numpy as np

from oracle import nn
from workloads import gauge_field, nn_init_weights


def _brute_conv(x, W, periodic):
    Ci, H, Wd = x.shape
    Co = W.shape[0]
    Ho, Wo = (H, Wd) if periodic else (H - 2, Wd - 2)
    y = np.zeros((Co, Ho, Wo))
    for o in range(Co):
        for i in range(Ho):
            for j in range(Wo):
                acc = 0.0
                for c in range(Ci):
                    for a in range(3):
                        for b in range(3):
                            if periodic:
                                acc += W[o, c, a, b] * x[c, (i + a - 1) % H, (j + b - 1) % Wd]
                            else:
                                acc += W[o, c, a, b] * x[c, i + a, j + b]
                y[o, i, j] = acc
    return y


def test_conv_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 7))
    W = rng.standard_normal((4, 3, 3, 3))
    for periodic in (True, False):
        assert np.allclose(nn.conv3x3(x, W, periodic), _brute_conv(x, W, periodic),
                           rtol=1e-13, atol=1e-13)


def test_periodic_conv_of_delta_and_constant():
    W = np.arange(2 * 1 * 9, dtype=float).reshape(2, 1, 3, 3)
    x = np.zeros((1, 6, 6))
    x[0, 2, 3] = 1.0
    y = nn.conv3x3(x, W, True)
    # a unit impulse at p lands at p - (a-1, b-1) weighted by W[:, :, a, b]
    for a in range(3):
        for b in range(3):
            assert np.all(y[:, 2 - (a - 1), 3 - (b - 1)] == W[:, 0, a, b])
    c = nn.conv3x3(np.ones((1, 4, 5)), W, True)
    assert np.allclose(c, W.sum(axis=(1, 2, 3))[:, None, None])


def test_network_is_translation_equivariant_and_homogeneous():
    N = 8
    rng = np.random.default_rng(1)
    th = gauge_field(N, seed=3)
    w = nn_init_weights(2)
    r = rng.standard_normal(2 * N * N) + 1j * rng.standard_normal(2 * N * N)
    e = nn.correction(r, th, N, w)
    # shifting residual and links together shifts the output
    sh = (2, 5)
    r_s = np.roll(r.reshape(N, N, 2), sh, axis=(0, 1)).reshape(-1)
    th_s = np.roll(th, sh, axis=(1, 2))
    e_s = nn.correction(r_s, th_s, N, w)
    assert np.allclose(e_s, np.roll(e.reshape(N, N, 2), sh, axis=(0, 1)).reshape(-1),
                       rtol=1e-12, atol=1e-13)
    # the RMS normalisation makes the correction positively homogeneous
    assert np.allclose(nn.correction(3.5 * r, th, N, w), 3.5 * e, rtol=1e-12, atol=1e-13)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    B, H = 2, 10
    X = rng.standard_normal((B, 8, H, H))
    T = rng.standard_normal((B, 4, H - 6, H - 6))
    w = nn_init_weights(5) * 3.0
    loss, g = nn.loss_and_grad(X, T, w)
    h = 1e-6
    # every output of the last layer and a sample of the hidden layers' weights
    idx = list(rng.choice(1152, 12, replace=False)) + \
        list(1152 + rng.choice(2304, 12, replace=False)) + \
        list(range(3456, 4032, 23))
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (nn.loss_and_grad(X, T, wp)[0] - nn.loss_and_grad(X, T, wm)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
    # and the directional derivative along a random direction (all weights)
    d = rng.standard_normal(w.size)
    fd = (nn.loss_and_grad(X, T, w + h * d)[0] - nn.loss_and_grad(X, T, w - h * d)[0]) / (2 * h)
    assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(g @ d))


def test_adam_first_step_moves_by_lr_times_sign():
    g = np.array([3.0, -0.25, 1e-3, -7.0])
    w0 = np.zeros(4)
    w, m, v = nn.adam_step(w0, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # bias-corrected first moments are g and g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(w, -0.01 * np.sign(g), rtol=1e-5)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_flatten_layout():
    w = np.arange(nn.N_WEIGHTS, dtype=float)
    W1, W2, W3 = nn.unflatten(w)
    assert W1[0, 0, 0, 0] == 0 and W1[15, 7, 2, 2] == 1151
    assert W2[0, 0, 0, 0] == 1152 and W3[0, 0, 0, 0] == 3456
    assert W3[3, 15, 2, 2] == nn.N_WEIGHTS - 1
    assert np.array_equal(nn.flatten([W1, W2, W3]), w)
