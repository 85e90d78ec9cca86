"""Pins of the oracle conv network (the learned CG aid): gradients against
FP64 central finite differences, the adjoint identity of the transposed
convolution, and that a trained network approximates A^{-1} of Eq. (7)."""
import numpy as np

from oracle import convnet, spectral


def test_conv_adjoint_identity():
    rng = np.random.default_rng(0)
    W = rng.standard_normal((5, 3, 3, 3))
    x = rng.standard_normal((3, 7, 9))
    g = rng.standard_normal((5, 7, 9))
    assert abs(np.sum(convnet.conv(x, W) * g) - np.sum(x * convnet.conv_t(g, W))) < 1e-10


def test_identity_init_is_identity():
    W = convnet.init_identity(np.random.default_rng(1), channels=4, noise=0.0)
    b = np.random.default_rng(2).standard_normal((6, 8))
    y, _ = convnet.forward(W, b)
    assert np.allclose(y, b, atol=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    W = convnet.init_identity(rng, channels=4, noise=0.3)
    b = rng.standard_normal((6, 7))
    t = rng.standard_normal((6, 7))
    L, G = convnet.loss_and_grad(W, b, t)
    h = 1e-6
    for layer in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W[layer].shape)
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[layer][idx] += h
            Wm[layer][idx] -= h
            fd = (convnet.loss(Wp, b, t) - convnet.loss(Wm, b, t)) / (2 * h)
            assert abs(fd - G[layer][idx]) <= 1e-7 * max(1.0, abs(fd)), (layer, idx, fd, G[layer][idx])


def test_trained_linear_net_approximates_inverse():
    """A few hundred plain gradient steps on one (b, A^{-1} b) pair bring the
    network well below the identity's error (the 7x7 receptive field covers
    A^{-1}'s kernel, which decays over theta*sigma cells)."""
    rng = np.random.default_rng(4)
    nx, ny, dx, dt, theta = 16, 16, 0.1, 0.1, 0.6
    b = rng.standard_normal((ny, nx))
    t = spectral.fft_solve(b, dx, dx, dt, theta)
    W = convnet.init_identity(rng, channels=4, noise=0.01)
    L0 = convnet.loss(W, b, t)
    m = [np.zeros_like(w) for w in W]
    v = [np.zeros_like(w) for w in W]
    lr, b1, b2 = 3e-3, 0.9, 0.999
    for k in range(1, 301):
        L, G = convnet.loss_and_grad(W, b, t)
        for i in range(3):
            m[i] = b1 * m[i] + (1 - b1) * G[i]
            v[i] = b2 * v[i] + (1 - b2) * G[i] ** 2
            W[i] -= lr * (m[i] / (1 - b1 ** k)) / (np.sqrt(v[i] / (1 - b2 ** k)) + 1e-12)
    assert convnet.loss(W, b, t) < 0.05 * L0


def test_window_gradient_matches_finite_differences():
    """The windowed loss (sums over a wrapped cx x cy window only) against
    central differences of the windowed loss itself."""
    rng = np.random.default_rng(5)
    W = convnet.init_identity(rng, channels=4, noise=0.3)
    b = rng.standard_normal((9, 11))
    t = rng.standard_normal((9, 11))
    win = (8, 6, 5, 4)        # wraps in both directions
    L, G = convnet.loss_and_grad(W, b, t, window=win)
    h = 1e-6
    for layer in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W[layer].shape)
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[layer][idx] += h
            Wm[layer][idx] -= h
            fd = (convnet.loss(Wp, b, t, win) - convnet.loss(Wm, b, t, win)) / (2 * h)
            assert abs(fd - G[layer][idx]) <= 1e-7 * max(1.0, abs(fd)), (layer, idx)


def test_windows_partitioning_the_field_sum_to_the_whole():
    """Unnormalised, the squared error is additive over cells: for windows
    that tile the field, sum_w (sum_w t^2) L_w equals (sum t^2) L, and the
    same for the gradients; a window covering the field is the whole loss."""
    rng = np.random.default_rng(6)
    W = convnet.init_identity(rng, channels=3, noise=0.3)
    ny, nx = 8, 12
    b = rng.standard_normal((ny, nx))
    t = rng.standard_normal((ny, nx))
    L, G = convnet.loss_and_grad(W, b, t)
    tt = float(np.sum(t * t))
    acc_L = 0.0
    acc_G = [np.zeros_like(w) for w in W]
    for oy in (1, 5):              # 2 x 3 windows of 4 x 4, offset so that they wrap
        for ox in (2, 6, 10):
            win = (ox, oy, 4, 4)
            m = convnet.window_mask((ny, nx), win)
            tw = float(np.sum(m * t * t))
            Lw, Gw = convnet.loss_and_grad(W, b, t, window=win)
            acc_L += tw * Lw
            for k in range(3):
                acc_G[k] += tw * Gw[k]
    assert abs(acc_L - tt * L) <= 1e-12 * tt * L
    for k in range(3):
        assert np.abs(acc_G[k] - tt * G[k]).max() <= 1e-12 * np.abs(tt * G[k]).max()
    Lf, Gf = convnet.loss_and_grad(W, b, t, window=(3, 2, nx, ny))
    assert abs(Lf - L) <= 1e-14 * L
