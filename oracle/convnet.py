"""FP64 reference of the small convolutional network used as initial guess
and preconditioner for the field CG (not part of the paper: the learned aid
is an addition; the paper solves Eq. (7) by plain CG).

TEST INFRASTRUCTURE ONLY (oracle side; never imported by the GPU package).

Network: three 3x3 convolutions with periodic padding and no activation,
1 -> C -> C -> 1 channels (C = 32):
    h1[c](i,j) = sum_{dy,dx} W1[c,0,dy,dx] x(i+dx-1, j+dy-1)
    h2[c]      = sum_{c', dy, dx} W2[c,c',dy,dx] h1[c'](i+dx-1, j+dy-1)
    y          = sum_{c', dy, dx} W3[0,c',dy,dx] h2[c'](i+dx-1, j+dy-1)
(arrays are [row j][column i]; dx shifts columns, dy rows). The target of
Eq. (7), dB = A^{-1} b, is linear in b, so a linear network keeps the
preconditioner a fixed linear operator.

Loss for one sample (b, t): L = sum (N(b) - t)^2 / sum t^2, over the whole
field or over a window of its cells (the network still acts on the whole
periodic field; only the sums are restricted).
"""
import numpy as np

C = 32


def init_identity(rng, channels=C, noise=0.01):
    """Weights that make N the identity map, plus small noise."""
    W1 = noise * rng.standard_normal((channels, 1, 3, 3))
    W2 = noise * rng.standard_normal((channels, channels, 3, 3)) / np.sqrt(channels)
    W3 = noise * rng.standard_normal((1, channels, 3, 3)) / np.sqrt(channels)
    W1[0, 0, 1, 1] += 1.0
    W2[0, 0, 1, 1] += 1.0
    W3[0, 0, 1, 1] += 1.0
    return [W1, W2, W3]


def shift(a, dy, dx):
    """a(i+dx, j+dy) with periodic wrap, for a[..., j, i]."""
    return np.roll(np.roll(a, -dy, axis=-2), -dx, axis=-1)


def conv(x, W):
    """x [Cin, ny, nx], W [Cout, Cin, 3, 3] -> [Cout, ny, nx] (cross-correlation)."""
    out = np.zeros((W.shape[0],) + x.shape[1:])
    for dy in range(3):
        for dx in range(3):
            xs = shift(x, dy - 1, dx - 1)
            out += np.einsum("oc,cji->oji", W[:, :, dy, dx], xs)
    return out


def conv_t(g, W):
    """Adjoint of conv with respect to its input: g [Cout, ny, nx] -> [Cin, ny, nx]."""
    out = np.zeros((W.shape[1],) + g.shape[1:])
    for dy in range(3):
        for dx in range(3):
            gi = np.einsum("oc,oji->cji", W[:, :, dy, dx], g)
            out += shift(gi, 1 - dy, 1 - dx)
    return out


def conv_wgrad(x, g):
    """dL/dW for out = conv(x, W) given g = dL/dout: [Cout, Cin, 3, 3]."""
    out = np.zeros((g.shape[0], x.shape[0], 3, 3))
    for dy in range(3):
        for dx in range(3):
            xs = shift(x, dy - 1, dx - 1)
            out[:, :, dy, dx] = np.einsum("oji,cji->oc", g, xs)
    return out


def forward(W, b):
    x = b[None]
    h1 = conv(x, W[0])
    h2 = conv(h1, W[1])
    y = conv(h2, W[2])
    return y[0], (x, h1, h2)


def window_mask(shape, window):
    """1 on the cx x cy cells from corner (ox, oy) of a periodic [ny][nx]
    field, 0 elsewhere; window None means every cell."""
    if window is None:
        return np.ones(shape)
    ox, oy, cx, cy = window
    ny, nx = shape
    m = np.zeros(shape)
    m[np.ix_((oy + np.arange(cy)) % ny, (ox + np.arange(cx)) % nx)] = 1.0
    return m


def loss_and_grad(W, b, t, window=None):
    m = window_mask(b.shape, window)
    y, (x, h1, h2) = forward(W, b)
    tt = float(np.sum(m * t * t))
    r = (y - t) * m
    L = float(np.sum(r * r)) / tt
    gy = (2.0 / tt) * r[None]
    g3 = conv_wgrad(h2, gy)
    gh2 = conv_t(gy, W[2])
    g2 = conv_wgrad(h1, gh2)
    gh1 = conv_t(gh2, W[1])
    g1 = conv_wgrad(x, gh1)
    return L, [g1, g2, g3]


def loss(W, b, t, window=None):
    m = window_mask(b.shape, window)
    y, _ = forward(W, b)
    return float(np.sum(m * (y - t) ** 2)) / float(np.sum(m * t * t))
