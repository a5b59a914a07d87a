"""Pins of the FP64 network reference (no GPU): closed forms and central
finite differences, independent of the chain-rule code they check."""
import numpy as np

from oracle import cnn


def test_delta_kernel_is_identity_and_shift():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 2))
    W = np.zeros((27, 2, 2))
    W[13] = np.eye(2)  # centre tap (1, 1, 1)
    assert np.allclose(cnn.conv3d(x, W, np.zeros(2)), x)
    # tap (1, 1, 2) reads x[v + (0, 0, 1)]: a shift along x with a zero edge
    W = np.zeros((27, 2, 2))
    W[14] = np.eye(2)
    out = cnn.conv3d(x, W, np.array([0.5, -1.0]))
    assert np.allclose(out[:, :, :-1], x[:, :, 1:] + [0.5, -1.0])
    assert np.allclose(out[:, :, -1], [0.5, -1.0])


def test_conv_matches_brute_force_sum():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 3, 4, 3))
    W = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(2)
    out = cnn.conv3d(x, W, b)
    Z, Y, X, _ = x.shape
    for z in range(Z):
        for y in range(Y):
            for xx in range(X):
                s = b.copy()
                for tap, (dz, dy, dx) in enumerate(cnn.TAPS):
                    zz, yy, xxx = z + dz - 1, y + dy - 1, xx + dx - 1
                    if 0 <= zz < Z and 0 <= yy < Y and 0 <= xxx < X:
                        s += x[zz, yy, xxx] @ W[tap]
                assert np.allclose(out[z, y, xx], s)


def test_gradient_matches_finite_differences():
    widths = (4, 3, 5, 2)
    rng = np.random.default_rng(2)
    n = cnn.n_params(widths)
    params = rng.standard_normal(n) * 0.3
    x = rng.standard_normal((3, 4, 4, 4))
    target = rng.standard_normal((3, 4, 4, 2))
    L, g = cnn.loss_grad(params, x, target, widths)
    assert np.isclose(L, cnn.loss(params, x, target, widths))
    idx = rng.choice(n, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(n)
        e[i] = h
        fd = (cnn.loss(params + e, x, target, widths) -
              cnn.loss(params - e, x, target, widths)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_input_gradient_of_one_layer_by_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 4, 3))
    W = rng.standard_normal((27, 3, 2))
    g = rng.standard_normal((2, 3, 4, 2))
    gx, gW, gb = cnn.conv3d_backward(x, W, g)
    f = lambda xx: np.sum(cnn.conv3d(xx, W, np.zeros(2)) * g)
    for _ in range(20):
        i = tuple(rng.integers(0, s) for s in x.shape)
        e = np.zeros_like(x)
        e[i] = 1e-6
        fd = (f(x + e) - f(x - e)) / 2e-6
        assert abs(fd - gx[i]) < 1e-6 * max(1.0, abs(fd))
    assert np.allclose(gb, g.reshape(-1, 2).sum(0))
