"""Pins of the FP64 network-layer reference (oracle/unet.py): brute-force
loops on tiny inputs, closed forms and adjoint identities."""
import numpy as np

from oracle import unet as U


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def brute_conv(x, w, b):
    D, H, W, ci = x.shape
    co = w.shape[1]
    y = np.zeros((D, H, W, co))
    for z in range(D):
        for yy in range(H):
            for xx in range(W):
                for o in range(co):
                    s = b[o]
                    for kz in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                zi, yi, xi = z + kz - 1, yy + ky - 1, xx + kx - 1
                                if 0 <= zi < D and 0 <= yi < H and 0 <= xi < W:
                                    t = (kz * 3 + ky) * 3 + kx
                                    for c in range(ci):
                                        s += x[zi, yi, xi, c] * w[t, o, c]
                    y[z, yy, xx, o] = s
    return y


def test_conv3d_against_scalar_loops():
    x, w, b = rand((3, 4, 5, 2), 1), rand((27, 3, 2), 2), rand(3, 3)
    assert np.allclose(U.conv3d(x, w, b), brute_conv(x, w, b), rtol=0, atol=1e-12)
    assert np.allclose(U.conv3d(x, w, b, relu=True), np.maximum(brute_conv(x, w, b), 0), rtol=0, atol=1e-12)


def test_conv3d_special_kernels():
    x = rand((4, 4, 4, 3), 4)
    w = np.zeros((27, 3, 3))
    w[13] = np.eye(3)                       # centre tap: identity
    assert np.allclose(U.conv3d(x, w), x)
    w = np.zeros((27, 3, 3))
    w[(2 * 3 + 1) * 3 + 1] = np.eye(3)      # tap kz=2 reads z+1: shift up with zero fill
    y = U.conv3d(x, w)
    assert np.allclose(y[:-1], x[1:]) and np.all(y[-1] == 0)


def test_conv3d_gradients_are_adjoints():
    x, w, gy = rand((4, 3, 5, 4), 5), rand((27, 6, 4), 6), rand((4, 3, 5, 6), 7)
    lhs = float((U.conv3d(x, w) * gy).sum())
    assert abs(lhs - float((x * U.conv3d_grad_input(gy, w)).sum())) < 1e-10 * abs(lhs)
    assert abs(lhs - float((w * U.conv3d_grad_weight(x, gy)).sum())) < 1e-10 * abs(lhs)
    assert np.allclose(U.bias_grad(gy), gy.sum(axis=(0, 1, 2)))


def test_conv3d_weight_gradient_by_finite_differences():
    x, w, gy = rand((3, 3, 3, 2), 8), rand((27, 2, 2), 9), rand((3, 3, 3, 2), 10)
    gw = U.conv3d_grad_weight(x, gy)
    for t, o, c in ((0, 0, 0), (13, 1, 0), (26, 1, 1)):
        e = np.zeros_like(w)
        e[t, o, c] = 1e-6
        fd = ((U.conv3d(x, w + e) - U.conv3d(x, w - e)) * gy).sum() / 2e-6
        assert abs(fd - gw[t, o, c]) < 1e-6 * max(1.0, abs(gw[t, o, c]))


def test_pool_and_upsample():
    x, y = rand((4, 6, 2, 3), 11), rand((2, 3, 1, 3), 12)
    assert np.allclose(U.avgpool2(U.upsample2(y)), y)
    assert np.isclose((U.avgpool2(x) * y).sum(), (x * U.avgpool2_grad(y)).sum())
    big = rand((4, 6, 2, 3), 13)
    assert np.isclose((U.upsample2(y) * big).sum(), (y * U.upsample2_grad(big)).sum())
    assert np.isclose(U.avgpool2(x)[0, 0, 0, 0], x[:2, :2, :2, 0].mean())


def test_relu_head_mse():
    y = np.array([[[[-1.0, 2.0]]]])
    assert np.array_equal(U.relu_grad(np.ones_like(y), y), np.array([[[[0.0, 1.0]]]]))
    h, w, x2, g = rand((2, 3, 4, 5), 14), rand(5, 15), rand((2, 3, 4), 16), rand((2, 3, 4), 17)
    x0 = U.head(h, w, 0.3, x2, 100.0)
    assert np.isclose(x0[1, 2, 3], x2[1, 2, 3] + (h[1, 2, 3] @ w + 0.3) / 100.0)
    dh, dw, db = U.head_grad(h, w, g, 100.0)
    lhs = ((x0 - x2 - 0.3 / 100.0) * g).sum()    # the part linear in h (and in w)
    assert np.isclose(lhs, (h * dh).sum()) and np.isclose(lhs, (w * dw).sum())
    assert np.isclose(db, g.sum() / 100.0)
    a, t = rand(50, 18), rand(50, 19)
    loss, grad = U.mse(a, t)
    assert np.isclose(loss, ((a - t) ** 2).mean())
    e = np.zeros(50)
    e[7] = 1e-6
    assert abs((U.mse(a + e, t)[0] - U.mse(a - e, t)[0]) / 2e-6 - grad[7]) < 1e-8


def test_adam_closed_forms():
    g = np.array([3.0, -0.5, 1e-3])
    p, m, v = U.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # after the bias corrections the first step is lr * g / (|g| + eps)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # it drives a convex quadratic to its minimum
    target = np.array([1.0, -2.0, 0.5])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(1, 3001):
        p, m, v = U.adam_step(p, 2 * (p - target), m, v, step, lr=0.01)
    assert np.allclose(p, target, atol=1e-3)


def test_pack_input():
    x1, x2 = rand((2, 2, 2), 20), rand((2, 2, 2), 21)
    t = U.pack_input(x1, x2, 100.0)
    assert t.shape == (2, 2, 2, 16)
    assert np.allclose(t[..., 0], 100 * x1) and np.allclose(t[..., 1], 100 * x2) and not t[..., 2:].any()
