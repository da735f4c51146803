"""FP64 reference of the warm-start network's layers (test infrastructure only).

Only tests/ may import this module; the GPU path never does.  Plain numpy in
float64, channel-last tensors (D, H, W, C) as the kernels store them:

* conv3d: 3x3x3 cross-correlation with zero padding 1, weights (27, Co, Ci)
  with tap = (kz*3 + ky)*3 + kx, the input sample for output voxel (z, y, x)
  and tap (kz, ky, kx) at (z + kz - 1, y + ky - 1, x + kx - 1);
* its two gradients, written out from that definition (the data gradient is
  the correlation of dy with the mirrored, transposed kernel; the weight
  gradient the correlation of x with dy);
* 2x2x2 average pooling, nearest 2x upsampling, ReLU, the 1x1x1 head with a
  residual on the second iterate, the mean squared error;
* one Adam step (Kingma and Ba, "Adam: a method for stochastic optimization",
  ICLR 2015, Algorithm 1, with the bias corrections written out).

The network itself is not part of the paper: it is the learned warm start of
the CGLS solver built around the projector.  Its pins are closed forms,
brute-force loops on tiny inputs and adjoint identities (tests/test_oracle_unet.py).
"""
import numpy as np

TAPS = [(kz, ky, kx) for kz in range(3) for ky in range(3) for kx in range(3)]


def _pad(x):
    return np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))


def conv3d(x, w, b=None, relu=False):
    """y[z,y,x,co] = b[co] + sum_tap sum_ci x[z+kz-1, y+ky-1, x+kx-1, ci] w[tap,co,ci]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    D, H, W, _ = x.shape
    xp = _pad(x)
    y = np.zeros((D, H, W, w.shape[1]))
    for t, (kz, ky, kx) in enumerate(TAPS):
        y += xp[kz:kz + D, ky:ky + H, kx:kx + W, :] @ w[t].T
    if b is not None:
        y += np.asarray(b, np.float64)
    return np.maximum(y, 0.0) if relu else y


def conv3d_grad_input(gy, w):
    """dL/dx of conv3d for dL/dy = gy: each output voxel sends
    gy[z,y,x,:] w[tap] to the input voxel its tap read."""
    gy = np.asarray(gy, np.float64)
    w = np.asarray(w, np.float64)
    D, H, W, _ = gy.shape
    gxp = np.zeros((D + 2, H + 2, W + 2, w.shape[2]))
    for t, (kz, ky, kx) in enumerate(TAPS):
        gxp[kz:kz + D, ky:ky + H, kx:kx + W, :] += gy @ w[t]
    return gxp[1:-1, 1:-1, 1:-1, :]


def conv3d_grad_weight(x, gy):
    """dL/dw[tap, co, ci] = sum over voxels of gy[v, co] x[v + tap - 1, ci]."""
    x = np.asarray(x, np.float64)
    gy = np.asarray(gy, np.float64)
    D, H, W, ci = x.shape
    co = gy.shape[3]
    xp = _pad(x)
    gw = np.zeros((27, co, ci))
    g2 = gy.reshape(-1, co)
    for t, (kz, ky, kx) in enumerate(TAPS):
        gw[t] = g2.T @ xp[kz:kz + D, ky:ky + H, kx:kx + W, :].reshape(-1, ci)
    return gw


def bias_grad(gy):
    return np.asarray(gy, np.float64).reshape(-1, gy.shape[3]).sum(axis=0)


def relu_grad(gy, y):
    """dL/d(pre-activation) given dL/dy and the ReLU output y."""
    return np.where(np.asarray(y) > 0.0, np.asarray(gy, np.float64), 0.0)


def avgpool2(x):
    x = np.asarray(x, np.float64)
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def avgpool2_grad(gy):
    return upsample2(gy) / 8.0


def upsample2(x):
    """Nearest-neighbour 2x upsampling along the three spatial axes."""
    x = np.asarray(x, np.float64)
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def upsample2_grad(gy):
    gy = np.asarray(gy, np.float64)
    D, H, W, C = gy.shape
    return gy.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def pack_input(x1, x2, scale, channels=16):
    """(D, H, W) iterates -> (D, H, W, channels): scale*x1, scale*x2, zeros."""
    out = np.zeros(np.shape(x1) + (channels,))
    out[..., 0] = scale * np.asarray(x1, np.float64)
    out[..., 1] = scale * np.asarray(x2, np.float64)
    return out


def head(h, w, b, x2, scale):
    """x0 = x2 + (sum_c w[c] h[..., c] + b) / scale."""
    return np.asarray(x2, np.float64) + (np.asarray(h, np.float64) @ np.asarray(w, np.float64) + float(b)) / scale


def head_grad(h, w, g, scale):
    """(dL/dh, dL/dw, dL/db) of head for dL/dx0 = g."""
    gs = np.asarray(g, np.float64) / scale
    h = np.asarray(h, np.float64)
    dh = gs[..., None] * np.asarray(w, np.float64)
    dw = (h * gs[..., None]).reshape(-1, h.shape[-1]).sum(axis=0)
    return dh, dw, float(gs.sum())


def mse(a, t):
    """(mean (a - t)^2, its gradient with respect to a)."""
    d = np.asarray(a, np.float64) - np.asarray(t, np.float64)
    return float((d * d).mean()), 2.0 * d / d.size


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns the new (p, m, v)."""
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
