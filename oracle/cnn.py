"""FP64 CPU oracle for the learned coarse-grid correction network.

TEST INFRASTRUCTURE.  Only ``tests/`` (and the benchmark's CPU-baseline
leg) may import this module; the GPU library never does, and the two share no
code.

The network is three 3 x 3 x 3 convolution layers (zero padding, stride 1)
on channels-last fields ``x[z][y][x][c]``:

    z1 = conv(x, w1) + b1,  y1 = relu(z1)
    z2 = conv(y1, w2) + b2, y2 = relu(z2)
    out = conv(y2, w3) + b3

with weights ``w[tap][cin][cout]``, tap = 9 (dz+1) + 3 (dy+1) + (dx+1) for
offsets dz, dy, dx in {-1, 0, 1}:

    conv(x, w)[p][co] = sum_tap sum_ci x[p + offset(tap)][ci] w[tap][ci][co]

(the cross-correlation convention of deep-learning convolutions).  The loss
is the masked mean square L = 1/(2 n) sum_mask |out - target|^2.  Backward is
the chain rule written out per layer; each function below states the formula
it computes.  All arithmetic in numpy float64.
"""
from __future__ import annotations

import numpy as np

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, dz, dy, dx):
    """s[p] = x[p + (dz, dy, dx)] with zeros outside (x is [D][H][W][C])."""
    D, H, W = x.shape[:3]
    p = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    return p[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W]


def conv3d(x, w, b=None):
    """conv(x, w)[p][co] = sum_tap x[p + off(tap)] @ w[tap] (+ b)."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    out = np.zeros(x.shape[:3] + (w.shape[2],))
    for t, (dz, dy, dx) in enumerate(OFFSETS):
        out += _shift(x, dz, dy, dx) @ w[t]
    if b is not None:
        out += np.asarray(b, np.float64)
    return out


def conv3d_loops(x, w, b=None):
    """The same definition as explicit loops (small inputs only)."""
    x = np.asarray(x, np.float64)
    D, H, W, Ci = x.shape
    Co = w.shape[2]
    out = np.zeros((D, H, W, Co))
    for z in range(D):
        for y in range(H):
            for xx in range(W):
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            t = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                            zz, yy, xs = z + dz, y + dy, xx + dx
                            if not (0 <= zz < D and 0 <= yy < H and 0 <= xs < W):
                                continue
                            for ci in range(Ci):
                                for co in range(Co):
                                    out[z, y, xx, co] += x[zz, yy, xs, ci] * w[t, ci, co]
    if b is not None:
        out += np.asarray(b, np.float64)
    return out


def conv3d_backward_data(dz, w):
    """dL/dx[q][ci] = sum_tap sum_co dL/dz[q - off(tap)][co] w[tap][ci][co]."""
    dz = np.asarray(dz, np.float64)
    w = np.asarray(w, np.float64)
    dx = np.zeros(dz.shape[:3] + (w.shape[1],))
    for t, (oz, oy, ox) in enumerate(OFFSETS):
        dx += _shift(dz, -oz, -oy, -ox) @ w[t].T
    return dx


def conv3d_backward_weight(x, dz):
    """dL/dw[tap][ci][co] = sum_p x[p + off(tap)][ci] dL/dz[p][co];
    dL/db[co] = sum_p dL/dz[p][co]."""
    x = np.asarray(x, np.float64)
    dz = np.asarray(dz, np.float64)
    Ci, Co = x.shape[3], dz.shape[3]
    dw = np.zeros((27, Ci, Co))
    for t, (oz, oy, ox) in enumerate(OFFSETS):
        dw[t] = _shift(x, oz, oy, ox).reshape(-1, Ci).T @ dz.reshape(-1, Co)
    return dw, dz.reshape(-1, Co).sum(0)


def net_forward(x, params):
    """params = (w1, b1, w2, b2, w3, b3); returns (out, cache)."""
    w1, b1, w2, b2, w3, b3 = params
    z1 = conv3d(x, w1, b1)
    y1 = np.maximum(z1, 0.0)
    z2 = conv3d(y1, w2, b2)
    y2 = np.maximum(z2, 0.0)
    out = conv3d(y2, w3, b3)
    return out, (np.asarray(x, np.float64), z1, y1, z2, y2)


def loss(out, target, mask):
    """L = 1/(2 n) sum_mask |out - target|^2, n = number of masked voxels."""
    m = np.asarray(mask, bool)
    d = (out - np.asarray(target, np.float64))[m]
    return 0.5 * float(np.sum(d * d)) / max(int(m.sum()), 1)


def loss_grad(out, target, mask):
    """dL/dout = mask (out - target) / n."""
    m = np.asarray(mask, bool)
    g = np.zeros_like(out)
    g[m] = (out - np.asarray(target, np.float64))[m] / max(int(m.sum()), 1)
    return g


def net_backward(dout, params, cache):
    """Parameter gradients (dw1, db1, dw2, db2, dw3, db3) by the chain rule,
    with relu'(z) = 1 for z > 0 and 0 otherwise."""
    w1, b1, w2, b2, w3, b3 = params
    x, z1, y1, z2, y2 = cache
    dw3, db3 = conv3d_backward_weight(y2, dout)
    dz2 = conv3d_backward_data(dout, w3) * (z2 > 0)
    dw2, db2 = conv3d_backward_weight(y1, dz2)
    dz1 = conv3d_backward_data(dz2, w2) * (z1 > 0)
    dw1, db1 = conv3d_backward_weight(x, dz1)
    return dw1, db1, dw2, db2, dw3, db3


def adam_step(param, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected, t >= 1:
    m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    p <- p - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).  Returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64 (the values the GPU stores)."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
