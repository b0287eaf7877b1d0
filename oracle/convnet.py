"""Oracle for the learned initial guess: a panel-wise 3-D convolutional
network and its online training, in plain NumPy FP64.

TEST INFRASTRUCTURE ONLY -- imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark; never by the product path.

What is computed (the learned-guess growth direction of the solver, whose
GMRES initial guess the paper takes from the previous time step, Sec. 3.3):

* tensors are channels-last per panel, ``X[p, d, h, w, c]`` with p the six
  panels as a batch, (d, h, w) = (k, j, i) of the cell and c the channel --
  the solver's vector layout ``[6][Nr][N][N][4]`` is this with c = 4;
* ``conv(X, W, b)``: 3x3x3 correlation with zero padding inside each panel
  (panels are independent volumes), ``W[co, t, ci]`` with tap
  ``t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1)``:
  ``Y[p, d, h, w, co] = b[co] + sum_{t, ci} X[p, d+dz, h+dy, w+dx, ci] W[co, t, ci]``;
* ``pool``: mean over 2x2x2 blocks; ``up``: copy to the 2x2x2 children;
* network with channel widths (c0, c1, c2, c3), four resolution levels and
  additive skips::

      e0 = relu(conv0(x))            in  -> c0   (full resolution)
      e1 = relu(conv1(pool(e0)))     c0  -> c1
      e2 = relu(conv2(pool(e1)))     c1  -> c2
      e3 = relu(conv3(pool(e2)))     c2  -> c3   (1/8 resolution)
      d2 = relu(conv4(up(e3)) + e2)  c3  -> c2
      d1 = relu(conv5(up(d2)) + e1)  c2  -> c1
      d0 = relu(conv6(up(d1)) + e0)  c1  -> c0
      y  = conv7(d0)                 c0  -> 4

* features: ``a = x^{n-1} / s``, ``e = (x^{n-1} - x^{n-2}) / s_d`` with s and
  s_d the per-component RMS over all cells (8 input channels); the guess is
  ``2 x^{n-1} - x^{n-2} + s_d * y`` (a correction to linear extrapolation);
* loss: mean over cells and the 4 components of ``(y - t)^2`` with
  ``t = (x^n - 2 x^{n-1} + x^{n-2}) / s_d``;
* Adam with bias correction on every weight and bias.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (32, 48, 64, 128)
ADAM = dict(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8)


def tap_offsets():
    """Offsets (dz, dy, dx) of the 27 taps in tap order."""
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))


def conv_fwd(x, w, b=None):
    """Y = conv(X, W) + b; x [P, D, H, W, Ci], w [Co, 27, Ci]."""
    P, D, H, Wd, _ = x.shape
    xp = _pad(x)
    y = np.zeros((P, D, H, Wd, w.shape[0]))
    for t, (dz, dy, dx) in enumerate(tap_offsets()):
        xs = xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd, :]
        y += xs @ w[:, t, :].T
    if b is not None:
        y += b
    return y


def conv_bwd_data(dy, w):
    """dX = dL/dX of Y = conv(X, W) given dY = dL/dY."""
    P, D, H, Wd, _ = dy.shape
    dxp = np.zeros((P, D + 2, H + 2, Wd + 2, w.shape[2]))
    for t, (dz, dy_, dx) in enumerate(tap_offsets()):
        dxp[:, 1 + dz:1 + dz + D, 1 + dy_:1 + dy_ + H, 1 + dx:1 + dx + Wd, :] += dy @ w[:, t, :]
    return dxp[:, 1:-1, 1:-1, 1:-1, :]


def conv_bwd_weight(x, dy):
    """(dW, db) of Y = conv(X, W) + b given dY."""
    P, D, H, Wd, Ci = x.shape
    Co = dy.shape[-1]
    xp = _pad(x)
    dw = np.zeros((Co, 27, Ci))
    dyf = dy.reshape(-1, Co)
    for t, (dz, dy_, dx) in enumerate(tap_offsets()):
        xs = xp[:, 1 + dz:1 + dz + D, 1 + dy_:1 + dy_ + H, 1 + dx:1 + dx + Wd, :].reshape(-1, Ci)
        dw[:, t, :] = dyf.T @ xs
    return dw, dyf.sum(axis=0)


def pool(x):
    P, D, H, W, C = x.shape
    return x.reshape(P, D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4, 6))


def up(x):
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def layer_shapes(widths=WIDTHS, cin=8, cout=4):
    c0, c1, c2, c3 = widths
    return [(c0, cin), (c1, c0), (c2, c1), (c3, c2), (c2, c3), (c1, c2), (c0, c1), (cout, c0)]


def param_count(widths=WIDTHS):
    return sum(co * 27 * ci + co for co, ci in layer_shapes(widths))


def unflatten(flat, widths=WIDTHS):
    """[(W, b)] in FP64 from the flat layout: per layer W[co][27][ci], then b[co]."""
    out, off = [], 0
    for co, ci in layer_shapes(widths):
        w = np.asarray(flat[off:off + co * 27 * ci], dtype=np.float64).reshape(co, 27, ci)
        off += co * 27 * ci
        b = np.asarray(flat[off:off + co], dtype=np.float64).copy()
        off += co
        out.append([w, b])
    assert off == len(flat)
    return out


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def _keep(bf16):
    """Storage rounding of a tensor: identity in FP64, or rounding to BF16 when the
    network is emulated with BF16 activations and gradients (every tensor that is
    stored between layers; sums inside a layer stay FP64)."""
    return bf16_round if bf16 else (lambda v: v)


def forward(params, x, bf16=False):
    """Network forward; returns y and the activations the backward needs.  With
    bf16=True every stored activation is rounded to BF16 (the output y is not)."""
    relu = lambda v: np.maximum(v, 0.0)
    k = _keep(bf16)
    (w0, b0), (w1, b1), (w2, b2), (w3, b3), (w4, b4), (w5, b5), (w6, b6), (w7, b7) = params
    a = {"x": x}
    a["e0"] = k(relu(conv_fwd(x, w0, b0)))
    a["p0"] = k(pool(a["e0"]))
    a["e1"] = k(relu(conv_fwd(a["p0"], w1, b1)))
    a["p1"] = k(pool(a["e1"]))
    a["e2"] = k(relu(conv_fwd(a["p1"], w2, b2)))
    a["p2"] = k(pool(a["e2"]))
    a["e3"] = k(relu(conv_fwd(a["p2"], w3, b3)))
    a["u3"] = up(a["e3"])
    a["d2"] = k(relu(conv_fwd(a["u3"], w4, b4) + a["e2"]))
    a["u2"] = up(a["d2"])
    a["d1"] = k(relu(conv_fwd(a["u2"], w5, b5) + a["e1"]))
    a["u1"] = up(a["d1"])
    a["d0"] = k(relu(conv_fwd(a["u1"], w6, b6) + a["e0"]))
    y = conv_fwd(a["d0"], w7, b7)
    return y, a


def backward(params, a, dy, bf16=False):
    """Gradients [(dW, db)] of the loss for every layer, given dL/dy.  With
    bf16=True, dy and every stored intermediate gradient is rounded to BF16."""
    g = [None] * 8
    mask = lambda v: (v > 0).astype(np.float64)
    k = _keep(bf16)
    dy = k(dy)
    g[7] = conv_bwd_weight(a["d0"], dy)
    dz6 = k(conv_bwd_data(dy, params[7][0]) * mask(a["d0"]))  # pre-activation of d0
    g[6] = conv_bwd_weight(a["u1"], dz6)
    dd1 = pool(k(conv_bwd_data(dz6, params[6][0]))) * 8.0  # adjoint of up = sum over children
    dz5 = k(dd1 * mask(a["d1"]))
    g[5] = conv_bwd_weight(a["u2"], dz5)
    dz4 = k(pool(k(conv_bwd_data(dz5, params[5][0]))) * 8.0 * mask(a["d2"]))
    g[4] = conv_bwd_weight(a["u3"], dz4)
    dz3 = k(pool(k(conv_bwd_data(dz4, params[4][0]))) * 8.0 * mask(a["e3"]))
    g[3] = conv_bwd_weight(a["p2"], dz3)
    # e2 feeds pool -> conv3 and the skip into d2's pre-activation
    dz2 = k((up(k(conv_bwd_data(dz3, params[3][0]))) / 8.0 + dz4) * mask(a["e2"]))
    g[2] = conv_bwd_weight(a["p1"], dz2)
    dz1 = k((up(k(conv_bwd_data(dz2, params[2][0]))) / 8.0 + dz5) * mask(a["e1"]))
    g[1] = conv_bwd_weight(a["p0"], dz1)
    dz0 = k((up(k(conv_bwd_data(dz1, params[1][0]))) / 8.0 + dz6) * mask(a["e0"]))
    g[0] = conv_bwd_weight(a["x"], dz0)
    return [list(t) for t in g]


def loss_and_grad(y, t):
    """Mean squared error over all entries and its gradient."""
    diff = y - t
    return float((diff**2).mean()), 2.0 * diff / diff.size


def features(xm1, xm2, eps=1e-30):
    """Inputs and scales from the previous two solutions ([6,Nr,N,N,4] each)."""
    d = xm1 - xm2
    s = np.sqrt((xm1**2).mean(axis=(0, 1, 2, 3))) + eps
    sd = np.sqrt((d**2).mean(axis=(0, 1, 2, 3))) + eps
    return np.concatenate([xm1 / s, d / sd], axis=-1), s, sd


def target(xn, xm1, xm2, sd):
    return (xn - 2.0 * xm1 + xm2) / sd


def guess(params, xm1, xm2):
    x, _, sd = features(xm1, xm2)
    y, _ = forward(params, x)
    return 2.0 * xm1 - xm2 + sd * y


class Adam:
    """Adam with bias correction (Kingma and Ba), one moment pair per tensor."""

    def __init__(self, params, lr=ADAM["lr"], beta1=ADAM["beta1"], beta2=ADAM["beta2"], eps=ADAM["eps"]):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [[np.zeros_like(w), np.zeros_like(b)] for w, b in params]
        self.v = [[np.zeros_like(w), np.zeros_like(b)] for w, b in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1, c2 = 1.0 - self.b1**self.t, 1.0 - self.b2**self.t
        for li in range(len(params)):
            for q in range(2):
                g = grads[li][q]
                self.m[li][q] = self.b1 * self.m[li][q] + (1 - self.b1) * g
                self.v[li][q] = self.b2 * self.v[li][q] + (1 - self.b2) * g * g
                params[li][q] = params[li][q] - self.lr * (self.m[li][q] / c1) / (np.sqrt(self.v[li][q] / c2) + self.eps)
        return params


def train_step(params, opt, xm2, xm1, xn):
    """One Adam step on the sample (x^{n-2}, x^{n-1}) -> x^n; returns the loss."""
    x, _, sd = features(xm1, xm2)
    y, a = forward(params, x)
    loss, dy = loss_and_grad(y, target(xn, xm1, xm2, sd))
    opt.step(params, backward(params, a, dy))
    return loss


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
