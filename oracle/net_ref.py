"""CPU oracle of the learned warm start: features, a 3-layer 3x3x3 conv net,
its gradients, the loss and the optimiser step.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy in float64
with explicit loops over the 27 taps; no blocking or fusion.  The only
precision the method fixes is BF16 weights and activations with FP32
accumulation; ``bf16`` reproduces the BF16 rounding (round to nearest even)
where the GPU stores BF16, and everything else stays in float64.

Layouts: activations are channel-first ``[C, nz, ny, nx]``; weights
``[C_out, C_in, 3, 3, 3]`` indexed by (dz+1, dy+1, dx+1); biases ``[C_out]``.
Outside the grid the input counts as zero (zero padding).

Network (edit-magnitude predictor): conv(6->16) ReLU, conv(16->16) ReLU,
conv(16->1), giving p, the predicted edit in units of xi.  The output layer
is linear (a ReLU there can switch the whole output off for good while
training on mostly-zero targets); the warm start clamps fhat - p*xi into
[L, fhat], so a negative p means "no edit".
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
CHANNELS = (6, 16, 16, 1)
N_FEATURES = 6


def bf16(a) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def _shift(x: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """out[..., z, y, x] = x[..., z+dz, y+dy, x+dx], zero outside the grid."""
    out = np.zeros_like(x)
    nz, ny, nx = x.shape[-3:]

    def rng(d, n):
        src = slice(max(d, 0), n + min(d, 0))
        dst = slice(max(-d, 0), n + min(-d, 0))
        return src, dst

    sz, tz = rng(dz, nz)
    sy, ty = rng(dy, ny)
    sx, tx = rng(dx, nx)
    out[..., tz, ty, tx] = x[..., sz, sy, sx]
    return out


def conv3d(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[co] = b[co] + sum_ci sum_taps W[co, ci, tap] * x[ci] shifted by the tap."""
    cout = W.shape[0]
    y = np.zeros((cout,) + x.shape[1:], dtype=np.float64)
    for (dz, dy, dx) in TAPS:
        xs = _shift(x, dz, dy, dx)                       # [ci, z, y, x]
        w = W[:, :, dz + 1, dy + 1, dx + 1]               # [co, ci]
        y += np.tensordot(w, xs, axes=([1], [0]))
    y += b.reshape((-1, 1, 1, 1))
    return y


def conv3d_backward(x: np.ndarray, W: np.ndarray, dy: np.ndarray):
    """Gradients of conv3d with respect to x, W and b, given dL/dy."""
    dx = np.zeros_like(x, dtype=np.float64)
    dW = np.zeros_like(W, dtype=np.float64)
    for (dz, dyy, dxx) in TAPS:
        xs = _shift(x, dz, dyy, dxx)
        w = W[:, :, dz + 1, dyy + 1, dxx + 1]             # [co, ci]
        dW[:, :, dz + 1, dyy + 1, dxx + 1] = np.tensordot(dy, xs, axes=([1, 2, 3], [1, 2, 3]))
        g = np.tensordot(w, dy, axes=([0], [0]))          # [ci, z, y, x] at the shifted position
        dx += _shift(g, -dz, -dyy, -dxx)
    db = dy.sum(axis=(1, 2, 3))
    return dx, dW, db


def init_params(seed: int = 0):
    """He-style uniform init (float64), weights then rounded to bf16 for use."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        bound = np.sqrt(6.0 / (cin * 27))
        W = rng.uniform(-bound, bound, size=(cout, cin, 3, 3, 3))
        b = np.zeros(cout)
        params.append((W, b))
    return params


def forward(x: np.ndarray, params, round_bf16: bool = True):
    """Returns (p, cache).  With round_bf16 the weights and every stored
    activation (input, hidden layers) are BF16 while sums stay exact."""
    acts = [bf16(x) if round_bf16 else x.astype(np.float64)]
    pre = []
    for li, (W, b) in enumerate(params):
        Wq = bf16(W) if round_bf16 else W
        z = conv3d(acts[-1], Wq, b)
        pre.append(z)
        if li < len(params) - 1:
            a = np.maximum(z, 0.0)
            acts.append(bf16(a) if round_bf16 else a)
        else:
            acts.append(z)
    return acts[-1][0], (acts, pre, params, round_bf16)


def backward(cache, dp: np.ndarray):
    """Parameter gradients [(dW, db), ...] for dL/dp."""
    acts, pre, params, round_bf16 = cache
    grads = [None] * len(params)
    g = dp[None].astype(np.float64)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        Wq = bf16(W) if round_bf16 else W
        if li < len(params) - 1:
            g = g * (pre[li] > 0)
        dx, dW, db = conv3d_backward(acts[li], Wq, g)
        grads[li] = (dW, db)
        g = dx
    return grads


def mse_loss(p: np.ndarray, t: np.ndarray, edit_weight: float = 0.0):
    """Weighted mean squared error over all vertices and its gradient: vertex i
    weighs 1 + edit_weight when its target edit t_i is positive, else 1."""
    d = p - t
    n = d.size
    w = 1.0 + edit_weight * (t > 0)
    return float((w * d * d).sum() / n), 2.0 * w * d / n


def box_mean(h: np.ndarray) -> np.ndarray:
    """Mean of h over the 3x3x3 box around each vertex, counting in-grid vertices only."""
    s = np.zeros(h.shape, dtype=np.float64)
    c = np.zeros(h.shape, dtype=np.float64)
    one = np.ones(h.shape, dtype=np.float64)
    for (dz, dy, dx) in TAPS:
        s += _shift(h.astype(np.float64), dz, dy, dx)
        c += _shift(one, dz, dy, dx)
    return s / c


def features(fhat: np.ndarray, xi: float, case_bits: np.ndarray, value_range: float) -> np.ndarray:
    """The six input channels of a field shaped (nz, ny, nx):
      0  (fhat - 3x3x3 box mean of fhat) / xi, clamped to [-8, 8]
      1  log10(xi / value_range) / 4 + 1      (constant over the field)
      2..5  the four false-critical-point flags of fhat against f
            (FPmax, FPmin, FNmax, FNmin; bits 0..3 of case_bits)."""
    x = np.zeros((N_FEATURES,) + fhat.shape, dtype=np.float64)
    local = (fhat.astype(np.float64) - box_mean(fhat)) / float(xi)
    x[0] = np.clip(local, -8.0, 8.0)
    x[1] = np.log10(float(xi) / float(value_range)) / 4.0 + 1.0
    for t in range(4):
        x[2 + t] = (case_bits >> t) & 1
    return x


def adam_step(w, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (bias-corrected); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
