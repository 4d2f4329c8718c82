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

Network (edit predictor): conv(12->16) ReLU, conv(16->16) ReLU, conv(16->1),
giving p, the predicted number of halvings (Eqs. 2-6) the correction loop
applies to the vertex.  Every edit of the loop moves g_i one step down the
chain fhat_i, halve(fhat_i), halve(halve(fhat_i)), ... towards L_i, so a
count reproduces an edit bit-exactly.  The output layer is linear (a ReLU
there can switch the whole output off for good while training on
mostly-zero targets).  The warm start applies k_i = floor(p_i - p_min) + 1
halvings, clamped to [0, 64] (p_min = 1/2 rounds p to the nearest count).
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
CHANNELS = (12, 16, 16, 1)
N_FEATURES = 12
MAX_WARM_HALVINGS = 64


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


def features(f: np.ndarray, fhat: np.ndarray, xi: float, case_bits: np.ndarray, value_range: float,
             dirs_f, dirs_h) -> np.ndarray:
    """The twelve input channels of a field shaped (nz, ny, nx).  dirs_f and
    dirs_h are the (up, dn) steepest-neighbour ids of f and fhat.
      0  (fhat - 3x3x3 box mean of fhat) / xi, clamped to [-8, 8]
      1  log10(xi / value_range) / 4 + 1      (constant over the field)
      2..5  the four false-critical-point flags of fhat against f
            (FPmax, FPmin, FNmax, FNmin; bits 0..3 of case_bits)
      6  (fhat - f) / xi, clamped to [-8, 8]  (room above the floor f - xi)
      7  (f - 3x3x3 box mean of f) / xi, clamped to [-8, 8]
      8  the vertex is dn_f(u) of an FPmin vertex u (that case's edit target)
      9  the vertex is up_fhat(u) of an FNmax vertex u (that case's edit target)
      10 the vertex is dn_f(u) of a neighbour u whose descent differs (dn_fhat(u) != dn_f(u))
      11 the vertex is up_fhat(u) of a neighbour u whose ascent differs (up_fhat(u) != up_f(u))."""
    x = np.zeros((N_FEATURES,) + fhat.shape, dtype=np.float64)
    f64, h64 = f.astype(np.float64), fhat.astype(np.float64)
    x[0] = np.clip((h64 - box_mean(fhat)) / float(xi), -8.0, 8.0)
    x[1] = np.log10(float(xi) / float(value_range)) / 4.0 + 1.0
    for t in range(4):
        x[2 + t] = (case_bits >> t) & 1
    x[6] = np.clip((h64 - f64) / float(xi), -8.0, 8.0)
    x[7] = np.clip((f64 - box_mean(f)) / float(xi), -8.0, 8.0)
    uf, df = (np.asarray(a).ravel() for a in dirs_f)
    uh, dh = (np.asarray(a).ravel() for a in dirs_h)
    ids = np.arange(uf.size)
    sources = [
        ((case_bits.ravel() >> 1) & 1).astype(bool), df,       # FPmin u -> dn_f(u)
        ((case_bits.ravel() >> 2) & 1).astype(bool), uh,       # FNmax u -> up_fhat(u)
        (dh != df) & (df != ids), df,                          # descent differs -> dn_f(u)
        (uh != uf) & (uh != ids), uh,                          # ascent differs -> up_fhat(u)
    ]
    for c in range(4):
        sel, tgt = sources[2 * c], sources[2 * c + 1]
        flat = np.zeros(uf.size)
        flat[tgt[sel]] = 1.0
        x[8 + c] = flat.reshape(fhat.shape)
    return x


def halve32(g: np.ndarray, L: np.ndarray) -> np.ndarray:
    """One decreasing edit in float32 (Eqs. 2-6 read with the float floor L):
    fl(fl(g + L) * 0.5), or L itself when that leaves g unchanged."""
    g = np.asarray(g, dtype=np.float32)
    L = np.asarray(L, dtype=np.float32)
    h = (g + L).astype(np.float32) * np.float32(0.5)
    return np.where(h == g, L, h).astype(np.float32)


def halving_count(fhat: np.ndarray, g: np.ndarray, L: np.ndarray, limit: int = 256) -> np.ndarray:
    """Number of halvings that take fhat_i to g_i (-1 where g_i is not on the chain)."""
    cur = np.asarray(fhat, dtype=np.float32).copy()
    g = np.asarray(g, dtype=np.float32)
    k = np.zeros(cur.shape, dtype=np.int64)
    for _ in range(limit):
        act = (cur != g) & (cur > g)
        if not act.any():
            break
        cur[act] = halve32(cur[act], L[act])
        k[act] += 1
    k[cur != g] = -1
    return k


def warm_start(p: np.ndarray, fhat: np.ndarray, L: np.ndarray, p_min: float) -> np.ndarray:
    """g0_i = fhat_i halved k_i times, k_i = floor(fl32(p_i - p_min)) + 1 clamped to
    [0, MAX_WARM_HALVINGS] (0 where p_i is not a number)."""
    q = np.floor((np.asarray(p, np.float32) - np.float32(p_min)).astype(np.float32)) + 1.0
    q = np.where(np.isnan(q), 0.0, q)
    k = np.clip(q, 0, MAX_WARM_HALVINGS).astype(np.int64)
    g = np.asarray(fhat, dtype=np.float32).copy()
    for j in range(MAX_WARM_HALVINGS):
        act = k > j
        if not act.any():
            break
        g[act] = halve32(g[act], L[act])
    return g


def adam_step(w, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (bias-corrected); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
