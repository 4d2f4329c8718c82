"""Pins of the learned-path oracle (oracle/net_ref.py) against library
primitives and finite differences; nothing here re-types the oracle's formulas."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from oracle import net_ref as nr


def test_bf16_matches_torch_rounding():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.normal(size=20000).astype(np.float32) * 10.0 ** rng.integers(-20, 20, 20000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, -0.0], np.float32)])
    a = a.astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(nr.bf16(a), ref)


def test_conv3d_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 5, 6, 7))
    W = rng.normal(size=(4, 3, 3, 3, 3))
    b = rng.normal(size=4)
    y = nr.conv3d(x, W, b)
    for co in range(4):
        ref = np.full(x.shape[1:], b[co])
        for ci in range(3):
            ref += ndi.correlate(x[ci], W[co, ci], mode="constant", cval=0.0)
        assert np.allclose(y[co], ref, rtol=1e-12, atol=1e-12)


def test_conv3d_backward_central_differences():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 3, 4, 5))
    W = rng.normal(size=(3, 2, 3, 3, 3))
    b = rng.normal(size=3)
    R = rng.normal(size=(3, 3, 4, 5))
    loss = lambda x_, W_, b_: float((nr.conv3d(x_, W_, b_) * R).sum())
    dx, dW, db = nr.conv3d_backward(x, W, R)
    h = 1e-6
    for _ in range(25):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        e = np.zeros_like(x); e[idx] = h
        assert abs((loss(x + e, W, b) - loss(x - e, W, b)) / (2 * h) - dx[idx]) < 1e-6
        idw = tuple(rng.integers(0, s) for s in W.shape)
        e = np.zeros_like(W); e[idw] = h
        assert abs((loss(x, W + e, b) - loss(x, W - e, b)) / (2 * h) - dW[idw]) < 1e-6
    for co in range(3):
        e = np.zeros_like(b); e[co] = h
        assert abs((loss(x, W, b + e) - loss(x, W, b - e)) / (2 * h) - db[co]) < 1e-6


def test_network_gradients_central_differences():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(6, 3, 4, 4))
    t = np.abs(rng.normal(size=(3, 4, 4)))
    params = nr.init_params(5)
    params = [(W, rng.normal(size=b.shape) * 0.1 + 0.2) for W, b in params]

    def L(ps):
        p, _ = nr.forward(x, ps, round_bf16=False)
        return nr.mse_loss(p, t)[0]

    p, cache = nr.forward(x, params, round_bf16=False)
    _, dp = nr.mse_loss(p, t)
    grads = nr.backward(cache, dp)
    h = 1e-6
    for li in range(3):
        W, b = params[li]
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h; Wm[idx] -= h
            pp = list(params); pp[li] = (Wp, b)
            pm = list(params); pm[li] = (Wm, b)
            num = (L(pp) - L(pm)) / (2 * h)
            assert abs(num - grads[li][0][idx]) < 1e-5 * max(1.0, abs(num))


def test_mse_gradient():
    rng = np.random.default_rng(4)
    p, t = rng.normal(size=(4, 5, 6)), rng.normal(size=(4, 5, 6))
    _, g = nr.mse_loss(p, t)
    h = 1e-7
    for _ in range(10):
        idx = tuple(rng.integers(0, s) for s in p.shape)
        e = np.zeros_like(p); e[idx] = h
        assert abs((nr.mse_loss(p + e, t)[0] - nr.mse_loss(p - e, t)[0]) / (2 * h) - g[idx]) < 1e-6


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    w0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    wt = torch.tensor(w0.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads, start=1):
        opt.zero_grad()
        wt.grad = torch.tensor(g)
        opt.step()
        w, m, v = nr.adam_step(w, g, m, v, k, 3e-3)
    assert np.allclose(w, wt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_box_mean_interior_and_boundary():
    rng = np.random.default_rng(6)
    h = rng.normal(size=(5, 6, 7))
    bm = nr.box_mean(h)
    assert np.allclose(bm[1:-1, 1:-1, 1:-1], ndi.uniform_filter(h, size=3, mode="constant")[1:-1, 1:-1, 1:-1])
    # corner: mean of the 8 in-grid vertices of the 2x2x2 corner block
    assert np.isclose(bm[0, 0, 0], h[:2, :2, :2].mean())
    assert np.isclose(bm[4, 5, 6], h[3:, 4:, 5:].mean())


def test_features_channels():
    f = np.zeros((4, 5, 6), np.float32)
    bits = np.zeros((4, 5, 6), np.uint8)
    bits[1, 2, 3] = 0b1010
    x = nr.features(f, 1e-3, bits, 1.0)
    assert x.shape == (6, 4, 5, 6)
    assert np.all(x[0] == 0)                         # constant field: no local structure
    assert np.allclose(x[1], 0.25)                   # log10(1e-3)/4 + 1
    assert x[3, 1, 2, 3] == 1 and x[5, 1, 2, 3] == 1 and x[2].sum() == 0 and x[4].sum() == 0
