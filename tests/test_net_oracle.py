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
    x = rng.normal(size=(12, 3, 4, 4))
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
    import oracle
    f = np.zeros((4, 5, 6), np.float32)
    fh = f.copy()
    fh[0, 0, 0] = np.float32(5e-4)
    bits = np.zeros((4, 5, 6), np.uint8)
    bits[1, 2, 3] = 0b1010
    x = nr.features(f, fh, 1e-3, bits, 1.0, oracle.dirs(f), oracle.dirs(fh))
    assert x.shape == (12, 4, 5, 6)
    assert np.all(x[7] == 0)                         # constant f: no local structure
    assert np.allclose(x[1], 0.25)                   # log10(1e-3)/4 + 1
    assert x[3, 1, 2, 3] == 1 and x[5, 1, 2, 3] == 1 and x[2].sum() == 0 and x[4].sum() == 0
    assert np.isclose(x[6, 0, 0, 0], 0.5) and np.count_nonzero(x[6]) == 1
    # the bump is 7/8 above the mean of its 2x2x2 corner block
    assert np.isclose(x[0, 0, 0, 0], 0.5 * 7 / 8)


def test_target_channels_on_a_hand_built_case():
    """The FPmin counterexample field: the only false case is FPmin at vertex 4,
    whose f-descent neighbour is vertex 1 (the loop edits exactly vertex 1)."""
    import oracle
    f = np.array([.80, .48, .30, .85, .50, .90, .75, .95, .99], np.float32).reshape(1, 3, 3)
    fh = f.copy().ravel()
    fh[4], fh[1] = np.float32(.46), np.float32(.52)
    fh = fh.reshape(1, 3, 3)
    bits = oracle.case_flags(f[0], fh[0])[None]
    df, dh = oracle.dirs(f), oracle.dirs(fh)
    x = nr.features(f, fh, 0.05, bits, 0.69, df, dh)
    assert x[3].ravel()[4] == 1 and x[2:6].sum() == 1        # FPmin at 4 only
    assert x[8].ravel()[1] == 1 and x[8].sum() == 1          # its target: dn_f(4) = 1
    assert x[9].sum() == 0
    # brute force of the direction-difference targets
    uf, dnf = (a.ravel() for a in df)
    uh, dnh = (a.ravel() for a in dh)
    want10 = np.zeros(9)
    want11 = np.zeros(9)
    for u in range(9):
        if dnh[u] != dnf[u] and dnf[u] != u:
            want10[dnf[u]] = 1
        if uh[u] != uf[u] and uh[u] != u:
            want11[uh[u]] = 1
    assert np.array_equal(x[10].ravel(), want10) and np.array_equal(x[11].ravel(), want11)


def test_weighted_mse_gradient():
    rng = np.random.default_rng(8)
    p = rng.normal(size=(3, 4, 5))
    t = np.where(rng.uniform(size=p.shape) < 0.5, 0.0, rng.uniform(0.5, 2.0, size=p.shape))
    lo, g = nr.mse_loss(p, t, edit_weight=7.0)
    # closed form on one vertex of each kind
    pos = np.argwhere(t > 0)[0]
    zer = np.argwhere(t == 0)[0]
    assert np.isclose(g[tuple(pos)], 2 * 8.0 * (p[tuple(pos)] - t[tuple(pos)]) / p.size)
    assert np.isclose(g[tuple(zer)], 2 * 1.0 * p[tuple(zer)] / p.size)
    h = 1e-7
    for _ in range(10):
        idx = tuple(rng.integers(0, s) for s in p.shape)
        e = np.zeros_like(p); e[idx] = h
        num = (nr.mse_loss(p + e, t, 7.0)[0] - nr.mse_loss(p - e, t, 7.0)[0]) / (2 * h)
        assert abs(num - g[idx]) < 1e-6


def test_halve32_matches_c_oracle_and_chain_lengths():
    import oracle
    rng = np.random.default_rng(9)
    L = rng.uniform(0, 1, 4000).astype(np.float32)
    g = (L + rng.uniform(0, 0.1, 4000) * rng.integers(0, 2, 4000)).astype(np.float32)
    ref = np.array([oracle.halve(a, b) for a, b in zip(g, L)], np.float32)
    assert np.array_equal(nr.halve32(g, L).view(np.uint32), ref.view(np.uint32))
    # closed-form chain lengths down to L = 0: a power of two 2^p takes p + 150
    # steps (exact halvings to 2^-149, then one rounding to 0); 0.1f takes 147
    zero = np.zeros(1, np.float32)
    for start, n in ((2.0 ** -3, 147), (2.0 ** -20, 130), (0.1, 147)):
        k = nr.halving_count(np.array([start], np.float32), zero, zero, limit=400)
        assert k[0] == n


def test_halving_count_inverts_repeated_halving():
    import oracle
    rng = np.random.default_rng(10)
    f = rng.uniform(0, 1, 500).astype(np.float32)
    xi = np.float32(0.01)
    L = oracle.lower_bound(f, xi)
    k = rng.integers(0, 6, 500)
    g = f.copy()
    for i in range(500):
        for _ in range(k[i]):
            g[i] = oracle.halve(g[i], L[i])
    got = nr.halving_count(f, g, L)
    # a count is unique unless the chain has already reached L (then any larger count also gives L)
    assert np.all((got == k) | ((g == L) & (got <= k)))
    off = g.copy()
    off[3] = np.nextafter(f[3], np.float32(2))                  # above fhat: not on the chain
    assert nr.halving_count(f, off, L)[3] == -1


def test_warm_start_counts():
    import oracle
    fh = np.full(7, 0.5, np.float32)
    L = oracle.lower_bound(fh, np.float32(0.05))
    p = np.array([0.49, 0.5, 1.49, 1.5, -3.0, np.nan, 1e9], np.float32)
    g = nr.warm_start(p, fh, L, 0.5)
    one = oracle.halve(np.float32(0.5), L[0])
    two = oracle.halve(one, L[0])
    assert g[0] == 0.5 and g[1] == one and g[2] == one and g[3] == two
    assert g[4] == 0.5 and g[5] == 0.5
    assert g[6] == L[0]                                         # 64 halvings run past the 22-step chain
