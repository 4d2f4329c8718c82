"""GPU parity of the learned warm start: BF16/MFMA convolution kernels, their
gradients, the optimiser and the warm-started fix, against oracle/net_ref.py.

Tolerances (derived, not tuned):
  * products of BF16 values are exact in FP32; FP32 accumulation of K terms is
    off by at most K * 2^-24 * S, S = sum of |terms| (K <= 432, so < 2^-15 S);
  * a stored BF16 value is off by at most 2^-9 relative (round to nearest);
  * a layer whose input is a BF16 tensor the GPU rounded itself may see any
    element 1 BF16 ulp (2^-8 relative) away from the oracle's, which moves a
    sum by at most 2^-8 * S.
So a pre-activation or gradient sum may differ by (2^-8 + 2^-15) S, a stored
BF16 output additionally by 2^-8 of itself; the tests allow 2^-7 S + 2^-8 |y|.
"""
import numpy as np
import pytest

import oracle
from oracle import net_ref as nr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def msz():
    import paper_2406_09423_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def flat_params(params) -> np.ndarray:
    """Oracle (W[co][ci][3][3][3], b) per layer -> the library's flat FP32 layout."""
    out = []
    cin_store = (16, 16, 16)
    for li, (W, b) in enumerate(params):
        co, ci = W.shape[:2]
        Wt = W.reshape(co, ci, 27).transpose(2, 1, 0)           # [tap][ci][co]
        if li < 2:
            full = np.zeros((27, cin_store[li], 16))
            full[:, :ci, :co] = Wt
            out += [full.ravel(), b.astype(np.float64)]
        else:
            out += [Wt[:, :, 0].ravel(), b.astype(np.float64)]
    flat = np.concatenate(out).astype(np.float32)
    assert flat.size == 14289
    return flat


def unflat_grads(g: np.ndarray):
    """Library gradient layout -> oracle shapes (dW[co][ci][3][3][3], db)."""
    o = 0
    res = []
    for li, (cin, cstore, cout) in enumerate(((12, 16, 16), (16, 16, 16), (16, 16, 1))):
        if li < 2:
            W = g[o:o + 27 * cstore * 16].reshape(27, cstore, 16)[:, :cin, :cout]
            o += 27 * cstore * 16
        else:
            W = g[o:o + 27 * 16].reshape(27, 16, 1)
            o += 27 * 16
        b = g[o:o + cout]
        o += cout
        res.append((W.transpose(2, 1, 0).reshape(cout, cin, 3, 3, 3).astype(np.float64), b.astype(np.float64)))
    return res


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """float values (already BF16-representable) -> raw int16 bits."""
    return (nr.bf16(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def bits_to_float(b: np.ndarray) -> np.ndarray:
    return (b.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def feature_case(shape, seed, xi=0.01):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0, 1, size=shape).astype(np.float32)
    fh = (f + rng.uniform(-xi, xi, size=shape)).astype(np.float32)
    fh = np.where(np.abs(f.astype(np.float64) - fh) > xi, f, fh).astype(np.float32)
    bits = oracle.case_flags(f, fh) if len(shape) == 3 else oracle.case_flags(f[0], fh[0])[None]
    x = nr.features(f, fh, xi, bits & 15, float(f.max()) - float(f.min()), oracle.dirs(f), oracle.dirs(fh))
    return f, fh, np.float32(xi), x


def to_dev_feat(x: np.ndarray):
    n = x[0].size
    feat = np.zeros((n, 16))
    feat[:, :12] = x.reshape(12, -1).T
    return torch.from_numpy(bf16_bits(feat)).cuda()


def random_params(seed):
    rng = np.random.default_rng(seed)
    params = nr.init_params(seed)
    return [(W, rng.uniform(0.0, 0.2, size=b.shape)) for W, b in params]


SHAPES = [(6, 9, 20), (1, 17, 33), (9, 8, 16)]


@pytest.mark.parametrize("shape", SHAPES)
def test_features_match_oracle(msz, shape):
    f, fh, xi, x = feature_case(shape, 1)
    got = msz.net_features(torch.from_numpy(f).cuda(), torch.from_numpy(fh).cuda(), xi).cpu().numpy()
    g = bits_to_float(got)
    ref = nr.bf16(x).reshape(12, -1).T
    assert np.array_equal(g[:, 1:7], ref[:, 1:7])                 # xi channel, flags, fhat - f exactly
    assert np.array_equal(g[:, 8:12], ref[:, 8:12])               # edit-target flags exactly
    assert np.all(g[:, 12:] == 0)
    # box-mean channels: the same double-precision formula summed in another order; one BF16 ulp at most
    for c in (0, 7):
        assert np.all(np.abs(g[:, c] - ref[:, c]) <= 2.0 ** -7 * np.abs(ref[:, c]) + 1e-30), c


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_layers_match_oracle(msz, shape):
    """Every layer's output within the propagated bound: the oracle runs on its own
    activations; the bound of layer l+1 adds conv(|W|, bound of layer l)."""
    f, fh, xi, x = feature_case(shape, 2)
    params = random_params(3)
    flat = torch.from_numpy(flat_params(params)).cuda()
    p, a1, a2 = msz.net_forward(flat, to_dev_feat(x), shape, hidden=True)
    p, a1, a2 = p.cpu().numpy(), bits_to_float(a1.cpu().numpy()), bits_to_float(a2.cpu().numpy())
    act = nr.bf16(x)                  # the GPU is fed exactly these BF16 features
    bound_in = np.zeros_like(act)
    for li, (W, b) in enumerate(params):
        Wq = nr.bf16(W)
        z = nr.conv3d(act, Wq, b)
        S = nr.conv3d(np.abs(act), np.abs(Wq), np.abs(b))
        carried = nr.conv3d(bound_in, np.abs(Wq), np.zeros_like(b))
        y = np.maximum(z, 0.0) if li < 2 else z     # linear output layer
        got = (a1, a2)[li].T[: W.shape[0]].reshape(z.shape) if li < 2 else p.reshape(z[0].shape)[None]
        bound = 2.0 ** -7 * S + carried + 2.0 ** -8 * np.abs(y) + 1e-30
        assert np.all(np.abs(got - y) <= bound), (li, float(np.max(np.abs(got - y) - bound)))
        act = nr.bf16(y) if li < 2 else y
        bound_in = bound + 2.0 ** -8 * np.abs(y)


def _bf16_spread(v, r):
    """The oracle's BF16 rounding c of v, and the largest distance from c of the
    BF16 rounding of any value within r of v (BF16 rounding is monotone, so the
    interval's ends bound it)."""
    c = nr.bf16(v)
    return c, np.maximum(np.abs(c - nr.bf16(v - r)), np.abs(nr.bf16(v + r) - c))


def _layerwise_gradient_bounds(x, params, a1, a2, p, t, edit_weight):
    """The backward pass of the oracle run on the GPU's own forward tensors
    (features x, hidden activations a1, a2, output p), with a per-element
    bound on the GPU's gradients.  Returns [(dW, db, bound_W, bound_b)] per layer.

    dL/dp is reproduced exactly (the GPU's FP32 operations, in its order, then
    BF16).  A weight gradient sum_v dz(v) a(v + tap) on the GPU differs from the
    float64 sum by its FP32 accumulation, at most (n + 16) 2^-23 of the sum of
    |terms| (one rounding per addition on any summation tree, counted at twice
    the round-to-nearest bound), plus sum_v e(v) |a(v + tap)| where the GPU's
    BF16 dz may differ by e.  A data gradient element sums K = 27 x (channels
    of dz) products (27 from the one-channel output gradient, 432 after it),
    off by at most K 2^-23 of its |terms|, and the difference e of its
    input spreads by the transposed convolution of e with |W|; its BF16
    rounding then differs from the oracle's only where that interval
    straddles a rounding boundary.  The ReLU masks come from the GPU's own
    activations, so they agree exactly."""
    n = p.size
    tf = t.astype(np.float32)
    scale = np.float32(2.0) / np.float32(n)
    w = np.where(tf > 0, np.float32(1.0) + np.float32(edit_weight), np.float32(1.0)).astype(np.float32)
    gz = ((scale * w).astype(np.float32) * (p.astype(np.float32) - tf).astype(np.float32)).astype(np.float32)
    dz = nr.bf16(gz)[None]                   # exactly the GPU's dL/dp
    e = np.zeros_like(dz)
    acts = [nr.bf16(x), a1, a2]
    masks = [None, a1 > 0, a2 > 0]
    acc = (n + 16) * 2.0 ** -23
    out = [None] * 3
    for li in (2, 1, 0):
        Wq = nr.bf16(params[li][0])
        a = acts[li]
        _, dW, db = nr.conv3d_backward(a, Wq, dz)
        _, dW_e, db_e = nr.conv3d_backward(np.abs(a), Wq, e)
        _, dW_t, db_t = nr.conv3d_backward(np.abs(a), Wq, np.abs(dz) + e)
        out[li] = (dW, db, dW_e + acc * dW_t + 1e-30, db_e + acc * db_t + 1e-30)
        if li == 0:
            break
        v, _, _ = nr.conv3d_backward(np.zeros_like(a), Wq, dz)
        spread, _, _ = nr.conv3d_backward(np.zeros_like(a), np.abs(Wq), e)
        tot, _, _ = nr.conv3d_backward(np.zeros_like(a), np.abs(Wq), np.abs(dz) + e)
        k_terms = 27 * dz.shape[0]           # non-zero products per element (adding a zero is exact)
        c, e_new = _bf16_spread(v, spread + k_terms * 2.0 ** -23 * tot)
        m = masks[li]
        dz, e = c * m, e_new * m
    return out


def test_gradients_match_oracle(msz):
    """Every parameter gradient element of the GPU's backward pass against the
    oracle's float64 backward run on the GPU's own forward tensors, within the
    per-element bound of _layerwise_gradient_bounds (the forward tensors
    themselves are checked against the oracle's in
    test_forward_layers_match_oracle); and the whole gradient against the
    oracle's own end-to-end float64 backward by norm."""
    shape = (6, 9, 20)
    f, fh, xi, x = feature_case(shape, 4)
    params = random_params(5)
    rng = np.random.default_rng(6)
    t = rng.uniform(0.5, 2.0, size=shape).astype(np.float32)
    flat = torch.from_numpy(flat_params(params)).cuda()
    t[rng.uniform(size=shape) < 0.6] = 0.0      # sparse targets, as in training
    feat = to_dev_feat(x)
    loss, g = msz.net_gradients(flat, feat, torch.from_numpy(t.ravel()).cuda(), shape, edit_weight=4.0)
    gg = unflat_grads(g.cpu().numpy())
    p_g, a1_g, a2_g = msz.net_forward(flat, feat, shape, hidden=True)
    p_g = p_g.cpu().numpy().reshape(shape)
    a1 = bits_to_float(a1_g.cpu().numpy()).T.reshape((16,) + shape)
    a2 = bits_to_float(a2_g.cpu().numpy()).T.reshape((16,) + shape)
    checked = 0
    for li, (dW, db, bW, bb) in enumerate(_layerwise_gradient_bounds(x, params, a1, a2, p_g, t, 4.0)):
        got_W, got_b = gg[li]
        assert got_W.shape == dW.shape and got_b.shape == db.shape
        assert np.all(np.abs(got_W - dW) <= bW), (li, float(np.max(np.abs(got_W - dW) - bW)))
        assert np.all(np.abs(got_b - db) <= bb), (li, float(np.max(np.abs(got_b - db) - bb)))
        # the bound is far below the gradients themselves
        big = np.abs(dW) > 1e-3 * np.abs(dW).max()
        assert np.median(bW[big] / np.abs(dW[big])) < 2.0 ** -6, li
        checked += got_W.size + got_b.size
    assert checked == (16 * 12 + 16 * 16 + 16) * 27 + 16 + 16 + 1   # every element of every tensor
    # end to end against the oracle's own forward and backward (float64 sums, BF16 storage)
    p, cache = nr.forward(x, params, round_bf16=True)
    lo, dp = nr.mse_loss(p, t.astype(np.float64), edit_weight=4.0)
    ref = nr.backward(cache, dp)
    assert abs(loss - lo) <= 2.0 ** -5 * lo
    for li in range(3):
        for k in range(2):
            got, want = gg[li][k], ref[li][k]
            assert np.linalg.norm(got - want) <= 2.0 ** -5 * np.linalg.norm(want) + 1e-12, (li, k)


def test_adam_matches_oracle(msz):
    rng = np.random.default_rng(7)
    w0 = rng.normal(size=14289)
    g = [rng.normal(size=14289) for _ in range(3)]
    w = torch.from_numpy(w0.astype(np.float32)).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    wr, mr, vr = w0.astype(np.float32).astype(np.float64), np.zeros(14289), np.zeros(14289)
    for k, gk in enumerate(g, start=1):
        gt = torch.from_numpy(gk.astype(np.float32)).cuda()
        msz.net_adam(w, gt, m, v, k, 1e-3)
        wr, mr, vr = nr.adam_step(wr, gk.astype(np.float32).astype(np.float64), mr, vr, k, 1e-3)
    assert np.allclose(w.cpu().numpy(), wr, rtol=0, atol=1e-6)


def test_fix_learned_converges(msz):
    """Any prediction only moves the start inside [L, fhat]; the loop still reaches zero error."""
    import synth
    f, fh, xi = synth.turb3d(n=48, nblobs=4)[0]
    params = random_params(8)
    flat = torch.from_numpy(flat_params(params)).cuda()
    fd, fhd = torch.from_numpy(f).cuda(), torch.from_numpy(fh).cuda()
    rc, d, g, st = msz.fix_learned(fd, fhd, xi, flat, timing=True)
    assert rc == msz.OK, st
    cnt = msz.count_false(fd, g)
    assert all(v == 0 for v in cnt.values())
    gh = g.cpu().numpy()
    assert (np.abs(f.astype(np.float64) - gh) <= float(xi)).all()
    assert st["timing"]["net"]["launches"] == 1


def test_halvings_match_oracle(msz):
    rng = np.random.default_rng(11)
    shape = (7, 13, 40)
    f = rng.uniform(0, 1, size=shape).astype(np.float32)
    xi = np.float32(0.02)
    fh = (f + rng.uniform(-xi, xi, size=shape)).astype(np.float32)
    fh = np.where(np.abs(f.astype(np.float64) - fh) > xi, f, fh).astype(np.float32)
    L = oracle.lower_bound(f, xi)
    k = rng.integers(0, 5, size=shape)
    k[0, 0, :8] = 40                                   # runs into the floor
    g = fh.copy()
    for j in range(int(k.max())):
        act = k > j
        g[act] = nr.halve32(g[act], L[act])
    g[1, 1, 1] = np.nextafter(fh[1, 1, 1], np.float32(2))  # above fhat: off the chain
    want = nr.halving_count(fh, g, L)
    got = msz.net_halvings(torch.from_numpy(f).cuda(), torch.from_numpy(fh).cuda(), torch.from_numpy(g).cuda(), xi)
    assert np.array_equal(got.cpu().numpy().astype(np.int64), want)
    assert want[1, 1, 1] == -1


@pytest.mark.parametrize("p_min,merged", [(0.5, False), (0.25, False), (1.5, False), (0.5, True)])
def test_fix_learned_bit_exact_with_oracle(msz, p_min, merged):
    """The warm start from the GPU's own prediction p, recomputed by the oracle,
    then the oracle's loop from it (with merged C rounds too): edits, g and
    round counts bit-identical."""
    import synth
    f, fh, xi = synth.turb3d(n=32, nblobs=4)[0]
    params = random_params(12)
    flat = torch.from_numpy(flat_params(params)).cuda()
    fd, fhd = torch.from_numpy(f).cuda(), torch.from_numpy(fh).cuda()
    feat = msz.net_features(fd, fhd, xi)
    p = msz.net_forward(flat, feat, f.shape).cpu().numpy().reshape(f.shape)
    L = oracle.lower_bound(f, xi)
    g0 = nr.warm_start(p, fh, L, p_min)
    assert (g0 != fh).any()
    rc_o, d_o, g_o, st_o = oracle.fix(f, fh, xi, warm_start=g0, merged_c=merged)
    rc, d, g, st = msz.fix_learned(fd, fhd, xi, flat, p_min=p_min, merged=merged, count_init=True)
    assert rc == rc_o == msz.OK
    assert np.array_equal(d.cpu().numpy().view(np.uint32), d_o.view(np.uint32))
    assert np.array_equal(g.cpu().numpy().view(np.uint32), g_o.view(np.uint32))
    assert list(st["rounds"]) == list(st_o["rounds"]) and st["rounds_r"] == st_o["rounds_r"]
    # the warm start's own mislabelled vertices (before the loop) and false cases
    assert st["mislabel_init"] == st_o["mislabel_init"] and st["false_init"] == st_o["false_init"]
