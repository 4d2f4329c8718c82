"""GPU edit encoding and decoding (msz_encode_edits / msz_decode_edits)
against the reference encoder, byte for byte, and round trips."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import edits_ref as E

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def msz():
    import paper_2406_09423_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _check(msz, x):
    n = x.size
    d = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    rc, blob, st = msz.encode_edits(d)
    assert rc == msz.OK
    got = blob.cpu().numpy().tobytes()
    want = E.encode(x)
    assert got == want, (len(got), len(want))
    assert st["n_edits"] == int(np.count_nonzero(x.view(np.uint32))) and st["bytes"] == len(want)
    rc, back = msz.decode_edits(blob, x.shape)
    assert rc == msz.OK
    assert (back.cpu().numpy().view(np.uint32) == x.view(np.uint32)).all()
    return st


@pytest.mark.parametrize("n,m", [(1, 0), (1, 1), (255, 255), (257, 257), (4097, 4097), (20000, 9000), (70000, 12289),
                                 (3_000_000, 5000)])
def test_random_edits_bit_exact(msz, n, m):
    _say("edits", n, m)
    rng = np.random.default_rng(n + 7 * m)
    x = np.zeros(n, dtype=np.float32)
    idx = rng.choice(n, size=m, replace=False) if m else np.zeros(0, np.int64)
    x[idx] = -rng.exponential(1e-3, size=m).astype(np.float32)
    _check(msz, x)


def test_extreme_values_and_gaps(msz):
    n = (1 << 22) + 3
    x = np.zeros(n, dtype=np.float32)
    x[[0, 1, 2, 1 << 20, (1 << 21) + 7, n - 1]] = [-1e-40, -0.0, -3.0e38, -1.0, 5.0, np.float32(-2.0 ** -149)]
    _check(msz, x)


def test_edits_of_the_loop(msz):
    """The edits msz_fix produces on the 128x128 bumps and a 3D field."""
    for f, fh, xi in (synth.bumps128()[0], synth.turb3d(n=48, nblobs=4)[0]):
        _, d, _, _ = oracle.fix(f, fh, xi)
        st = _check(msz, d)
        _say("loop edits", f.shape, st)
        assert st["n_edits"] > 0


def test_malformed_input_is_rejected(msz):
    rng = np.random.default_rng(5)
    x = np.zeros(50000, dtype=np.float32)
    x[rng.choice(50000, size=9000, replace=False)] = -1.0
    d = torch.from_numpy(x).cuda()
    rc, blob, _ = msz.encode_edits(d)
    assert rc == msz.OK
    rc, _ = msz.decode_edits(blob, (50001,))  # header names another size
    assert rc == msz.EINVAL
    rc, _ = msz.decode_edits(blob[: blob.numel() - 64].clone(), x.shape)  # the last chunk cut short
    assert rc == msz.EINVAL
    small = torch.empty(600, dtype=torch.uint8, device="cuda")
    rc, _, _ = msz.encode_edits(d, out=small)  # capacity too small
    assert rc == msz.EINVAL
