"""msz_fix_noalloc (the entry point for callers that cannot allocate) against
msz_fix through the C ABI: edited values, deltas and every statistic bit for
bit, on calls in a row that reuse the library's static device scratch with a
smaller field after a larger one, plus its size limit and argument checks."""
import sys

import numpy as np
import pytest

import synth

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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bits(t):
    return t.cpu().numpy().view(np.uint32)


def _case(shape, exponent, rel, seed):
    rng = np.random.default_rng(seed)
    f = synth.gaussian_random_field(shape, exponent, rng).astype(np.float32)
    f = ((f - f.min()) / (f.max() - f.min())).astype(np.float32)
    xi = synth.xi_for(f, rel)
    return f, synth.quantize(f, xi), xi


def _same_as_fix(msz, f, fh, xi, **kw):
    fd, fhd = _dev(f), _dev(fh)
    rc, d, g, st = msz.fix(fd, fhd, xi, **kw)
    g_n = torch.empty_like(fd)
    rc_n, d_n, _, st_n = msz.fix_noalloc(fd, fhd, xi, g_out=g_n, **kw)
    torch.cuda.synchronize()
    _say(f"  {f.shape} {kw}: rc {rc_n}, rounds {st_n['rounds']} + {st_n['rounds_r']}, {st_n['n_edited']} edits")
    assert rc_n == rc, (rc_n, rc)
    assert (_bits(g_n) == _bits(g)).all(), "edited values differ"
    assert (_bits(d_n) == _bits(d)).all(), "deltas differ"
    assert st_n == st, (st_n, st)
    return rc_n, st_n


def test_noalloc_matches_fix_twice_in_a_row(msz):
    """A 128^3 field (near the scratch limit), then a smaller ragged 2D one, then
    the 3D field again with merged C rounds: each bit-identical to msz_fix."""
    big = _case((128, 128, 128), 11.0 / 3.0, 1e-3, 7001)
    small = _case((257, 300), 3.0, 1e-3, 7002)
    _say("no-alloc: 128^3, then 257x300, then 128^3 merged")
    rc, st = _same_as_fix(msz, *big, count_init=True)
    assert rc == msz.OK and sum(st["rounds"]) + st["rounds_r"] > 0
    rc, st = _same_as_fix(msz, *small)
    assert rc == msz.OK and st["mislabel_init"] == -1 and st["n_edited"] > 0
    rc, _ = _same_as_fix(msz, *big, merged=True)
    assert rc == msz.OK


def test_noalloc_cap_and_tiny(msz):
    """A capped run (ENOCONV, the bounded delta still written) and a 1-vertex
    field, after the larger runs above left the scratch dirty."""
    f, fh, xi = _case((90, 70), 3.0, 1e-2, 7003)
    rc, _ = _same_as_fix(msz, f, fh, xi, max_rounds=2)
    assert rc == msz.ENOCONV
    one = np.array([[0.5]], dtype=np.float32)
    rc, st = _same_as_fix(msz, one, one, np.float32(0.01))
    assert rc == msz.OK and st["n_edited"] == 0


def test_noalloc_limits_and_arguments(msz):
    """Beyond the static scratch: ETOOBIG before any device work; a workspace
    or the timing flag: EINVAL."""
    import ctypes
    limit = msz.NOALLOC_SCRATCH_BYTES
    assert msz.workspace_bytes((150, 150, 150)) < limit < msz.workspace_bytes((160, 160, 160))
    f = torch.zeros((160, 160, 160), dtype=torch.float32, device="cuda")
    rc, _, _, st = msz.fix_noalloc(f, f, 0.1)
    assert rc == msz.ETOOBIG and st["status"] == msz.ETOOBIG
    assert "static scratch" in msz.strerror(rc)
    small = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    e = torch.empty_like(small)
    for ws, flags in ((torch.empty(1 << 20, dtype=torch.uint8, device="cuda"), 0), (None, msz.FLAG_TIMING)):
        opt = msz.Options()
        if ws is not None:
            opt.workspace = ws.data_ptr()
            opt.workspace_bytes = ws.numel()
        opt.flags = flags
        st = msz.Stats()
        rc = msz.lib().msz_fix_noalloc(small.data_ptr(), small.data_ptr(), msz.dims_of(small.shape), 0.1,
                                       e.data_ptr(), ctypes.byref(opt), ctypes.byref(st), msz._stream())
        assert rc == msz.EINVAL
