"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit.

Labels, directions-derived counts, edited values, deltas and round statistics
must be identical (the plain loop is deterministic: integer decisions and
single IEEE float operations in both implementations).
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def assert_fix_parity(msz, f, fh, xi, **kw):
    okw = {("merged_c" if k == "merged" else k): v for k, v in kw.items() if k != "tile"}
    rc_o, d_o, g_o, st_o = oracle.fix(f, fh, xi, **okw)
    ws = kw.pop("warm_start", None)
    tile = kw.pop("tile", 0)
    rc, d, g, st = msz.fix(dev(f), dev(fh), xi, warm_start=None if ws is None else dev(ws), tile=tile,
                           count_init=True, **kw)
    torch.cuda.synchronize()
    assert rc == rc_o, (rc, rc_o, st, st_o)
    if rc in (msz.OK, msz.ESTALL, msz.ENOCONV):
        assert (_bits(host(g)) == _bits(g_o)).all(), "edited values differ"
        assert (_bits(host(d)) == _bits(d_o)).all(), "deltas differ"
        assert st == st_o
    return rc, st


# ------------------------------------------------------------ labels ---

LABEL_SHAPES = [(1, 1), (1, 7), (9, 1), (64, 64), (70, 130), (129, 65), (200, 333),
                (1, 1, 1), (2, 3, 4), (16, 16, 16), (17, 33, 19), (40, 50, 61), (5, 80, 3),
                (17, 33, 20), (3, 70, 132)]


@pytest.mark.parametrize("shape", LABEL_SHAPES)
def test_labels_bit_exact(msz, shape):
    _say("labels", shape)
    rng = np.random.default_rng(11)
    for levels in (0, 5):
        h = rng.uniform(0, 1, size=shape)
        if levels:
            h = np.round(h * (levels - 1))
        h = h.astype(np.float32)
        M, m = msz.labels(dev(h))
        Mo, mo = oracle.labels(h)
        assert (host(M) == Mo).all() and (host(m) == mo).all()


def test_labels_smooth_fields_long_paths(msz):
    """Smooth fields give integral lines crossing many label tiles."""
    rng = np.random.default_rng(12)
    h2 = synth.gaussian_random_field((700, 900), 4.0, rng).astype(np.float32)
    M, m = msz.labels(dev(h2))
    Mo, mo = oracle.labels(h2)
    assert (host(M) == Mo).all() and (host(m) == mo).all()
    h3 = synth.gaussian_random_field((70, 90, 110), 4.0, rng).astype(np.float32)
    M, m = msz.labels(dev(h3))
    Mo, mo = oracle.labels(h3)
    assert (host(M) == Mo).all() and (host(m) == mo).all()
    # constant field: closed form
    c = np.full((37, 45, 29), 0.5, np.float32)
    M, m = msz.labels(dev(c))
    assert (host(M) == c.size - 1).all() and (host(m) == 0).all()


def test_nz1_equals_2d(msz):
    rng = np.random.default_rng(13)
    h = np.round(rng.uniform(0, 4, size=(90, 150))).astype(np.float32)
    M2, m2 = msz.labels(dev(h))
    M3, m3 = msz.labels(dev(h[None]))
    assert (host(M2) == host(M3)[0]).all() and (host(m2) == host(m3)[0]).all()


def test_count_false_bit_exact(msz):
    rng = np.random.default_rng(14)
    for shape in [(100, 120), (30, 31, 32)]:
        f = rng.uniform(0, 1, size=shape).astype(np.float32)
        g = (f + rng.uniform(-0.02, 0.02, size=shape)).astype(np.float32)
        assert msz.count_false(dev(f), dev(g)) == oracle.count_false(f, g)


# -------------------------------------------------------------- fix ---

def test_fix_bumps128(msz):
    f, fh, xi = synth.bumps128()[0]
    _say("fix bumps128")
    rc, st = assert_fix_parity(msz, f, fh, xi)
    assert rc == msz.OK and st["n_edited"] > 0


@pytest.mark.parametrize("shape", [(3, 3), (4, 7), (13, 11), (64, 65), (33, 68), (3, 3, 3), (5, 6, 7),
                                   (20, 17, 9), (20, 17, 12)])
def test_fix_random_small(msz, shape):
    rng = np.random.default_rng(15)
    for k in range(6):
        f, fh, xi = synth.random_small(rng, shape, xi=0.1, levels=(0, 4, 9)[k % 3])
        assert_fix_parity(msz, f, fh, xi)


@pytest.mark.parametrize("merged", [False, True])
@pytest.mark.parametrize("shape", [(256, 128), (64, 16, 16), (32, 32, 16)])
def test_fix_dense_troublemakers(msz, shape, merged):
    """Random fields under a bound of a tenth of their range: more than a
    quarter of the vertices start mislabelled and most directions differ, so
    each label tile lists thousands of vertices in a troublemaker pass and the
    blocks' LDS target lists take many targets per pass (edited when half
    full; any beyond their capacity at once).  Bit for bit with the oracle
    under both schedules."""
    rng = np.random.default_rng(41)
    for levels in (0, 4):
        f, fh, xi = synth.random_small(rng, shape, xi=0.1, levels=levels)
        _say("dense troublemakers", shape, "levels", levels, "merged" if merged else "default")
        rc, st = assert_fix_parity(msz, f, fh, xi, merged=merged)
        assert rc == msz.OK and st["mislabel_init"] * 4 > f.size and st["rounds_r"] > 0


def test_fix_ragged_multi_tile_2d_and_3d(msz):
    rng = np.random.default_rng(16)
    f = synth.gaussian_random_field((301, 517), 3.0, rng).astype(np.float32)
    xi = synth.xi_for(f, 1e-3)
    _say("fix 2D 301x517")
    assert assert_fix_parity(msz, f, synth.quantize(f, xi), xi)[0] == msz.OK
    f3 = synth.gaussian_random_field((37, 70, 95), 11.0 / 3.0, rng).astype(np.float32)
    xi3 = synth.xi_for(f3, 1e-3)
    _say("fix 3D 37x70x95")
    assert assert_fix_parity(msz, f3, synth.quantize(f3, xi3), xi3)[0] == msz.OK


def test_full_and_incremental_passes(msz):
    """An apply that changes many values is followed by a full pass over g, one
    that changes few by a refresh of the flagged vertices only (and R rounds
    redo only the changed label tiles).  A fine checkerboard under a flat
    decompression has false maxima at about a sixth of the vertices, so its
    FNmax rounds start dense and thin out; the schedule shows both kinds of
    pass and the result is still the oracle's, bit for bit."""
    rng = np.random.default_rng(19)
    for shape in ((90, 120), (20, 22, 24)):
        parity = np.indices(shape).sum(axis=0) % 2
        f = (0.5 + 1e-3 * parity + 1e-4 * rng.uniform(0, 1, size=shape)).astype(np.float32)
        xi = np.float32(1e-2)
        fh = synth.quantize(f, xi)
        _say("fix checkerboard", shape)
        rc, st = assert_fix_parity(msz, f, fh, xi)
        assert rc == msz.OK and st["rounds_r"] >= 1 and st["false_init"][2] * 4 * (7 if len(shape) == 2 else 15) > f.size
        rc2, _, _, st2 = msz.fix(dev(f), dev(fh), xi, timing=True)
        assert rc2 == rc and st2["rounds"] == st["rounds"]
        names = [msz.PHASES[k] for k in msz.last_schedule() if k >= 0]
        assert names.count("dirs_detect") >= 2, names.count("dirs_detect")  # the first pass and a full one
        assert names.count("refresh") >= 1


def test_fix_turbulence_64(msz):
    f, fh, xi = synth.turb3d(n=64, nblobs=8)[0]
    _say("fix 3D 64^3 turbulence")
    assert assert_fix_parity(msz, f, fh, xi)[0] == msz.OK


@pytest.mark.parametrize("tile", [1, 2, 3])
def test_tile_variants_identical(msz, tile):
    rng = np.random.default_rng(17)
    f = synth.gaussian_random_field((33, 41, 75), 3.0, rng).astype(np.float32)
    xi = synth.xi_for(f, 1e-3)
    assert_fix_parity(msz, f, synth.quantize(f, xi), xi, tile=tile)
    f2 = synth.gaussian_random_field((130, 250), 3.0, rng).astype(np.float32)
    xi2 = synth.xi_for(f2, 1e-3)
    if tile <= msz.tile_variants(2):
        assert_fix_parity(msz, f2, synth.quantize(f2, xi2), xi2, tile=tile)


def test_fix_warm_start(msz):
    f, fh, xi = synth.bumps128()[0]
    L = oracle.lower_bound(f, xi)
    mid = np.maximum(L, fh - np.float32(0.3) * (fh - L)).astype(np.float32)
    assert_fix_parity(msz, f, fh, xi, warm_start=mid)


@pytest.mark.parametrize("merged", [False, True])
def test_fix_degenerate_shapes(msz, merged):
    """One vertex, single rows and columns, 3D slabs one vertex thick, and
    xi = 0 (every floor equals f, so fhat == f is the only valid input and no
    edit is possible): bit-identical to the oracle under both schedules."""
    rng = np.random.default_rng(20)
    for shape in [(1, 1), (1, 9), (9, 1), (1, 1, 1), (1, 1, 9), (9, 1, 1), (1, 9, 1), (2, 1, 5), (1, 6, 6)]:
        for levels in (0, 3):
            f, fh, xi = synth.random_small(rng, shape, xi=0.2, levels=levels)
            _say("fix degenerate", shape, levels, "merged" if merged else "")
            assert_fix_parity(msz, f, fh, xi, merged=merged)
    f = rng.uniform(0, 1, size=(7, 9)).astype(np.float32)
    rc, st = assert_fix_parity(msz, f, f, np.float32(0.0), merged=merged)
    assert rc == msz.OK and st["n_edited"] == 0


def test_fix_identity(msz):
    rng = np.random.default_rng(18)
    f = rng.uniform(0, 1, size=(50, 60)).astype(np.float32)
    rc, d, g, st = msz.fix(dev(f), dev(f), 0.01)
    assert rc == 0 and st["n_edited"] == 0 and not host(d).any()


# ------------------------------------------------------ error paths ---

def test_error_paths(msz):
    f, fh, xi = synth.bumps128()[0]
    bad = fh.copy()
    bad[5, 5] = f[5, 5] + np.float32(2.5) * xi
    assert msz.fix(dev(f), dev(bad), xi)[0] == msz.EBOUND
    nan = fh.copy()
    nan[0, 0] = np.nan
    assert msz.fix(dev(f), dev(nan), xi)[0] == msz.ENONFINITE
    assert msz.fix(dev(f), dev(fh), float("inf"))[0] == msz.ENONFINITE
    assert msz.fix(dev(f), dev(fh), -1.0)[0] == msz.EINVAL
    assert_fix_parity(msz, f, fh, xi, max_rounds=1)
    assert_fix_parity(msz, f, fh, xi, max_rounds=7)
    small_ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    assert msz.fix(dev(f), dev(fh), xi, workspace=small_ws)[0] == msz.EINVAL
    # arrays must be 16-byte aligned: a view starting one float in is rejected
    big_f = dev(np.concatenate([f.ravel(), f.ravel()[:1]]))[1:].reshape(f.shape)
    assert msz.fix(big_f, dev(fh), xi)[0] == msz.EINVAL
    with pytest.raises(msz.MszError):
        msz.labels(dev(nan))
    # an unknown option flag is rejected before any work
    fd, fhd = dev(f), dev(fh)
    e = torch.empty_like(fd)
    opt = msz.Options()
    opt.flags = 1 << 20
    st = msz.Stats()
    rc = msz.lib().msz_fix(fd.data_ptr(), fhd.data_ptr(), msz.dims_of(f.shape), float(xi), e.data_ptr(),
                           ctypes.byref(opt), ctypes.byref(st), msz._stream())
    assert rc == msz.EINVAL


def test_floor_collision_stalls(msz):
    f0 = np.float32(0.5 + 2.0 ** -23)
    f1 = np.float32(0.5 + 2.0 ** -24)
    xi = np.float32(4.5)
    f = np.array([[f0, f1]], np.float32)
    L = oracle.lower_bound(f, xi)
    fh = np.array([[L[0, 0], np.float32(0.0)]], np.float32)
    assert assert_fix_parity(msz, f, fh, xi)[0] == msz.ESTALL


def test_fpmin_counterexample(msz):
    f = np.array([.80, .48, .30, .85, .50, .90, .75, .95, .99], np.float32).reshape(3, 3)
    fh = f.copy()
    fh[1, 1] = np.float32(.46)
    fh[0, 1] = np.float32(.52)
    rc, st = assert_fix_parity(msz, f, fh, np.float32(0.05))
    assert rc == msz.OK and st["rounds"] == [0, 2, 0, 0]


# ----------------------------------------------- full-size workloads ---

def _full_invariants(msz, f, fh, xi, g, d, st):
    fd, gd = dev(f), dev(g)
    cnt = msz.count_false(fd, gd)
    assert all(v == 0 for v in cnt.values()), cnt
    assert (np.abs(f.astype(np.float64) - g.astype(np.float64)) <= float(xi)).all()
    assert (g <= fh).all()
    rec = (fh + d).astype(np.float32)
    assert int((rec != g).sum()) == st["n_inexact"]


def _oracle_threads():
    """Threads for each of two concurrent oracle runs (the oracle's per-vertex
    direction loop; its result does not depend on the split)."""
    import os
    try:
        cpus = len(os.sched_getaffinity(0))
    except AttributeError:
        cpus = os.cpu_count() or 1
    return max(1, min(16, cpus) // 2)


def _full_parity_both_schedules(msz, f, fh, xi, name):
    """The whole oracle run under the default and the merged C schedule (two
    host threads, started before the GPU runs) against the GPU's runs of the
    same schedules: edited values, deltas and every statistic bit for bit;
    the default run also by the invariants of a converged result."""
    from concurrent.futures import ThreadPoolExecutor
    nt = _oracle_threads()
    with ThreadPoolExecutor(max_workers=2) as pool:
        fut = {m: pool.submit(oracle.fix, f, fh, xi, merged_c=m, threads=nt) for m in (False, True)}
        gpu = {}
        for m in (False, True):
            rc, d, g, st = msz.fix(dev(f), dev(fh), xi, merged=m, count_init=True)
            torch.cuda.synchronize()
            gpu[m] = (rc, host(d), host(g), st)
            _say(f"  {name} gpu {'merged' if m else 'default'}: rc {rc}, rounds {st['rounds']} + {st['rounds_r']}")
        for m in (False, True):
            rc_o, d_o, g_o, st_o = fut[m].result()
            _say(f"  {name} oracle {'merged' if m else 'default'}: rc {rc_o}, rounds {st_o['rounds']} + {st_o['rounds_r']}")
            rc, d, g, st = gpu[m]
            assert rc == rc_o == msz.OK, (m, rc, rc_o)
            assert (_bits(g) == _bits(g_o)).all(), ("edited values differ", m, int((_bits(g) != _bits(g_o)).sum()))
            assert (_bits(d) == _bits(d_o)).all(), ("deltas differ", m)
            assert st == st_o, (m, st, st_o)
    rc, d, g, st = gpu[False]
    _full_invariants(msz, f, fh, xi, g, d, st)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("rel", [1e-4, 1e-3])
def test_full_ocean2d_bit_exact(msz, rel):
    """3600x2400 ocean-like field at xi = 1e-4 and 1e-3 of the range: the whole
    oracle run of each schedule against the GPU's."""
    f, fh, xi = synth.ocean2d(rels=(rel,))[0]
    _say(f"full 3600x2400 xi={rel:g}")
    _full_parity_both_schedules(msz, f, fh, xi, "ocean2d")


@pytest.mark.timeout(900)
def test_full_turb256_bit_exact(msz):
    """The 256^3 turbulence field with 64 blobs at xi = 1e-3 of the range: the
    whole oracle run of each schedule against the GPU's."""
    f, fh, xi = synth.turb3d()[0]
    _say("full 256^3")
    _full_parity_both_schedules(msz, f, fh, xi, "turb256")


# ------------------------------------------------------------ batched ---

def _batch_case(seed):
    rng = np.random.default_rng(seed)
    shapes = [(37, 70), (128, 96), (1, 5), (20, 33, 17), (48, 48, 48), (3, 200), (16, 16, 16), (250, 301)]
    fields = []
    for k, shape in enumerate(shapes):
        f = synth.gaussian_random_field(shape, 3.0, rng).astype(np.float32)
        rel = (1e-4, 1e-3, 1e-2)[k % 3]
        xi = synth.xi_for(f, rel) if f.max() > f.min() else np.float32(0.01)
        fields.append((f, synth.quantize(f, xi), xi))
    return fields


@pytest.mark.parametrize("seed,tiles,count_init", [(21, None, False), (22, "mixed", True)])
def test_batch_bit_exact_with_single_fix(msz, seed, tiles, count_init):
    fields = _batch_case(seed)
    tl = None
    if tiles == "mixed":
        tl = [(j % (msz.tile_variants(f.ndim) + 1)) for j, (f, _, _) in enumerate(fields)]
    _say("batch of", len(fields), "tiles", tl)
    rc, res = msz.fix_batch([(dev(f), dev(fh), xi) for f, fh, xi in fields], tiles=tl, count_init=count_init)
    torch.cuda.synchronize()
    for j, (f, fh, xi) in enumerate(fields):
        st_b, d_b, g_b, s_b = res[j]
        rc_s, d_s, g_s, s_s = msz.fix(dev(f), dev(fh), xi, count_init=count_init)
        assert (s_b["mislabel_init"] >= 0) == count_init
        assert st_b == rc_s == s_b["status"], (j, st_b, rc_s)
        assert (_bits(host(g_b)) == _bits(host(g_s))).all(), j
        assert (_bits(host(d_b)) == _bits(host(d_s))).all(), j
        assert s_b == s_s, (j, s_b, s_s)
    assert rc == msz.OK


def test_batch_error_and_cap(msz):
    fields = _batch_case(23)[:4]
    f, fh, xi = fields[1]
    bad = fh.copy()
    bad.ravel()[7] = f.ravel()[7] + np.float32(3) * xi
    jobs = [(dev(a), dev(b), x) for a, b, x in fields] + [(dev(f), dev(bad), xi)]
    rc, res = msz.fix_batch(jobs, max_rounds=2)
    assert res[-1][0] == msz.EBOUND
    for j, (a, b, x) in enumerate(fields):
        rc_s, d_s, g_s, s_s = msz.fix(dev(a), dev(b), x, max_rounds=2)
        assert res[j][0] == rc_s
        assert (_bits(host(res[j][2])) == _bits(host(g_s))).all()
    assert rc != msz.OK


@pytest.mark.timeout(900)
@pytest.mark.parametrize("merged", [False, True])
def test_full_batch96_bit_exact(msz, merged):
    """The 96-field batch of the batched form (about 1.35e8 vertices) in one
    run, under the default and the merged C schedule: every field's edited
    values, deltas and statistics (the start field's mislabel count included)
    bit for bit against the oracle's run of the same schedule on that field
    alone, and every field reaches zero segmentation error within its bound.
    The oracle runs on a pool of host threads, started before the GPU run,
    largest fields first."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    fields = synth.batch_fields(0)
    try:
        cpus = len(os.sched_getaffinity(0))
    except AttributeError:
        cpus = os.cpu_count() or 1
    order = sorted(range(len(fields)), key=lambda j: -fields[j][0].size)
    _say(f"full 96-field batch, {'merged' if merged else 'default'} schedule, oracle on {min(16, cpus)} threads")
    with ThreadPoolExecutor(max_workers=max(1, min(16, cpus))) as pool:
        fut = {j: pool.submit(oracle.fix, *fields[j], merged_c=merged) for j in order}
        rc, res = msz.fix_batch([(dev(f), dev(fh), xi) for f, fh, xi in fields], merged=merged, count_init=True)
        torch.cuda.synchronize()
        assert rc == msz.OK
        for j, (f, fh, xi) in enumerate(fields):
            st_b, d_b, g_b, s_b = res[j]
            assert st_b == msz.OK, j
            _full_invariants(msz, f, fh, xi, host(g_b), host(d_b), s_b)
        for j in order:
            rc_o, d_o, g_o, st_o = fut[j].result()
            st_b, d_b, g_b, s_b = res[j]
            assert rc_o == st_b == msz.OK, (j, rc_o, st_b)
            assert (_bits(host(g_b)) == _bits(g_o)).all(), ("edited values differ", j, fields[j][0].shape)
            assert (_bits(host(d_b)) == _bits(d_o)).all(), ("deltas differ", j)
            assert s_b == st_o, (j, s_b, st_o)


def test_full_turb512_learned_properties(msz):
    """The 512^3 field of the learned form: warm-started and plain loops both reach
    zero segmentation error within xi; the warm start needs fewer rounds.  The
    end-to-end times and edit counts of both are reported (the warm start does
    not pay on this field: its network costs more than the rounds it saves)."""
    import time
    from paper_2406_09423_amd import train_net
    f, fh, xi = synth.turb512()[0]
    _say("full 512^3 learned")
    fd, fhd = dev(f), dev(fh)
    params = train_net.load_weights()
    pm = train_net.stored_p_min()
    msz.fix_learned(fd, fhd, xi, params, p_min=pm)      # warm-up (first-call setup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc_l, d_l, g_l, st_l = msz.fix_learned(fd, fhd, xi, params, p_min=pm)
    torch.cuda.synchronize()
    t_l = time.perf_counter() - t0
    assert rc_l == msz.OK
    cnt = msz.count_false(fd, g_l)
    assert all(v == 0 for v in cnt.values()), cnt
    gl = host(g_l)
    assert (np.abs(f.astype(np.float64) - gl.astype(np.float64)) <= float(xi)).all()
    assert (gl <= fh).all()
    del gl, d_l, g_l
    msz.fix(fd, fhd, xi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc_p, d_p, g_p, st_p = msz.fix(fd, fhd, xi)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    assert rc_p == msz.OK
    cnt = msz.count_false(fd, g_p)
    assert all(v == 0 for v in cnt.values()), cnt
    rounds = lambda st: sum(st["rounds"]) + st["rounds_r"]
    _say(f"  learned {1e3 * t_l:.2f} ms, {rounds(st_l)} rounds, {st_l['n_edited']} edits; "
         f"plain {1e3 * t_p:.2f} ms, {rounds(st_p)} rounds, {st_p['n_edited']} edits; "
         f"speedup {t_p / t_l:.2f}")
    assert rounds(st_l) < rounds(st_p), (rounds(st_l), rounds(st_p))


@pytest.mark.parametrize("merged", [False, True])
def test_turb512_chunk_summaries_bit_exact(msz, merged):
    """At 512^3 the one-field kernel keeps chunk summaries of its flag arrays
    and skips chunks with nothing flagged; the batch kernel never does.  The
    field corrected alone and corrected in a batch (beside a tiny field, so
    that the batch kernels run) must agree bit for bit, with equal stats."""
    f, fh, xi = synth.turb512()[0]
    _say(f"512^3 summaries vs batch, merged={merged}")
    fd, fhd = dev(f), dev(fh)
    del f, fh
    rc, d1, g1, st1 = msz.fix(fd, fhd, xi, merged=merged)
    assert rc == msz.OK
    b1, b2 = _bits(host(g1)), _bits(host(d1))
    del d1, g1
    rng = np.random.default_rng(5)
    tf = rng.uniform(0, 1, size=(9, 10, 11)).astype(np.float32)
    rc_b, res = msz.fix_batch([(fd, fhd, xi), (dev(tf), dev(synth.quantize(tf, np.float32(0.05))), 0.05)],
                              merged=merged)
    assert rc_b == msz.OK
    st_b, d2, g2, st2 = res[0]
    assert st_b == msz.OK and st1 == st2
    assert (_bits(host(g2)) == b1).all() and (_bits(host(d2)) == b2).all()


# ------------------------------------------------------- merged C rounds ---

def _merged_case(name):
    rng = np.random.default_rng(31)
    if name == "bumps128":
        return [synth.bumps128()[0]]
    if name == "ocean":
        f = synth.gaussian_random_field((240, 360), 3.0, rng).astype(np.float32)
        f = ((f - f.min()) / (f.max() - f.min())).astype(np.float32)
        return [(f, synth.quantize(f, np.float32(x)), np.float32(x)) for x in (1e-4, 1e-3)]
    if name == "turb":
        f = synth.gaussian_random_field((37, 70, 95), 11.0 / 3.0, rng).astype(np.float32)
        xi = synth.xi_for(f, 1e-3)
        return [(f, synth.quantize(f, xi), xi)]
    shape = (90, 120) if name == "checker2d" else (20, 22, 24)
    parity = np.indices(shape).sum(axis=0) % 2
    f = (0.5 + 1e-3 * parity + 1e-4 * rng.uniform(0, 1, size=shape)).astype(np.float32)
    xi = np.float32(1e-2)
    return [(f, synth.quantize(f, xi), xi)]


@pytest.mark.parametrize("name", ["bumps128", "ocean", "checker2d", "checker3d", "turb"])
def test_merged_c_bit_exact(msz, name):
    """Merged C rounds (all four case types per round, Sec. 6.1): edited
    values, deltas and statistics bit-identical to the oracle's merged
    schedule, and zero segmentation error.  The checkerboards start with dense
    rounds (full passes over g), the others are sparse."""
    for f, fh, xi in _merged_case(name):
        _say("merged C rounds", name, f.shape, float(xi))
        rc, st = assert_fix_parity(msz, f, fh, xi, merged=True)
        assert rc == msz.OK
        rc_p, _, _, st_p = msz.fix(dev(f), dev(fh), xi)
        assert rc_p == msz.OK
        _say("  rounds merged", st["rounds"], st["rounds_r"], "plain", st_p["rounds"], st_p["rounds_r"])


def test_merged_c_cap_and_batch(msz):
    """The round cap ends a merged C phase like the oracle's, and a batch with
    merged rounds gives every field its single-call result."""
    f, fh, xi = synth.bumps128()[0]
    _say("merged C rounds, cap 3")
    rc, st = assert_fix_parity(msz, f, fh, xi, merged=True, max_rounds=3)
    assert rc == msz.ENOCONV
    fields = _batch_case(24)[:6]
    _say("merged batch of", len(fields))
    rcb, res = msz.fix_batch([(dev(a), dev(b), x) for a, b, x in fields], merged=True)
    assert rcb == msz.OK
    for j, (a, b, x) in enumerate(fields):
        rc_s, d_s, g_s, s_s = msz.fix(dev(a), dev(b), x, merged=True)
        st_b, d_b, g_b, s_b = res[j]
        assert st_b == rc_s == msz.OK, (j, st_b, rc_s)
        assert (_bits(host(g_b)) == _bits(host(g_s))).all(), j
        assert (_bits(host(d_b)) == _bits(host(d_s))).all(), j
        assert s_b == s_s, (j, s_b, s_s)
