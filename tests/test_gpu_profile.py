"""Profiling records of the step kernels (msz_last_launches): one record per
launch, phases matching the step schedule, the whole-field operations
reporting exactly their per-vertex bytes times the vertex count, and timed
runs giving the same results as untimed ones."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


# bytes per vertex of the operations that visit every vertex once per launch
WHOLE_FIELD = {"validate": 16, "dirs": 5, "dirs_detect": 9, "delta": 16}


@pytest.mark.parametrize("shape", [(77, 130), (21, 40, 35)])
def test_single_field_records(msz, shape):
    rng = np.random.default_rng(61)
    f = synth.gaussian_random_field(shape, 3.0, rng).astype(np.float32)
    xi = synth.xi_for(f, 1e-3)
    fd, fhd = _dev(f), _dev(synth.quantize(f, xi))
    rc, d0, g0, st0 = msz.fix(fd, fhd, xi)
    rc_t, d1, g1, st1 = msz.fix(fd, fhd, xi, timing=True)
    assert rc == rc_t == msz.OK
    assert (_bits(g0) == _bits(g1)).all() and (_bits(d0) == _bits(d1)).all()
    st1.pop("timing")
    assert st0 == st1
    recs = msz.last_launches()
    sched = msz.last_schedule()
    assert len(recs) == len(sched) and len(recs) % 48 == 0
    kern = "step1_3d" if len(shape) == 3 else "step1_2d"
    n = f.size
    seen = set()
    for r, ph in zip(recs, sched):
        assert r["kernel"] == kern
        assert (r["phase"] is None) == (ph < 0)
        if ph < 0:
            assert r["bytes"] == 0
            continue
        assert r["phase"] == msz.PHASES[ph] and r["us"] > 0
        if r["phase"] in WHOLE_FIELD:
            assert r["bytes"] == WHOLE_FIELD[r["phase"]] * n, r
            seen.add(r["phase"])
        elif r["phase"] == "label_final":
            # 16 per vertex, plus 4 per gather along the exit chains (fewer than
            # two per vertex on a smooth field)
            assert 16 * n <= r["bytes"] < 24 * n, r
        else:
            assert r["bytes"] > 0, r
    assert seen == set(WHOLE_FIELD)


def test_batch_records(msz):
    rng = np.random.default_rng(62)
    fields = []
    for k, shape in enumerate([(50, 70), (30, 31, 33), (200, 9), (16, 16, 16)]):
        f = synth.gaussian_random_field(shape, 3.0, rng).astype(np.float32)
        xi = synth.xi_for(f, (1e-4, 1e-3, 1e-2)[k % 3])
        fields.append((_dev(f), _dev(synth.quantize(f, xi)), float(xi)))
    rc, res = msz.fix_batch(fields)
    rc_t, res_t = msz.fix_batch(fields, timing=True)
    assert rc == rc_t == msz.OK
    for (s0, d0, g0, st0), (s1, d1, g1, st1) in zip(res, res_t):
        assert s0 == s1 == msz.OK and st0 == st1
        assert (_bits(g0) == _bits(g1)).all() and (_bits(d0) == _bits(d1)).all()
    recs = msz.last_launches()
    assert recs and all(r["phase"] is None for r in recs)
    assert {r["kernel"] for r in recs} == {"batch_2d", "batch_3d"}
    # every field is validated, its deltas written and its directions of f
    # and g computed at least once: a lower bound on the bytes
    nv = sum(f.numel() for f, _, _ in fields)
    assert sum(r["bytes"] for r in recs) >= (16 + 5 + 9 + 16 + 16) * nv
    assert sum(r["us"] for r in recs) > 0
