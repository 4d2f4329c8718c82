"""The R loop's stopping rule (Sec. 5.2): a field g has a vertex whose maximum
(minimum) label differs from f's exactly when it has a max (min)
troublemaker -- a mislabelled vertex whose steepest ascent (descent) in g
differs from f's.  The GPU's detection resolves labels only at vertices
whose direction differs and stops the loop when it finds no troublemaker;
this checks, with the oracle's directions and labels on fields of every
kind (random, plateaued, perturbed, with and without false critical
points), that the two conditions always agree, and that each troublemaker
found is one the oracle's own definition gives."""
import numpy as np
import pytest

import oracle


def _families(f, g):
    """(mislabelled, troublemakers) per family: max (ascent) and min (descent)."""
    uf, df = oracle.dirs(f)
    ug, dg = oracle.dirs(g)
    Mf, mf = oracle.labels(f)
    Mg, mg = oracle.labels(g)
    wrong_max, wrong_min = Mg != Mf, mg != mf
    tm_max = wrong_max & (ug != uf)
    tm_min = wrong_min & (dg != df)
    return (wrong_max, tm_max), (wrong_min, tm_min)


def _fields(rng, shape):
    f = rng.uniform(0, 1, size=shape).astype(np.float32)
    yield f, (f + rng.normal(0, 0.05, size=shape)).astype(np.float32)           # perturbed
    yield f, np.round(f * 4).astype(np.float32) / 4                             # plateaus (ties by index)
    yield f, f.copy()                                                           # identical
    yield f, rng.permutation(f.ravel()).reshape(shape).astype(np.float32)       # unrelated
    smooth = np.cumsum(np.cumsum(rng.normal(size=shape), axis=0), axis=-1).astype(np.float32)
    q = (np.round(smooth / 3.0) * 3.0).astype(np.float32)                       # quantized, smooth
    yield smooth, q
    g = smooth.copy()                                                           # a few values lowered
    idx = rng.choice(g.size, size=max(1, g.size // 50), replace=False)
    g.ravel()[idx] -= np.float32(2.0)
    yield smooth, g


@pytest.mark.parametrize("shape", [(9, 13), (31, 40), (1, 17), (6, 7, 8), (12, 5, 9)])
def test_mislabelled_iff_troublemaker(shape):
    rng = np.random.default_rng(1000 + sum(shape))
    seen_both = seen_none = 0
    for f, g in _fields(rng, shape):
        for wrong, tm in _families(f, g):
            assert wrong.any() == tm.any()
            assert not (tm & ~wrong).any()          # a troublemaker is mislabelled by definition
            seen_both += int(wrong.any())
            seen_none += int(not wrong.any())
    assert seen_both > 0 and seen_none > 0          # both outcomes occur among the cases


def test_first_differing_vertex_on_the_path_is_a_troublemaker():
    """The argument itself, vertex by vertex: following the descent in g from
    any min-mislabelled vertex, the first vertex whose descent differs from
    f's is a min troublemaker (and likewise for ascents and maxima)."""
    rng = np.random.default_rng(77)
    for shape in [(20, 23), (7, 8, 9)]:
        smooth = np.cumsum(np.cumsum(rng.normal(size=shape), axis=0), axis=-1).astype(np.float32)
        g = (np.round(smooth / 2.0) * 2.0).astype(np.float32)
        uf, df = [a.ravel() for a in oracle.dirs(smooth)]
        ug, dg = [a.ravel() for a in oracle.dirs(g)]
        (wM, tM), (wm, tm) = [(a.ravel(), b.ravel()) for a, b in _families(smooth, g)]
        checked = 0
        for wrong, tmk, pg, pf in ((wm, tm, dg, df), (wM, tM, ug, uf)):
            for i in np.flatnonzero(wrong):
                u = int(i)
                while pg[u] == pf[u] and pg[u] != u:
                    u = int(pg[u])
                assert pg[u] != pf[u], "the paths agree to a common extremum, so the labels would agree"
                assert tmk[u]
                checked += 1
        assert checked > 0
