"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expectation comes from a
closed form, a special case, exact rational arithmetic, a literal brute-force
restatement of the definitions (tests/literal.py) or an invariant of the
problem statement.
"""
import random
from fractions import Fraction

import numpy as np
import pytest

import literal as lit
import oracle
import synth


# ------------------------------------------------------------ arithmetic ---

def _rand_float(rng, lo_exp=-149, hi_exp=4):
    """Random float32 covering subnormals, normals and signs."""
    kind = rng.random()
    if kind < 0.15 and lo_exp <= -126:
        v = rng.randint(1, 2 ** 23 - 1) * 2.0 ** -149          # subnormal
    else:
        v = rng.uniform(1, 2) * 2.0 ** rng.randint(max(lo_exp, -126), hi_exp)
    return np.float32(v if rng.random() < 0.7 else -v)


def test_halve_matches_exact_rounding():
    """Eqs. 2-6 evaluated as fl(fl(g+L)/2): oracle bits == exact-rational RNE bits."""
    rng = random.Random(1)
    pairs = []
    for _ in range(3000):
        a, b = _rand_float(rng), _rand_float(rng)
        g, L = (a, b) if a >= b else (b, a)
        pairs.append((g, L))
    # adjacent floats, equal values, zero floor, subnormal floor
    for v in (np.float32(0.45), np.float32(1e-40), np.float32(-3.0), np.float32(0.0)):
        pairs += [(lit.next_up(v), v), (v, v), (lit.next_up(lit.next_up(v)), v)]
    for g, L in pairs:
        h = oracle.halve(g, L)
        e = lit.halve_exact(g, L)
        assert h.view(np.uint32) == e.view(np.uint32), (g, L, h, e)
        assert L <= h <= g
        if g != L:
            assert h < g, "every edit must strictly lower g until it reaches the floor"


def test_halving_chain_lengths():
    """Closed forms: with L = 0 the chain is exact division by 2 down to the subnormals.

    g0 = m * 2^e (m odd) stays exact for e - k >= -149; from 2^-149 one more step
    rounds 2^-150 to 0 (ties to even).  So a power of two 2^p needs p + 149 + 1 steps.
    """
    for p in (-3, 0, -20):
        g0 = np.float32(2.0 ** p)
        n = 0
        g = g0
        while g != 0:
            g = oracle.halve(g, np.float32(0.0))
            n += 1
            assert n < 400
        assert n == p + 149 + 1
    # f = xi gives L = 0; starting from 2 xi the chain runs through the subnormals
    xi = np.float32(0.05)
    L = oracle.lower_bound(np.array([xi], np.float32), xi)[0]
    assert L == 0.0
    chain = lit.halving_chain(np.float32(2 * xi), L)
    n, g = 0, np.float32(2 * xi)
    while g != L:
        g = oracle.halve(g, L)
        n += 1
    assert n == len(chain) - 1
    assert n == 147   # 0.1f = 13421773 * 2^-27: exact halvings to 2^-149 granularity, then rounding


def test_lower_bound_is_exact_ceiling():
    rng = random.Random(2)
    fs, xis = [], []
    for _ in range(2000):
        fs.append(_rand_float(rng, -60, 3))
        xis.append(abs(_rand_float(rng, -60, 2)))
    fs += [np.float32(0.05), np.float32(1e-30), np.float32(-1e-30), np.float32(0.5)]
    xis += [np.float32(0.05), np.float32(1e-3), np.float32(1e-3), np.float32(4.5)]
    for f, xi in zip(fs, xis):
        L = oracle.lower_bound(np.array([f], np.float32), xi)[0]
        assert L == lit.lower_bound_exact(f, xi), (f, xi)
        assert Fraction(float(L)) >= Fraction(float(f)) - Fraction(float(xi))
        assert Fraction(float(lit.next_down(L))) < Fraction(float(f)) - Fraction(float(xi))


def test_delta_reconstructs():
    rng = random.Random(3)
    for _ in range(2000):
        fh = _rand_float(rng, -20, 2)
        g = np.float32(fh - abs(float(_rand_float(rng, -30, 1))))
        d, ok = oracle.delta(g, fh)
        if ok:
            assert np.float32(fh + d) == g
    # representable differences (Sterbenz) always reconstruct exactly
    for _ in range(500):
        fh = np.float32(rng.uniform(0.5, 1.0))
        g = np.float32(rng.uniform(float(fh) / 2, float(fh)))
        d, ok = oracle.delta(g, fh)
        assert ok and d == np.float32(float(g) - float(fh))


# ------------------------------------------------------- order, directions ---

def _rand_field(rng, shape, levels=0):
    a = rng.uniform(0, 1, size=shape)
    if levels:
        a = np.round(a * (levels - 1))
    return a.astype(np.float32)


SHAPES = [(3, 3), (4, 5), (5, 2), (1, 6), (2, 3, 3), (3, 3, 3), (2, 2, 4), (1, 3, 4)]


@pytest.mark.parametrize("shape", SHAPES)
def test_dirs_and_labels_match_literal(shape):
    rng = np.random.default_rng(4)
    mesh = lit.Mesh(shape)
    for levels in (0, 3, 1):
        for _ in range(4):
            h = _rand_field(rng, shape, levels)
            up, dn = oracle.dirs(h)
            lup, ldn = lit.dirs(mesh, h.ravel())
            assert up.ravel().tolist() == lup
            assert dn.ravel().tolist() == ldn
            M, m = oracle.labels(h)
            lM, lm = lit.labels(mesh, h.ravel())
            assert M.ravel().tolist() == lM
            assert m.ravel().tolist() == lm


def test_neighbour_counts_closed_form():
    """Interior vertices have 6 (2D) / 14 (3D) neighbours; corners of the split have fewer."""
    mesh2 = lit.Mesh((5, 5))
    # the split diagonal runs through corners 0 and 24: they keep 3 edges, the other two corners 2
    assert len(mesh2.nb[12]) == 6 and len(mesh2.nb[0]) == 3 and len(mesh2.nb[4]) == 2
    assert len(mesh2.nb[24]) == 3 and len(mesh2.nb[20]) == 2
    mesh3 = lit.Mesh((3, 3, 3))
    # the (0,0,0)-(1,1,1) diagonal corners keep all 7 edges of their octant
    assert len(mesh3.nb[13]) == 14 and len(mesh3.nb[0]) == 7 and len(mesh3.nb[26]) == 7
    assert len(mesh3.nb[2]) == 4


def test_constant_field_closed_form():
    """Constant field: ties go to the larger index, so every ascent ends at N-1, every descent at 0."""
    for shape in [(7, 9), (4, 5, 6), (1, 1, 8)]:
        h = np.full(shape, 0.25, np.float32)
        M, m = oracle.labels(h)
        n = h.size
        assert (M == n - 1).all() and (m == 0).all()
        up, dn = oracle.dirs(h)
        ids = np.arange(n).reshape(shape)
        assert (up >= ids).all() and (dn <= ids).all()


def test_ramp_field_closed_form():
    """f = linear index: strictly increasing, same labels as the constant field; -0 == +0 ties by index."""
    for shape in [(6, 7), (3, 4, 5)]:
        h = np.arange(np.prod(shape), dtype=np.float32).reshape(shape)
        M, m = oracle.labels(h)
        assert (M == h.size - 1).all() and (m == 0).all()
    z = np.zeros((3, 3), np.float32)
    z.ravel()[::2] = -0.0
    M, m = oracle.labels(z)
    assert (M == 8).all() and (m == 0).all()


def test_nz1_equals_2d():
    rng = np.random.default_rng(5)
    for _ in range(5):
        h = _rand_field(rng, (6, 7), levels=4)
        M2, m2 = oracle.labels(h)
        M3, m3 = oracle.labels(h[None])
        assert (M2 == M3[0]).all() and (m2 == m3[0]).all()
        up2, dn2 = oracle.dirs(h)
        up3, dn3 = oracle.dirs(h[None])
        assert (up2 == up3[0]).all() and (dn2 == dn3[0]).all()


def test_separated_bumps_known_maxima():
    """Four well separated positive Gaussians: the maxima are exactly the four centres."""
    ny = nx = 40
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    centres = [(10, 10), (10, 29), (29, 10), (29, 29)]
    h = sum(np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * 5.0 ** 2)) * a
            for (cy, cx), a in zip(centres, (1.0, 0.9, 0.8, 0.7)))
    h = h.astype(np.float32)
    M, m = oracle.labels(h)
    roots = sorted(set(M.ravel().tolist()))
    assert roots == sorted(cy * nx + cx for cy, cx in centres)
    # each vertex flows to the centre of the bump nearest to it (Voronoi cells here are quadrants)
    for (cy, cx) in centres:
        assert M[cy, cx] == cy * nx + cx
        assert M[cy + 2 if cy < 20 else cy - 2, cx] == cy * nx + cx
    # 3D: one blob, one maximum
    z, y, x = np.mgrid[0:12, 0:12, 0:12].astype(np.float64)
    h3 = np.exp(-((x - 6) ** 2 + (y - 5) ** 2 + (z - 4) ** 2) / 18.0).astype(np.float32)
    M3, _ = oracle.labels(h3)
    assert (M3 == 4 * 144 + 5 * 12 + 6).all()


def test_label_invariants():
    rng = np.random.default_rng(6)
    for shape in [(30, 40), (9, 10, 11)]:
        h = _rand_field(rng, shape, levels=50)
        up, dn = oracle.dirs(h)
        M, m = oracle.labels(h)
        upf, Mf = up.ravel(), M.ravel()
        assert (upf[Mf] == Mf).all()                 # labels are maxima
        assert (Mf[upf] == Mf).all()                 # constant along every ascending step
        dnf, mf = dn.ravel(), m.ravel()
        assert (dnf[mf] == mf).all() and (mf[dnf] == mf).all()


# ---------------------------------------------------------------- detection ---

@pytest.mark.parametrize("shape", [(4, 4), (3, 5), (2, 3, 3), (3, 3, 2)])
def test_case_flags_match_definitions(shape):
    rng = np.random.default_rng(7)
    mesh = lit.Mesh(shape)
    for levels in (0, 4):
        for _ in range(6):
            f = _rand_field(rng, shape, levels)
            g = _rand_field(rng, shape, levels)
            flags = oracle.case_flags(f, g).ravel()
            fl, gl = f.ravel(), g.ravel()
            for i in range(mesh.n):
                for t, pred in enumerate(lit.PREDICATES):
                    assert bool(flags[i] >> t & 1) == pred(mesh, fl, gl, i), (i, t)
            cnt = oracle.count_false(f, g)
            for t, name in enumerate(oracle.CASE_NAMES):
                assert cnt[name] == sum(lit.PREDICATES[t](mesh, fl, gl, i) for i in range(mesh.n))
            Mf, mf = lit.labels(mesh, fl)
            Mg, mg = lit.labels(mesh, gl)
            assert cnt["wrong_any"] == sum((Mf[i] != Mg[i]) or (mf[i] != mg[i]) for i in range(mesh.n))


# ----------------------------------------------------------- whole loop ---

def _fpmin_case():
    f = np.array([.80, .48, .30, .85, .50, .90, .75, .95, .99], np.float32).reshape(3, 3)
    fh = f.copy()
    fh[1, 1] = np.float32(.46)
    fh[0, 1] = np.float32(.52)
    return f, fh, np.float32(0.05)


def test_fpmin_counterexample_two_rounds():
    """The single FPmin at the centre is fixed by lowering its f-descent neighbour (vertex 1) twice."""
    f, fh, xi = _fpmin_case()
    cnt = oracle.count_false(f, fh)
    assert cnt["fp_min"] == 1 and cnt["fp_max"] + cnt["fn_max"] + cnt["fn_min"] == 0
    rc, d, g, st = oracle.fix(f, fh, xi)
    assert rc == oracle.OK
    assert st["rounds"] == [0, 2, 0, 0] and st["rounds_r"] == 0
    L1 = lit.lower_bound_exact(f[0, 1], xi)
    g1 = lit.halve_exact(lit.halve_exact(fh[0, 1], L1), L1)
    assert g[0, 1] == g1
    assert abs(float(g1) - 0.4525) < 1e-6
    changed = np.argwhere(g != fh)
    assert changed.tolist() == [[0, 1]]


def test_fpmin_literal_reading_stalls():
    """Lowering the centre's highest neighbour (the printed Eq. 3) never ends the false minimum."""
    f, fh, xi = _fpmin_case()
    rc, d, g, st = oracle.fix(f, fh, xi, fpmin_literal=True)
    assert rc == oracle.ESTALL
    assert g[0, 1] == fh[0, 1]                       # vertex 1 is never touched
    assert g[1, 1] == fh[1, 1]                       # the centre is still the false minimum
    assert g[2, 2] == lit.lower_bound_exact(f[2, 2], xi)


def _check_invariants(f, fh, xi, rc, d, g, st):
    assert rc == oracle.OK
    cnt = oracle.count_false(f, g)
    assert all(v == 0 for v in cnt.values()), cnt
    f64, g64 = f.astype(np.float64), g.astype(np.float64)
    assert (np.abs(f64 - g64) <= float(xi)).all()    # exact for these magnitudes
    assert (g <= fh).all()
    rec = (fh + d).astype(np.float32)
    ok = rec == g
    assert (~ok).sum() == st["n_inexact"]
    assert st["n_edited"] == int((g != fh).sum())


def test_literal_loop_bit_exact_small_grids():
    """The oracle's whole schedule == the literal restatement (path-walk troublemakers, shuffled apply)."""
    rng = np.random.default_rng(8)
    prng = random.Random(8)
    total_rounds = 0
    mislabelled = 0
    cases = 0
    for shape in [(3, 3), (4, 4), (3, 5), (5, 4), (2, 2, 2), (2, 3, 3), (3, 3, 3)]:
        for levels in (0, 5):
            for _ in range(5):
                f, fh, xi = synth.random_small(rng, shape, xi=0.15, levels=levels)
                rc, d, g, st = oracle.fix(f, fh, xi)
                status, lg, lst = lit.fix(f, fh, xi, rng=prng)
                assert status == {0: "ok", -4: "stall", -5: "noconv"}[rc]
                assert (g.view(np.uint32) == lg.view(np.uint32)).all()
                assert st["rounds"] == lst["rounds"] and st["rounds_r"] == lst["rounds_r"]
                assert st["outer_iters"] == lst["outer_iters"]
                # Appendix B's N_f of the start field: brute-force traced labels of fhat against f's
                mesh = lit.Mesh(shape)
                Mh, mh = lit.labels(mesh, fh.ravel())
                Mf, mf = lit.labels(mesh, f.ravel())
                assert st["mislabel_init"] == sum(a != b or c != e for a, b, c, e in zip(Mh, Mf, mh, mf))
                if rc == oracle.OK:
                    _check_invariants(f, fh, xi, rc, d, g, st)
                total_rounds += sum(st["rounds"]) + st["rounds_r"]
                mislabelled += st["mislabel_init"]
                cases += 1
    assert total_rounds > cases  # the cases really exercise the loop
    assert mislabelled > cases


def test_merged_c_rounds_bit_exact_with_literal():
    """The merged C phase (all four types per round, Sec. 6.1) == the literal
    restatement of that schedule, and it reaches zero segmentation error."""
    rng = np.random.default_rng(81)
    prng = random.Random(81)
    total, fewer = 0, 0
    for shape in [(3, 3), (4, 4), (3, 5), (5, 4), (2, 2, 2), (2, 3, 3), (3, 3, 3)]:
        for levels in (0, 5):
            for _ in range(5):
                f, fh, xi = synth.random_small(rng, shape, xi=0.15, levels=levels)
                rc, d, g, st = oracle.fix(f, fh, xi, merged_c=True)
                status, lg, lst = lit.fix(f, fh, xi, rng=prng, merged=True)
                assert status == {0: "ok", -4: "stall", -5: "noconv"}[rc]
                assert (g.view(np.uint32) == lg.view(np.uint32)).all()
                assert st["rounds"] == lst["rounds"] and st["rounds_r"] == lst["rounds_r"]
                assert st["outer_iters"] == lst["outer_iters"]
                if rc == oracle.OK:
                    _check_invariants(f, fh, xi, rc, d, g, st)
                rc1, _, _, st1 = oracle.fix(f, fh, xi)
                total += 1
                fewer += max(st["rounds"]) < sum(st1["rounds"])
    assert fewer > 0  # some cases really had several types in one round


def test_merged_c_rounds_bumps128():
    f, fh, xi = synth.bumps128()[0]
    rc, d, g, st = oracle.fix(f, fh, xi, merged_c=True)
    _check_invariants(f, fh, xi, rc, d, g, st)
    assert rc == oracle.OK and st["n_edited"] > 0


def test_values_stay_on_halving_chain():
    """Every final g_i is reached from fhat_i by repeated halving toward L_i (Eq. 1)."""
    f, fh, xi = synth.bumps128()[0]
    f, fh = f[:48, :48].copy(), fh[:48, :48].copy()
    rc, d, g, st = oracle.fix(f, fh, xi)
    _check_invariants(f, fh, xi, rc, d, g, st)
    L = oracle.lower_bound(f, xi)
    idx = np.argwhere(g != fh)
    assert len(idx) > 0
    for (y, x) in idx[:60]:
        chain = lit.halving_chain(fh[y, x], L[y, x])
        assert any(c.view(np.uint32) == g[y, x].view(np.uint32) for c in chain)


def test_bumps128_converges_with_invariants():
    f, fh, xi = synth.bumps128()[0]
    rc, d, g, st = oracle.fix(f, fh, xi)
    _check_invariants(f, fh, xi, rc, d, g, st)
    assert sum(st["false_init"]) > 0 and st["n_edited"] > 0


def test_exhaustive_orderings_2x3():
    """Every ordering of a 2x3 grid as f, with three random in-bound decompressions each."""
    rng = np.random.default_rng(9)
    xi = np.float32(1.0)
    worst = 0
    for perm in lit.all_orderings(6):
        f = (np.array(perm, np.float32) / np.float32(5)).reshape(2, 3)
        for _ in range(3):
            fh = rng.uniform(0, 1, size=(2, 3)).astype(np.float32)
            rc, d, g, st = oracle.fix(f, fh, xi)
            _check_invariants(f, fh, xi, rc, d, g, st)
            worst = max(worst, sum(st["rounds"]) + st["rounds_r"])
    assert worst > 0


def test_identity_and_order_preserving_inputs():
    rng = np.random.default_rng(10)
    f = rng.uniform(0, 1, size=(20, 30)).astype(np.float32)
    rc, d, g, st = oracle.fix(f, f, np.float32(0.01))
    assert rc == 0 and st["n_edited"] == 0 and not d.any()
    assert sum(st["rounds"]) + st["rounds_r"] == 0 and st["mislabel_init"] == 0
    # same order as f (exact shift by a power of two fraction): nothing to fix
    fi = rng.permutation(600).astype(np.float32).reshape(20, 30)
    rc, d, g, st = oracle.fix(fi, fi + np.float32(0.25), np.float32(0.5))
    assert rc == 0 and st["n_edited"] == 0 and sum(st["false_init"]) == 0 and st["mislabel_init"] == 0
    # reversed order: every vertex's labels are wrong except where both agree by chance (none here:
    # the max of f is the min of -f)
    rc, d, g, st = oracle.fix(fi, -fi, np.float32(1200.0))
    assert st["mislabel_init"] == fi.size


def test_warm_start_resume():
    """Resuming from the converged field does nothing; from a mid-way field it converges."""
    f, fh, xi = synth.bumps128()[0]
    rc, d, g, st = oracle.fix(f, fh, xi)
    rc2, d2, g2, st2 = oracle.fix(f, fh, xi, warm_start=g)
    assert rc2 == 0 and (g2 == g).all() and sum(st2["rounds"]) + st2["rounds_r"] == 0
    L = oracle.lower_bound(f, xi)
    mid = np.maximum(L, fh - np.float32(0.3) * (fh - L)).astype(np.float32)
    rc3, d3, g3, st3 = oracle.fix(f, fh, xi, warm_start=mid)
    _check_invariants(f, fh, xi, rc3, d3, g3, st3)
    bad = mid.copy()
    bad[3, 3] = L[3, 3] - np.float32(1e-3)
    assert oracle.fix(f, fh, xi, warm_start=bad)[0] == oracle.EBOUND


# ------------------------------------------------------------ error paths ---

def test_error_paths():
    f, fh, xi = synth.bumps128()[0]
    bad = fh.copy()
    bad[5, 5] = f[5, 5] + np.float32(2.5) * xi
    assert oracle.fix(f, bad, xi)[0] == oracle.EBOUND
    nan = fh.copy()
    nan[0, 0] = np.nan
    assert oracle.fix(f, nan, xi)[0] == oracle.ENONFINITE
    assert oracle.fix(f, fh, np.float32(np.inf))[0] == oracle.ENONFINITE
    assert oracle.fix(f, fh, np.float32(-1.0))[0] == oracle.EINVAL
    rc, d, g, st = oracle.fix(f, fh, xi, max_rounds=1)
    assert rc == oracle.ENOCONV and sum(st["rounds"]) + st["rounds_r"] == 1
    assert (g <= fh).all() and (g >= oracle.lower_bound(f, xi)).all()
    with pytest.raises(oracle.OracleError):
        oracle.dirs(np.zeros((0, 3), np.float32))


def test_floor_collision_stalls():
    """f_1 < f_0 but float rounding of f - xi gives both the same floor L; index 1 > 0 keeps 1 on top."""
    f0 = np.float32(0.5 + 2.0 ** -23)
    f1 = np.float32(0.5 + 2.0 ** -24)
    xi = np.float32(4.5)
    f = np.array([[f0, f1]], np.float32)
    L = oracle.lower_bound(f, xi)
    assert L[0, 0] == L[0, 1] and f1 < f0
    fh = np.array([[L[0, 0], np.float32(0.0)]], np.float32)
    rc, d, g, st = oracle.fix(f, fh, xi)
    assert rc == oracle.ESTALL
    assert g[0, 1] == L[0, 1]
