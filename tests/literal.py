"""Literal, brute-force restatement of the paper's definitions for tiny grids.

Used only to pin the C oracle.  It is written independently of it and
differently on purpose:
  * neighbours come from a predicate (offset components all in {0,1} or all in
    {0,-1}), not from a table;
  * float32 results are computed with exact rational arithmetic and an
    explicit round-to-nearest-even, not with the machine's float unit;
  * false critical points follow Definitions 1-3 word for word ("for all
    neighbours" loops);
  * labels are traced step by step with no memo;
  * R-loop troublemakers are found by walking each mislabelled vertex's
    integral line to the first divergence (Sec. 5.2), not by the per-vertex
    predicate;
  * edits inside a round are applied in a random order.
"""
from __future__ import annotations

import itertools
import random
from fractions import Fraction

import numpy as np

# ---------------------------------------------------------------- float32 ---

def rne32(q: Fraction) -> np.float32:
    """Round an exact rational to the nearest float32, ties to even."""
    if q == 0:
        return np.float32(0.0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    quantum = Fraction(2) ** (max(e, -126) - 23)
    m = a / quantum
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    val = sign * fl * quantum
    return np.float32(float(val))


def F(x) -> Fraction:
    return Fraction(float(np.float32(x)))


def next_up(x: np.float32) -> np.float32:
    return np.nextafter(np.float32(x), np.float32(np.inf))


def next_down(x: np.float32) -> np.float32:
    return np.nextafter(np.float32(x), np.float32(-np.inf))


def halve_exact(g, L) -> np.float32:
    """Eqs. 2-6 with the float reading: fl(fl(g + L) * 1/2), snapped to L if it equals g."""
    s = rne32(F(g) + F(L))
    h = rne32(F(s) * Fraction(1, 2))
    if F(h) == F(g):
        return np.float32(L)
    return h


def lower_bound_exact(f, xi) -> np.float32:
    """Smallest float32 >= f - xi, exactly."""
    target = F(f) - F(xi)
    c = rne32(target)
    while F(c) < target:
        c = next_up(c)
    while F(next_down(c)) >= target:
        c = next_down(c)
    return c


# ------------------------------------------------------------------- mesh ---

def _is_edge(d) -> bool:
    if all(v == 0 for v in d):
        return False
    return all(v in (0, 1) for v in d) or all(v in (0, -1) for v in d)


def coords(shape, i):
    """(x, y[, z]) of linear id i for a field shaped (ny, nx) or (nz, ny, nx)."""
    if len(shape) == 2:
        ny, nx = shape
        return (i % nx, i // nx)
    nz, ny, nx = shape
    return (i % nx, (i // nx) % ny, i // (nx * ny))


def neighbours(shape, i):
    n = int(np.prod(shape))
    ci = coords(shape, i)
    return [j for j in range(n) if j != i and _is_edge(tuple(a - b for a, b in zip(coords(shape, j), ci)))]


class Mesh:
    def __init__(self, shape):
        self.shape = tuple(shape)
        self.n = int(np.prod(shape))
        self.nb = [neighbours(self.shape, i) for i in range(self.n)]


# ------------------------------------------------------------------ order ---

def key(h, i):
    return (float(h[i]), i)


def dirs(mesh: Mesh, h):
    up = [max([i] + mesh.nb[i], key=lambda j: key(h, j)) for i in range(mesh.n)]
    dn = [min([i] + mesh.nb[i], key=lambda j: key(h, j)) for i in range(mesh.n)]
    return up, dn


def trace(ptr, i):
    path = [i]
    while ptr[path[-1]] != path[-1]:
        path.append(ptr[path[-1]])
    return path


def labels(mesh: Mesh, h):
    up, dn = dirs(mesh, h)
    return [trace(up, i)[-1] for i in range(mesh.n)], [trace(dn, i)[-1] for i in range(mesh.n)]


# --------------------------------------------------------- Definitions 1-3 ---

def is_max(mesh, h, i):
    return all(key(h, i) > key(h, j) for j in mesh.nb[i])


def is_min(mesh, h, i):
    return all(key(h, i) < key(h, j) for j in mesh.nb[i])


def fp_max(mesh, f, g, i):   # Def. 1
    return is_max(mesh, g, i) and any(key(f, i) < key(f, j) for j in mesh.nb[i])


def fp_min(mesh, f, g, i):   # Def. 2
    return is_min(mesh, g, i) and any(key(f, i) > key(f, j) for j in mesh.nb[i])


def fn_max(mesh, f, g, i):   # Def. 3
    return (not is_max(mesh, g, i)) and all(key(f, i) > key(f, j) for j in mesh.nb[i])


def fn_min(mesh, f, g, i):   # Def. 3
    return (not is_min(mesh, g, i)) and all(key(f, i) < key(f, j) for j in mesh.nb[i])


PREDICATES = (fp_max, fp_min, fn_max, fn_min)


def highest_neighbour(mesh, h, i):
    return max(mesh.nb[i], key=lambda j: key(h, j))


def lowest_neighbour(mesh, h, i):
    return min(mesh.nb[i], key=lambda j: key(h, j))


def c_target(mesh, t, f, g, i):
    if t == 0:                    # FPmax: lower the vertex itself (Eq. 2)
        return i
    if t == 1:                    # FPmin: lower the neighbour that is lower in f (Lemma-1 reading)
        return lowest_neighbour(mesh, f, i)
    if t == 2:                    # FNmax: lower the highest neighbour in g (Eq. 4)
        return highest_neighbour(mesh, g, i)
    return i                      # FNmin: lower the vertex itself (Eq. 5)


def r_targets(mesh, f, g, Mf, mf):
    """Walk every mislabelled vertex's integral lines to the first divergence (Sec. 5.2)."""
    upf, dnf = dirs(mesh, f)
    upg, dng = dirs(mesh, g)
    Mg, mg = labels(mesh, g)
    targets = set()
    for i in range(mesh.n):
        if mg[i] != mf[i]:
            for u in trace(dng, i):
                if dng[u] != dnf[u]:
                    targets.add(dnf[u])   # reroute a wrong minimum through the f-descent
                    break
        if Mg[i] != Mf[i]:
            for u in trace(upg, i):
                if upg[u] != upf[u]:
                    targets.add(upg[u])   # push the wrong ascent neighbour down
                    break
    return targets


def fix(f, fhat, xi, rng: random.Random | None = None, max_rounds: int = 100000, merged: bool = False):
    """The synchronous-round schedule; returns (status, g, stats) with status in {'ok','stall','noconv'}.
    merged: every C round takes the cases of all four types from one snapshot
    (the parallel C-loop of Sec. 6.1) instead of one type per sub-loop."""
    rng = rng or random.Random(0)
    shape = f.shape
    mesh = Mesh(shape)
    f = [np.float32(v) for v in f.ravel()]
    g = [np.float32(v) for v in fhat.ravel()]
    L = [lower_bound_exact(v, xi) for v in f]
    Mf, mf = labels(mesh, f)
    stats = {"rounds": [0, 0, 0, 0], "rounds_r": 0, "outer_iters": 0}
    rounds = 0

    def apply(targets):
        nonlocal rounds
        order = sorted(targets)
        rng.shuffle(order)
        changed = 0
        for t in order:
            h = halve_exact(g[t], L[t])
            if F(h) != F(g[t]):
                changed += 1
            g[t] = h
        return changed

    def any_c():
        return any(p(mesh, f, g, i) for p in PREDICATES for i in range(mesh.n))

    while True:
        stats["outer_iters"] += 1
        while merged:
            found = [[i for i in range(mesh.n) if PREDICATES[t](mesh, f, g, i)] for t in range(4)]
            if not any(found):
                break
            if rounds >= max_rounds:
                return "noconv", np.array(g, np.float32).reshape(shape), stats
            if apply({c_target(mesh, t, f, g, i) for t in range(4) for i in found[t]}) == 0:
                return "stall", np.array(g, np.float32).reshape(shape), stats
            rounds += 1
            for t in range(4):
                stats["rounds"][t] += bool(found[t])
        while not merged:
            for t in range(4):
                while True:
                    cases = [i for i in range(mesh.n) if PREDICATES[t](mesh, f, g, i)]
                    if not cases:
                        break
                    if rounds >= max_rounds:
                        return "noconv", np.array(g, np.float32).reshape(shape), stats
                    if apply({c_target(mesh, t, f, g, i) for i in cases}) == 0:
                        return "stall", np.array(g, np.float32).reshape(shape), stats
                    rounds += 1
                    stats["rounds"][t] += 1
            if not any_c():
                break
        while True:
            Mg, mg = labels(mesh, g)
            if Mg == Mf and mg == mf:
                return "ok", np.array(g, np.float32).reshape(shape), stats
            tg = r_targets(mesh, f, g, Mf, mf)
            if rounds >= max_rounds:
                return "noconv", np.array(g, np.float32).reshape(shape), stats
            if apply(tg) == 0:
                return "stall", np.array(g, np.float32).reshape(shape), stats
            rounds += 1
            stats["rounds_r"] += 1
            if any_c():
                break


def halving_chain(start, L):
    """All values visited by repeated halving from start down to L (inclusive)."""
    chain = [np.float32(start)]
    while F(chain[-1]) != F(L):
        chain.append(halve_exact(chain[-1], L))
    return chain


def all_orderings(n):
    return itertools.permutations(range(n))
