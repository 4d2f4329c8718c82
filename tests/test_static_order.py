"""Host-side check of the neighbour order the direction kernel relies on.

The kernel feeds the neighbours of a vertex in a fixed order: first those
with a smaller vertex id, nearest id first, then those with a larger id,
nearest first, so that ties in value are broken by id without comparing ids.
This checks, for every vertex of every small grid, that the fixed slot order
is the true id order of the in-grid neighbours.
"""
import itertools

OFF = {0: (1, 0, 0), 1: (-1, 0, 0), 2: (0, 1, 0), 3: (0, -1, 0), 4: (1, 1, 0), 5: (-1, -1, 0),
       6: (0, 0, 1), 7: (0, 0, -1), 8: (1, 0, 1), 9: (-1, 0, -1), 10: (0, 1, 1), 11: (0, -1, -1),
       12: (1, 1, 1), 13: (-1, -1, -1)}
BELOW = {2: [1, 3, 5], 3: [1, 3, 5, 7, 9, 11, 13]}
ABOVE = {2: [0, 2, 4], 3: [0, 2, 4, 6, 8, 10, 12]}


def _check(ndim, nx, ny, nz):
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        i = x + nx * (y + ny * z)

        def nid(s):
            dx, dy, dz = OFF[s]
            xx, yy, zz = x + dx, y + dy, z + dz
            if 0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz:
                return xx + nx * (yy + ny * zz)
            return None

        below = [nid(s) for s in BELOW[ndim] if nid(s) is not None]
        above = [nid(s) for s in ABOVE[ndim] if nid(s) is not None]
        assert all(a < i for a in below) and all(a > i for a in above)
        assert below == sorted(below, reverse=True) and above == sorted(above)


def test_static_neighbour_order_2d():
    for nx, ny in itertools.product(range(1, 8), repeat=2):
        _check(2, nx, ny, 1)


def test_static_neighbour_order_3d():
    for nx, ny, nz in itertools.product(range(1, 6), repeat=3):
        _check(3, nx, ny, nz)
