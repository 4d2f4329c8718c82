"""Serial CPU oracle for the MSz correction loop (arXiv 2406.09423).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
(``paper_2406_09423_amd``) never does, and the two share no code.

The arithmetic lives in ``msz_ref.c`` (plain serial C, built with
``-ffp-contract=off`` and without fast-math); this module only marshals numpy
arrays through ctypes.  Fields are C-contiguous float32 arrays shaped
``(ny, nx)`` for 2D grids and ``(nz, ny, nx)`` for 3D grids, so the vertex id
is ``x + nx*(y + ny*z)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msz_ref.c")
_SO = os.path.join(_HERE, "libmsz_ref.so")

OK, EINVAL, ENONFINITE, EBOUND, ESTALL, ENOCONV, ENOMEM = 0, -1, -2, -3, -4, -5, -7
FPMAX, FPMIN, FNMAX, FNMIN = 0, 1, 2, 3
CASE_NAMES = ("fp_max", "fp_min", "fn_max", "fn_min")


def build() -> str:
    """Compile the oracle into ``oracle/libmsz_ref.so`` (always recompiles)."""
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class _Options(ctypes.Structure):
    _fields_ = [("max_rounds", ctypes.c_int64), ("warm_start", ctypes.c_void_p),
                ("g_out", ctypes.c_void_p), ("fpmin_literal", ctypes.c_int32),
                ("merged_c", ctypes.c_int32), ("threads", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64 * 4), ("rounds_r", ctypes.c_int64),
                ("outer_iters", ctypes.c_int64), ("n_edited", ctypes.c_int64),
                ("false_init", ctypes.c_int64 * 4), ("mislabel_init", ctypes.c_int64),
                ("n_inexact", ctypes.c_int64),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Counts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("fp_max", "fp_min", "fn_max", "fn_min", "wrong_max", "wrong_min", "wrong_any")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P, I, I64, F = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
        L.msz_ref_lower_bound.argtypes = [P, I64, F, P]
        L.msz_ref_halve.argtypes = [F, F]
        L.msz_ref_halve.restype = F
        L.msz_ref_dirs.argtypes = [P, I, I, I, I, P, P]
        L.msz_ref_labels.argtypes = [P, I, I, I, I, P, P]
        L.msz_ref_count_false.argtypes = [P, P, I, I, I, I, P]
        L.msz_ref_case_flags.argtypes = [P, P, I, I, I, I, P]
        L.msz_ref_delta.argtypes = [F, F, P]
        L.msz_ref_fix.argtypes = [P, P, I, I, I, I, F, P, P, P]
        for fn in (L.msz_ref_lower_bound, L.msz_ref_dirs, L.msz_ref_labels, L.msz_ref_count_false,
                   L.msz_ref_case_flags, L.msz_ref_delta, L.msz_ref_fix):
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def grid_args(shape) -> tuple[int, int, int, int]:
    """(ndim, nx, ny, nz) of a field shaped (ny, nx) or (nz, ny, nx)."""
    if len(shape) == 2:
        return 2, int(shape[1]), int(shape[0]), 1
    if len(shape) == 3:
        return 3, int(shape[2]), int(shape[1]), int(shape[0])
    raise ValueError(f"field must be 2D or 3D, got shape {shape}")


def _f32(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


def lower_bound(f, xi: float) -> np.ndarray:
    f = _f32(f)
    L = np.empty_like(f)
    _check(lib().msz_ref_lower_bound(_ptr(f), f.size, np.float32(xi), _ptr(L)), "lower_bound")
    return L


def halve(g: float, L: float) -> np.float32:
    return np.float32(lib().msz_ref_halve(np.float32(g), np.float32(L)))


def delta(g: float, fhat: float) -> tuple[np.float32, bool]:
    out = np.zeros(1, np.float32)
    ok = lib().msz_ref_delta(np.float32(g), np.float32(fhat), _ptr(out))
    return out[0], bool(ok)


def dirs(h) -> tuple[np.ndarray, np.ndarray]:
    """Steepest ascent / descent neighbour ids, shaped like the field."""
    h = _f32(h)
    up = np.empty(h.shape, np.int32)
    dn = np.empty(h.shape, np.int32)
    _check(lib().msz_ref_dirs(_ptr(h), *grid_args(h.shape), _ptr(up), _ptr(dn)), "dirs")
    return up, dn


def labels(h) -> tuple[np.ndarray, np.ndarray]:
    """(max_label, min_label) extremum ids, shaped like the field."""
    h = _f32(h)
    M = np.empty(h.shape, np.int32)
    m = np.empty(h.shape, np.int32)
    _check(lib().msz_ref_labels(_ptr(h), *grid_args(h.shape), _ptr(M), _ptr(m)), "labels")
    return M, m


def count_false(f, g) -> dict:
    f, g = _f32(f), _f32(g)
    assert f.shape == g.shape
    c = _Counts()
    _check(lib().msz_ref_count_false(_ptr(f), _ptr(g), *grid_args(f.shape), ctypes.byref(c)),
           "count_false")
    return {k: int(getattr(c, k)) for k, _ in _Counts._fields_}


def case_flags(f, g) -> np.ndarray:
    f, g = _f32(f), _f32(g)
    out = np.empty(f.shape, np.uint8)
    _check(lib().msz_ref_case_flags(_ptr(f), _ptr(g), *grid_args(f.shape), _ptr(out)), "case_flags")
    return out


def stats_dict(st: _Stats) -> dict:
    return {
        "rounds": [int(x) for x in st.rounds],
        "rounds_r": int(st.rounds_r),
        "outer_iters": int(st.outer_iters),
        "n_edited": int(st.n_edited),
        "false_init": [int(x) for x in st.false_init],
        "mislabel_init": int(st.mislabel_init),
        "n_inexact": int(st.n_inexact),
        "status": int(st.status),
    }


def fix(f, fhat, xi: float, *, max_rounds: int = 0, warm_start=None, fpmin_literal: bool = False,
        merged_c: bool = False, threads: int = 1):
    """Run the correction loop.  Returns (status, delta, g, stats).  ``threads``
    splits the per-vertex direction loop over that many threads (the result
    does not depend on it); everything else runs serially."""
    f, fhat = _f32(f), _f32(fhat)
    assert f.shape == fhat.shape
    edits = np.zeros(f.shape, np.float32)
    g = np.zeros(f.shape, np.float32)
    opt = _Options()
    opt.max_rounds = int(max_rounds)
    ws = None
    if warm_start is not None:
        ws = _f32(warm_start)
        assert ws.shape == f.shape
        opt.warm_start = _ptr(ws)
    opt.g_out = _ptr(g)
    opt.fpmin_literal = 1 if fpmin_literal else 0
    opt.merged_c = 1 if merged_c else 0
    opt.threads = int(threads)
    st = _Stats()
    rc = lib().msz_ref_fix(_ptr(f), _ptr(fhat), *grid_args(f.shape), np.float32(xi), _ptr(edits),
                           ctypes.byref(opt), ctypes.byref(st))
    return int(rc), edits, g, stats_dict(st)
