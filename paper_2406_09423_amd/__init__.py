"""MSz correction loop on AMD Instinct MI355X (gfx950).

A thin ctypes binding over ``libmsz.so`` (the C ABI in ``include/msz.h``).
Every step of the correction runs in the library's HIP kernels; this module
only passes device pointers, sizes and the current stream.  PyTorch provides
device memory and streams.  There is no CPU fallback: if ``libmsz.so`` has
not been built, the first call raises.

Fields are contiguous float32 CUDA tensors shaped ``(ny, nx)`` (2D, 6
neighbours) or ``(nz, ny, nx)`` (3D, Freudenthal 14 neighbours), so that the
vertex id is ``x + nx*(y + ny*z)``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsz.so")

OK, EINVAL, ENONFINITE, EBOUND, ESTALL, ENOCONV, EDEVICE, ENOMEM, ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7, -8
NOALLOC_SCRATCH_BYTES = 96 << 20  # the static device scratch of msz_fix_noalloc
CASE_NAMES = ("fp_max", "fp_min", "fn_max", "fn_min")
PHASES = ("validate", "dirs", "dirs_detect", "refresh", "apply", "label_tile", "label_jump",
          "label_final", "detect_r", "delta", "net")
NET_PARAMS = 14289
NET_FEATURES = 16
N_PHASES = len(PHASES)
FLAG_TIMING = 1
FLAG_MERGED_C = 2  # merged C rounds (all four case types per round)
FLAG_COUNT_INIT = 4  # count the start field's mislabelled vertices (stats["mislabel_init"], else -1)
FLAG_PREEMPTIVE = 8  # merged C rounds whose shared targets are edited without claims (not deterministic)


class Dims(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64 * 4), ("rounds_r", ctypes.c_int64),
                ("outer_iters", ctypes.c_int64), ("n_edited", ctypes.c_int64),
                ("false_init", ctypes.c_int64 * 4), ("mislabel_init", ctypes.c_int64),
                ("n_inexact", ctypes.c_int64), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("phase_ms", ctypes.c_float * N_PHASES), ("phase_launches", ctypes.c_int32 * N_PHASES)]

    def timing(self) -> dict:
        """Per-kernel GPU time (ms) and launches, filled when the call ran with timing on."""
        return {name: {"ms": float(self.phase_ms[k]), "launches": int(self.phase_launches[k])}
                for k, name in enumerate(PHASES)}

    def as_dict(self) -> dict:
        return {
            "rounds": [int(x) for x in self.rounds],
            "rounds_r": int(self.rounds_r),
            "outer_iters": int(self.outer_iters),
            "n_edited": int(self.n_edited),
            "false_init": [int(x) for x in self.false_init],
            "mislabel_init": int(self.mislabel_init),
            "n_inexact": int(self.n_inexact),
            "status": int(self.status),
        }


class FalseCounts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("fp_max", "fp_min", "fn_max", "fn_min", "wrong_max", "wrong_min", "wrong_any")]


class Options(ctypes.Structure):
    _fields_ = [("max_rounds", ctypes.c_int64), ("warm_start", ctypes.c_void_p),
                ("g_out", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("tile_override", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p), ("fhat", ctypes.c_void_p), ("d", Dims),
                ("xi", ctypes.c_float), ("tile", ctypes.c_int32), ("edits_out", ctypes.c_void_p),
                ("g_out", ctypes.c_void_p), ("stats", ctypes.POINTER(Stats))]


class EditStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "n_edits", "bytes", "index_bits", "value_bits")]


class Launch(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("phase", ctypes.c_int32), ("us", ctypes.c_double),
                ("bytes", ctypes.c_int64)]


KERNELS = ("step1_2d", "step1_3d", "batch_2d", "batch_3d")  # MSZ_KERNEL_*: device names below
KERNEL_SYMBOLS = ("k_eng_step1<2>", "k_eng_step1<3>", "k_eng_step<2>", "k_eng_step<3>")


class MszError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libmsz.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2406_09423_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, F, I32 = ctypes.c_void_p, ctypes.c_float, ctypes.c_int32
        L.msz_fix.argtypes = [P, P, Dims, F, P, ctypes.POINTER(Options), ctypes.POINTER(Stats), P]
        L.msz_fix_noalloc.argtypes = [P, P, Dims, F, P, ctypes.POINTER(Options), ctypes.POINTER(Stats), P]
        L.msz_labels.argtypes = [P, Dims, P, P, P]
        L.msz_count_false.argtypes = [P, P, Dims, ctypes.POINTER(FalseCounts), P]
        L.msz_fix_batch.argtypes = [ctypes.POINTER(Job), I32, ctypes.POINTER(Options), P]
        L.msz_workspace_bytes.argtypes = [Dims]
        L.msz_workspace_bytes.restype = ctypes.c_size_t
        L.msz_batch_workspace_bytes.argtypes = [ctypes.POINTER(Job), I32]
        L.msz_batch_workspace_bytes.restype = ctypes.c_size_t
        L.msz_tile_variants.argtypes = [I32]
        L.msz_last_launches.argtypes = [P, I32]
        L.msz_last_launches.restype = I32
        L.msz_last_schedule.argtypes = [P, I32]
        L.msz_last_schedule.restype = I32
        L.msz_strerror.argtypes = [ctypes.c_int]
        L.msz_strerror.restype = ctypes.c_char_p
        L.msz_net_workspace_bytes.argtypes = [Dims]
        L.msz_net_workspace_bytes.restype = ctypes.c_size_t
        L.msz_learned_workspace_bytes.argtypes = [Dims]
        L.msz_learned_workspace_bytes.restype = ctypes.c_size_t
        L.msz_net_features.argtypes = [P, P, Dims, F, P, P, ctypes.c_size_t, P]
        L.msz_net_forward.argtypes = [P, P, Dims, P, P, P, P, ctypes.c_size_t, P]
        L.msz_net_halvings.argtypes = [P, P, P, Dims, F, P, P, ctypes.c_size_t, P]
        L.msz_net_gradients.argtypes = [P, P, P, F, Dims, P, ctypes.POINTER(ctypes.c_float), P,
                                        ctypes.c_size_t, P]
        L.msz_net_adam.argtypes = [P, P, P, P, I32, I32, F, P]
        L.msz_fix_learned.argtypes = [P, P, Dims, F, P, F, P, ctypes.POINTER(Options),
                                      ctypes.POINTER(Stats), P]
        L.msz_edits_bound.argtypes = [ctypes.c_int64]
        L.msz_edits_bound.restype = ctypes.c_size_t
        L.msz_encode_edits.argtypes = [P, ctypes.c_int64, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(EditStats), P]
        L.msz_decode_edits.argtypes = [P, ctypes.c_size_t, P, ctypes.c_int64, P]
        for fn in (L.msz_fix, L.msz_fix_noalloc, L.msz_labels, L.msz_count_false, L.msz_fix_batch, L.msz_tile_variants,
                   L.msz_net_features, L.msz_net_forward, L.msz_net_gradients, L.msz_net_adam,
                   L.msz_fix_learned, L.msz_net_halvings, L.msz_encode_edits, L.msz_decode_edits):
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().msz_strerror(int(code)).decode()
    except ImportError:
        return str(code)


def dims_of(shape) -> Dims:
    if len(shape) == 2:
        return Dims(2, int(shape[1]), int(shape[0]), 1)
    if len(shape) == 3:
        return Dims(3, int(shape[2]), int(shape[1]), int(shape[0]))
    raise ValueError(f"fields are 2D (ny, nx) or 3D (nz, ny, nx), got shape {tuple(shape)}")


def _flags(timing: bool, merged: bool, count_init: bool, preemptive: bool = False) -> int:
    return ((FLAG_TIMING if timing else 0) | (FLAG_MERGED_C if merged else 0) | (FLAG_COUNT_INIT if count_init else 0)
            | (FLAG_PREEMPTIVE if preemptive else 0))


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_field(t, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 tensor")


def workspace_bytes(shape) -> int:
    return int(lib().msz_workspace_bytes(dims_of(shape)))


def tile_variants(ndim: int) -> int:
    return int(lib().msz_tile_variants(int(ndim)))


def fix(f, fhat, xi: float, *, max_rounds: int = 0, warm_start=None, want_g: bool = True,
        workspace=None, tile: int = 0, edits_out=None, g_out=None, timing: bool = False,
        merged: bool = False, count_init: bool = False, preemptive: bool = False, stream=None):
    """Runs the correction loop on the GPU.

    Returns ``(status, delta, g, stats)``: ``delta`` with fl(fhat + delta) == g,
    ``g`` the edited field (None unless ``want_g``), ``stats`` a dict (with a
    per-kernel ``"timing"`` entry when ``timing`` is set; ``mislabel_init`` is
    -1 unless ``count_init``).
    """
    import torch
    _check_field(f, "f")
    _check_field(fhat, "fhat")
    if f.shape != fhat.shape:
        raise ValueError("f and fhat differ in shape")
    d = dims_of(f.shape)
    edits = edits_out if edits_out is not None else torch.empty_like(f)
    g = g_out if g_out is not None else (torch.empty_like(f) if want_g else None)
    opt = Options()
    opt.max_rounds = int(max_rounds)
    if warm_start is not None:
        _check_field(warm_start, "warm_start")
        opt.warm_start = warm_start.data_ptr()
    opt.g_out = g.data_ptr() if g is not None else None
    if workspace is not None:
        opt.workspace = workspace.data_ptr()
        opt.workspace_bytes = workspace.numel() * workspace.element_size()
    opt.tile_override = int(tile)
    opt.flags = _flags(timing, merged, count_init, preemptive)
    st = Stats()
    rc = lib().msz_fix(f.data_ptr(), fhat.data_ptr(), d, float(xi), edits.data_ptr(),
                       ctypes.byref(opt), ctypes.byref(st), _stream(stream))
    out = st.as_dict()
    if timing:
        out["timing"] = st.timing()
    return int(rc), edits, g, out


def fix_noalloc(f, fhat, xi: float, *, max_rounds: int = 0, warm_start=None, edits_out=None, g_out=None,
                tile: int = 0, merged: bool = False, count_init: bool = False, preemptive: bool = False, stream=None):
    """msz_fix_noalloc: the correction loop with all scratch in the library's
    static device array (no allocation inside the call).  ``edits_out`` and
    ``g_out`` (optional) are caller-owned outputs; returns ``(status, delta,
    g, stats)`` like :func:`fix`."""
    import torch
    _check_field(f, "f")
    _check_field(fhat, "fhat")
    if f.shape != fhat.shape:
        raise ValueError("f and fhat differ in shape")
    edits = edits_out if edits_out is not None else torch.empty_like(f)
    opt = Options()
    opt.max_rounds = int(max_rounds)
    if warm_start is not None:
        _check_field(warm_start, "warm_start")
        opt.warm_start = warm_start.data_ptr()
    opt.g_out = g_out.data_ptr() if g_out is not None else None
    opt.tile_override = int(tile)
    opt.flags = _flags(False, merged, count_init, preemptive)
    st = Stats()
    rc = lib().msz_fix_noalloc(f.data_ptr(), fhat.data_ptr(), dims_of(f.shape), float(xi), edits.data_ptr(),
                               ctypes.byref(opt), ctypes.byref(st), _stream(stream))
    return int(rc), edits, g_out, st.as_dict()


def last_launches() -> list:
    """Every step-kernel launch of this thread's last timed fix / fix_batch:
    dicts with the kernel name, phase (None for batch or idle steps), duration
    (us, GPU clock stamps) and the algorithmic bytes its blocks visited."""
    n = int(lib().msz_last_launches(None, 0))
    buf = (Launch * max(n, 1))()
    lib().msz_last_launches(ctypes.cast(buf, ctypes.c_void_p), n)
    return [{"kernel": KERNELS[buf[k].kernel], "phase": PHASES[buf[k].phase] if buf[k].phase >= 0 else None,
             "us": float(buf[k].us), "bytes": int(buf[k].bytes)} for k in range(n)]


def last_schedule() -> list:
    """Phase index of every step of this thread's last timed fix (-1: idle step)."""
    n = int(lib().msz_last_schedule(None, 0))
    buf = (ctypes.c_int32 * max(n, 1))()
    lib().msz_last_schedule(ctypes.cast(buf, ctypes.c_void_p), n)
    return [int(buf[k]) for k in range(n)]


def labels(field, stream=None):
    """(max_label, min_label) int32 tensors of extremum vertex ids."""
    import torch
    _check_field(field, "field")
    M = torch.empty(field.shape, dtype=torch.int32, device=field.device)
    m = torch.empty_like(M)
    rc = lib().msz_labels(field.data_ptr(), dims_of(field.shape), M.data_ptr(), m.data_ptr(),
                          _stream(stream))
    if rc != OK:
        raise MszError(rc, "msz_labels")
    return M, m


def count_false(f, g, stream=None) -> dict:
    _check_field(f, "f")
    _check_field(g, "g")
    c = FalseCounts()
    rc = lib().msz_count_false(f.data_ptr(), g.data_ptr(), dims_of(f.shape), ctypes.byref(c),
                               _stream(stream))
    if rc != OK:
        raise MszError(rc, "msz_count_false")
    return {k: int(getattr(c, k)) for k, _ in FalseCounts._fields_}


def edits_bound(n: int) -> int:
    return int(lib().msz_edits_bound(int(n)))


def encode_edits(edits, out=None, stream=None):
    """Lossless encoding of an edit field (msz_encode_edits).  Returns
    ``(status, blob, stats)``: ``blob`` a uint8 device tensor of the encoded
    bytes (a view of ``out`` when given)."""
    import torch
    _check_field(edits, "edits")
    n = edits.numel()
    if out is None:
        out = torch.empty(max(edits_bound(n), 16), dtype=torch.uint8, device=edits.device)
    size = ctypes.c_size_t(0)
    st = EditStats()
    rc = lib().msz_encode_edits(edits.data_ptr(), n, out.data_ptr(), out.numel(), ctypes.byref(size),
                                ctypes.byref(st), _stream(stream))
    return int(rc), out[: size.value], {k: int(getattr(st, k)) for k, _ in EditStats._fields_}


def decode_edits(blob, shape, out=None, stream=None):
    """Dense float32 edits of ``shape`` from an encoded blob (msz_decode_edits)."""
    import torch
    if blob.dtype != torch.uint8 or not blob.is_cuda or not blob.is_contiguous():
        raise ValueError("blob must be a contiguous uint8 CUDA tensor")
    n = 1
    for s_ in shape:
        n *= int(s_)
    if out is None:
        out = torch.empty(tuple(int(s_) for s_ in shape), dtype=torch.float32, device=blob.device)
    rc = lib().msz_decode_edits(blob.data_ptr(), blob.numel(), out.data_ptr(), n, _stream(stream))
    return int(rc), out


def fix_batch(fields, *, max_rounds: int = 0, want_g: bool = True, workspace=None, tiles="auto", outs=None,
              merged: bool = False, count_init: bool = False, preemptive: bool = False, timing: bool = False,
              stream=None):
    """Corrects a list of (f, fhat, xi) together in one device-scheduled run (msz_fix_batch).

    With ``timing`` every step-kernel launch is recorded (see :func:`last_launches`).

    ``tiles``: each field's direction tile variant, "auto" (the autotuner's
    table, autotune.py) or None (the default tile).  ``outs`` optionally gives
    preallocated (delta_j, g_j) pairs.  Returns
    ``(status, [(status_j, delta_j, g_j, stats_j), ...])``.
    """
    import torch
    n = len(fields)
    if isinstance(tiles, str):
        if tiles != "auto":
            raise ValueError(f"tiles must be 'auto', None or a list, got {tiles!r}")
        from . import autotune
        tiles = autotune.tiles_for([f.shape for f, _, _ in fields])
    jobs = (Job * n)()
    stats = [Stats() for _ in range(n)]
    pairs = []
    for j, (f, fh, xi) in enumerate(fields):
        _check_field(f, f"f[{j}]")
        _check_field(fh, f"fhat[{j}]")
        if outs is not None:
            e, g = outs[j]
        else:
            e = torch.empty_like(f)
            g = torch.empty_like(f) if want_g else None
        jobs[j].f, jobs[j].fhat = f.data_ptr(), fh.data_ptr()
        jobs[j].d = dims_of(f.shape)
        jobs[j].xi = float(xi)
        jobs[j].tile = int(tiles[j]) if tiles is not None else 0
        jobs[j].edits_out = e.data_ptr()
        jobs[j].g_out = g.data_ptr() if g is not None else None
        jobs[j].stats = ctypes.pointer(stats[j])
        pairs.append((e, g))
    opt = Options()
    opt.max_rounds = int(max_rounds)
    opt.flags = _flags(timing, merged, count_init, preemptive)
    if workspace is not None:
        opt.workspace = workspace.data_ptr()
        opt.workspace_bytes = workspace.numel() * workspace.element_size()
    rc = lib().msz_fix_batch(jobs, n, ctypes.byref(opt), _stream(stream))
    res = [(stats[j].status, pairs[j][0], pairs[j][1], stats[j].as_dict()) for j in range(n)]
    return int(rc), res


def batch_workspace_bytes(shapes) -> int:
    n = len(shapes)
    jobs = (Job * n)()
    for j, s in enumerate(shapes):
        jobs[j].d = dims_of(s)
    return int(lib().msz_batch_workspace_bytes(jobs, n))


# ------------------------------------------------------------------ learned ---

def _ws_arg(workspace):
    if workspace is None:
        return None, 0
    return workspace.data_ptr(), workspace.numel() * workspace.element_size()


def net_workspace_bytes(shape) -> int:
    return int(lib().msz_net_workspace_bytes(dims_of(shape)))


def learned_workspace_bytes(shape) -> int:
    return int(lib().msz_learned_workspace_bytes(dims_of(shape)))


def net_features(f, fhat, xi: float, *, workspace=None, stream=None):
    """BF16 features [n][16] of (f, fhat, xi), returned as an int16 tensor of raw bits."""
    import torch
    _check_field(f, "f")
    _check_field(fhat, "fhat")
    feat = torch.empty((f.numel(), NET_FEATURES), dtype=torch.int16, device=f.device)
    wp, wb = _ws_arg(workspace)
    rc = lib().msz_net_features(f.data_ptr(), fhat.data_ptr(), dims_of(f.shape), float(xi), feat.data_ptr(),
                                wp, wb, _stream(stream))
    if rc != OK:
        raise MszError(rc, "msz_net_features")
    return feat


def net_forward(params, feat, shape, *, hidden: bool = False, workspace=None, stream=None):
    """p[n] (float32); with ``hidden`` also the two hidden activations ([n][16] BF16 bits)."""
    import torch
    n = feat.shape[0]
    p = torch.empty(n, dtype=torch.float32, device=feat.device)
    a1 = a2 = None
    if hidden:
        a1 = torch.empty((n, 16), dtype=torch.int16, device=feat.device)
        a2 = torch.empty((n, 16), dtype=torch.int16, device=feat.device)
    wp, wb = _ws_arg(workspace)
    rc = lib().msz_net_forward(params.data_ptr(), feat.data_ptr(), dims_of(shape), p.data_ptr(),
                               a1.data_ptr() if a1 is not None else None,
                               a2.data_ptr() if a2 is not None else None, wp, wb, _stream(stream))
    if rc != OK:
        raise MszError(rc, "msz_net_forward")
    return (p, a1, a2) if hidden else p


def net_gradients(params, feat, target, shape, *, edit_weight: float = 0.0, grad_out=None, workspace=None,
                  stream=None):
    """(loss, grad) of the weighted mean squared error; grad has the parameter layout."""
    import torch
    g = grad_out if grad_out is not None else torch.empty_like(params)
    loss = ctypes.c_float(0.0)
    wp, wb = _ws_arg(workspace)
    rc = lib().msz_net_gradients(params.data_ptr(), feat.data_ptr(), target.data_ptr(), float(edit_weight),
                                 dims_of(shape), g.data_ptr(), ctypes.byref(loss), wp, wb, _stream(stream))
    if rc != OK:
        raise MszError(rc, "msz_net_gradients")
    return float(loss.value), g


def net_halvings(f, fhat, g, xi: float, *, workspace=None, stream=None):
    """Per-vertex number of halvings from fhat to g (-1 off the chain), float32."""
    import torch
    _check_field(g, "g")
    k = torch.empty_like(g)
    wp, wb = _ws_arg(workspace)
    rc = lib().msz_net_halvings(f.data_ptr(), fhat.data_ptr(), g.data_ptr(), dims_of(f.shape), float(xi),
                                k.data_ptr(), wp, wb, _stream(stream))
    if rc != OK:
        raise MszError(rc, "msz_net_halvings")
    return k


def net_adam(params, grad, m, v, step: int, lr: float, stream=None):
    rc = lib().msz_net_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), params.numel(),
                            int(step), float(lr), _stream(stream))
    if rc != OK:
        raise MszError(rc, "msz_net_adam")


def fix_learned(f, fhat, xi: float, params, *, p_min: float = 0.5, max_rounds: int = 0, want_g: bool = True,
                workspace=None, edits_out=None, g_out=None, timing: bool = False, merged: bool = False,
                count_init: bool = False, preemptive: bool = False, stream=None):
    """msz_fix warm-started by the network; same return value as fix()."""
    import torch
    _check_field(f, "f")
    _check_field(fhat, "fhat")
    edits = edits_out if edits_out is not None else torch.empty_like(f)
    g = g_out if g_out is not None else (torch.empty_like(f) if want_g else None)
    opt = Options()
    opt.max_rounds = int(max_rounds)
    opt.g_out = g.data_ptr() if g is not None else None
    if workspace is not None:
        opt.workspace = workspace.data_ptr()
        opt.workspace_bytes = workspace.numel() * workspace.element_size()
    opt.flags = _flags(timing, merged, count_init, preemptive)
    st = Stats()
    rc = lib().msz_fix_learned(f.data_ptr(), fhat.data_ptr(), dims_of(f.shape), float(xi), params.data_ptr(),
                               float(p_min), edits.data_ptr(), ctypes.byref(opt), ctypes.byref(st),
                               _stream(stream))
    out = st.as_dict()
    if timing:
        out["timing"] = st.timing()
    return int(rc), edits, g, out
