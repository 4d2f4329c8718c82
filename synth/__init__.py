"""Seeded synthetic inputs for the MSz correction loop.

This module holds input generation only, none of the correction method's
arithmetic: it is shared by the tests, the oracle timing leg and the GPU
benchmark so that both sides see identical bytes.

Fields are generated in float64 with numpy's PCG64 (``default_rng(seed)``),
normalised, then rounded to float32 (round-to-nearest-even).  The stand-in
for the paper's error-bounded compressor (SZ3/ZFP, not available) is a
uniform quantiser, ``fhat = 2 xi * rint(f / (2 xi))`` evaluated in double and
rounded to float32, followed by a one-ulp nudge toward ``f`` wherever float32
rounding pushed it past the bound, so that ``|f - fhat| <= xi`` holds.

Array layout: C-contiguous, shape ``(ny, nx)`` in 2D and ``(nz, ny, nx)`` in
3D (x fastest).
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 240609423


def seed_for(config: int, k: int = 0) -> int:
    """Seed of field ``k`` of workload ``config`` (0-based workload number)."""
    return BASE_SEED + 1000 * config + k


def _normalise(a: np.ndarray) -> np.ndarray:
    lo, hi = float(a.min()), float(a.max())
    return (a - lo) / (hi - lo) if hi > lo else np.zeros_like(a)


def gaussian_random_field(shape, power_exponent: float, rng: np.random.Generator) -> np.ndarray:
    """Float64 field in [0, 1] with power spectrum ~ k^-power_exponent.

    White N(0,1) noise is filtered in Fourier space by the amplitude
    k^(-power_exponent/2) (k in integer wavenumbers, the k = 0 mode zeroed),
    transformed back and min-max normalised.
    """
    shape = tuple(int(s) for s in shape)
    white = rng.standard_normal(shape)
    spec = np.fft.rfftn(white)
    axes_k = [np.fft.fftfreq(n) * n for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1]) * shape[-1]]
    k2 = np.zeros(spec.shape, dtype=np.float64)
    for ax, kk in enumerate(axes_k):
        sh = [1] * len(shape)
        sh[ax] = kk.size
        k2 = k2 + (kk.reshape(sh) ** 2)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (-power_exponent / 4.0), 0.0)  # (k^2)^(-p/4) = k^(-p/2)
    spec *= amp
    del k2, amp
    out = np.fft.irfftn(spec, s=shape, axes=tuple(range(len(shape))))
    return _normalise(out)


def _gauss_1d(n: int, c: float, sigma: float) -> np.ndarray:
    x = np.arange(n, dtype=np.float64)
    return np.exp(-0.5 * ((x - c) / sigma) ** 2)


def bumps_2d(nx: int, ny: int, nbumps: int, rng: np.random.Generator, noise_std: float) -> np.ndarray:
    """Sum of Gaussian bumps (centres U[0,n), sigma U[3,15] px, amplitude U[-1,1]) + N(0, noise_std)."""
    out = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(nbumps):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        s = rng.uniform(3, 15)
        a = rng.uniform(-1, 1)
        out += a * np.outer(_gauss_1d(ny, cy, s), _gauss_1d(nx, cx, s))
    if noise_std > 0:
        out += rng.normal(0.0, noise_std, size=out.shape)
    return out


def blobs_3d(shape, nblobs: int, rng: np.random.Generator, amp: float = 0.5) -> np.ndarray:
    """Sum of separable Gaussian blobs: centres U[0,n)^3, sigma U[3,15], amplitude U[-amp, amp]."""
    nz, ny, nx = shape
    out = np.zeros(shape, dtype=np.float64)
    for _ in range(nblobs):
        cx, cy, cz = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)
        s = rng.uniform(3, 15)
        a = rng.uniform(-amp, amp)
        gz, gy, gx = _gauss_1d(nz, cz, s), _gauss_1d(ny, cy, s), _gauss_1d(nx, cx, s)
        out += a * (gz[:, None, None] * np.outer(gy, gx)[None, :, :])
    return out


def xi_for(f32: np.ndarray, rel: float) -> np.float32:
    """Absolute bound xi = float32(rel * (max f - min f))."""
    return np.float32(rel * (float(f32.max()) - float(f32.min())))


def quantize(f32: np.ndarray, xi: float) -> np.ndarray:
    """Quantising decompressor fhat = float32(2 xi * rint(f / (2 xi))), nudged into |f - fhat| <= xi."""
    f64 = f32.astype(np.float64)
    x = float(np.float32(xi))
    if x == 0.0:
        return f32.copy()
    q = (2.0 * x) * np.rint(f64 / (2.0 * x))
    fh = q.astype(np.float32)
    for _ in range(4):
        d = f64 - fh.astype(np.float64)   # exact for the magnitudes generated here
        hi = d < -x                       # fhat too high
        lo = d > x                        # fhat too low
        if not (hi.any() or lo.any()):
            break
        fh[hi] = np.nextafter(fh[hi], np.float32(-np.inf))
        fh[lo] = np.nextafter(fh[lo], np.float32(np.inf))
    return fh


# ---------------------------------------------------------------------------
# The five workloads.  Each returns a list of (f, fhat, xi) with float32 arrays.
# ---------------------------------------------------------------------------

def bumps128(k: int = 0, n: int = 128, rel: float = 1e-3):
    """2D 128x128: 32 Gaussian bumps + N(0, 1e-3) noise; xi = 1e-3 x range; 6-neighbour mesh."""
    rng = np.random.default_rng(seed_for(0, k))
    f = bumps_2d(n, n, 32, rng, 1e-3).astype(np.float32)
    xi = xi_for(f, rel)
    return [(f, quantize(f, xi), xi)]


def ocean2d(k: int = 0, nx: int = 3600, ny: int = 2400, rels=(1e-4, 1e-3)):
    """2D 3600x2400 GRF, power ~k^-3, in [0,1]; xi in {1e-4, 1e-3} (range is 1)."""
    rng = np.random.default_rng(seed_for(1, k))
    f = gaussian_random_field((ny, nx), 3.0, rng).astype(np.float32)
    out = []
    for rel in rels:
        xi = xi_for(f, rel)
        out.append((f, quantize(f, xi), xi))
    return out


def turb3d(k: int = 0, n: int = 256, rel: float = 1e-3, nblobs: int = 64):
    """3D n^3 GRF, power ~k^-11/3, + 64 Gaussian blobs, renormalised to [0,1]; xi = 1e-3 x range."""
    rng = np.random.default_rng(seed_for(2, k))
    base = gaussian_random_field((n, n, n), 11.0 / 3.0, rng)
    base += blobs_3d((n, n, n), nblobs, rng, amp=0.5)
    f = _normalise(base).astype(np.float32)
    del base
    xi = xi_for(f, rel)
    return [(f, quantize(f, xi), xi)]


def batch_shapes(k: int = 0, n2d: int = 64, n3d: int = 32, lo2: int = 64, hi2: int = 2048,
                 lo3: int = 32, hi3: int = 192):
    """Shapes and relative bounds of the uneven batch: 2D sides iid U{lo2..hi2}, 3D cubes U{lo3..hi3}."""
    rng = np.random.default_rng(seed_for(3, k))
    shapes = []
    for _ in range(n2d):
        nx, ny = int(rng.integers(lo2, hi2 + 1)), int(rng.integers(lo2, hi2 + 1))
        shapes.append((ny, nx))
    for _ in range(n3d):
        s = int(rng.integers(lo3, hi3 + 1))
        shapes.append((s, s, s))
    rels = [float(rng.choice([1e-4, 1e-3, 1e-2])) for _ in shapes]
    return shapes, rels


def batch_fields(k: int = 0, **kw):
    """The uneven batch: every field a k^-3 GRF in [0,1] with its own xi."""
    shapes, rels = batch_shapes(k, **kw)
    out = []
    for j, (shape, rel) in enumerate(zip(shapes, rels)):
        rng = np.random.default_rng(seed_for(3, 100 + 1000 * k + j))
        f = gaussian_random_field(shape, 3.0, rng).astype(np.float32)
        xi = xi_for(f, rel)
        out.append((f, quantize(f, xi), xi))
    return out


def turb512(k: int = 0, n: int = 512, rel: float = 1e-3):
    """3D n^3 GRF with power ~k^-11/3 in [0,1]; xi = 1e-3 x range (learned warm-start workload)."""
    rng = np.random.default_rng(seed_for(4, k))
    f = gaussian_random_field((n, n, n), 11.0 / 3.0, rng).astype(np.float32)
    xi = xi_for(f, rel)
    return [(f, quantize(f, xi), xi)]


TRAIN_RELS = (1e-4, 3e-4, 1e-3, 3e-3, 1e-2)


def train_field(k: int, n: int = 128):
    """Training field k (seeds disjoint from the held-out ones): k^-11/3 GRF, rotating relative xi."""
    rng = np.random.default_rng(seed_for(5, k))
    f = gaussian_random_field((n, n, n), 11.0 / 3.0, rng).astype(np.float32)
    xi = xi_for(f, TRAIN_RELS[k % len(TRAIN_RELS)])
    return f, quantize(f, xi), xi


def heldout_field(k: int, n: int = 128, rel: float = 1e-3):
    """Held-out field k of side n (seed block of its own)."""
    rng = np.random.default_rng(seed_for(6, k))
    f = gaussian_random_field((n, n, n), 11.0 / 3.0, rng).astype(np.float32)
    xi = xi_for(f, rel)
    return f, quantize(f, xi), xi


def random_small(rng: np.random.Generator, shape, xi: float = 0.05, levels: int = 0):
    """Tiny random field + a random in-bound decompression, for property tests.

    levels > 0 quantises f to that many values in [0, 1] to create ties."""
    f = rng.uniform(0.0, 1.0, size=shape)
    if levels > 0:
        f = np.round(f * (levels - 1)) / (levels - 1)
    f = f.astype(np.float32)
    fh = (f.astype(np.float64) + rng.uniform(-xi, xi, size=shape)).astype(np.float32)
    # keep |f - fhat| <= xi exactly after float32 rounding
    d = f.astype(np.float64) - fh.astype(np.float64)
    fh = np.where(np.abs(d) > xi, f, fh).astype(np.float32)
    return f, fh, np.float32(xi)
