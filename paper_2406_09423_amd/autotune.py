"""Tile autotuner for the steepest-direction stencil.

The direction kernels stage a (TY + 2) x 66 halo tile of each plane in LDS and
stream z-chunks of ZC planes (3D), re-reading two halo planes per chunk, so a
variant trades halo re-reads ((TY + 2) / TY and (ZC + 2) / ZC) against the
number of work items that fill the chip.  Variants (msz_tile_variants):
  2D: 1 = 64 x 16 tiles, 2 = 64 x 32
  3D: 1 = 64 x 16 x 16-plane chunks, 2 = 64 x 16 x 8, 3 = 64 x 16 x 32, 4 = 64 x 32 x 16
The tuner times every variant on a seeded representative field of each size
class (fields are binned by vertex count) and stores the fastest per class;
msz_fix_batch then takes each field's variant from this table.

  python -m paper_2406_09423_amd.autotune [--out tile_table.json] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_table.json")

# Upper bounds (exclusive) of the vertex-count classes; the last class is open.
EDGES = {2: (1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22), 3: (1 << 15, 1 << 18, 1 << 21, 1 << 24)}
# Phases whose kernels run the direction stencil (the only ones a variant changes).
STENCIL_PHASES = ("dirs_detect",)


def n_classes(ndim: int) -> int:
    return len(EDGES[ndim]) + 1


def size_class(shape) -> str:
    """'2d:k' / '3d:k', k = the index of the first edge above the vertex count."""
    ndim = len(shape)
    if ndim not in (2, 3):
        raise ValueError(f"fields are 2D or 3D, got shape {tuple(shape)}")
    n = math.prod(int(s) for s in shape)
    k = sum(1 for e in EDGES[ndim] if n >= e)
    return f"{ndim}d:{k}"


def representative(cls: str):
    """A field shape near the geometric middle of the class's vertex range."""
    ndim, k = int(cls[0]), int(cls.split(":")[1])
    edges = EDGES[ndim]
    lo = edges[k - 1] if k > 0 else edges[0] // 4
    hi = edges[k] if k < len(edges) else edges[-1] * 4
    n = math.sqrt(lo * hi)
    side = max(8, int(round(n ** (1.0 / ndim))))
    return (side,) * ndim


def variants(ndim: int) -> list:
    import paper_2406_09423_amd as msz
    return list(range(1, msz.tile_variants(ndim) + 1))


def _field(shape, seed: int):
    import numpy as np

    import synth
    rng = np.random.default_rng(synth.seed_for(7, seed))
    f = synth.gaussian_random_field(shape, 3.0 if len(shape) == 2 else 11.0 / 3.0, rng).astype(np.float32)
    xi = synth.xi_for(f, 1e-3)
    return f, synth.quantize(f, xi), xi


def time_variant(fd, fhd, xi, tile: int, ws, reps: int) -> float:
    """Mean microseconds per stencil launch of msz_fix with this tile variant."""
    import paper_2406_09423_amd as msz
    total_ms, launches = 0.0, 0
    msz.fix(fd, fhd, xi, workspace=ws, tile=tile)
    for _ in range(reps):
        rc, _, _, st = msz.fix(fd, fhd, xi, workspace=ws, tile=tile, timing=True)
        if rc != msz.OK:
            raise RuntimeError(f"msz_fix with tile {tile}: {msz.strerror(rc)}")
        for ph in STENCIL_PHASES:
            total_ms += st["timing"][ph]["ms"]
            launches += st["timing"][ph]["launches"]
    return 1e3 * total_ms / max(launches, 1)


def tune(classes=None, reps: int = 5, log=print) -> dict:
    import torch

    import paper_2406_09423_amd as msz
    if classes is None:
        classes = [f"{d}d:{k}" for d in (2, 3) for k in range(n_classes(d))]
    table = {"device": torch.cuda.get_device_name(0), "reps": reps, "classes": {}}
    for j, cls in enumerate(classes):
        shape = representative(cls)
        f, fh, xi = _field(shape, j)
        fd, fhd = torch.from_numpy(f).cuda(), torch.from_numpy(fh).cuda()
        ws = torch.empty(msz.workspace_bytes(shape), dtype=torch.uint8, device="cuda")
        us = {v: time_variant(fd, fhd, xi, v, ws, reps) for v in variants(len(shape))}
        best = min(us, key=us.get)
        table["classes"][cls] = {"shape": list(shape), "variant": best,
                                 "us_per_launch": {str(v): round(t, 3) for v, t in us.items()}}
        log(f"autotune {cls} {shape}: " + ", ".join(f"v{v} {t:.1f} us" for v, t in us.items()) + f" -> v{best}")
    return table


def load_table(path: str = TABLE_PATH):
    """The stored table, or None when no tuning has been stored."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def tile_for(shape, table=None) -> int:
    """The tuned variant of a field's class, or 0 (the default tile) when untuned."""
    table = table if table is not None else load_table()
    if not table:
        return 0
    entry = table.get("classes", {}).get(size_class(shape))
    return int(entry["variant"]) if entry else 0


def tiles_for(shapes, table=None) -> list:
    table = table if table is not None else load_table()
    return [tile_for(s, table) for s in shapes]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    t0 = time.perf_counter()
    table = tune(reps=args.reps, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    table["seconds"] = round(time.perf_counter() - t0, 1)
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(json.dumps(table), flush=True)


if __name__ == "__main__":
    main()
