"""One timed plain correction of the 512^3 turbulence field, for profiler runs.

    python3 -m paper_2406_09423_amd.profile_turb512 OUT.json [CACHE.npz]

Runs ``msz_fix`` once as a warm-up and once with per-launch timing, and writes
each step-kernel launch of the timed call (its operation, the GPU clock-stamp
duration in µs and the algorithmic bytes the device counted) to OUT.json, so
that per-dispatch counters of a ``rocprofv3 --pmc`` run of this program can be
matched to the loop's operations.  The field (``synth.turb512()``) is kept in
CACHE.npz (default ``/tmp/f512.npz``) between runs, since its generation takes
longer than the correction.
"""
import json
import os
import sys

import numpy as np


def main(argv):
    if len(argv) < 2:
        print(__doc__, file=sys.stderr)
        return 2
    out_path = argv[1]
    cache = argv[2] if len(argv) > 2 else "/tmp/f512.npz"
    import torch

    import paper_2406_09423_amd as msz

    msz.lib()
    if os.path.exists(cache):
        z = np.load(cache)
        f, fh, xi = z["f"], z["fh"], z["xi"]
    else:
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import synth

        f, fh, xi = synth.turb512()[0]
        np.savez(cache, f=f, fh=fh, xi=xi)
    fd, fhd = torch.from_numpy(f).cuda(), torch.from_numpy(fh).cuda()
    ws = torch.empty(msz.workspace_bytes(fd.shape), dtype=torch.uint8, device="cuda")
    e, g = torch.empty_like(fd), torch.empty_like(fd)
    msz.fix(fd, fhd, float(xi), workspace=ws, edits_out=e, g_out=g)
    torch.cuda.synchronize()
    rc, _, _, _ = msz.fix(fd, fhd, float(xi), workspace=ws, edits_out=e, g_out=g, timing=True)
    torch.cuda.synchronize()
    recs = msz.last_launches()
    with open(out_path, "w") as fh_out:
        json.dump({"phases": [r["phase"] for r in recs], "us": [r["us"] for r in recs],
                   "bytes": [r["bytes"] for r in recs]}, fh_out)
    print("ok", rc, len(recs), flush=True)
    return 0 if rc == msz.OK else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv))
