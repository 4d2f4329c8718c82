"""Benchmark of the MSz correction loop on one MI355X.

A step corrects the 3600x2400 k^-3 Gaussian-random-field pair (xi = 1e-4 and
1e-3 of the value range) to zero segmentation error with the plain loop; the
fields are resident in HBM before the clock starts.  The same run also times
the two other forms on their own workloads, and the encoding of the edits
(reported under "forms"):
  edits    the plain loop's edits on the pair, losslessly encoded on the GPU
           (sorted index gaps and values, Huffman coded) and decoded back
  merged   the same pair with merged C rounds (all four case types fixed in
           one round, the parallel C-loop of Sec. 6.1)
  batched  96 uneven k^-3 fields (64 2D with sides 64..2048, 32 3D cubes
           32^3..192^3, xi in {1e-4, 1e-3, 1e-2} x range) in one launch
  learned  a 512^3 k^-11/3 field at xi = 1e-3 x range: the warm-started loop
           (features + network + loop) against the plain loop on that field.
Every result is checked for zero segmentation error outside the clock.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--forms plain,edits,merged,batched,learned]
                  [--no-cpu-baseline] [--batch-cpu-baseline] [--calib-copy] [--schedule-out FILE]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gvertices/s corrected to zero MS-label error @xi; plain vs batched vs learned"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_2406_09423_amd/csrc/msz_kernels.hip", "paper_2406_09423_amd/csrc/msz_internal.h")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "traffic_ocean2d.json")
CALIB_BYTES = 1 << 30   # bytes read (and written) by the calibration copy

# Algorithmic (compulsory) HBM bytes per vertex of each kernel kind, per launch.
BYTES_PER_VERTEX = {
    "dirs_detect": 4 + 1 + 1 + 1 + 2,  # read g, dirs_f; write dirs_g, case bytes; clear dirty flags and marks
    "dirs": 4 + 1,              # read the field, write dirs
    "refresh": 1,               # read the dirty flags (the refreshed vertices are sparse)
    "apply": 1,                 # read the case bytes or marks (edited vertices are sparse)
    "label_tile": 1 + 8,        # read dirs, write both pointer arrays
    "label_jump": 0,            # touches only the tiles' face layers
    "detect_r": 2 + 8 + 8 + 8,  # dirs x2, pointers x2, pointer-of-pointer x2, labels of f x2
    "delta": 4 + 4 + 4 + 4,     # read g, fhat; write delta, g
    "validate": 4 + 4 + 4 + 4,  # read f, fhat; write L, g
    "label_final": 8 + 8 + 8,   # read q x2, gather q[q] x2, write labels x2
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none or the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    with open(TRAFFIC_SUMMARY) as fh:
        s = json.load(fh)
    if s.get("source_hash") != kernel_source_hash():
        return None
    k = s.get("kernels", {}).get(kernel)
    return int(k["bytes_per_launch"]) if k else None


def checked(msz, f, g, xi):
    cnt = msz.count_false(f, g)
    if any(v != 0 for v in cnt.values()):
        raise RuntimeError(f"segmentation error left: {cnt}")
    err = (f.double() - g.double()).abs().max().item()
    if err > xi:
        raise RuntimeError(f"bound broken: {err} > {xi}")


def bench_plain(msz, torch, dev, args):
    import synth
    log("bench: generating the 3600x2400 pair")
    pairs = synth.ocean2d()
    fields = [(torch.from_numpy(f).to(dev), torch.from_numpy(fh).to(dev), float(xi)) for f, fh, xi in pairs]
    n_per = fields[0][0].numel()
    ws = torch.empty(msz.workspace_bytes(fields[0][0].shape), dtype=torch.uint8, device=dev)
    outs = [(torch.empty_like(f), torch.empty_like(f)) for f, _, _ in fields]

    schedules = []  # with --schedule-out: every call timed, its step schedule kept

    def step(timing=False):
        res = []
        for (f, fh, xi), (e, g) in zip(fields, outs):
            rc, _, _, st = msz.fix(f, fh, xi, workspace=ws, edits_out=e, g_out=g,
                                   timing=timing or args.schedule_out is not None)
            if rc != msz.OK:
                raise RuntimeError(f"msz_fix failed: {msz.strerror(rc)}")
            if args.schedule_out is not None:
                schedules.append({"xi": xi, "phases": msz.last_schedule()})
            res.append(st)
        return res

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sts = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    verts = n_per * len(fields)
    log(f"bench: plain {ms_per_step:.3f} ms/step, {verts / ms_per_step / 1e6:.3f} Gvertices/s")
    for (f, fh, xi), (e, g) in zip(fields, outs):
        checked(msz, f, g, xi)
    # the same steps again with every device step timed (the step kernel stamps
    # its first block's start and its last block's end with the GPU's
    # constant-rate clock): per-kernel durations for the roofline
    log(f"bench: {args.steps} instrumented steps")
    phase_ms, phase_n = {}, {}
    t2 = time.perf_counter()
    for _ in range(args.steps):
        for st in step(timing=True):
            for name, v in st["timing"].items():
                phase_ms[name] = phase_ms.get(name, 0.0) + v["ms"]
                phase_n[name] = phase_n.get(name, 0) + v["launches"]
    torch.cuda.synchronize()
    ms_instrumented = (time.perf_counter() - t2) * 1e3 / args.steps

    dominant = max((k for k in phase_ms if phase_n.get(k)), key=lambda k: phase_ms[k])
    avg_ms = phase_ms[dominant] / phase_n[dominant]
    bpl = BYTES_PER_VERTEX.get(dominant, 0) * n_per
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if bpl else None
    traffic = stored_traffic(dominant)
    roofline = {
        "kernel": dominant,
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": traffic,
        "avg_launch_us": round(avg_ms * 1e3, 2),
        "bytes_per_launch": bpl,
        "launches_per_step": phase_n[dominant] / args.steps,
        "timing": "GPU clock stamps of every step kernel in an instrumented pass of the same steps "
                  f"({ms_instrumented:.3f} ms/step with the stamps)",
    }
    phases = {}
    for k in phase_ms:
        if not phase_n[k]:
            continue
        us = phase_ms[k] / phase_n[k] * 1e3
        b = BYTES_PER_VERTEX.get(k)
        phases[k] = {"ms_per_step": round(phase_ms[k] / args.steps, 4),
                     "launches_per_step": phase_n[k] / args.steps, "avg_us": round(us, 2),
                     "algorithmic_GBps": round(b * n_per / (us * 1e-6) / 1e9, 1) if b else None}
    rounds = [{"xi": xi, "rounds": st["rounds"], "rounds_r": st["rounds_r"], "outer_iters": st["outer_iters"],
               "n_edited": st["n_edited"]} for (_, _, xi), st in zip(fields, sts)]
    if args.schedule_out is not None:
        with open(args.schedule_out, "w") as fh:
            json.dump({"phase_names": list(msz.PHASES), "calls": schedules}, fh)
    return pairs, verts, ms_per_step, roofline, phases, rounds, [e for e, _ in outs]


def batch_oracle_all_cores(host_fields):
    """The serial C oracle over the whole batch, one field per task on a pool
    of host threads (the oracle is a C library: ctypes releases the GIL)."""
    import concurrent.futures

    import oracle
    oracle.build()
    workers = max(1, min(16, os.cpu_count() or 1))
    verts = sum(f.size for f, _, _ in host_fields)
    # largest fields first, so the slowest one does not start last
    order = sorted(host_fields, key=lambda t: -t[0].size)
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        rcs = list(ex.map(lambda t: oracle.fix(*t)[0], order))
    dt = time.perf_counter() - t0
    assert all(rc == 0 for rc in rcs)
    return {"value": round(verts / dt / 1e9, 6), "unit": "Gvertices/s", "cores": workers, "kind": "oracle",
            "sample": "the whole 96-field batch, one field per task on a pool of host threads", "seconds": round(dt, 2)}


def bench_batched(msz, torch, dev, steps, cpu_all_cores=False):
    import synth
    from paper_2406_09423_amd import autotune
    log("bench: generating the 96-field batch")
    host_fields = synth.batch_fields(0)
    fields = [(torch.from_numpy(f).to(dev), torch.from_numpy(fh).to(dev), float(xi)) for f, fh, xi in host_fields]
    shapes = [f.shape for f, _, _ in fields]
    tiles = autotune.tiles_for(shapes)
    verts = sum(f.numel() for f, _, _ in fields)
    outs = [(torch.empty_like(f), torch.empty_like(f)) for f, _, _ in fields]
    ws = torch.empty(msz.batch_workspace_bytes(shapes), dtype=torch.uint8, device=dev)

    def run(merged=False):
        rc, res = msz.fix_batch(fields, workspace=ws, tiles=tiles, outs=outs, merged=merged)
        if rc != msz.OK:
            raise RuntimeError(f"msz_fix_batch failed: {msz.strerror(rc)}")
        return res

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    for (f, fh, xi), (_, _, g, _) in zip(fields, res):
        checked(msz, f, g, xi)
    # the same fields one msz_fix call after another, for comparison
    ws1 = torch.empty(max(msz.workspace_bytes(s) for s in shapes), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (f, fh, xi), (e, g), tl in zip(fields, outs, tiles):
        rc, _, _, _ = msz.fix(f, fh, xi, workspace=ws1, edits_out=e, g_out=g, tile=tl)
        if rc != msz.OK:
            raise RuntimeError(f"msz_fix failed: {msz.strerror(rc)}")
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3
    log(f"bench: batched {ms:.2f} ms ({verts / ms / 1e6:.3f} Gv/s), one by one {ms_seq:.2f} ms")
    rounds = [sum(st["rounds"]) + st["rounds_r"] for _, _, _, st in res]
    # the same batch with merged C rounds (all four case types per round)
    run(merged=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res_m = run(merged=True)
    torch.cuda.synchronize()
    ms_m = (time.perf_counter() - t0) * 1e3 / steps
    for (f, fh, xi), (_, _, g, _) in zip(fields, res_m):
        checked(msz, f, g, xi)
    log(f"bench: batched with merged C rounds {ms_m:.2f} ms ({verts / ms_m / 1e6:.3f} Gv/s)")
    cpu = None
    if cpu_all_cores:
        log("bench: oracle over the batch on all host cores")
        cpu = batch_oracle_all_cores(host_fields)
        log(f"bench: oracle batch {cpu['seconds']} s on {cpu['cores']} threads")
    del host_fields
    return {"workload": "96 uneven k^-3 fields: 64 2D (sides U{64..2048}), 32 3D (U{32..192}^3), "
                        "xi in {1e-4,1e-3,1e-2} x range; one device-scheduled run",
            "vertices": verts, "ms": round(ms, 3), "value": round(verts / ms / 1e6, 4), "unit": "Gvertices/s",
            "steps": steps, "sequential_ms": round(ms_seq, 3),
            "speedup_vs_sequential": round(ms_seq / ms, 3), "max_rounds": max(rounds),
            "merged_c_ms": round(ms_m, 3), "merged_c_value": round(verts / ms_m / 1e6, 4),
            "tiles": {v: tiles.count(v) for v in sorted(set(tiles))}, "cpu_all_cores": cpu}


def bench_learned(msz, torch, dev, steps):
    import numpy as np

    import synth
    from paper_2406_09423_amd import train_net
    if not os.path.exists(train_net.WEIGHTS_PATH):
        return {"skipped": "no trained weights stored"}
    params = train_net.load_weights()
    p_min = train_net.stored_p_min()
    log("bench: generating the 512^3 field")
    f, fh, xi = synth.turb512()[0]
    fd, fhd = torch.from_numpy(f).to(dev), torch.from_numpy(fh).to(dev)
    del f, fh
    xi = float(xi)
    ws = torch.empty(msz.learned_workspace_bytes(fd.shape), dtype=torch.uint8, device=dev)
    e, g = torch.empty_like(fd), torch.empty_like(fd)
    out = {"workload": "512^3 k^-11/3 Gaussian random field, xi = 1e-3 x range", "vertices": fd.numel(),
           "p_min": p_min, "steps": steps}
    for name, fn in (("plain", lambda t: msz.fix(fd, fhd, xi, workspace=ws, edits_out=e, g_out=g, timing=t)),
                     ("learned", lambda t: msz.fix_learned(fd, fhd, xi, params, p_min=p_min, workspace=ws,
                                                           edits_out=e, g_out=g, timing=t))):
        fn(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rc, _, _, st = fn(False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        if rc != msz.OK:
            raise RuntimeError(f"{name} failed: {msz.strerror(rc)}")
        checked(msz, fd, g, xi)
        _, _, _, stt = fn(True)
        n = fd.numel()
        phases = {}
        for k, v in stt["timing"].items():  # one timed call: per-operation step times on 512^3
            if not v["launches"] or k == "net":
                continue
            us = v["ms"] / v["launches"] * 1e3
            b = BYTES_PER_VERTEX.get(k)
            phases[k] = {"launches": v["launches"], "avg_us": round(us, 2),
                         "algorithmic_GBps": round(b * n / (us * 1e-6) / 1e9, 1) if b else None,
                         "frac_of_hbm_peak": round(b * n / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if b else None}
        out[name] = {"ms": round(ms, 3), "value": round(n / ms / 1e6, 4),
                     "rounds": sum(st["rounds"]) + st["rounds_r"], "outer_iters": st["outer_iters"],
                     "n_edited": st["n_edited"], "net_ms": round(stt["timing"]["net"]["ms"], 3),
                     "phases": phases}
        log(f"bench: {name} 512^3 {ms:.2f} ms, rounds {out[name]['rounds']}")
    out["speedup"] = round(out["plain"]["ms"] / out["learned"]["ms"], 4)
    out["unit"] = "Gvertices/s"
    # the same two with merged C rounds (all four case types per round)
    for name, fn in (("plain_merged", lambda: msz.fix(fd, fhd, xi, workspace=ws, edits_out=e, g_out=g, merged=True)),
                     ("learned_merged", lambda: msz.fix_learned(fd, fhd, xi, params, p_min=p_min, workspace=ws,
                                                                edits_out=e, g_out=g, merged=True))):
        try:
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                rc, _, _, st = fn()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            if rc != msz.OK:
                raise RuntimeError(f"{name} failed: {msz.strerror(rc)}")
            checked(msz, fd, g, xi)
            out[name] = {"ms": round(ms, 3), "value": round(fd.numel() / ms / 1e6, 4),
                         "c_rounds_by_type": st["rounds"], "r_rounds": st["rounds_r"], "n_edited": st["n_edited"]}
            log(f"bench: {name} 512^3 {ms:.2f} ms")
        except RuntimeError as err:  # reported, not fatal: the default forms above are the measured ones
            out[name] = {"failed": str(err)}
    return out


def bench_merged(msz, torch, dev, pairs, steps, plain_ms):
    """The ocean2d pair with merged C rounds (all four case types per round,
    the parallel C-loop of Sec. 6.1): time per step, rounds, zero error."""
    fields = [(torch.from_numpy(f).to(dev), torch.from_numpy(fh).to(dev), float(xi)) for f, fh, xi in pairs]
    ws = torch.empty(msz.workspace_bytes(fields[0][0].shape), dtype=torch.uint8, device=dev)
    outs = [(torch.empty_like(f), torch.empty_like(f)) for f, _, _ in fields]

    def step(timing=False):
        res = []
        for (f, fh, xi), (e, g) in zip(fields, outs):
            rc, _, _, st = msz.fix(f, fh, xi, workspace=ws, edits_out=e, g_out=g, merged=True, timing=timing)
            if rc != msz.OK:
                raise RuntimeError(f"msz_fix (merged C rounds) failed: {msz.strerror(rc)}")
            res.append(st)
        return res

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sts = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    for (f, fh, xi), (e, g) in zip(fields, outs):
        checked(msz, f, g, xi)
    verts = sum(f.numel() for f, _, _ in fields)
    log(f"bench: merged C rounds {ms:.3f} ms/step ({verts / ms / 1e6:.3f} Gv/s), plain {plain_ms:.3f} ms/step")
    return {"workload": "the ocean2d pair (3600x2400 at xi = 1e-4 and 1e-3), merged C rounds",
            "ms_per_step": round(ms, 3), "value": round(verts / ms / 1e6, 4), "unit": "Gvertices/s",
            "steps": steps, "speedup_vs_plain": round(plain_ms / ms, 3),
            "rounds": [{"xi": p[2], "rounds": st["rounds"], "rounds_r": st["rounds_r"],
                        "outer_iters": st["outer_iters"], "n_edited": st["n_edited"]}
                       for p, st in zip(fields, sts)]}


def bench_edits(msz, torch, edits, pairs, reps=3):
    """Lossless encoding of the plain loop's edits on the ocean2d pair (Sec. 6.3):
    sizes, the edit ratio, and encode / decode times, each decode checked bit
    for bit against the edits."""
    out = []
    for e, (_, _, xi) in zip(edits, pairs):
        n = e.numel()
        buf = torch.empty(msz.edits_bound(n), dtype=torch.uint8, device=e.device)
        dec = torch.empty_like(e)
        msz.encode_edits(e, out=buf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rc, blob, st = msz.encode_edits(e, out=buf)
        torch.cuda.synchronize()
        t_enc = (time.perf_counter() - t0) * 1e3 / reps
        if rc != msz.OK:
            raise RuntimeError(f"msz_encode_edits: {msz.strerror(rc)}")
        t0 = time.perf_counter()
        for _ in range(reps):
            rc, _ = msz.decode_edits(blob, e.shape, out=dec)
        torch.cuda.synchronize()
        t_dec = (time.perf_counter() - t0) * 1e3 / reps
        if rc != msz.OK or not torch.equal(dec.view(torch.int32), e.view(torch.int32)):
            raise RuntimeError("decoded edits differ")
        m = st["n_edits"]
        out.append({"xi": float(xi), "vertices": n, "edits": m, "edit_ratio": round(m / n, 6),
                    "bytes": st["bytes"], "bits_per_edit": round(8 * st["bytes"] / max(m, 1), 3),
                    "index_bits_per_edit": round(st["index_bits"] / max(m, 1), 3),
                    "value_bits_per_edit": round(st["value_bits"] / max(m, 1), 3),
                    "bits_per_vertex": round(8 * st["bytes"] / n, 5),
                    "encode_ms": round(t_enc, 3), "decode_ms": round(t_dec, 3)})
        log(f"bench: edits xi={float(xi):g}: {m} edits, {st['bytes']} bytes "
            f"({8 * st['bytes'] / max(m, 1):.2f} bits/edit), encode {t_enc:.2f} ms, decode {t_dec:.2f} ms")
    return {"workload": "edits of the plain loop on the ocean2d pair, encoded on the GPU and decoded back",
            "fields": out}


def calibration_copy(torch, dev):
    """A plain device copy of CALIB_BYTES, so that a counter run sees a kernel of known traffic."""
    a = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--forms", default="plain,edits,merged,batched,learned")
    ap.add_argument("--form-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-cpu-baseline", action="store_true",
                    help="also time the oracle over the whole batch on all host cores (minutes)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 1 GiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--schedule-out", default=None,
                    help="time every plain-form call and write each call's step schedule to this JSON file "
                         "(to attribute the step kernels of a kernel trace)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: each field's "
              "correction loop runs on a single GPU", file=sys.stderr)
        sys.exit(2)
    forms = [x for x in args.forms.split(",") if x]

    import torch

    import paper_2406_09423_amd as msz

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    msz.lib()
    if args.calib_copy:
        calibration_copy(torch, dev)
    pairs, verts, ms_per_step, roofline, phases, rounds, edits = bench_plain(msz, torch, dev, args)
    value = verts / (ms_per_step * 1e-3) / 1e9

    extra = {}
    if "edits" in forms:
        extra["edits"] = bench_edits(msz, torch, edits, pairs)
    if "merged" in forms:
        extra["merged"] = bench_merged(msz, torch, dev, pairs, args.form_steps, ms_per_step)
    if "batched" in forms:
        extra["batched"] = bench_batched(msz, torch, dev, args.form_steps, args.batch_cpu_baseline)
    if "learned" in forms:
        extra["learned"] = bench_learned(msz, torch, dev, args.form_steps)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        f, fh, xi = pairs[0]
        log("bench: oracle on the xi = 1e-4 field (serial C, one core)")
        tc = time.perf_counter()
        rc, _, _, _ = oracle.fix(f, fh, xi)
        dt = time.perf_counter() - tc
        assert rc == 0
        cpu = {"value": round(f.size / dt / 1e9, 6), "unit": "Gvertices/s", "cores": 1, "kind": "oracle",
               "sample": "half a step: the xi = 1e-4 field of the 3600x2400 pair (8.64 M vertices), "
                         "serial C oracle on one core", "seconds": round(dt, 2)}

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gvertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ocean2d: 3600x2400 k^-3 Gaussian random field in [0,1], quantised at "
                               "xi = 1e-4 and 1e-3; plain loop, both fields per step",
                   "vertices_per_step": verts, "form": "plain"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases": phases,
        "rounds": rounds,
        "forms": extra,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
