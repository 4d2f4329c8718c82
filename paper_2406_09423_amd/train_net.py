"""Trains the warm-start network on the GPU with the library's own kernels.

Training pairs come from the plain correction loop: for each seeded 128^3
field, the target of vertex i is the number of halvings the loop applied to
it (msz_net_halvings: its edit, exactly), and the inputs are the library's
features of (f, fhat, xi).  Loss: mean squared error in which vertices with a non-zero
target weigh 1 + edit_weight (edited vertices are a few percent of a field,
so an unweighted loss settles on a small positive edit everywhere);
optimiser: Adam on FP32 master weights; forward and backward run in BF16 on
MFMA (msz_net_gradients).  The warm start applies a prediction only where it
exceeds p_min, so that vertices the network is unsure about keep fhat.

  python -m paper_2406_09423_amd.train_net --fields 200 --epochs 6 --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2406_09423_amd as msz  # noqa: E402

WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "net_weights.npy")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, small positive biases, in the library's flat layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cstore, cout, last in ((12, 16, 16, False), (16, 16, 16, False), (16, 16, 1, True)):
        bound = np.sqrt(6.0 / (cin * 27))
        W = np.zeros((27, cstore, 16 if not last else 1))
        W[:, :cin, :cout] = rng.uniform(-bound, bound, size=(27, cin, cout))
        parts += [W.ravel(), np.full(cout, 0.01)]
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == msz.NET_PARAMS
    return flat


INFO_PATH = os.path.splitext(WEIGHTS_PATH)[0] + ".json"


def stored_p_min(path: str = INFO_PATH) -> float:
    """The count threshold chosen when the stored weights were trained (0.5 if unrecorded)."""
    if not os.path.exists(path):
        return 0.5
    with open(path) as fh:
        return float(json.load(fh).get("p_min", 0.5))


def load_weights(path: str = WEIGHTS_PATH):
    import torch
    w = np.load(path, allow_pickle=False).astype(np.float32)
    assert w.size == msz.NET_PARAMS
    return torch.from_numpy(w).cuda()


def make_pair(f, fh, xi, ws):
    """(features, target) of one field on the GPU, from the plain loop."""
    import torch
    fd, fhd = torch.from_numpy(f).cuda(), torch.from_numpy(fh).cuda()
    rc, d, g, st = msz.fix(fd, fhd, xi, workspace=ws)
    if rc != msz.OK:
        raise RuntimeError(f"plain loop failed: {msz.strerror(rc)}")
    t = msz.net_halvings(fd, fhd, g, xi).reshape(-1)
    if bool((t < 0).any()):
        raise RuntimeError("an edit of the plain loop is off its halving chain")
    feat = msz.net_features(fd, fhd, xi)
    return feat, t, st


def train(n_fields: int = 200, side: int = 128, epochs: int = 6, lr: float = 2e-3, seed: int = 0,
          edit_weight: float = 8.0, log_every: int = 50):
    import torch

    import synth
    shape = (side, side, side)
    ws = torch.empty(msz.workspace_bytes(shape), dtype=torch.uint8, device="cuda")
    nws = torch.empty(msz.net_workspace_bytes(shape), dtype=torch.uint8, device="cuda")
    data = []
    t0 = time.perf_counter()
    for k in range(n_fields):
        f, fh, xi = synth.train_field(k, n=side)
        feat, t, st = make_pair(f, fh, xi, ws)
        data.append((feat, t))
        if (k + 1) % log_every == 0:
            log(f"train data: {k + 1}/{n_fields} fields ({time.perf_counter() - t0:.1f} s)")
    params = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    rng = np.random.default_rng(seed)
    history = []
    step = 0
    t1 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(n_fields)
        losses = []
        for k in order:
            feat, t = data[k]
            loss, _ = msz.net_gradients(params, feat, t, shape, edit_weight=edit_weight, grad_out=grad,
                                        workspace=nws)
            step += 1
            msz.net_adam(params, grad, m, v, step, lr)
            losses.append(loss)
        history.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{epochs}: mean loss {history[-1]:.5f} ({time.perf_counter() - t1:.1f} s)")
    torch.cuda.synchronize()
    return params, {"loss_per_epoch": history, "fields": n_fields, "side": side, "epochs": epochs, "lr": lr,
                    "edit_weight": edit_weight, "train_seconds": time.perf_counter() - t1,
                    "data_seconds": t1 - t0}


def evaluate(params, fields, reps: int = 3, p_mins=(0.5,)):
    """Rounds and time of the plain loop against the warm-started loop on each field."""
    import torch
    out = []
    for f, fh, xi in fields:
        fd, fhd = torch.from_numpy(f).cuda(), torch.from_numpy(fh).cuda()
        ws = torch.empty(msz.learned_workspace_bytes(f.shape), dtype=torch.uint8, device="cuda")
        res = {}
        runs = [("plain", lambda: msz.fix(fd, fhd, xi, workspace=ws))]
        for pm in p_mins:
            runs.append((f"learned@{pm:g}",
                         lambda pm=pm: msz.fix_learned(fd, fhd, xi, params, p_min=pm, workspace=ws)))
        for name, fn in runs:
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                rc, d, g, st = fn()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3 / reps
            assert rc == msz.OK
            cnt = msz.count_false(fd, g)
            assert all(c == 0 for c in cnt.values())
            res[name] = {"ms": ms, "rounds": sum(st["rounds"]) + st["rounds_r"], "n_edited": st["n_edited"]}
        out.append(res)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fields", type=int, default=200)
    ap.add_argument("--side", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--edit-weight", type=float, default=8.0)
    ap.add_argument("--p-min", type=float, nargs="+", default=[0.5])
    ap.add_argument("--out", default=WEIGHTS_PATH)
    ap.add_argument("--eval", type=int, default=4, help="held-out 128^3 fields to evaluate")
    args = ap.parse_args()
    import synth
    params, info = train(args.fields, args.side, args.epochs, args.lr, edit_weight=args.edit_weight)
    np.save(args.out, params.cpu().numpy())
    held = [synth.heldout_field(k, n=args.side) for k in range(args.eval)]
    info["heldout"] = evaluate(params, held, p_mins=args.p_min)
    # the threshold with the lowest mean time over the held-out fields
    mean_ms = {pm: float(np.mean([r[f"learned@{pm:g}"]["ms"] for r in info["heldout"]])) for pm in args.p_min}
    info["p_min"] = min(mean_ms, key=mean_ms.get)
    info["plain_ms_mean"] = float(np.mean([r["plain"]["ms"] for r in info["heldout"]]))
    info["learned_ms_mean"] = mean_ms
    with open(os.path.splitext(args.out)[0] + ".json", "w") as fh:
        json.dump(info, fh, indent=1)
    print(json.dumps(info), flush=True)


if __name__ == "__main__":
    main()
