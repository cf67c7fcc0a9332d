"""Autotuner and learned kernel-parameter predictor for the FP64 block-product
kernels (the paper autotunes its GPU block-product kernels per (m, n, k) and
trains a performance model on the autotuning data to predict parameters for
the (m, n, k) it did not tune; "Batched execution" subsection).

* ``sweep``: exhaustive timing of every catalogue entry on synthetic stacks
  for a list of (m, n, k, stack size) points, through ``bsm_smm_bench``;
  results go to a JSON-lines file, one point per line.
* ``best_table`` / ``install``: the fastest entry per (m, n, k) becomes the
  library's tuning table (``bsm_set_smm_table``).
* ``train``: a 3-layer, width-64 FP32 MLP maps features of a point to the
  predicted log-time of every catalogue entry; its choice is the arg-min.
  It is trained on 80% of the (m, n, k) triples and evaluated on the
  held-out 20% by its regret t(predicted) / t(best) - 1; exhaustive tuning is
  both the fallback for shapes the model is not trusted on and the reference
  the regret is measured against.

Usage (GPU for sweep, CPU for train):
    python -m paper_2003_03868_amd.tune sweep --grid 4:32 --out sweep.jsonl
    python -m paper_2003_03868_amd.tune train --data sweep.jsonl --out model.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

# (family, wpg, prefetch): family 0 = 16x16x4 FP64 MFMA, 1 = 4x4x4 FP64 MFMA,
# 2 = (m, n)-specialised kernel (only m, n in {5, 13, 23, 26}, k <= 26),
# 3 = compile-time-shape kernel (only m = n = k in {5, 13, 23, 26, 32}).
CATALOGUE = [(f, w, p) for f in (0, 1) for w in (1, 2, 4) for p in (0, 1)]
CLASS_ENTRY = (2, 1, 1)
FIXED_ENTRY = (3, 1, 1)
CLASS_SIZES = (5, 13, 23, 26)
FIXED_SIZES = (5, 6, 13, 23, 26, 32)
ALL_ENTRIES = CATALOGUE + [CLASS_ENTRY, FIXED_ENTRY]


def entries_for(m: int, n: int, k: int):
    cat = list(CATALOGUE)
    if m in CLASS_SIZES and n in CLASS_SIZES and (k == 0 or k <= 26):
        cat.append(CLASS_ENTRY)
    if m == n == k and m in FIXED_SIZES:
        cat.append(FIXED_ENTRY)
    return cat


def features(m, n, k, stack, per_c):
    """Model inputs: block shape, log2 of the stack size, products per C
    block (how much one C block's accumulator is reused)."""
    kk = k if k > 0 else 16.75   # mean of the mixed-k cycle {5, 13, 23, 26}
    return [m / 32.0, n / 32.0, kk / 32.0, math.log2(stack) / 16.0, per_c / 64.0,
            (m * n * kk) / 32768.0, ((m + 3) // 4 * 4 - m) / 4.0, ((n + 15) // 16 * 16 - n) / 16.0]


# -------------------------------------------------------------------- sweep

def sweep(points, out_path, reps=3, log_every=200):
    """points: iterable of (m, n, k, n_cblocks, prods_per_cblock)."""
    from paper_2003_03868_amd import bsm
    import torch
    torch.cuda.init()
    done = set()
    if os.path.exists(out_path):
        for line in open(out_path):
            d = json.loads(line)
            done.add((d["m"], d["n"], d["k"], d["n_c"], d["per_c"]))
    t0 = time.time()
    with open(out_path, "a") as f:
        for i, (m, n, k, n_c, per_c) in enumerate(points):
            if (m, n, k, n_c, per_c) in done:
                continue
            cat = entries_for(m, n, k)
            ms = bsm.bsm_smm_bench(m, n, k, n_c, per_c, cat, reps=reps)
            f.write(json.dumps(dict(m=m, n=n, k=k, n_c=n_c, per_c=per_c,
                                    entries=[list(e) for e in cat], ms=ms)) + "\n")
            if i % log_every == 0:
                f.flush()
                print(f"[tune] {i} points, ({m},{n},{k}) x {n_c * per_c}: best "
                      f"{min(ms):.4f} ms, {time.time() - t0:.0f} s", flush=True)


def load_records(path):
    return [json.loads(line) for line in open(path)]


def best_table(records):
    """(m, n, k) -> best (family, wpg, prefetch), by the largest stack measured."""
    best = {}
    for r in records:
        key = (r["m"], r["n"], r["k"])
        stack = r["n_c"] * r["per_c"]
        i = int(np.argmin(r["ms"]))
        if key not in best or stack > best[key][0]:
            best[key] = (stack, tuple(r["entries"][i]))
    return {k: v[1] for k, v in best.items()}


def install(table):
    from paper_2003_03868_amd import bsm
    bsm.bsm_set_smm_table(sorted(table.items()))


_HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(_HERE, "tuned", "gfx950_smm_table.txt")
MODEL_PATH = os.path.join(_HERE, "tuned", "gfx950_mlp.json")


def load_table(path=TABLE_PATH):
    """The committed exhaustive tuning table: (m, n, k) -> (family, wpg, prefetch)."""
    tab = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        m, n, k, f, w, p = (int(v) for v in line.split())
        tab[(m, n, k)] = (f, w, p)
    return tab


def table_from_model(model, keys, stack=60000, per_c=32):
    """MLP choice for every (m, n, k) key (batched forward pass)."""
    keys = list(keys)
    X = [features(m, n, k, stack, per_c) for (m, n, k) in keys]
    out = _forward(model, X)
    tab = {}
    for (m, n, k), row in zip(keys, out):
        valid = {tuple(e) for e in entries_for(m, n, k)}
        for i in np.argsort(row):
            if tuple(model["entries"][i]) in valid:
                tab[(m, n, k)] = tuple(model["entries"][i])
                break
    return tab


def install_default(kind="exhaustive"):
    """Install the committed tuning into the library: "exhaustive" (the
    measured table), "mlp" (the model's choice for the same shapes) or
    "none" (built-in choices)."""
    from paper_2003_03868_amd import bsm
    if kind == "none":
        bsm.bsm_set_smm_table(None)
        return {}
    tab = load_table()
    if kind == "mlp":
        tab = table_from_model(json.load(open(MODEL_PATH)), tab.keys())
    bsm.bsm_set_smm_table(None)
    install(tab)
    return tab


# ---------------------------------------------------------------------- MLP

def _dataset(records):
    X, Y, M = [], [], []
    idx = {e: i for i, e in enumerate(ALL_ENTRIES)}
    for r in records:
        X.append(features(r["m"], r["n"], r["k"], r["n_c"] * r["per_c"], r["per_c"]))
        y = np.full(len(idx), np.nan)
        best = min(r["ms"])
        for e, t in zip(r["entries"], r["ms"]):
            y[idx[tuple(e)]] = math.log(t / best)
        Y.append(y)
    X = np.asarray(X, np.float32)
    Y = np.asarray(Y, np.float32)
    M = ~np.isnan(Y)
    return X, np.nan_to_num(Y, nan=0.0), M


def split_triples(records, holdout=0.2, seed=0):
    triples = sorted({(r["m"], r["n"], r["k"]) for r in records})
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(triples))
    n_out = int(round(holdout * len(triples)))
    held = {triples[i] for i in perm[:n_out]}
    train = [r for r in records if (r["m"], r["n"], r["k"]) not in held]
    test = [r for r in records if (r["m"], r["n"], r["k"]) in held]
    return train, test, held


def train(records, holdout=0.2, seed=0, epochs=400, width=64, lr=3e-3):
    """Train the 3-layer MLP; returns (model dict, report dict)."""
    import torch
    torch.manual_seed(seed)
    tr, te, held = split_triples(records, holdout, seed)
    Xtr, Ytr, Mtr = _dataset(tr)
    net = torch.nn.Sequential(
        torch.nn.Linear(Xtr.shape[1], width), torch.nn.ReLU(),
        torch.nn.Linear(width, width), torch.nn.ReLU(),
        torch.nn.Linear(width, Ytr.shape[1]))
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    xt, yt, mt = torch.from_numpy(Xtr), torch.from_numpy(Ytr), torch.from_numpy(Mtr)
    n = xt.shape[0]
    bs = 512
    for ep in range(epochs):
        perm = torch.randperm(n)
        for s in range(0, n, bs):
            b = perm[s:s + bs]
            pred = net(xt[b])
            loss = (((pred - yt[b]) ** 2) * mt[b]).sum() / mt[b].sum()
            opt.zero_grad()
            loss.backward()
            opt.step()
    model = {"width": width, "n_in": int(Xtr.shape[1]), "entries": [list(e) for e in ALL_ENTRIES],
             "state": {k: v.tolist() for k, v in net.state_dict().items()}}
    rep = {"train_points": len(tr), "test_points": len(te), "heldout_triples": len(held),
           "train": regret(model, tr), "test": regret(model, te)}
    return model, rep


def _forward(model, X):
    st = model["state"]
    h = np.asarray(X, np.float32)
    h = np.maximum(h @ np.asarray(st["0.weight"], np.float32).T + np.asarray(st["0.bias"], np.float32), 0)
    h = np.maximum(h @ np.asarray(st["2.weight"], np.float32).T + np.asarray(st["2.bias"], np.float32), 0)
    return h @ np.asarray(st["4.weight"], np.float32).T + np.asarray(st["4.bias"], np.float32)


def predict(model, m, n, k, stack, per_c, valid=None):
    """Predicted best (family, wpg, prefetch) among the entries valid for
    (m, n, k) (or among `valid`, e.g. the entries a record measured)."""
    out = _forward(model, [features(m, n, k, stack, per_c)])[0]
    valid = {tuple(e) for e in (valid if valid is not None else entries_for(m, n, k))}
    order = np.argsort(out)
    for i in order:
        if tuple(model["entries"][i]) in valid:
            return tuple(model["entries"][i])
    raise RuntimeError("no valid entry")


def regret(model, records):
    """Slowdown of the predicted entry against the exhaustive best."""
    rs = []
    for r in records:
        e = predict(model, r["m"], r["n"], r["k"], r["n_c"] * r["per_c"], r["per_c"],
                    valid=r["entries"])
        t = dict((tuple(x), y) for x, y in zip(r["entries"], r["ms"]))[e]
        rs.append(t / min(r["ms"]) - 1.0)
    rs = np.asarray(rs)
    if rs.size == 0:
        return {}
    return {"mean": float(rs.mean()), "median": float(np.median(rs)),
            "p90": float(np.percentile(rs, 90)), "max": float(rs.max()),
            "exact_best": float((rs == 0).mean()), "within_10pct": float((rs <= 0.10).mean())}


def default_regret(records, entry=(1, 1, 1)):
    """Slowdown of a fixed default entry, for comparison with the model."""
    rs = []
    for r in records:
        d = dict((tuple(x), y) for x, y in zip(r["entries"], r["ms"]))
        rs.append(d[entry] / min(r["ms"]) - 1.0)
    rs = np.asarray(rs)
    return {"mean": float(rs.mean()), "median": float(np.median(rs)), "max": float(rs.max())}


# ---------------------------------------------------------------------- CLI

def _grid(spec):
    lo, hi = (int(x) for x in spec.split(":"))
    return range(lo, hi + 1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sw = sub.add_parser("sweep")
    sw.add_argument("--grid", default="4:32")
    sw.add_argument("--stack", type=int, default=30000, help="products per point")
    sw.add_argument("--per-c", type=int, default=16)
    sw.add_argument("--extra-stacks", default="1000,10000",
                    help="other stack sizes, on a seeded 10%% sample of the triples")
    sw.add_argument("--class-mixed", action="store_true",
                    help="also the 16 (m, n) classes of {5,13,23,26} with mixed k")
    sw.add_argument("--limit", type=int, default=0)
    sw.add_argument("--only", default="", help="semicolon list of m,n,k points to sweep")
    sw.add_argument("--reps", type=int, default=3)
    sw.add_argument("--out", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--data", required=True)
    tr.add_argument("--out", required=True)
    tr.add_argument("--epochs", type=int, default=400)
    args = ap.parse_args(argv)
    if args.cmd == "sweep":
        g = list(_grid(args.grid))
        pts = [(m, n, k, max(1, args.stack // args.per_c), args.per_c) for m in g for n in g for k in g]
        rng = np.random.default_rng(1)
        for st in [int(x) for x in args.extra_stacks.split(",") if x]:
            sel = rng.choice(len(g) ** 3, max(1, len(g) ** 3 // 10), replace=False)
            for i in sel:
                m, n, k = pts[i][:3]
                pts.append((m, n, k, max(1, st // args.per_c), args.per_c))
        if args.class_mixed:
            pts += [(m, n, 0, max(1, args.stack // args.per_c), args.per_c)
                    for m in CLASS_SIZES for n in CLASS_SIZES]
        if args.only:
            pts = [tuple(int(v) for v in q.split(",")) + (max(1, args.stack // args.per_c), args.per_c)
                   for q in args.only.split(";")]
        if args.limit:
            pts = pts[:args.limit]
        sweep(pts, args.out, reps=args.reps)
    else:
        recs = [r for r in load_records(args.data) if r["k"] > 0]
        model, rep = train(recs, epochs=args.epochs)
        rep["default_entry_test"] = default_regret(split_triples(recs)[1])
        json.dump({"model": model, "report": rep}, open(args.out, "w"))
        print(json.dumps(rep, indent=1))


if __name__ == "__main__":
    sys.exit(main())
