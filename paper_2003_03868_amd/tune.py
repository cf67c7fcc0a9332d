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
  An ensemble of such MLPs (different initialisations and batch orders) is
  trained on 80% of the (m, n, k) triples and evaluated on the held-out 20%
  by its regret t(predicted) / t(best) - 1.  A shape is trusted to the
  model when every member picks the same entry; the others fall back to
  exhaustive tuning, which is also the reference the regret is measured
  against.
* ``real``: per-class kernel times of the sign iteration on the mixed-size
  workload with the exhaustive, the model's and the built-in choices: the
  regret on the stacks a real multiply builds (GPU).

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


POOL = 1024   # operand blocks per k value in the synthetic stacks (bsm_smm_bench)


def operand_reuse(stack, k):
    """Products per operand block of a synthetic stack: the operand reuse
    that the block occupancy of a real product sets (a C block row of
    occupancy o over nb block columns reads each A block for o nb products)."""
    nk = 4 if k == 0 else 1
    return stack / (2.0 * nk * POOL)


def features(m, n, k, stack, per_c):
    """Model inputs: block shape, log2 of the stack size, products per C
    block (how much one C block's accumulator is reused), padding to the
    4- and 16-wide tiles, and the operand reuse (occupancy)."""
    kk = k if k > 0 else 16.75   # mean of the mixed-k cycle {5, 13, 23, 26}
    return [m / 32.0, n / 32.0, kk / 32.0, math.log2(stack) / 16.0, per_c / 64.0,
            (m * n * kk) / 32768.0, ((m + 3) // 4 * 4 - m) / 4.0, ((n + 15) // 16 * 16 - n) / 16.0,
            math.log2(operand_reuse(stack, k)) / 8.0]


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


def members_of(model):
    """The MLPs of an ensemble model (a single MLP is an ensemble of one)."""
    return model["members"] if "members" in model else [model]


def table_from_model(model, keys, stack=60000, per_c=32, fallback=None):
    """Model choice for every (m, n, k) key (batched forward passes).  With
    `fallback` (the exhaustive table), keys whose ensemble members disagree
    take the fallback's entry.  Returns the table; `table_from_model.trusted`
    holds the keys the model decided."""
    keys = list(keys)
    X = [features(m, n, k, stack, per_c) for (m, n, k) in keys]
    picks = []
    for mem in members_of(model):
        out = _forward(mem, X)
        row_pick = []
        for (m, n, k), row in zip(keys, out):
            valid = {tuple(e) for e in entries_for(m, n, k)}
            for i in np.argsort(row):
                if tuple(mem["entries"][i]) in valid:
                    row_pick.append(tuple(mem["entries"][i]))
                    break
        picks.append(row_pick)
    tab, trusted = {}, set()
    for q, key in enumerate(keys):
        votes = [p[q] for p in picks]
        agree = all(v == votes[0] for v in votes)
        if agree or fallback is None or key not in fallback:
            tab[key] = max(set(votes), key=votes.count)
            if agree:
                trusted.add(key)
        else:
            tab[key] = tuple(fallback[key])
    table_from_model.trusted = trusted
    return tab


def install_default(kind="exhaustive"):
    """Install the committed tuning into the library: "exhaustive" (the
    measured table), "mlp" (the model's choice for the same shapes, the
    exhaustive entry where its members disagree), "mlp_raw" (the model's
    choice everywhere) or "none" (built-in choices)."""
    from paper_2003_03868_amd import bsm
    if kind == "none":
        bsm.bsm_set_smm_table(None)
        return {}
    tab = load_table()
    if kind == "mlp":
        tab = table_from_model(json.load(open(MODEL_PATH)), tab.keys(), fallback=tab)
    elif kind == "mlp_raw":
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


def train(records, holdout=0.2, seed=0, epochs=400, width=64, lr=3e-3, init_seed=None):
    """Train the 3-layer MLP; returns (model dict, report dict)."""
    import torch
    torch.set_num_threads(1)      # a small net: one thread avoids oversubscription
    torch.manual_seed(seed if init_seed is None else init_seed)
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


def train_ensemble(records, members=5, holdout=0.2, seed=0, epochs=400):
    """Members trained on the same split from different initialisations and
    batch orders; returns (ensemble model, report)."""
    ms = []
    for i in range(members):
        t0 = time.time()
        ms.append(train(records, holdout, seed, epochs, init_seed=seed + 101 * i)[0])
        print(f"[tune] member {i} trained in {time.time() - t0:.0f} s", flush=True)
    model = {"members": ms}
    tr, te, held = split_triples(records, holdout, seed)
    rep = {"train_points": len(tr), "test_points": len(te), "heldout_triples": len(held),
           "members": members,
           "test_single": regret(ms[0], te), "test_ensemble": regret(model, te),
           "test_with_fallback": regret(model, te, fallback=True),
           "trusted_share_test": trusted_share(model, te)}
    return model, rep


def trusted_share(model, records):
    """Share of records whose shape every member decides alike."""
    if not records:
        return 0.0
    n = 0
    for r in records:
        picks = {predict(mem, r["m"], r["n"], r["k"], r["n_c"] * r["per_c"], r["per_c"],
                         valid=r["entries"]) for mem in members_of(model)}
        n += len(picks) == 1
    return n / len(records)


def _forward(model, X):
    st = model["state"]
    h = np.asarray(X, np.float32)
    h = np.maximum(h @ np.asarray(st["0.weight"], np.float32).T + np.asarray(st["0.bias"], np.float32), 0)
    h = np.maximum(h @ np.asarray(st["2.weight"], np.float32).T + np.asarray(st["2.bias"], np.float32), 0)
    return h @ np.asarray(st["4.weight"], np.float32).T + np.asarray(st["4.bias"], np.float32)


def predict(model, m, n, k, stack, per_c, valid=None):
    """Predicted best (family, wpg, prefetch) among the entries valid for
    (m, n, k) (or among `valid`, e.g. the entries a record measured); for an
    ensemble, the most frequent member choice."""
    valid = {tuple(e) for e in (valid if valid is not None else entries_for(m, n, k))}
    votes = []
    for mem in members_of(model):
        out = _forward(mem, [features(m, n, k, stack, per_c)])[0]
        for i in np.argsort(out):
            if tuple(mem["entries"][i]) in valid:
                votes.append(tuple(mem["entries"][i]))
                break
        else:
            raise RuntimeError("no valid entry")
    return max(votes, key=votes.count) if len(set(votes)) > 1 else votes[0]


def regret(model, records, fallback=False):
    """Slowdown of the predicted entry against the exhaustive best; with
    fallback, records whose members disagree take the exhaustive best."""
    rs = []
    for r in records:
        d = dict((tuple(x), y) for x, y in zip(r["entries"], r["ms"]))
        picks = [predict(mem, r["m"], r["n"], r["k"], r["n_c"] * r["per_c"], r["per_c"],
                         valid=r["entries"]) for mem in members_of(model)]
        if fallback and len(set(picks)) > 1:
            rs.append(0.0)
            continue
        e = max(picks, key=picks.count)
        rs.append(d[e] / min(r["ms"]) - 1.0)
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


# ------------------------------------------------------- regret on real stacks

CLASS_NAMES = [f"{m}x{n}" for m in CLASS_SIZES for n in CLASS_SIZES]


def real_regret(sites=4096, seed=0, reps=2):
    """Per-class block-product time of the FP64 sign iteration (eps 1e-6,
    tol 1e-6) on the mixed-size workload, one launch per (m, n) class, with
    the exhaustive table, the model's table (fallback where its members
    disagree) and the built-in choices; minimum over reps runs.  Regret of a
    class = t(table) / t(exhaustive) - 1 on the multiplies' own stacks."""
    import torch

    import synth
    from paper_2003_03868_amd import bsm
    prev = os.environ.get("BSM_SMM_VARIANT")
    os.environ["BSM_SMM_VARIANT"] = "4"         # one launch per class
    try:
        torch.cuda.init()
        h = synth.neighbour_hamiltonian(sites, density=0.1, cutoff=6.0, seed=seed,
                                        size_choices=CLASS_SIZES)
        dh = bsm.Matrix.from_bsr(h, device=True)
        o = bsm.bsm_sign_opts_default()
        o.eps_filter, o.tol = 1e-6, 1e-6
        times, choices = {}, {}
        for kind in ("exhaustive", "mlp", "mlp_raw", "none"):
            tab = install_default(kind)
            choices[kind] = {f"{m}x{n}": list(tab.get((m, n, 0), ("built-in",)))
                             for m in CLASS_SIZES for n in CLASS_SIZES}
            best = None
            for _ in range(reps):
                st, xh, stats = bsm.bsm_sign_iterate(dh.handle, 0.0, o)
                bsm.bsm_destroy(xh)
                if st != bsm.OK:
                    raise RuntimeError(f"sign iteration failed: {bsm.bsm_last_error()}")
                cm = list(stats.class_ms)
                best = cm if best is None else [min(a, b) for a, b in zip(best, cm)]
            times[kind] = best
            print(f"[tune] {kind}: block products {sum(best):.0f} ms", flush=True)
        install_default("exhaustive")
        dh.destroy()
    finally:
        if prev is None:
            os.environ.pop("BSM_SMM_VARIANT", None)
        else:
            os.environ["BSM_SMM_VARIANT"] = prev
    ex = times["exhaustive"]
    reg = {k: {CLASS_NAMES[c]: (times[k][c] / ex[c] - 1.0) if ex[c] > 0 else 0.0 for c in range(16)}
           for k in ("mlp", "mlp_raw", "none")}
    return {"sites": sites, "seed": seed, "class_ms": {k: dict(zip(CLASS_NAMES, v)) for k, v in times.items()},
            "choices": choices, "regret_mlp": reg["mlp"], "regret_mlp_raw": reg["mlp_raw"],
            "regret_none": reg["none"], "total_ms": {k: sum(v) for k, v in times.items()}}


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
    tr.add_argument("--members", type=int, default=5)
    rl = sub.add_parser("real")
    rl.add_argument("--sites", type=int, default=4096)
    rl.add_argument("--seed", type=int, default=0)
    rl.add_argument("--reps", type=int, default=2)
    rl.add_argument("--out", default="")
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
    elif args.cmd == "real":
        rep = real_regret(args.sites, args.seed, args.reps)
        if args.out:
            json.dump(rep, open(args.out, "w"), indent=1)
        print(json.dumps(rep["regret_mlp"], indent=1))
    else:
        allrec = load_records(args.data)
        recs = [r for r in allrec if r["k"] > 0]
        model, rep = train_ensemble(recs, members=args.members, epochs=args.epochs)
        rep["default_entry_test"] = default_regret(split_triples(recs)[1])
        cls = [r for r in allrec if r["k"] == 0]
        rep["class_mixed_k"] = regret(model, cls)
        rep["class_mixed_k_with_fallback"] = regret(model, cls, fallback=True)
        rep["class_mixed_k_trusted"] = trusted_share(model, cls)
        model["report"] = rep
        json.dump(model, open(args.out, "w"))
        print(json.dumps(rep, indent=1))


if __name__ == "__main__":
    sys.exit(main())
