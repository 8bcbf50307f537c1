"""Training and evaluation of the learned variant picker.

1. collect(): for random problem shapes, the exhaustive autotuner
   (lpx_autotune, with a cache-flush buffer overwritten before every timed
   launch) times every candidate record; each (shape, record) becomes one
   row: its 13 features (lpx_features) and the median time.
2. train(): the 12-64-64-1 cost model learns log time from those rows.
   Every step runs the library's kernels: lpx_mlp_forward -> lpx_mlp_loss ->
   lpx_mlp_backward -> lpx_adam_step (torch only gathers minibatches).
   Rows are split into training and validation by shape; training stops
   when the validation regret stops improving.
3. evaluate(): on held-out shapes, each shape is tuned exhaustively (the
   judge of the picker) and the learned pick, the untuned default and the
   best record are read off the same timings.

Run as ``python -m paper_1405_7470_amd.picker --out DIR`` on a GPU.
"""
import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import inputs, lpx

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "data", "picker.lpxpick")


def _problem_tensors(sh, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    K, Np, E, layout = sh["K"], sh["Np"], sh["E"], sh["layout"]
    D = torch.randn((K, Np, Np), device="cuda", generator=g) / math.sqrt(Np)
    ushape = (E, Np) if layout == "em" else (Np, E)
    u = torch.rand(ushape, device="cuda", generator=g) * 2 - 1
    out = torch.empty(lpx.out_shape(K, Np, E, layout), device="cuda")
    return D, u, out


def tune_shape(sh, flush, warmup=1, reps=5, seed=0):
    """(records, median microseconds per record; inf = not supported)."""
    D, u, out = _problem_tensors(sh, seed)
    _, times = lpx.autotune(D, u, out, sh["layout"], sh["precision"], warmup=warmup, reps=reps,
                            flush=flush)
    recs = lpx.enumerate_records(sh["K"], sh["Np"], sh["E"], sh["layout"], sh["precision"])
    del D, u, out
    return recs, times


def collect(shapes, flush_mb=512, reps=5, db_path=None, log=print):
    """Exhaustive timings of every candidate for each shape; returns rows."""
    flush = torch.empty(flush_mb * (1 << 20) // 4, device="cuda")
    rows = []
    db = open(db_path, "a") if db_path else None
    t0 = time.time()
    for si, sh in enumerate(shapes):
        recs, times = tune_shape(sh, flush, reps=reps, seed=si)
        for ri, (r, t) in enumerate(zip(recs, times)):
            if not math.isfinite(t):
                continue
            row = {"shape_id": si, "shape": sh, "rec_index": ri, "record": r.as_dict(),
                   "features": lpx.features(sh["K"], sh["Np"], sh["E"], sh["layout"], r),
                   "us": float(t)}
            rows.append(row)
            if db:
                db.write(json.dumps(row) + "\n")
        if log and (si % 25 == 0 or si == len(shapes) - 1):
            log(f"collect: {si + 1}/{len(shapes)} shapes, {len(rows)} timings, "
                f"{time.time() - t0:.0f} s", flush=True)
    if db:
        db.close()
    return rows


def _he_init(rng):
    p = np.zeros(lpx.MLP_PARAMS, np.float32)
    p[0:768] = rng.normal(0, math.sqrt(2 / 12), 768)
    p[832:4928] = rng.normal(0, math.sqrt(2 / 64), 4096)
    p[4992:5056] = rng.normal(0, math.sqrt(2 / 64), 64)
    return p


def _regret(pred, rows_by_shape):
    """Geometric-mean regret t[argmin pred] / t_best over shapes."""
    logs = []
    for idx in rows_by_shape:
        t = np.array([r["us"] for r in idx["rows"]])
        pick = int(np.argmin(pred[idx["slice"]]))
        logs.append(math.log(t[pick] / t.min()))
    return math.exp(float(np.mean(logs))) if logs else float("nan")


def _group(rows):
    """Rows grouped by shape, each with its slice into the row list."""
    groups, start = [], 0
    for i in range(1, len(rows) + 1):
        if i == len(rows) or rows[i]["shape_id"] != rows[start]["shape_id"]:
            groups.append({"slice": slice(start, i), "rows": rows[start:i]})
            start = i
    return groups


def train(rows, epochs=300, batch=256, lr=1e-3, seed=0, val_frac=0.15, patience=40, log=print,
          split_seed=0):
    """Trains the cost model with the library's kernels; returns
    (params, mean, std, history).  split_seed fixes the validation shapes,
    seed the initialisation and minibatch order."""
    rng = np.random.default_rng(seed)
    shape_ids = sorted({r["shape_id"] for r in rows})
    np.random.default_rng(split_seed).shuffle(shape_ids)
    nval = max(1, int(len(shape_ids) * val_frac))
    val_ids = set(shape_ids[:nval])
    tr = [r for r in rows if r["shape_id"] not in val_ids]
    va = [r for r in rows if r["shape_id"] in val_ids]
    Xtr = np.array([r["features"] for r in tr], np.float32)
    ytr = np.log(np.array([r["us"] for r in tr], np.float32))
    Xva = np.array([r["features"] for r in va], np.float32)
    mean = Xtr.mean(axis=0)
    std = Xtr.std(axis=0)
    std[std == 0] = 1.0
    dev = torch.device("cuda")
    Xtr_d = torch.from_numpy((Xtr - mean) / std).to(dev)
    ytr_d = torch.from_numpy(ytr).to(dev)
    Xva_d = torch.from_numpy((Xva - mean) / std).to(dev)
    va_groups = _group(va)

    P = torch.from_numpy(_he_init(rng)).to(dev)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    act = torch.empty((batch, 2 * lpx.MLP_HIDDEN), device=dev)
    work = torch.empty((batch, 2 * lpx.MLP_HIDDEN), device=dev)
    grads = torch.empty_like(P)
    yb = torch.empty(batch, device=dev)
    dy = torch.empty(batch, device=dev)
    loss = torch.empty(1, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    n = Xtr_d.shape[0]
    best = (float("inf"), None, -1)
    history = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device=dev, generator=gen)
        tot = 0.0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb = Xtr_d.index_select(0, idx).contiguous()
            tb = ytr_d.index_select(0, idx).contiguous()
            lpx.mlp_forward(P, xb, act=act, y=yb)
            lpx.mlp_loss(yb, tb, dy=dy, loss=loss)
            lpx.mlp_backward(P, xb, act, dy, grads=grads, work=work)
            step += 1
            lpx.adam_step(P, grads, M, V, step, lr=lr)
            tot += loss.item()
        pred = lpx.mlp_forward(P, Xva_d).cpu().numpy()
        reg = _regret(pred, va_groups)
        nb = max(1, n // batch)
        history.append({"epoch": ep, "train_mse": tot / nb, "val_regret": reg})
        if reg < best[0] - 1e-6:
            best = (reg, P.clone(), ep)
        if log and ep % 10 == 0:
            log(f"train: epoch {ep} mse {tot / nb:.4f} val regret {reg:.4f}", flush=True)
        if ep - best[2] >= patience:
            break
    params = best[1].cpu().numpy()
    return params, mean, std, history


def evaluate(shapes, model_path, flush_mb=512, reps=5, log=print):
    """Regret of the learned pick against exhaustive tuning on held-out
    shapes, with the untuned default beside it (all from one timing pass)."""
    flush = torch.empty(flush_mb * (1 << 20) // 4, device="cuda")
    picker = lpx.Picker(model_path)
    res = []
    t0 = time.time()
    for si, sh in enumerate(shapes):
        tp = time.perf_counter()
        rec = lpx.pick_variant(sh["K"], sh["Np"], sh["E"], sh["layout"], sh["precision"],
                               mode=lpx.PICK_LEARNED, picker=picker)
        pick_us = (time.perf_counter() - tp) * 1e6
        tt = time.perf_counter()
        recs, times = tune_shape(sh, flush, reps=reps, seed=10_000 + si)
        tune_s = time.perf_counter() - tt
        times = np.array(times)
        li = recs.index(rec)
        di = recs.index(lpx.default_record(sh["precision"]))
        res.append({"shape": sh, "t_learned": float(times[li]), "t_best": float(np.nanmin(times)),
                    "t_untuned": float(times[di]), "learned": lpx.describe(rec),
                    "best": lpx.describe(recs[int(np.argmin(times))]),
                    "pick_us": pick_us, "tune_s": tune_s})
        if log and (si % 25 == 0 or si == len(shapes) - 1):
            log(f"evaluate: {si + 1}/{len(shapes)} shapes, {time.time() - t0:.0f} s", flush=True)
    picker.close()
    r = np.array([x["t_learned"] / x["t_best"] for x in res])
    g = np.array([x["t_untuned"] / x["t_learned"] for x in res])
    summary = {
        "shapes": len(res),
        "geomean_learned_over_best": float(np.exp(np.mean(np.log(r)))),
        "fraction_within_10pct": float(np.mean(r <= 1.10)),
        "sum_ratio": float(sum(x["t_learned"] for x in res) / sum(x["t_best"] for x in res)),
        "geomean_untuned_over_learned": float(np.exp(np.mean(np.log(g)))),
        "median_pick_us": float(np.median([x["pick_us"] for x in res])),
        "median_exhaustive_tune_s": float(np.median([x["tune_s"] for x in res])),
    }
    return summary, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="picker_out")
    ap.add_argument("--train-shapes", type=int, default=560)
    ap.add_argument("--eval-shapes", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--model", default=MODEL_PATH)
    ap.add_argument("--seeds", type=int, default=3,
                    help="initialisations trained; the lowest validation regret is kept")
    ap.add_argument("--eval-only", action="store_true",
                    help="evaluate the existing model on the held-out shapes only")
    ap.add_argument("--summary", default=None,
                    help="also write a text summary of the evaluation to this file")
    ap.add_argument("--timings", default=None,
                    help="train from the rows of an earlier collection (timings.jsonl, "
                         "or .gz) instead of timing the training shapes again")
    ap.add_argument("--widen-from", default=None,
                    help="write --model from a model file of the 12-feature cost model "
                         "(no tile-order feature): its weights with a zero weight for the "
                         "order feature, so its picks are unchanged (ties go to the cyclic "
                         "order, listed first)")
    ap.add_argument("--command", default=None,
                    help="with --summary-from: the command that wrote the eval.json")
    ap.add_argument("--summary-from", default=None,
                    help="write --summary from the eval.json of an earlier evaluation "
                         "(no GPU work)")
    args = ap.parse_args()
    if args.widen_from:
        widen_model(args.widen_from, args.model)
        return
    if args.summary_from:
        d = json.load(open(args.summary_from))
        args.out = os.path.dirname(args.summary_from)
        write_summary(args.summary, d["summary"], d["per_shape"], args)
        return
    os.makedirs(args.out, exist_ok=True)
    eval_shapes = inputs.picker_shapes(args.eval_shapes, seed=2)
    if args.eval_only:
        summary, res = evaluate(eval_shapes, args.model)
        json.dump({"summary": summary, "per_shape": res},
                  open(os.path.join(args.out, "eval.json"), "w"), indent=1)
        if args.summary:
            write_summary(args.summary, summary, res, args)
        print(json.dumps(summary), flush=True)
        return
    os.makedirs(os.path.dirname(args.model), exist_ok=True)
    if args.timings:
        import gzip
        opener = gzip.open if args.timings.endswith(".gz") else open
        with opener(args.timings, "rt") as fh:
            rows = [json.loads(line) for line in fh if line.strip()]
        print(f"loaded {len(rows)} timings from {args.timings}", flush=True)
    else:
        train_shapes = inputs.picker_shapes(args.train_shapes, seed=1)
        db = os.path.join(args.out, "timings.jsonl")
        if os.path.exists(db):
            os.remove(db)
        rows = collect(train_shapes, db_path=db)
    best = None
    for seed in range(args.seeds):
        params, mean, std, hist = train(rows, epochs=args.epochs, seed=seed)
        reg = min(h["val_regret"] for h in hist)
        print(f"seed {seed}: best val regret {reg:.4f}", flush=True)
        if best is None or reg < best[0]:
            best = (reg, params, mean, std, hist)
    _, params, mean, std, hist = best
    lpx.picker_save(args.model, params, mean, std)
    json.dump(hist, open(os.path.join(args.out, "train_history.json"), "w"))
    print(f"saved {args.model}; best val regret {min(h['val_regret'] for h in hist):.4f}",
          flush=True)
    summary, res = evaluate(eval_shapes, args.model)
    json.dump({"summary": summary, "per_shape": res},
              open(os.path.join(args.out, "eval.json"), "w"), indent=1)
    if args.summary:
        write_summary(args.summary, summary, res, args)
    print(json.dumps(summary), flush=True)


def widen_model(old_path, new_path, old_nf=12):
    """A 12-feature model file (magic, version and dimensions, mean[12],
    std[12], params, checksum) as a 13-feature one: W1 gains a zero column
    for the order feature, whose standardisation is (0, 1)."""
    raw = open(old_path, "rb").read()
    nh = lpx.MLP_HIDDEN
    nparams = nh * old_nf + nh + nh * nh + nh + nh + 1
    if len(raw) != 8 + 16 + 4 * (2 * old_nf + nparams) + 4:
        raise ValueError(f"{old_path} is not a {old_nf}-feature model file")
    v = np.frombuffer(raw[24:-4], dtype="<f4")
    mean, std, p = v[:old_nf], v[old_nf:2 * old_nf], v[2 * old_nf:]
    W1 = p[:nh * old_nf].reshape(nh, old_nf)
    W1n = np.concatenate([W1, np.zeros((nh, 1), np.float32)], axis=1)
    pn = np.concatenate([W1n.ravel(), p[nh * old_nf:]]).astype(np.float32)
    assert pn.size == lpx.MLP_PARAMS
    lpx.picker_save(new_path, pn, np.append(mean, 0.0), np.append(std, 1.0))


def write_summary(path, summary, res, args):
    """A short text record of a held-out evaluation: the summary figures,
    the regret distribution and the worst shapes."""
    r = sorted(((x["t_learned"] / x["t_best"], x) for x in res), key=lambda p: p[0])
    q = np.quantile([v for v, _ in r], [0.5, 0.9, 0.99, 1.0])
    by = {}
    for v, x in r:
        k = (x["shape"]["layout"], x["shape"]["precision"])
        by.setdefault(k, []).append(v)
    lines = [
        "# Learned picker: regret on held-out shapes",
        "",
        f"Command: `{args.command or ('python -m paper_1405_7470_amd.picker --eval-only --eval-shapes %d --out %s' % (args.eval_shapes, args.out))}` "
        f"(model `{os.path.relpath(args.model)}`), then `python -m paper_1405_7470_amd.picker "
        f"--summary-from {os.path.join(args.out, 'eval.json')} --summary {path}`.",
        "",
        f"Held-out shapes: {summary['shapes']} (seed 2: Np uniform in [8, 128], "
        "E = floor(2^U(10, 21)), layout and precision uniform, K = 3), each tuned "
        "exhaustively over every supported record with a cache flush before each timed launch; "
        "learned pick, untuned default and best read off the same timing pass.",
        "",
        "| figure | value |",
        "|---|---|",
        f"| geomean t_learned / t_best | {summary['geomean_learned_over_best']:.4f} |",
        f"| fraction of shapes within 10% of best | {summary['fraction_within_10pct']:.3f} |",
        f"| sum t_learned / sum t_best | {summary['sum_ratio']:.4f} |",
        f"| geomean t_untuned / t_learned (gain over no model) | "
        f"{summary['geomean_untuned_over_learned']:.3f} |",
        f"| median pick latency (us) | {summary['median_pick_us']:.1f} |",
        f"| median exhaustive tuning time (s) | {summary['median_exhaustive_tune_s']:.3f} |",
        f"| regret quantiles 50/90/99/100% | {q[0]:.3f} / {q[1]:.3f} / {q[2]:.3f} / {q[3]:.3f} |",
        "",
        "| layout/precision | shapes | geomean regret | within 10% |",
        "|---|---|---|---|",
    ]
    for k in sorted(by):
        v = np.array(by[k])
        lines.append(f"| {k[0]}/{k[1]} | {len(v)} | {float(np.exp(np.mean(np.log(v)))):.4f} | "
                     f"{float(np.mean(v <= 1.10)):.3f} |")
    lines += ["", "Worst five shapes:", "", "| K | Np | E | layout | precision | regret | learned "
              "| best |", "|---|---|---|---|---|---|---|---|"]
    for v, x in r[-5:][::-1]:
        sh = x["shape"]
        lines.append(f"| {sh['K']} | {sh['Np']} | {sh['E']} | {sh['layout']} | "
                     f"{sh['precision']} | {v:.3f} | {x['learned']} | {x['best']} |")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
