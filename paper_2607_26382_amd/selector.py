"""Learned first-floor selection (addition (4)): labelled data from the guarded
solver, training with the library's MLP kernels, exact offline replay of the
guarded ladder, and the stored model.

The selector replaces only the choice of the first rung k0 in the floor policy
(Alg. floor_policy); the ladder above k0 and the recomputed FP64 residual
guard stay as they are, so a wrong prediction costs iterations, never
correctness.  Inputs are the two probe features of Sec. 3.4 (log10 r50,
log10 r100) and six density statistics computed on the device
(tg_density_features); the label is the lowest admissible rung, i.e. the
lowest ladder floor whose independent solve passes the guard.

Every solve in a batch is bitwise the solve the same state would get alone, so
the outcome of an attempt (iterations, guard verdict) depends only on (state,
rung).  Recording the outcome at every rung therefore lets any choice of k0 be
replayed exactly offline: the replayed attempts are the ones the online policy
makes.

Usage (GPU):
  python -m paper_2607_26382_amd.selector label --n 20000 --seed0 5000000 --out train.npz
  python -m paper_2607_26382_amd.selector label --n 2000 --seed0 6000000 --dims 64,32,32 --out heldout.npz
  python -m paper_2607_26382_amd.selector train --data train.npz --out selector_model.json
  python -m paper_2607_26382_amd.selector evaluate --model selector_model.json --data heldout.npz
"""
import argparse
import itertools
import json
import math
import os
import sys
import time

import numpy as np

RUNGS = (1e-9, 1e-6, 1e-4, 1e-3)
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_model.json")
SIZES = (8, 64, 64, 4)


# ---------------------------------------------------------------------------
# labelled data
def _batch_size(dims):
    n_e = dims[0] * dims[1] * dims[2]
    return 256 if n_e <= 8192 else 128 if n_e <= 27648 else 102


def label_states(seeds, dims=None, prec=None, tau=1e-6, log=print):
    """Probe features, density statistics and the outcome at every rung for
    the selector mixture states of `seeds` (grid from the mixture unless
    `dims`).  Returns a dict of arrays (one row per seed)."""
    import torch

    from . import synth
    from . import topoguard as tg

    prec = tg.BF16X3MFMA if prec is None else prec
    states = [synth.selector_state(s, dims) for s in seeds]
    n = len(seeds)
    out = dict(seed=np.asarray(seeds, dtype=np.int64), dims=np.zeros((n, 3), np.int32),
               kind=np.zeros(n, np.int8), r50=np.zeros(n), r100=np.zeros(n),
               feat=np.zeros((n, 8), np.float32), probe_iters=np.zeros(n, np.int32),
               iters=np.zeros((n, len(RUNGS)), np.int32), acc=np.zeros((n, len(RUNGS)), bool),
               eta=np.full((n, len(RUNGS)), np.nan), label=np.full(n, -1, np.int32))
    for i, (d, _, k) in enumerate(states):
        out["dims"][i] = d
        out["kind"][i] = 0 if k == "blobs" else 1
    by_dims = {}
    for i, (d, _, _) in enumerate(states):
        by_dims.setdefault(tuple(d), []).append(i)
    solve = tg.solver_opts(restart=30, max_iters=200, tol=tau, prec=prec)
    pol = tg.policy(rungs=RUNGS, tau=tau, selector=tg.SELECT_FIXED, fixed_rung=0, solve=solve,
                    want_features=True)
    done, t0 = 0, time.time()
    for d, idx in sorted(by_dims.items()):
        bs = _batch_size(d)
        grids = [tg.Grid(*d, max_restart=100, device="cuda") for _ in range(bs)]
        f = torch.tensor(grids[0].edge_load(), device="cuda")
        for c0 in range(0, len(idx), bs):
            chunk = idx[c0:c0 + bs]
            m = len(chunk)
            batch = tg.Batch(grids[:m])
            rhos = [torch.tensor(states[i][1], device="cuda") for i in chunk]
            fs = [f] * m
            _, res = batch.select_floor(rhos, fs, pol)
            for q, i in enumerate(chunk):
                r = res[q]
                out["r50"][i], out["r100"][i] = r["r50"], r["r100"]
                out["feat"][i] = np.asarray(r["features"], dtype=np.float32)
                out["probe_iters"][i] = r["probe_iters"]
                out["label"][i] = r["rung"]
                for a in r["attempts"]:
                    out["iters"][i, a["rung"]] = a["iterations"]
                    out["acc"][i, a["rung"]] = a["accepted"]
                    out["eta"][i, a["rung"]] = a["true_eta"]
            # outcomes above the accepted rung, for exact replay of any k0
            for k in range(1, len(RUNGS)):
                sub = [q for q, i in enumerate(chunk) if 0 <= out["label"][i] < k]
                if not sub:
                    continue
                b2 = tg.Batch([grids[q] for q in sub])
                b2.set_density([rhos[q] for q in sub], 3.0, [RUNGS[k]] * len(sub))
                _, rs = b2.solve([f] * len(sub), solve)
                for q, rr in zip(sub, rs):
                    i = chunk[q]
                    out["iters"][i, k] = rr["iterations"]
                    out["eta"][i, k] = rr["true_eta"]
                    out["acc"][i, k] = bool(np.isfinite(rr["true_eta"]) and rr["true_eta"] <= tau)
                del b2
            del batch
            done += m
            log(f"labelled {done}/{n} states ({d[0]}x{d[1]}x{d[2]}), {time.time() - t0:.1f} s", flush=True)
        del grids
    return out


# ---------------------------------------------------------------------------
# exact replay of the guarded ladder from a first rung
def replay(data, k0):
    """Attempts the guarded ladder makes from first rung k0[i] for every state:
    returns dict(rung, attempts, iters_selected, iters_rejected, first_ok)."""
    acc = np.asarray(data["acc"], bool)
    it = np.asarray(data["iters"], np.int64)
    n, R = acc.shape
    k0 = np.asarray(k0, np.int64)
    # first admissible rung at or above k (R if none)
    nxt = np.full((n, R + 1), R, np.int64)
    for k in range(R - 1, -1, -1):
        nxt[:, k] = np.where(acc[:, k], k, nxt[:, k + 1])
    cum = np.concatenate([np.zeros((n, 1), np.int64), np.cumsum(it, axis=1)], axis=1)
    rows = np.arange(n)
    stop = nxt[rows, k0]                       # accepted rung, or R
    ok = stop < R
    rung = np.where(ok, stop, -1)
    attempts = np.where(ok, stop - k0 + 1, R - k0)
    rejected = cum[rows, stop] - cum[rows, k0]
    selected = np.where(ok, it[rows, np.minimum(stop, R - 1)], 0)
    return dict(rung=rung, attempts=attempts, iters_selected=selected, iters_rejected=rejected,
                first_ok=ok & (stop == k0))


def rule_k0(data, t_high=1e-2, t_plateau=1e-4, t_ratio=0.6):
    """Eq. trigger: escalate iff r50 >= t_high or (r100 >= t_plateau and
    r100 / r50 >= t_ratio); escalation starts the ladder at rung 1."""
    r50, r100 = data["r50"], data["r100"]
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(r50 > 0, r100 / r50, 1.0)
    fire = (r50 >= t_high) | ((r100 >= t_plateau) & (ratio >= t_ratio))
    return fire.astype(np.int32)


def summarize(data, k0):
    """Policy metrics of first rungs k0 on labelled data."""
    rp = replay(data, k0)
    label = data["label"]
    probe = data["probe_iters"].astype(np.int64)
    admissible = label >= 0
    total = probe + rp["iters_selected"] + rp["iters_rejected"]
    return dict(
        n=int(len(k0)),
        certified=int(np.count_nonzero(rp["rung"] >= 0)),
        first_attempt_accept=float(np.mean(rp["first_ok"])),
        mean_attempts=float(np.mean(rp["attempts"])),
        wasted_iters_per_state=float(np.mean(rp["iters_rejected"])),
        total_iters_per_state=float(np.mean(total)),
        at_lowest_admissible=float(np.mean(rp["rung"][admissible] == label[admissible])) if admissible.any() else 1.0,
        first_at_lowest=float(np.mean(np.asarray(k0)[admissible] == label[admissible])) if admissible.any() else 1.0,
        above_lowest_admissible=int(np.count_nonzero(rp["rung"][admissible] > label[admissible])),
        k0_hist=np.bincount(np.asarray(k0), minlength=len(RUNGS)).tolist(),
    )


def cost_key(s):
    """Ordering of policies: most first attempts at the lowest admissible rung
    (accepted at once and nothing preserved lost), then fewest iterations."""
    return (-s["first_at_lowest"], s["total_iters_per_state"])


def tune_rule(data):
    """Re-tunes the rule's three thresholds on labelled data over a 288-point
    grid (8 x 6 x 6), keeping the combination with the lowest cost_key."""
    th = np.logspace(-4, -0.5, 8)
    tp = np.logspace(-7, -2, 6)
    tr = np.linspace(0.3, 0.95, 6)
    best = None
    for a, b, c in itertools.product(th, tp, tr):
        s = summarize(data, rule_k0(data, a, b, c))
        if best is None or cost_key(s) < cost_key(best[1]):
            best = ((float(a), float(b), float(c)), s)
    return best[0]


# ---------------------------------------------------------------------------
# training (device kernels)
def init_params(seed):
    """He-normal weights from default_rng(seed), zero biases (W[out][in])."""
    rng = np.random.default_rng(seed)
    flat = []
    for fi, fo in zip(SIZES[:-1], SIZES[1:]):
        flat.append((rng.standard_normal((fo, fi)) * math.sqrt(2.0 / fi)).ravel())
        flat.append(np.zeros(fo))
    return np.concatenate(flat).astype(np.float32)


def standardization(X):
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std = np.where(std > 1e-6, std, 1.0)
    return mean.astype(np.float32), std.astype(np.float32)


def train(data, epochs=30, batch=256, lr=1e-3, seed=0, log=print):
    """Adam on the mean cross-entropy of the lowest-admissible-rung labels
    (states with no admissible rung are left out), run by the MLP kernels."""
    import torch

    from . import topoguard as tg

    keep = data["label"] >= 0
    X = np.asarray(data["feat"][keep], dtype=np.float32)
    y = np.asarray(data["label"][keep], dtype=np.int32)
    mean, std = standardization(X)
    mlp = tg.MLP(init_params(seed), mean, std, max_batch=batch)
    Xd = torch.tensor(X, device="cuda")
    yd = torch.tensor(y, device="cuda")
    rng = np.random.default_rng(seed + 1)
    hist = []
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(len(y)), device="cuda")
        tot = 0.0
        for b0 in range(0, len(y), batch):
            ix = perm[b0:b0 + batch]
            loss = mlp.train_step(Xd[ix], yd[ix], lr)
            tot += loss * len(ix)
        hist.append(tot / len(y))
        log(f"epoch {ep + 1}/{epochs}: mean loss {hist[-1]:.4f}", flush=True)
    return mlp, mean, std, hist


def predict(mlp, feat):
    import torch

    logits = mlp.forward(torch.tensor(np.asarray(feat, dtype=np.float32), device="cuda")).cpu().numpy()
    return np.argmax(logits, axis=1).astype(np.int32)   # first maximum: ties to the lower rung


def save_model(path, mlp, mean, std, meta):
    obj = dict(sizes=list(SIZES), rungs=list(RUNGS), params=[float(v) for v in mlp.get_params()],
               mean=[float(v) for v in mean], std=[float(v) for v in std], meta=meta)
    with open(path, "w") as fh:
        json.dump(obj, fh)


def load_model(path=MODEL_PATH, device="cuda"):
    """The stored selector as a tg.MLP on the device."""
    from . import topoguard as tg

    with open(path) as fh:
        obj = json.load(fh)
    if tuple(obj["sizes"]) != SIZES:
        raise ValueError("stored selector has another architecture")
    return tg.MLP(np.asarray(obj["params"], np.float32), np.asarray(obj["mean"], np.float32),
                  np.asarray(obj["std"], np.float32), device=device), obj


def load_data(path):
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def concat(parts):
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def evaluate(mlp, data, tuned=None):
    """Held-out comparison: plain rule, re-tuned rule, MLP, and the two fixed
    baselines (always rho0 first; always the top rung)."""
    res = dict(rule=summarize(data, rule_k0(data)))
    if tuned is not None:
        res["rule_tuned"] = summarize(data, rule_k0(data, *tuned))
    res["mlp"] = summarize(data, predict(mlp, data["feat"]))
    res["always_rho0"] = summarize(data, np.zeros(len(data["label"]), np.int32))
    res["always_top"] = summarize(data, np.full(len(data["label"]), len(RUNGS) - 1, np.int32))
    res["label_hist"] = np.bincount(data["label"] + 1, minlength=len(RUNGS) + 1).tolist()   # [none, r0..]
    return res


# ---------------------------------------------------------------------------
def _main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2607_26382_amd.selector")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("label")
    a.add_argument("--n", type=int, required=True)
    a.add_argument("--seed0", type=int, required=True)
    a.add_argument("--dims", default=None)
    a.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--out", default=MODEL_PATH)
    t.add_argument("--epochs", type=int, default=30)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--heldout", nargs="*", default=[])
    e = sub.add_parser("evaluate")
    e.add_argument("--model", default=MODEL_PATH)
    e.add_argument("--data", nargs="+", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "label":
        dims = tuple(int(v) for v in args.dims.split(",")) if args.dims else None
        d = label_states(list(range(args.seed0, args.seed0 + args.n)), dims)
        np.savez_compressed(args.out, **d)
        print(json.dumps(dict(states=args.n, label_hist=np.bincount(d["label"] + 1, minlength=5).tolist())))
    elif args.cmd == "train":
        data = concat([load_data(p) for p in args.data])
        tuned = tune_rule(data)
        mlp, mean, std, hist = train(data, epochs=args.epochs, seed=args.seed)
        meta = dict(train_states=int(len(data["label"])), train_files=[os.path.basename(p) for p in args.data],
                    epochs=args.epochs, seed=args.seed, loss_hist=hist, tuned_rule=list(tuned),
                    train_eval=evaluate(mlp, data, tuned))
        if args.heldout:
            ho = concat([load_data(p) for p in args.heldout])
            meta["heldout_eval"] = evaluate(mlp, ho, tuned)
            meta["heldout_states"] = int(len(ho["label"]))
        save_model(args.out, mlp, mean, std, meta)
        print(json.dumps(meta.get("heldout_eval", meta["train_eval"]), indent=1))
    else:
        mlp, obj = load_model(args.model)
        data = concat([load_data(p) for p in args.data])
        print(json.dumps(evaluate(mlp, data, obj["meta"].get("tuned_rule")), indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(_main())
