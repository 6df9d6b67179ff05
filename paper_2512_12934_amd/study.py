"""Labelled data from batched channel runs, and the surrogate trained on it.

``generate`` runs a sweep of T-junction instances as one batch, probing a
cross-section of every member at a fixed interval, and returns the labels of
each instance (droplet diameter over width, dimensionless period).
``features`` and ``Scaler`` turn instance parameters and labels into the
normalised arrays the surrogate trains on.  ``evaluate`` compares the
surrogate with the labels of held-out runs and times both.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import cases, labels


def features(params):
    """(log10 Ca, q, log10 M, W / 128) per instance."""
    return np.array([[math.log10(Ca), q, math.log10(M), W / 128.0] for (W, Ca, q, M) in params], np.float64)


class Scaler:
    """Affine normalisation to zero mean and unit spread, per column."""

    def __init__(self, a):
        a = np.asarray(a, np.float64)
        self.mu = a.mean(0)
        self.sd = np.where(a.std(0) > 0, a.std(0), 1.0)

    def fwd(self, a):
        return (np.asarray(a, np.float64) - self.mu) / self.sd

    def inv(self, a):
        return np.asarray(a, np.float64) * self.sd + self.mu


def generate(params, steps, every=100, storage="f32", chunk=256, device="cuda:0", log=print):
    """Run every instance of ``params`` (list of (W, Ca, q, M)) for ``steps``
    steps, batched ``chunk`` at a time; returns (labels, seconds): labels[i]
    is a dict with D_over_W, T_star (None where undefined) and the series."""
    import torch
    from .lbm import Batch
    out = []
    t_total = 0.0
    for c0 in range(0, len(params), chunk):
        cs = [cases.sweep_case(*p) for p in params[c0:c0 + chunk]]
        b = Batch(cs, storage=storage, device=device)
        regs = [labels.tjunction_regions(c) for c in cs]
        thr = [labels.threshold(c) for c in cs]
        n = steps // every
        series = torch.zeros((len(cs), n), dtype=torch.int64, device=device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n):
            b.step(every)
            for i, m in enumerate(b.members):
                m.probe(0, regs[i][1][0], regs[i][1][1], thr[i], series[i, k:k + 1])
        torch.cuda.synchronize()
        t_total += time.perf_counter() - t0
        s = series.cpu().numpy()
        for i, (c, m) in enumerate(zip(cs, b.members)):
            comps, _ = m.components(0, regs[i][0][0], regs[i][0][1], thr[i])
            D = labels.droplets(comps, regs[i][0], c.dim)
            T = labels.period(s[i], every)
            W, u_c = c.meta["W"], c.meta["u_c"]
            out.append({"D_over_W": float(np.mean(D)) / W if D else None,
                        "T_star": None if T is None else T * u_c / W,
                        "passages": int(len(labels.passages(s[i]))), "series": s[i]})
        log(f"[study] instances {c0}..{c0 + len(cs)}: {steps} steps in {t_total:.1f} s so far")
        del b
    return out, t_total


def usable(lab):
    return lab["D_over_W"] is not None and lab["T_star"] is not None


def evaluate(sur, xs, ys, X_raw, Y_true, threshold=0.05):
    """Held-out comparison: mean absolute percentage error of the surrogate's
    mean prediction against the LBM labels, on all queries and on those the
    ensemble keeps (no fallback); the fallback rate; seconds per query."""
    import torch
    Xn = xs.fwd(X_raw).astype(np.float32)
    # the network predicts normalised labels; the kernel maps every member's
    # outputs back to D/W and T* before the ensemble statistics, so the
    # disagreement test is relative to the physical values
    query = lambda: sur.predict(Xn, threshold=threshold, out_scale=ys.sd, out_shift=ys.mu)
    query()   # the first call pays one-time costs (kernel loading, allocations)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        mean, sd, fb = query()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    pred = mean.cpu().numpy().astype(np.float64)
    fb = fb.cpu().numpy().astype(bool)
    ape = np.abs(pred - Y_true) / np.abs(Y_true)
    keep = ~fb
    return {"mape_all": ape.mean(0).tolist(),
            "mape_kept": ape[keep].mean(0).tolist() if keep.any() else None,
            "fallback_rate": float(fb.mean()), "seconds_per_query": dt / len(Xn), "n": int(len(Xn))}


def save_labels(path, p_tr, lab_tr, p_te, lab_te, seconds, steps):
    """Parameters and labels of both sets as .npz (NaN where undefined)."""
    nan = float("nan")
    lab = lambda L: np.array([[l["D_over_W"] if l["D_over_W"] is not None else nan,
                               l["T_star"] if l["T_star"] is not None else nan, l["passages"]] for l in L])
    np.savez(path, params_train=np.array(p_tr, np.float64), labels_train=lab(lab_tr),
             params_test=np.array(p_te, np.float64), labels_test=lab(lab_te),
             lbm_seconds=np.array(seconds, np.float64), steps=steps)


def load_labels(path):
    """The sets written by save_labels: (p_tr, lab_tr, p_te, lab_te, seconds, steps)."""
    z = np.load(path)
    lab = lambda a: [{"D_over_W": None if np.isnan(r[0]) else float(r[0]),
                      "T_star": None if np.isnan(r[1]) else float(r[1]), "passages": int(r[2])} for r in a]
    tup = lambda a: [tuple(float(v) for v in r) for r in a]
    return (tup(z["params_train"]), lab(z["labels_train"]), tup(z["params_test"]), lab(z["labels_test"]),
            z["lbm_seconds"].tolist(), int(z["steps"]))


def fit_and_evaluate(p_tr, lab_tr, p_te, lab_te, seconds, steps, members=5, epochs=3000, lr=3e-3,
                  threshold=0.05):
    """Train the ensemble on the usable training labels and evaluate it on the
    usable held-out ones; seconds = LBM time of the two sets."""
    from .surrogate import Surrogate
    keep_tr = [i for i, l in enumerate(lab_tr) if usable(l)]
    keep_te = [i for i, l in enumerate(lab_te) if usable(l)]
    out = {"train_runs": len(p_tr), "test_runs": len(p_te), "steps": steps,
           "usable_train": len(keep_tr), "usable_test": len(keep_te),
           "lbm_seconds_per_run": sum(seconds) / (len(p_tr) + len(p_te))}
    if len(keep_tr) < 8 or not keep_te:
        out["note"] = "too few labelled runs"
        return out
    Xtr = features([p_tr[i] for i in keep_tr])
    Ytr = np.array([[lab_tr[i]["D_over_W"], lab_tr[i]["T_star"]] for i in keep_tr])
    Xte = features([p_te[i] for i in keep_te])
    Yte = np.array([[lab_te[i]["D_over_W"], lab_te[i]["T_star"]] for i in keep_te])
    xs, ys = Scaler(Xtr), Scaler(Ytr)
    sur = Surrogate(members=members, max_n=max(len(Xtr), 64), seed=0)
    loss = sur.train(xs.fwd(Xtr).astype(np.float32), ys.fwd(Ytr).astype(np.float32), epochs, lr)
    out["train_loss"] = loss.tolist()
    out["held_out"] = evaluate(sur, xs, ys, Xte, Yte, threshold)
    out["gain_seconds_per_query"] = out["lbm_seconds_per_run"] / out["held_out"]["seconds_per_query"]
    return out


def run(n_train, n_test, steps, W_range, every=100, members=5, epochs=3000, lr=3e-3, threshold=0.05,
        seed_train=12935, seed_test=12936, chunk=256, labels_out=None, log=print):
    """Label n_train + n_test batched runs (chunk instances per batch), train
    the ensemble on the usable training labels, and evaluate it on the held-out
    ones; labels_out (optional) receives the parameters and labels as .npz."""
    p_tr = cases.sweep_params(n_train, seed_train, W_range)
    p_te = cases.sweep_params(n_test, seed_test, W_range)
    lab_tr, t_tr = generate(p_tr, steps, every, chunk=chunk, log=log)
    lab_te, t_te = generate(p_te, steps, every, chunk=chunk, log=log)
    if labels_out:
        save_labels(labels_out, p_tr, lab_tr, p_te, lab_te, [t_tr, t_te], steps)
    out = fit_and_evaluate(p_tr, lab_tr, p_te, lab_te, [t_tr, t_te], steps, members, epochs, lr, threshold)
    out["W_range"] = list(W_range)
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="label batched T-junction runs, train and evaluate the surrogate")
    ap.add_argument("--train", type=int, default=512)
    ap.add_argument("--test", type=int, default=64)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--wmin", type=int, default=16)
    ap.add_argument("--wmax", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--chunk", type=int, default=256, help="instances per batch")
    ap.add_argument("--out", default=None)
    ap.add_argument("--labels-out", default=None, help="write parameters and labels to this .npz")
    ap.add_argument("--labels-in", default=None, help="train and evaluate on labels saved by --labels-out")
    ap.add_argument("--threshold", type=float, default=0.05, help="ensemble disagreement that falls back")
    a = ap.parse_args(argv)
    if a.labels_in:
        res = fit_and_evaluate(*load_labels(a.labels_in), epochs=a.epochs, threshold=a.threshold)
    else:
        res = run(a.train, a.test, a.steps, (a.wmin, a.wmax), epochs=a.epochs, threshold=a.threshold,
                  chunk=a.chunk, labels_out=a.labels_out)
    s = json.dumps(res)
    print(s, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(s + "\n")


if __name__ == "__main__":
    main()
