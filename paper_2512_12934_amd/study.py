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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mean, sd, fb = sur.predict(Xn, threshold=threshold)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pred = ys.inv(mean.cpu().numpy())
    fb = fb.cpu().numpy().astype(bool)
    ape = np.abs(pred - Y_true) / np.abs(Y_true)
    keep = ~fb
    return {"mape_all": ape.mean(0).tolist(),
            "mape_kept": ape[keep].mean(0).tolist() if keep.any() else None,
            "fallback_rate": float(fb.mean()), "seconds_per_query": dt / len(Xn), "n": int(len(Xn))}


def run(n_train, n_test, steps, W_range, every=100, members=5, epochs=3000, lr=3e-3, threshold=0.05,
        seed_train=12935, seed_test=12936, log=print):
    """Label n_train + n_test batched runs, train the ensemble on the usable
    training labels, and judge it on the held-out ones."""
    from .surrogate import Surrogate
    p_tr = cases.sweep_params(n_train, seed_train, W_range)
    p_te = cases.sweep_params(n_test, seed_test, W_range)
    lab_tr, t_tr = generate(p_tr, steps, every, log=log)
    lab_te, t_te = generate(p_te, steps, every, log=log)
    keep_tr = [i for i, l in enumerate(lab_tr) if usable(l)]
    keep_te = [i for i, l in enumerate(lab_te) if usable(l)]
    out = {"train_runs": n_train, "test_runs": n_test, "steps": steps, "W_range": list(W_range),
           "usable_train": len(keep_tr), "usable_test": len(keep_te),
           "lbm_seconds_per_run": (t_tr + t_te) / (n_train + n_test)}
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


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="label batched T-junction runs, train and judge the surrogate")
    ap.add_argument("--train", type=int, default=512)
    ap.add_argument("--test", type=int, default=64)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--wmin", type=int, default=16)
    ap.add_argument("--wmax", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.train, a.test, a.steps, (a.wmin, a.wmax), epochs=a.epochs)
    s = json.dumps(res)
    print(s, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(s + "\n")


if __name__ == "__main__":
    main()
