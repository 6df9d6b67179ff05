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


def generate(params, steps, every=100, storage="f16", chunk=256, device="cuda:0", log=print):
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
