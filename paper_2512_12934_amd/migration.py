"""Droplet migration through the outlet, original against corrected outflow
(Sec. III C, Figs. 6 and 8).

A droplet of radius 30 starts at x = 100 in the middle of a channel of 500 x
100 fluid nodes (2-D) or 500 x 100 x 100 (3-D), carried by the inflow of the
continuous phase through the left face, and leaves through the convective
outlet on the right.  The same run is made with the outlet velocity
correction of eqs. (22)-(23) (corrected) and without it (original, eqs.
20-21 only).  The inflow speed is not given in the text; 0.02 is taken
(Reynolds number 12 on the channel width).  Recorded every ``every`` steps:
the droplet position x_d (the centroid of the largest connected region whose
component-1 density exceeds the mean of the two phase densities), its
deformation (L - B) / (L + B) in the mid plane, and the total mass against
its initial value.

    python -m paper_2512_12934_amd.migration --dim 2
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import cases, labels


def migration_case(dim=2, chi_on=True, length=500, width=100, R=30.0, x0=100.0, u_in=0.02, nu=0.17):
    """The migration channel: walls on the lateral faces, plug inflow u_in of
    the continuous phase at x = 0, outlet at x = length - 1; phases at the
    coexisting densities of G12 = 0.9 (both viscosities nu)."""
    yc = (width + 1) / 2.0
    drop = (x0, yc, R) if dim == 2 else (x0, yc, yc, R)
    c = cases.channel(length, width, u_in, nu=(nu, nu), droplet=drop, major=cases.COEX_G09[0],
                      minor=cases.COEX_G09[1], dim=dim, chi_on=chi_on)
    c.name = f"migration{dim}d_{'corrected' if chi_on else 'original'}"
    c.meta.update(x0=x0, R=R)
    return c


def droplet_state(rho_k, case, min_nodes=None):
    """(x_d, deformation, nodes) of the droplet: the largest face-connected
    region of the dispersed phase (films that collect along the corner edges
    of a square channel are separate regions).  x_d = nan once less than a
    tenth of the initial droplet is left in the domain."""
    from scipy import ndimage
    nx, ny, nz = case.n
    thr = labels.threshold(case)
    m = ((np.asarray(rho_k) > thr) & (case.solid == 0)).reshape(nz, ny, nx)
    lab, n = ndimage.label(m, structure=ndimage.generate_binary_structure(3, 1))
    if min_nodes is None:
        R = case.meta["R"]
        min_nodes = 0.1 * (np.pi * R * R if case.dim == 2 else 4.0 / 3.0 * np.pi * R ** 3)
    if n == 0:
        return float("nan"), float("nan"), 0
    sizes = np.bincount(lab.ravel())[1:]
    big = int(np.argmax(sizes)) + 1
    if sizes[big - 1] < min_nodes:
        return float("nan"), float("nan"), int(sizes[big - 1])
    g = lab == big
    zz, yy, xx = np.nonzero(g)
    xd = float(xx.mean())
    mid = g[nz // 2] if case.dim == 3 else g[0]
    y2, x2 = np.nonzero(mid)
    D = float("nan")
    if x2.size >= 3:
        lam = np.linalg.eigvalsh(np.cov(np.vstack([x2 - x2.mean(), y2 - y2.mean()]), bias=True))
        L, B = 2.0 * np.sqrt(max(lam[1], 0.0)), 2.0 * np.sqrt(max(lam[0], 0.0))
        D = float((L - B) / (L + B))
    return xd, D, int(g.sum())


def run(dim=2, steps=50000, every=1000, storage="f32", device="cuda:0", log=print, **kw):
    """Both outlets, stepped alternately on one stream.  Returns the record
    per variant and the stepping rate."""
    import torch
    from .lbm import LBM
    out = {}
    rate = {}
    for chi_on in (False, True):
        c = migration_case(dim, chi_on, **kw)
        s = LBM(c, storage=storage, device=device, tile_config="auto")
        s.set_graph_steps(16)
        rec = {"t": [], "x_d": [], "D": [], "nodes": [], "mass_dev": []}
        t_step = 0.0
        for k in range(steps // every):
            t0 = time.perf_counter()
            s.step(every)
            torch.cuda.synchronize()
            t_step += time.perf_counter() - t0
            rho, _ = s.moments()
            xd, D, n = droplet_state(rho[0], c)
            fl = s.mass_flux()
            rec["t"].append((k + 1) * every)
            rec["x_d"].append(xd)
            rec["D"].append(D)
            rec["nodes"].append(n)
            rec["mass_dev"].append(sum(fl["mass"]) / sum(fl["mass0"]) - 1.0)
        name = "corrected" if chi_on else "original"
        out[name] = rec
        rate[name] = c.fluid_nodes * steps / t_step / 1e6
        if log:
            log(f"[migration] {dim}-D {name}: {rate[name]:.0f} MLUPS; x_d " +
                " ".join(f"{v:.1f}" for v in rec["x_d"][::5]), flush=True)
        del s
        torch.cuda.empty_cache()
    return out, rate


def compare(rec):
    """Position deviation of the corrected run from the original one, before
    the droplet front reaches the outlet and while it passes it; mean and
    largest |m - m0| / m0 of both runs."""
    o, c = rec["original"], rec["corrected"]
    xo, xc = np.array(o["x_d"]), np.array(c["x_d"])
    both = np.isfinite(xo) & np.isfinite(xc)
    dev = np.abs(xc - xo) / np.maximum(xo, 1.0)
    res = {"max_position_deviation": float(dev[both].max()) if both.any() else None,
           "mass_dev_mean_abs": {k: float(np.mean(np.abs(rec[k]["mass_dev"]))) for k in rec},
           "mass_dev_max_abs": {k: float(np.max(np.abs(rec[k]["mass_dev"]))) for k in rec}}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dim", type=int, default=2)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--u-in", type=float, default=0.02)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    rec, rate = run(args.dim, args.steps, args.every, args.storage, u_in=args.u_in)
    res = {"dim": args.dim, "steps": args.steps, "MLUPS": rate, **compare(rec)}
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({**res, "records": rec}, fh)


if __name__ == "__main__":
    main()
