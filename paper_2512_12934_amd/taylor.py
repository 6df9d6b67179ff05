"""Taylor deformation on the GPU (Sec. III A, Fig. 4): droplets sheared
between plates moving in opposite directions, at viscosity ratios M = 30 and
110, for several capillary numbers and both s_eps policies, all advanced
together as one batch.

The deformation of each droplet is (L - B) / (L + B), with L and B the half
length and half width of the droplet.  They are taken from the second
moments of the dispersed region (nodes whose component-1 density is above the
mean of the two phase densities): for an ellipse of half axes a and b the
eigenvalues of the covariance of its area are a^2 / 4 and b^2 / 4.  The
paper's claims checked here: the deformation grows linearly with Ca, and
taking s_eps from the most viscous phase leaves it unchanged.

    python -m paper_2512_12934_amd.taylor --steps 60000
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import cases, labels


def deformation(rho_k, case) -> tuple:
    """(D, area or volume) of the droplet of component 1 in the x-y plane
    through the droplet (2-D: the whole field; 3-D: the mid z-plane)."""
    nx, ny, nz = case.n
    r = np.asarray(rho_k).reshape(nz, ny, nx)
    r = r[nz // 2] if case.dim == 3 else r[0]
    thr = labels.threshold(case)
    m = r > thr
    m[0, :] = m[-1, :] = False
    yy, xx = np.nonzero(m)
    if xx.size < 3:
        return float("nan"), int(xx.size)
    cov = np.cov(np.vstack([xx - xx.mean(), yy - yy.mean()]), bias=True)
    lam = np.linalg.eigvalsh(cov)
    L, B = 2.0 * np.sqrt(max(lam[1], 0.0)), 2.0 * np.sqrt(max(lam[0], 0.0))
    return float((L - B) / (L + B)), int(xx.size)


def study_cases(Ms=(30, 110), Cas=(0.025, 0.05, 0.075, 0.1), policies=(0, 1), nx=320, H=160, R=32.0,
                dim=2):
    out = []
    for M in Ms:
        for pol in policies:
            for Ca in Cas:
                out.append(cases.taylor(M, Ca, nx=nx, H=H, R=R, dim=dim, s_eps_policy=pol))
    return out


def run(case_list, steps, every, storage="f32", device="cuda:0", log=print):
    """Advance all cases as one batch; the deformation of each, every
    ``every`` steps.  Returns (rows, seconds of device stepping)."""
    import torch
    from .lbm import Batch
    b = Batch(case_list, storage=storage, device=device)
    b.set_graph_steps(16)
    series = [[] for _ in case_list]
    t_step = 0.0
    for k in range(steps // every):
        t0 = time.perf_counter()
        b.step(every)
        torch.cuda.synchronize()
        t_step += time.perf_counter() - t0
        for i, c in enumerate(case_list):
            rho, _ = b[i].moments()
            series[i].append(deformation(rho[0], c))
        log(f"[taylor] step {(k + 1) * every}: " +
            " ".join(f"{s[-1][0]:.4f}" for s in series), flush=True) if log else None
    rows = []
    for c, s in zip(case_list, series):
        D = np.array([d for d, _ in s])
        rows.append({"M": c.meta["M"], "Ca": c.meta["Ca"], "policy": "maxvisc" if c.s_eps_policy == 0 else "fixed",
                     "U": c.meta["U"], "D": float(np.mean(D[-3:])), "D_spread_last3": float(np.ptp(D[-3:])),
                     "area_first_last": (s[0][1], s[-1][1]), "series": D.tolist()})
    nodes = sum(c.fluid_nodes for c in case_list)
    return rows, t_step, nodes


def linear_fit(Ca, D):
    """Least-squares line D = a Ca + b; returns (a, b, R^2)."""
    Ca, D = np.asarray(Ca, float), np.asarray(D, float)
    A = np.vstack([Ca, np.ones_like(Ca)]).T
    (a, b), *_ = np.linalg.lstsq(A, D, rcond=None)
    r2 = 1 - ((D - A @ [a, b]) ** 2).sum() / ((D - D.mean()) ** 2).sum()
    return float(a), float(b), float(r2)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=60000)
    ap.add_argument("--every", type=int, default=5000)
    ap.add_argument("--nx", type=int, default=320)
    ap.add_argument("--H", type=int, default=160)
    ap.add_argument("--R", type=float, default=32.0)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--M", type=float, nargs="+", default=[30, 110])
    ap.add_argument("--Ca", type=float, nargs="+", default=[0.025, 0.05, 0.075, 0.1])
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    cl = study_cases(Ms=args.M, Cas=args.Ca, nx=args.nx, H=args.H, R=args.R)
    rows, secs, nodes = run(cl, args.steps, args.every, storage=args.storage)
    fits = {}
    for M in sorted({r["M"] for r in rows}):
        for pol in ("maxvisc", "fixed"):
            sel = [r for r in rows if r["M"] == M and r["policy"] == pol]
            fits[f"M{M:g}_{pol}"] = linear_fit([r["Ca"] for r in sel], [r["D"] for r in sel])
    res = {"rows": [{k: v for k, v in r.items() if k != "series"} for r in rows], "fits": fits,
           "members": len(cl), "fluid_nodes": nodes, "steps": args.steps,
           "MLUPS": nodes * args.steps / secs / 1e6}
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({**res, "series": [r["series"] for r in rows]}, fh)


if __name__ == "__main__":
    main()
