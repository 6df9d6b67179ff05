"""Droplet labels of a channel run: droplet diameter and generation period.

The paper compares droplet sizes and generation periods of its T-junction
and co-flow runs (Sec. III D) without defining them operationally.  Readings
taken here:

* the dispersed phase is the set of fluid nodes whose dispersed-component
  density exceeds the mean of the two bulk densities;
* a droplet is a face-connected component of it inside the main channel
  downstream of the junction, and its diameter is that of the disc (2-D) or
  ball (3-D) of the same area or volume;
* the generation period is the median interval between droplet passages
  through a cross-section of the main channel, after the first two passages
  are discarded; fewer than three remaining passages leave it undefined
  (censored).  The median keeps one irregular passage (a droplet that breaks
  up in the channel, a front that recedes and returns between two samples)
  from moving the period.  T* = T u_c / W.

The GPU does the node work (``lbm_probe``: passage counts; ``lbm_components``:
connected components); this module turns counts and components into labels.
"""
from __future__ import annotations

import math

import numpy as np


def diameter(size: float, dim: int) -> float:
    """Equivalent diameter of a droplet of ``size`` nodes."""
    if dim == 2:
        return 2.0 * math.sqrt(size / math.pi)
    return (6.0 * size / math.pi) ** (1.0 / 3.0)


def threshold(case) -> float:
    """Half-way between the bulk densities of the dispersed component."""
    major = max(case.rho0[0].max(), case.rho0[1].max())
    minor = min(case.rho0[0][case.solid == 0].min(), case.rho0[1][case.solid == 0].min())
    return 0.5 * (major + minor)


def passages(series, on: int = 1) -> np.ndarray:
    """Sample indices at which the probe count rises from below ``on`` to at
    least ``on`` (a droplet front reaching the cross-section)."""
    s = np.asarray(series) >= on
    return np.nonzero(s[1:] & ~s[:-1])[0] + 1


def period(series, every: int, skip: int = 2):
    """Median interval (in steps) between passages after the first ``skip``;
    None when fewer than three passages remain."""
    ev = passages(series)[skip:]
    if len(ev) < 3:
        return None
    return float(np.median(np.diff(ev)) * every)


def tjunction_regions(case):
    """(region box, probe box) of a T-junction case: the main channel from one
    channel width past the side channel to two nodes before the outlet, and
    the cross-section at its middle."""
    W = case.meta["W"]
    x0 = case.meta["x_side"] + case.meta["side_width"] + W // 2
    x1 = case.n[0] - 2
    xp = (x0 + x1) // 2
    region = ((x0, 1, 0), (x1, W + 1, 1))
    probe = ((xp, 1, 0), (xp + 1, W + 1, 1))
    return region, probe


def droplets(components, region, dim):
    """Diameters of the components that lie strictly inside the region along
    the channel axis (not cut by its upstream or downstream end)."""
    (lo, hi) = region
    out = []
    for c in components:
        if c["lo"][0] > lo[0] and c["hi"][0] < hi[0]:
            out.append(diameter(c["size"], dim))
    return out


def label_run(sim, case, steps: int, every: int = 100, k: int = 0):
    """Advance ``sim`` (an LBM context or batch member) by ``steps`` steps,
    probing every ``every`` steps; returns a dict with the passage series,
    the period T, T* and the droplet diameters at the end."""
    import torch
    region, probe = tjunction_regions(case)
    thr = threshold(case)
    n = steps // every
    series = torch.zeros(n, dtype=torch.int64, device=sim.device)
    for i in range(n):
        sim.step(every)
        sim.probe(k, probe[0], probe[1], thr, series[i:i + 1])
    comps, total = sim.components(k, region[0], region[1], thr)
    s = series.cpu().numpy()
    T = period(s, every)
    W, u_c = case.meta["W"], case.meta["u_c"]
    D = droplets(comps, region, case.dim)
    return {"series": s, "T": T, "T_star": None if T is None else T * u_c / W, "D": D,
            "D_over_W": float(np.mean(D)) / W if D else None, "n_components": total}
