"""Droplet labels on the GPU: passage counts and connected components must
equal, exactly, a CPU labelling (scipy.ndimage) of the same FP32 density
field, and the droplet sizes must agree with those of the FP64 oracle run."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2512_12934_amd import cases, labels

pytestmark = pytest.mark.gpu


def _cpu_components(rho_k, case, lo, hi, thr):
    nx, ny, nz = case.n
    f = np.float32(thr)
    field = rho_k.reshape(nz, ny, nx).astype(np.float32) > f
    field &= (case.solid.reshape(nz, ny, nx) == 0)
    box = np.zeros_like(field)
    box[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = True
    field &= box
    structure = ndimage.generate_binary_structure(3, 1)
    lab, n = ndimage.label(field, structure=structure)
    out = []
    idx = np.arange(field.size).reshape(field.shape)
    for j in range(1, n + 1):
        m = lab == j
        zz, yy, xx = np.nonzero(m)
        out.append({"first": int(idx[m].min()), "size": int(m.sum()),
                    "lo": (int(xx.min()), int(yy.min()), int(zz.min())),
                    "hi": (int(xx.max()) + 1, int(yy.max()) + 1, int(zz.max()) + 1)})
    return sorted(out, key=lambda c: c["first"]), int(field.sum())


CASES = [
    ("drops2d", lambda: cases.drops()),
    ("drops3d", lambda: cases.drops(shape=(40, 32, 36), count=6, r_range=(3.0, 7.0))),
    ("tjunction_small", lambda: cases.tjunction(W=20, length=90, x_side=30, side_width=14, side_len=18)),
]


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_components_and_probe_equal_cpu_labelling(name, make, storage):
    import torch
    from paper_2512_12934_amd.lbm import LBM
    c = make()
    print(f"[gpu] labels {name} storage={storage}", flush=True)
    g = LBM(c, storage=storage)
    g.step(40)
    thr = labels.threshold(c)
    lo = (1, 1, 0)
    hi = (c.n[0] - 1, c.n[1] - 1, c.n[2] - 1 if c.dim == 3 else 1)
    if c.dim == 3:
        lo = (1, 1, 1)
    comps, n = g.components(0, lo, hi, thr)
    rho, _ = g.moments()
    ref, count = _cpu_components(rho[0], c, lo, hi, thr)
    assert n == len(ref) and n > 0
    assert comps == ref
    out = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    g.probe(0, lo, hi, thr, out)
    assert int(out.item()) == count
    # a thin cross-section
    xs = c.n[0] // 2
    g.probe(0, (xs, lo[1], lo[2]), (xs + 1, hi[1], hi[2]), thr, out)
    _, count_x = _cpu_components(rho[0], c, (xs, lo[1], lo[2]), (xs + 1, hi[1], hi[2]), thr)
    assert int(out.item()) == count_x


def test_droplet_sizes_agree_with_oracle():
    from paper_2512_12934_amd.lbm import LBM
    c = cases.drops()
    g = LBM(c)
    s = oracle.Sim(c)
    g.step(100)
    s.step(100)
    thr = labels.threshold(c)
    lo, hi = (0, 0, 0), (c.n[0], c.n[1], 1)
    comps, n = g.components(0, lo, hi, thr)
    ro, _, _ = s.moments()
    ref, _ = _cpu_components(ro[0], c, lo, hi, thr)
    assert n == len(ref)
    dg = sorted(labels.diameter(x["size"], 2) for x in comps)
    do = sorted(labels.diameter(x["size"], 2) for x in ref)
    print("  diameters gpu", np.round(dg, 3), "oracle", np.round(do, 3), flush=True)
    assert np.allclose(dg, do, rtol=0.01)


def _coflow_quarter_labels(storage, steps=45000, every=100):
    """Droplet period (probe across the channel core at mid-length) and the
    mean equivalent diameter of the droplets found between 10 and 50 nodes
    downstream of the inlet, sampled every 1000 steps."""
    import torch
    from paper_2512_12934_amd.lbm import LBM
    c = cases.coflow3d_quarter()
    thr = labels.threshold(c)
    n0, n1 = c.n[0], c.n[1]
    s = LBM(c, storage=storage)
    series = torch.zeros(steps // every, dtype=torch.int64, device="cuda:0")
    # the core of the channel cross-section, a quarter of the width from the
    # walls: the films of the dispersed phase along the corner edges of the
    # square channel stay outside
    m = n1 // 4
    plo, phi = (n0 // 2, m, m), (n0 // 2 + 1, n1 - m, n1 - m)
    diam = []
    for k in range(steps // every):
        s.step(every)
        s.probe(0, plo, phi, thr, series[k:k + 1])
        if (k + 1) % 10 == 0:
            comps, _ = s.components(0, (10, 1, 1), (50, n1 - 1, n1 - 1), thr)
            diam += [labels.diameter(cc["size"], 3) for cc in comps
                     if cc["lo"][0] > 10 and cc["hi"][0] < 50 and min(cc["lo"][1], cc["lo"][2]) >= m - 2
                     and max(cc["hi"][1], cc["hi"][2]) <= n1 - m + 2]
    T = labels.period(series.cpu().numpy(), every)
    return T, float(np.mean(diam)) if diam else None, len(diam)


def test_coflow_quarter_drips_like_the_oracle():
    """The 1/4-scale co-flow device (phases at the coexisting densities) drips
    at a regular period in 3-D.  Its labels are compared with those of the
    FP64 oracle on the same device (tests/golden/coflow_quarter_oracle_labels.json,
    written by make_coflow_quarter_labels.py with the same probe and windows):
    FP32 and binary16 (reference-density offset) storage both within 1% of
    the oracle on the period and on the mean droplet diameter.  The period is
    sampled every 100 steps against periods of about 4700, and droplets are
    measured wherever they are every 1000 steps between 10 and 50 nodes from
    the inlet (they shrink slowly as they travel)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "coflow_quarter_oracle_labels.json")))
    T32, D32, n32 = _coflow_quarter_labels("f32")
    T16, D16, n16 = _coflow_quarter_labels("f16")
    To, Do = gold["period_steps"], gold["diameter"]
    print(f"  oracle: period {To} steps, D {Do:.2f} ({gold['diameter_samples']} samples); "
          f"FP32: period {T32} steps, D {D32:.2f} ({n32} samples); "
          f"FP16: period {T16} steps, D {D16:.2f} ({n16} samples)", flush=True)
    assert T32 is not None and T16 is not None and D32 is not None and D16 is not None
    assert abs(T32 - To) < 0.01 * To
    assert abs(D32 - Do) < 0.01 * Do
    assert abs(T16 - To) < 0.01 * To
    assert abs(D16 - Do) < 0.01 * Do
