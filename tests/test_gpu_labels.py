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
