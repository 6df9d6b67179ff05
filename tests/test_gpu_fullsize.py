"""Parity at the benchmark's full sizes, in the launch configuration that
bench.py times (tile_config "auto" for the single context, the batch's own
tuned configuration for the sweep).

* The 600 x 120 x 120 co-flow device (8.64M fluid nodes, D3Q19): a few steps
  against the FP64 oracle on every fluid node, FP32 and binary16-offset
  storage.  Tolerances follow the per-step bound of test_gpu_parity (about
  1e-5 of the node density per step in FP32); binary16 adds the rounding of
  the stored offsets, 2^-11 of values that are a few percent of the density.
* The 256-instance sweep (W 32..128, binary16): members of the batch against
  the same instances stepped alone, bitwise.
"""
import numpy as np
import pytest

import oracle
from paper_2512_12934_amd import cases

pytestmark = pytest.mark.gpu


_ORACLE = {}


def _oracle_coflow(c, steps):
    """The oracle's fields after `steps` steps of the full device (computed
    once for both storage modes)."""
    if steps not in _ORACLE:
        print(f"[gpu] oracle, {steps} steps of {c.n}", flush=True)
        s = oracle.Sim(c)
        s.step(steps)
        ro, uo, _ = s.moments()
        _ORACLE[steps] = (ro, uo, s.diag())
        s.close()
    return _ORACLE[steps]


@pytest.mark.parametrize("storage,tol", [("f32", 3e-5), ("f16", 1e-3)])
def test_coflow_full_size(storage, tol):
    from paper_2512_12934_amd.lbm import LBM
    c = cases.coflow3d()
    steps = 3
    print(f"[gpu] coflow3d full size {c.n} storage={storage}", flush=True)
    g = LBM(c, storage=storage, tile_config="auto")
    g.step(steps)
    rg, ug = g.moments()
    fg = g.mass_flux()
    del g
    ro, uo, do = _oracle_coflow(c, steps)
    fluid = c.solid == 0
    rt = ro[:, fluid].sum(axis=0)
    er = (np.abs(rg[:, fluid] - ro[:, fluid]) / rt).max()
    eu = np.abs(ug[:, fluid] - uo[:, fluid]).max() / np.abs(uo[:, fluid]).max()
    print(f"  rho err / node density {er:.3e}, u err / max|u| {eu:.3e}", flush=True)
    assert np.isfinite(rg[:, fluid]).all() and np.isfinite(ug[:, fluid]).all()
    assert er < tol and eu < 10 * tol
    for k in range(2):
        assert abs(fg["mass"][k] - do["mass"][k]) < tol * do["mass"][k]
    # the eq. 23 sums and the outlet correction of the last step
    for key in ("q_in", "q_out", "chi"):
        print(f"  {key}: gpu {fg[key]:.9g} oracle {do[key]:.9g}", flush=True)
        assert abs(fg[key] - do[key]) <= 10 * tol * abs(do[key])


def test_batch_full_sweep_members_bitwise():
    from paper_2512_12934_amd.lbm import LBM, Batch
    cs = cases.sweep(256)
    print(f"[gpu] sweep batch of {len(cs)} members, binary16", flush=True)
    b = Batch(cs, storage="f16")
    b.step(24)
    picks = [0, 1, 97, 128, 255]
    for i in picks:
        s = LBM(cs[i], storage="f16", tile_config=b.tile_config)
        s.set_graph_steps(0)
        s.step(24)
        assert np.array_equal(b.members[i].get_state(), s.get_state()), i
        fm, fs = b.members[i].mass_flux(), s.mass_flux()
        for key in ("q_in", "q_out", "chi", "u_conv"):
            assert fm[key] == fs[key], (i, key)


@pytest.mark.parametrize("storage,tol", [("f32", 3e-5), ("f16", 1e-3)])
def test_tjunction_4096x1026_full_size(storage, tol):
    """The largest T-junction of the sweep distribution (W 512, 4096 x 1026
    box, 2.36M fluid nodes, D2Q9) in the configuration the autotuner picks
    for it (the fused node update): three steps against the FP64 oracle on
    every fluid node, and the eq. 23 sums of the last step."""
    from paper_2512_12934_amd.lbm import LBM
    c = cases.sweep_case(512, 0.01, 0.5, 1.0)
    steps = 3
    print(f"[gpu] T-junction full size {c.n} storage={storage}", flush=True)
    g = LBM(c, storage=storage, tile_config="auto")
    g.step(steps)
    rg, ug = g.moments()
    fg = g.mass_flux()
    del g
    s = oracle.Sim(c)
    s.step(steps)
    ro, uo, _ = s.moments()
    do = s.diag()
    s.close()
    fluid = c.solid == 0
    rt = ro[:, fluid].sum(axis=0)
    er = (np.abs(rg[:, fluid] - ro[:, fluid]) / rt).max()
    eu = np.abs(ug[:, fluid] - uo[:, fluid]).max() / np.abs(uo[:, fluid]).max()
    print(f"  rho err / node density {er:.3e}, u err / max|u| {eu:.3e}", flush=True)
    assert np.isfinite(rg[:, fluid]).all() and np.isfinite(ug[:, fluid]).all()
    assert er < tol and eu < 10 * tol
    for key in ("q_in", "q_out", "chi"):
        assert abs(fg[key] - do[key]) <= 10 * tol * abs(do[key]), key
