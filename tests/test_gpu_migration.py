"""Droplet migration through the outlet (Sec. III C, Figs. 6 and 8), the
original convective outflow against the corrected one: the droplet moves
the same way (positions within 5% while it is in the domain) and the
corrected outlet keeps the total mass, where the original lets it drift.
2-D at the paper's size (500 x 100, R = 30); 3-D at half the paper's size
(250 x 50 x 50, R = 15; the full 500 x 100 x 100 run is the study module's
default)."""
import numpy as np
import pytest

from paper_2512_12934_amd import migration

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,kw,steps", [(2, {}, 40000),
                                          (3, dict(length=250, width=50, R=15.0, x0=50.0), 20000)])
def test_corrected_outlet_keeps_mass_and_motion(dim, kw, steps):
    print(f"[gpu] migration {dim}-D {kw} steps={steps}", flush=True)
    rec, rate = migration.run(dim, steps, 1000, log=None, **kw)
    res = migration.compare(rec)
    o, c = rec["original"], rec["corrected"]
    print(f"  x_d original  {np.round(o['x_d'][::4], 1)}\n  x_d corrected {np.round(c['x_d'][::4], 1)}", flush=True)
    print(f"  {res}  MLUPS {rate}", flush=True)
    # the droplet travelled and left the domain in both runs
    assert np.isfinite(o["x_d"][0]) and np.isfinite(c["x_d"][0])
    assert not np.isfinite(o["x_d"][-1]) and not np.isfinite(c["x_d"][-1])
    assert res["max_position_deviation"] < 0.05
    mo, mc = res["mass_dev_mean_abs"]["original"], res["mass_dev_mean_abs"]["corrected"]
    assert mc < 0.05 and mc < 0.2 * mo
    assert res["mass_dev_max_abs"]["corrected"] < res["mass_dev_max_abs"]["original"]
