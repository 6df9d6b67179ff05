"""FP32 and FP16-offset storage against the FP64 oracle on the Laplace case
(64 x 64 periodic, droplet R = 16): fields at step 1000, the droplet's
equivalent diameter, and the surface tension from the Laplace fit over
R = 10 .. 20.

FP32 storage holds the fields to 1e-4 relative (L2 norm) at step 1000; its
velocity error is an absolute floor of about 1e-7 that does not grow.
binary16 storage of f - w_i r (r: the reading node's density of the previous
step) holds the diameter and the surface tension to 1%.  The fixed offset
f - w_i (storage "f16fixed") does not: each component is also present at the
minority density, where f - w_i is close to -w_i and the 11-bit significand
leaves a relative error near 1e-3 on every such population; bulk nodes round
alike, so the error is systematic and the minority density drifts."""
import numpy as np
import pytest

import oracle
from paper_2512_12934_amd import cases

pytestmark = pytest.mark.gpu


def _dp_reff(rho, c):
    p = (rho[0] + rho[1]) / 3 + c.G12 * rho[0] * rho[1]
    thr = 0.5 * (rho[0].max() + rho[0].min())
    Reff = np.sqrt((rho[0] > thr).sum() / np.pi)
    n = c.n[0]
    return p[n // 2 + n * (n // 2)] - p[0], Reff


def _gamma(pts):
    pts = np.array(pts)
    x, y = 1 / pts[:, 1], pts[:, 0]
    A = np.vstack([x, np.ones_like(x)]).T
    (g, _), *_ = np.linalg.lstsq(A, y, rcond=None)
    return g


_cache = {}


def _errors():
    """Field, diameter and surface-tension errors of both storages (once)."""
    if _cache:
        return _cache
    from paper_2512_12934_amd.lbm import LBM
    c = cases.laplace()
    s = oracle.Sim(c)
    s.step(1000)
    ro, uo, _ = s.moments()
    for storage in ("f32", "f16", "f16fixed"):
        g = LBM(c, storage=storage)
        g.step(1000)
        rg, ug = g.moments()
        er = np.abs(rg - ro).max() / np.abs(ro).max()
        eu = np.abs(ug - uo).max() / np.abs(uo).max()
        er2 = np.linalg.norm(rg - ro) / np.linalg.norm(ro)
        eu2 = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
        _, Rg = _dp_reff(rg, c)
        _, Ro = _dp_reff(ro, c)
        _cache[storage] = {"rho": er, "u": eu, "rho_l2": er2, "u_l2": eu2, "D": abs(Rg - Ro) / Ro}
    pts = {"oracle": [], "f32": [], "f16": [], "f16fixed": []}
    for R in (10, 12, 14, 16, 18, 20):
        c = cases.laplace(R=R, major=0.93, minor=0.1)
        s = oracle.Sim(c)
        s.step(2000)
        pts["oracle"].append(_dp_reff(s.moments()[0], c))
        for storage in ("f32", "f16", "f16fixed"):
            g = LBM(c, storage=storage)
            g.step(2000)
            pts[storage].append(_dp_reff(g.moments()[0], c))
    gam = {k: _gamma(v) for k, v in pts.items()}
    for storage in ("f32", "f16", "f16fixed"):
        _cache[storage]["gamma"] = abs(gam[storage] - gam["oracle"]) / gam["oracle"]
    for storage in ("f32", "f16", "f16fixed"):
        e = _cache[storage]
        print(f"  {storage}: max-norm rho {e['rho']:.2e} u {e['u']:.2e}; L2 rho {e['rho_l2']:.2e} u {e['u_l2']:.2e}; "
              f"diameter {e['D']:.2e}  gamma {e['gamma']:.2e}", flush=True)
    return _cache


def test_fp32_fields_diameter_and_surface_tension():
    """Relative errors in the L2 norm over the box below 1e-4; the largest
    single-node velocity error, relative to the largest velocity (a spurious
    current of ~1e-3, so FP32 rounding of ~1e-7 sits near 1e-4), below 2e-4."""
    e = _errors()["f32"]
    assert e["rho_l2"] < 1e-4 and e["u_l2"] < 1e-4
    assert e["rho"] < 1e-4 and e["u"] < 2e-4
    assert e["D"] < 1e-3 and e["gamma"] < 1e-3


def test_fp32_velocity_error_is_a_floor_not_a_drift():
    """On the static droplet the FP32 velocity error against the oracle is an
    absolute floor of about 1e-7, one step's rounding: it is already 8e-8
    after the first step and does not grow through step 3000, while the
    spurious velocity field itself decays a thousandfold (0.23 at step 1,
    1.1e-3 at step 1000, 2e-4 at step 3000).  The relative max-norm error at
    step 1000 (1.4e-4 of the largest velocity) therefore measures how small
    that field has become, not an accumulation of rounding."""
    from paper_2512_12934_amd.lbm import LBM
    c = cases.laplace()
    print(f"[gpu] {c.name} n={c.n} storage=f32", flush=True)
    g = LBM(c, storage="f32")
    s = oracle.Sim(c)
    done, errs = 0, []
    for t in (1, 100, 1000, 3000):
        g.step(t - done)
        s.step(t - done)
        done = t
        _, ug = g.moments()
        _, uo, _ = s.moments()
        errs.append(np.abs(ug - uo).max())
        print(f"  step {t}: max |u_gpu - u_oracle| {errs[-1]:.3e}, max |u_oracle| {np.abs(uo).max():.3e}", flush=True)
    assert max(errs) < 2.5e-7
    assert max(errs) < 3.0 * errs[0]


def test_fp16_tjunction_fields_step_1000():
    """The 800 x 100 T-junction (open faces, walls with adhesion) at step
    1000 in binary16 storage against the FP64 oracle.  With the reference
    density the measured errors are 1.6e-3 (rho, max-norm), 1.9e-3 (u,
    max-norm relative to the largest velocity), 2e-6 on chi and 6e-5 on the
    component masses; the bars are about three times those.  The fixed
    offset f - w_i misses them by far (rho 4e-2, u 0.42, chi 1.5e-2): its
    rounding is systematic at the minority density."""
    from paper_2512_12934_amd.lbm import LBM
    c = cases.tjunction()
    s = oracle.Sim(c)
    s.step(1000)
    ro, uo, _ = s.moments()
    do = s.diag()
    fl = c.solid == 0
    err = {}
    for storage in ("f16", "f16fixed"):
        print(f"[gpu] {c.name} n={c.n} storage={storage}", flush=True)
        g = LBM(c, storage=storage)
        g.step(1000)
        rg, ug = g.moments()
        dg = g.mass_flux()
        err[storage] = (np.abs(rg[:, fl] - ro[:, fl]).max() / np.abs(ro[:, fl]).max(),
                        np.abs(ug[:, fl] - uo[:, fl]).max() / np.abs(uo[:, fl]).max(),
                        abs(dg["chi"] - do["chi"]),
                        max(abs(dg["mass"][k] - do["mass"][k]) / do["mass"][k] for k in range(2)))
        print(f"  {storage}: rho {err[storage][0]:.2e}  u {err[storage][1]:.2e}  chi {err[storage][2]:.2e}  "
              f"mass {err[storage][3]:.2e}", flush=True)
    e = err["f16"]
    assert e[0] < 5e-3 and e[1] < 6e-3 and e[2] < 1e-5 and e[3] < 2e-4
    f = err["f16fixed"]
    assert f[0] > 5e-3 and f[1] > 6e-3


def test_fp16_offset_meets_one_percent():
    e = _errors()["f16"]
    assert e["D"] < 0.01 and e["gamma"] < 0.01
    # the fields themselves stay close as well
    assert e["rho_l2"] < 1e-3 and e["u_l2"] < 1e-2


def test_fp16_fixed_offset_reported():
    """The fixed offset f - w_i in binary16, as the precision extension states
    it, measured on the same quantities: its errors are reported here and it
    is far less accurate than the reference-density offset (at least ten
    times the field error), which is why that offset is the binary16 mode the
    benchmark and the batches use."""
    e = _errors()
    fx, rf = e["f16fixed"], e["f16"]
    assert np.isfinite([fx["rho_l2"], fx["u_l2"], fx["D"], fx["gamma"]]).all()
    assert fx["rho_l2"] > 10 * rf["rho_l2"]


def test_fp16_fixed_offset_drifts_in_the_coflow_device():
    """On the 1/4-scale co-flow device at step 1000 the fixed offset moves the
    densities by far more than 1% of the oracle's, while the reference-density
    offset stays within 1e-3 (measured 3e-4)."""
    from paper_2512_12934_amd.lbm import LBM
    c = cases.coflow3d_quarter()
    s = oracle.Sim(c)
    s.step(1000)
    ro, _, _ = s.moments()
    fluid = c.solid == 0
    err = {}
    for storage in ("f16", "f16fixed"):
        print(f"[gpu] coflow quarter 1000 steps storage={storage}", flush=True)
        g = LBM(c, storage=storage)
        g.step(1000)
        rg, _ = g.moments()
        err[storage] = float(np.abs(rg[:, fluid] - ro[:, fluid]).max() / np.abs(ro[:, fluid]).max())
    print(f"  rho max-norm relative error at step 1000: f16 {err['f16']:.2e}, f16fixed {err['f16fixed']:.2e}",
          flush=True)
    assert err["f16"] < 1e-3
    assert err["f16fixed"] > 1e-2
