"""Whole-step cross-check of the FP64 oracle against an independent dense
NumPy restatement of the method (``tests/brute_lbm.py``: whole-array
operations, pull streaming, ghost layers by padding) on tiny grids.  Both
follow the same readings of the paper, so this pins the oracle's
implementation (indices, loop bounds, face rules, stage order), not its
readings; those are pinned by the physics and table tests."""
import numpy as np
import pytest

import oracle
from paper_2512_12934_amd import cases

from brute_lbm import Brute


def _tiny_cases():
    out = {}
    out["periodic2d"] = cases.random_box((9, 7), seed=1, dim=2, u_amp=0.01, Fb=(1e-4, -2e-4, 0.0))
    out["walled2d_adhesion"] = cases.random_box((11, 9), seed=2, dim=2, periodic=(False, False, True), walls=True,
                                                Gw=(0.05, -0.05), u_amp=0.01)
    out["periodic3d"] = cases.random_box((6, 5, 5), seed=3, dim=3, u_amp=0.01, Fb=(1e-4, 0.0, 2e-4))
    out["walled3d"] = cases.random_box((7, 6, 6), seed=4, dim=3, periodic=(True, False, False), walls=True,
                                       Gw=(0.03, -0.03), u_amp=0.005)
    out["tjunction_alpha"] = cases.tjunction(W=8, length=24, x_side=8, side_width=6, side_len=5)
    out["tjunction_no_alpha"] = cases.tjunction(W=8, length=24, x_side=8, side_width=6, side_len=5,
                                                alpha_on=False, chi_on=False)
    out["channel_droplet"] = cases.channel(20, 9, 0.02, droplet=(14, 5, 3), major=0.93, minor=0.1,
                                           nu=(0.1, 0.05))
    out["coflow3d"] = cases.coflow3d(length=12, width=6, inner=2)
    seps = cases.laplace(n=12, R=4, nu=(0.5, 0.05), major=0.93, minor=0.1)
    out["laplace_maxvisc"] = seps
    out["laplace_fixed"] = seps.copy(s_eps_policy=1)
    out["taylor2d"] = cases.taylor(30, 0.1, nx=14, H=10, R=3.5, nu_c=0.1)
    out["taylor3d"] = cases.taylor(5, 0.1, nx=8, H=6, R=2.5, nu_c=0.1, dim=3)
    return out


CASES = _tiny_cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_matches_brute_force(name):
    c = CASES[name]
    o, b = oracle.Sim(c), Brute(c)
    fluid = np.asarray(c.solid).reshape(-1) == 0
    for _ in range(4):
        o.step(1)
        b.step()
        fo = o.get_f()[:, :, fluid]
        fb = b.f_nodes()[:, :, fluid]
        assert np.isfinite(fb).all()
        err = np.abs(fo - fb).max() / np.abs(fb).max()
        assert err < 1e-13, (name, err)
