"""Host checks of the cylindrical co-flow generator (eq. 28): the fluid set
is the cylinder minus the capillary wall, the inlet patches put each phase
on its own part of the inlet face, and the C ABI accepts the configuration
(lbm_workspace_bytes validates it without a GPU)."""
import numpy as np
import pytest

from paper_2512_12934_amd import cases


@pytest.mark.parametrize("focus", [None, (24, 6, 5)])
def test_cylinder_fluid_set_is_eq28(focus):
    c = cases.coflow_cylinder(length=40, R=8, r_in=3, t_wall=2, L_cap=12, focus=focus)
    x, y, z = c.grid()
    c0 = 9
    r2 = (y - c0) ** 2 + (z - c0) ** 2
    R = np.full(c.n[0], 8.0)
    if focus:
        R[focus[0]:focus[0] + focus[1]] = focus[2]
    in_tube = r2 <= R[x] ** 2
    wall = (x < 12) & (r2 > 9) & (r2 <= 25)
    assert np.array_equal(c.solid == 0, in_tube & ~wall)
    # a cross-section of the tube is a lattice disc: its area is near pi R^2
    sec = (x == 30) & (c.solid == 0)
    assert abs(sec.sum() - np.pi * R[30] ** 2) < 2 * np.pi * R[30]
    # the dispersed phase starts inside the capillary only
    core = (x < 12) & (r2 <= 9)
    assert np.array_equal(c.rho0[0] > 0.5, core)


def test_cylinder_inlet_patches_split_the_face():
    c = cases.coflow_cylinder(length=40, R=8, r_in=3, t_wall=2, L_cap=12)
    x, y, z = c.grid()
    face = (x == 0) & (c.solid == 0)
    inner = c.inlets[1]
    in_sq = (y >= inner["lo"][1]) & (y < inner["hi"][1]) & (z >= inner["lo"][2]) & (z < inner["hi"][2])
    r2 = (y - 9) ** 2 + (z - 9) ** 2
    # fluid nodes of the square patch are exactly the capillary interior
    assert np.array_equal(face & in_sq, face & (r2 <= 9))
    assert c.meta["A_core"] == int((face & (r2 <= 9)).sum())
    with pytest.raises(ValueError):
        cases.coflow_cylinder(length=40, R=8, r_in=5, t_wall=1, L_cap=12)


def test_cylinder_config_accepted_by_the_library():
    from paper_2512_12934_amd.lbm import workspace_bytes
    for focus in (None, (24, 6, 5)):
        c = cases.coflow_cylinder(length=40, R=8, r_in=3, t_wall=2, L_cap=12, focus=focus)
        assert workspace_bytes(c) > 0
        assert workspace_bytes(c, storage="f16") > 0
