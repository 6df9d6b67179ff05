"""Batched step: many uneven instances advanced together must give, member by
member, exactly the bits of the same instances stepped one at a time, and
the members agree with the FP64 oracle like single contexts do."""
import numpy as np
import pytest

import oracle
from paper_2512_12934_amd import cases

pytestmark = pytest.mark.gpu


def _tj_batch():
    # uneven sizes and physics, as in the sweep, but small
    return [cases.sweep_case(W, Ca, q, M) for (W, Ca, q, M) in
            [(16, 0.01, 0.5, 1.0), (20, 0.003, 1.5, 4.0), (24, 0.05, 0.2, 0.6), (13, 0.02, 1.0, 8.0),
             (18, 0.001, 0.8, 2.0)]]


def _coflow_batch():
    return [cases.coflow3d(length=L, width=w, inner=i) for (L, w, i) in [(30, 8, 2), (40, 10, 4), (24, 6, 2)]]


def _fused_config(dim):
    """The first configuration whose node update recomputes psi itself."""
    from paper_2512_12934_amd.lbm import tile_config_desc, tile_configs
    return next(i for i in range(tile_configs(dim)) if tile_config_desc(dim, i)["psrc"] == 0)


@pytest.mark.parametrize("make", [_tj_batch, _coflow_batch], ids=["tjunction", "coflow"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("tile", ["default", "fused"])
def test_batch_equals_single_contexts_bitwise(make, storage, tile):
    from paper_2512_12934_amd.lbm import LBM, Batch
    cs = make()
    cfg = -1 if tile == "default" else _fused_config(cs[0].dim)
    print(f"[gpu] batch of {len(cs)} {cs[0].name} storage={storage} tile_config={cfg}", flush=True)
    b = Batch(cs, storage=storage, tile_config=cfg)
    b.set_graph_steps(8)
    singles = [LBM(c, storage=storage, tile_config=b.tile_config) for c in cs]
    b.step(21)                         # two replayed graphs and an eager tail
    for s in singles:
        s.set_graph_steps(0)
        s.step(21)
    for i, (m, s) in enumerate(zip(b.members, singles)):
        assert np.array_equal(m.get_state(), s.get_state()), i
        fm, fs = m.mass_flux(), s.mass_flux()
        for key in ("q_in", "q_out", "chi", "u_conv"):
            assert fm[key] == fs[key], (i, key)
        assert m.steps == 21


def test_batch_member_matches_oracle():
    from paper_2512_12934_amd.lbm import Batch
    cs = _tj_batch()
    b = Batch(cs)
    b.step(20)
    for i in (0, 3):
        s = oracle.Sim(cs[i])
        s.step(20)
        fg = b[i].get_state()
        fo = s.get_f()
        fluid = cs[i].solid == 0
        scale = fo[:, :, fluid].sum(axis=(0, 1))
        err = (np.abs(fg[:, :, fluid] - fo[:, :, fluid]) / scale).max()
        print(f"  member {i}: 20-step max err {err:.3e}", flush=True)
        assert err < 1e-4


def test_batch_refuses_after_a_member_stepped_alone():
    from paper_2512_12934_amd.lbm import Batch, LBMError, lib
    cs = _tj_batch()[:2]
    b = Batch(cs)
    b.step(2)
    assert lib().lbm_step(b[1]._h, 1) == 0   # the member steps on its own
    with pytest.raises(LBMError):
        b.step(1)
    assert lib().lbm_step(b[1]._h, 1) == 0   # parities agree again
    b.step(1)


def test_member_stepped_alone_after_batch_steps_bitwise():
    """A member stepped on its own after batch steps (whose density pass runs
    at the start of each batch step) computes the densities of its state first,
    and matches a context stepped alone all along."""
    from paper_2512_12934_amd.lbm import LBM, Batch
    cs = _tj_batch()[:2]
    print("[gpu] member stepped alone after batch steps", flush=True)
    b = Batch(cs)
    s = LBM(cs[1], tile_config=b.tile_config)
    b.step(5)
    b[1].step(4)
    s.step(9)
    assert np.array_equal(b[1].get_state(), s.get_state())
