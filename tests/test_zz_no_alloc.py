"""The allocation-free labelling entry point (lbm_components_static) against
lbm_components on the same contexts: identical component lists (integer
results, bit-exact), on two calls in a row, the second on a smaller
domain, plus the size limit's error."""
import numpy as np
import pytest

from paper_2512_12934_amd import cases, labels

pytestmark = pytest.mark.gpu


def _box(c):
    if c.dim == 3:
        return (1, 1, 1), (c.n[0] - 1, c.n[1] - 1, c.n[2] - 1)
    return (1, 1, 0), (c.n[0] - 1, c.n[1] - 1, 1)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_static_components_equal_allocating_entry_point(storage):
    from paper_2512_12934_amd.lbm import LBM
    big = cases.drops(shape=(40, 32, 36), count=6, r_range=(3.0, 7.0))
    small = cases.drops(shape=(96, 48, 1), count=9, seed=8, r_range=(2.0, 6.0))
    for c in (big, small):
        print(f"[gpu] no-alloc labels {c.name} {c.n} storage={storage}", flush=True)
        g = LBM(c, storage=storage)
        g.step(30)
        lo, hi = _box(c)
        thr = labels.threshold(c)
        want, n_want = g.components(0, lo, hi, thr)
        got, n_got = g.components(0, lo, hi, thr, static=True)
        assert n_want > 1 and n_got == n_want
        assert got == want
        # a short output buffer receives the first components in the same order
        part, n_part = g.components(0, lo, hi, thr, max_out=2, static=True)
        assert n_part == n_want and part == want[:2]
        g.close()


def test_static_components_reject_oversized_domain():
    from paper_2512_12934_amd.lbm import LBM, LBMError, LBM_EINVAL, lib
    n = (2048, 2050, 1)           # 4,198,400 nodes, above the 2^22-node scratch
    N = n[0] * n[1]
    c = cases.Case("big", 2, n, (True, True, True), (0.1, 0.1), 0.9, solid=np.zeros(N, np.uint8),
                   rho0=np.stack([np.full(N, 0.5), np.full(N, 0.5)]))
    g = LBM(c, storage="f16")
    with pytest.raises(LBMError) as ei:
        g.components(0, (0, 0, 0), (n[0], n[1], 1), 0.6, static=True)
    assert ei.value.status == LBM_EINVAL
    assert "static labelling scratch" in str(ei.value)
    g.close()
