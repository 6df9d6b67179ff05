"""The C-ABI libraries load and export every entry point of their headers
(include/lbm.h: the solver, liblbm.so; include/lbm_probe.h: the measurement
library, libprobe.so); configuration validation (pure host code) answers
without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="lbm.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^\s*(?:lbm_status|size_t|void|int64_t|int|lbm_ctx|const char)\s*\*?\s*((?:lbm|surr)_\w+)\s*\(",
                                 src, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2512_12934_amd import build
    if build.stale():
        build.build()
    from paper_2512_12934_amd import lbm
    return lbm.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    # measurement code stays out of the solver library
    assert not hasattr(lib, "lbm_stream_probe")


def test_probe_library_exports_its_header(lib):
    from paper_2512_12934_amd import lbm
    names = _declared("lbm_probe.h")
    assert names == ["lbm_stream_probe"]
    pl = lbm.probe_lib()
    for n in names:
        assert hasattr(pl, n), n


def test_workspace_bytes_validates(lib):
    from paper_2512_12934_amd import cases, lbm
    c = cases.tjunction(W=20, length=90, x_side=30, side_width=14, side_len=18)
    ws = lbm.workspace_bytes(c)
    assert ws > 2 * 2 * 9 * c.N * 4
    assert lbm.workspace_bytes(c, "f16") < ws
    bad = c.copy(nu=(0.1, -1.0))
    assert lbm.workspace_bytes(bad) == 0
    # an open face not covered by a patch
    bad = c.copy(outlet=None)
    assert lbm.workspace_bytes(bad) == 0
    # a 2-node axis
    small = cases.random_box((8, 2), seed=0)
    assert lbm.workspace_bytes(small) == 0


def test_create_rejects_invalid_config_before_any_device_work(lib):
    from paper_2512_12934_amd import cases, lbm
    c = cases.laplace(n=16, R=4).copy(nu=(0.0, 0.1))
    cfg, keep = lbm.make_config(c)
    h = C.c_void_p()
    st = lib.lbm_create(C.byref(cfg), None, 0, None, C.byref(h))
    assert st == lbm.LBM_EINVAL
    assert b"viscosities" in lib.lbm_last_error(None)
    assert lib.lbm_step(None, 1) == lbm.LBM_EINVAL


def test_batch_workspace_validates(lib):
    from paper_2512_12934_amd import cases, lbm
    a = cases.tjunction(W=20, length=90, x_side=30, side_width=14, side_len=18)
    b = cases.tjunction(W=24, length=120, x_side=36, side_width=24, side_len=24)
    n = 2
    cfgs = (lbm.Config * n)()
    keep = []
    for i, c in enumerate((a, b)):
        cfg, k = lbm.make_config(c)
        cfgs[i] = cfg
        keep.append(k)
    total = lib.lbm_batch_workspace_bytes(cfgs, n)
    assert total >= lbm.workspace_bytes(a) + lbm.workspace_bytes(b)
    # members must share the lattice
    c3 = cases.coflow3d(length=12, width=5, inner=2)
    cfg3, k3 = lbm.make_config(c3)
    cfgs[1] = cfg3
    assert lib.lbm_batch_workspace_bytes(cfgs, n) == 0
    h = C.c_void_p()
    assert lib.lbm_batch_create(cfgs, n, None, 0, None, C.byref(h)) == lbm.LBM_EINVAL
    assert b"share" in lib.lbm_batch_last_error(None)
    assert lib.lbm_batch_step(None, 1) == lbm.LBM_EINVAL
    assert lib.lbm_batch_size(None) == 0
    assert lib.lbm_batch_member(None, 0) is None


def test_size_limit_depends_on_storage(lib):
    """A context holds each component's populations in one buffer addressed
    with 32-bit byte offsets: a D3Q19 box of 700 x 200 x 200 needs 2.28 GB per
    component in FP32 (refused, with the reason) and half that in binary16
    (accepted)."""
    import numpy as np
    from paper_2512_12934_amd import cases, lbm
    n = (700, 200, 200)
    N = n[0] * n[1] * n[2]
    c = cases.Case("big", 3, n, (True, True, True), (0.1, 0.1), 0.9, solid=np.zeros(N, np.uint8),
                   rho0=np.ones((2, N)))
    assert lbm.workspace_bytes(c, "f32") == 0
    assert lbm.workspace_bytes(c, "f16") > 2 * 2 * 19 * N * 2
    cfg, keep = lbm.make_config(c, "f32")
    h = C.c_void_p()
    assert lib.lbm_create(C.byref(cfg), None, 0, None, C.byref(h)) == lbm.LBM_EINVAL
    assert b"too large" in lib.lbm_last_error(None)


def test_all_solid_box_is_valid(lib):
    """A box with no fluid node is a valid (empty) problem: it has a
    workspace, and its work list is empty."""
    import numpy as np
    from paper_2512_12934_amd import cases, lbm
    c = cases.random_box((20, 12, 9), seed=1, dim=3)
    c = c.copy(solid=np.ones(c.N, np.uint8))
    assert lbm.workspace_bytes(c) > 0


def test_stream_probe_rejects_bad_arguments(lib):
    """Argument checks of the measurement hook answer before any device call
    (the pointers below are never dereferenced)."""
    from paper_2512_12934_amd.lbm import LBM_EINVAL, probe_lib
    pl = probe_lib()
    r = C.c_double(0.0)
    fake = C.c_void_p(4096)
    call = lambda nbytes, kind, reps=1: pl.lbm_stream_probe(fake, fake, C.c_size_t(nbytes), kind, reps, None,
                                                            C.byref(r))
    assert call(1 << 20, 7) == LBM_EINVAL            # unknown kind
    assert call(1 << 20, -1) == LBM_EINVAL
    assert call(1 << 20, 0, reps=0) == LBM_EINVAL
    assert call(1000, 0) == LBM_EINVAL               # not a multiple of 16
    # the pull pattern needs room for 20 planes of 128 x 128 nodes x 38 populations
    assert call(38 * 4 * 128 * 128 * 19, 4) == LBM_EINVAL
    assert call(1 << 31, 5) == LBM_EINVAL            # beyond 32-bit buffer offsets
    assert pl.lbm_stream_probe(None, fake, C.c_size_t(1 << 20), 0, 1, None, C.byref(r)) == LBM_EINVAL
