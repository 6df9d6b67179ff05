"""The streaming probes behind the practical-ceiling figures of the bench:
the D3Q19 pull probes move every population from the right neighbour slot
(so their rate is that of the node update's access pattern), and every
probe reports a positive rate."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

D3Q19 = {(0, 0, 0)} | {(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                       if 1 <= abs(a) + abs(b) + abs(c) <= 2}


@pytest.mark.parametrize("kind", [4, 5])
def test_pull_probe_moves_each_population_from_its_neighbour(kind):
    import torch
    from paper_2512_12934_amd.lbm import LBM_OK, probe_lib as lib
    PX = PY = 128
    nz = 20
    M = nz * PX * PY
    nbytes = 38 * 4 * M
    print(f"[gpu] pull probe kind {kind}, box 128x128x{nz}", flush=True)
    src = torch.arange(38 * M, dtype=torch.int32, device="cuda:0")
    dst = torch.full_like(src, -1)
    r = C.c_double(0.0)
    s = torch.cuda.current_stream()
    st = lib().lbm_stream_probe(src.data_ptr(), dst.data_ptr(), nbytes, kind, 1, s.cuda_stream, C.byref(r))
    assert st == LBM_OK and r.value > 0.0
    d = dst.cpu().numpy().reshape(38, nz, PY, PX).astype(np.int64)
    # planes outside [2, nz - 2) are not written
    assert (d[:, :2] == -1).all() and (d[:, nz - 2:] == -1).all()
    j = np.arange(M, dtype=np.int64).reshape(nz, PY, PX)[2:nz - 2]
    shifts = []
    for c in range(38):
        k = d[c, 2:nz - 2] - c * M                # the source node of each slot
        sh = j - k
        assert (sh == sh.flat[0]).all(), c          # one shift per plane
        s0 = int(sh.flat[0])
        # decode the shift into a lattice offset e with sh = e_x + 128 e_y + 128^2 e_z
        ez = int(np.round(s0 / (PX * PY)))
        ey = int(np.round((s0 - ez * PX * PY) / PX))
        ex = s0 - ez * PX * PY - ey * PX
        shifts.append((ex, ey, ez))
    assert shifts[:19] == shifts[19:]               # both components alike
    assert set(shifts[:19]) == D3Q19 and len(set(shifts[:19])) == 19


def test_pull_pairs_probe_moves_each_pair_from_its_neighbour():
    import torch
    from paper_2512_12934_amd.lbm import LBM_OK, probe_lib as lib
    PX = PY = 128
    nz = 20
    M = nz * PX * PY
    nbytes = 19 * 8 * M
    print(f"[gpu] pull pairs probe, box 128x128x{nz}", flush=True)
    src = torch.arange(19 * M, dtype=torch.int64, device="cuda:0")
    dst = torch.full_like(src, -1)
    r = C.c_double(0.0)
    s = torch.cuda.current_stream()
    st = lib().lbm_stream_probe(src.data_ptr(), dst.data_ptr(), nbytes, 6, 1, s.cuda_stream, C.byref(r))
    assert st == LBM_OK and r.value > 0.0
    d = dst.cpu().numpy().reshape(19, nz, PY, PX)
    assert (d[:, :2] == -1).all() and (d[:, nz - 2:] == -1).all()
    j = np.arange(M, dtype=np.int64).reshape(nz, PY, PX)[2:nz - 2]
    shifts = []
    for c in range(19):
        sh = j - (d[c, 2:nz - 2] - c * M)
        assert (sh == sh.flat[0]).all(), c
        s0 = int(sh.flat[0])
        ez = int(np.round(s0 / (PX * PY)))
        ey = int(np.round((s0 - ez * PX * PY) / PX))
        shifts.append((s0 - ez * PX * PY - ey * PX, ey, ez))
    assert set(shifts) == D3Q19 and len(set(shifts)) == 19


def test_stream_probe_rates_positive():
    from paper_2512_12934_amd.lbm import stream_probe
    rates = stream_probe(nbytes=64 << 20, reps=2)
    print(f"[gpu] stream probe rates {rates}", flush=True)
    assert set(rates) == {"copy_b32", "copy_b128", "read_b128", "copy_b32x8", "pull_d3q19", "pull_d3q19_ahead",
                          "pull_d3q19_pairs"}
    assert all(v > 0 for v in rates.values())
