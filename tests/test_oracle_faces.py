"""Pins of the oracle's face rules on planted states, one stage at a time:
the mirror ghost layers (eqs. 24-25), the non-equilibrium extrapolation of
the inlet (eq. 13) with its half-force velocity (reading A13), and the
convective outflow (eqs. 20-21).  Each expected value follows from a
property of the rule (a closed form for a linear field, exact transmission of
a linear travelling profile), not from re-typing the oracle's expression, so
a plausible slip (a copied instead of mirrored ghost, a swapped weight,
extrapolation from the wrong node) fails here."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2512_12934_amd import cases

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_constants.json")))


def _w8_2d(r2):
    return float(Fraction(GOLD["e8_weights_2d"]["w_by_r2"].get(str(r2), "0")))


def _box(n, periodic, rho, u=None, **kw):
    N = int(np.prod(n))
    c = cases.Case("planted", 2 if n[2] == 1 else 3, tuple(n), tuple(periodic), (0.1, 0.1), 0.9,
                   solid=np.zeros(N, np.uint8), rho0=np.asarray(rho, float).reshape(2, N), **kw)
    if u is not None:
        c.u0 = np.asarray(u, float).reshape(3, N)
    return c


# ------------------------------------------------------------ ghost layers

def test_mirror_ghosts_on_a_linear_profile():
    """eqs. 24-25: beyond an open face the two ghost layers repeat x1 and x2
    (g1 <- x1, g2 <- x2).  For psi_2 = a + b x and uniform psi_1, the x-force
    on component 1 is -G12 psi_1 sum_e w e_x psi_2(x + e).  Grouping the
    stencil by e_x (W1 over e_x = 1, W2 over e_x = 2, printed weights):
    interior nodes see b (2 W1 + 8 W2) = b; the face node sees
    psi_2(1) - psi_2(g1) = b and psi_2(2) - psi_2(g2) = b, so b (W1 + 2 W2); the
    second node sees b (2 W1 + 6 W2).  A copied ghost (g2 <- x1) would give
    b (W1 + 4 W2) at the face, a wrap a jump of order b n."""
    nx, ny = 12, 4
    a, b, c1 = 0.3, 0.01, 0.5
    x = np.tile(np.arange(nx), ny)
    rho = np.stack([np.full(nx * ny, c1), a + b * x])
    case = _box((nx, ny, 1), (False, True, True), rho)
    s = oracle.Sim(case)
    _, _, F = s.moments()
    W1 = _w8_2d(1) + 2 * _w8_2d(2) + 2 * _w8_2d(5)
    W2 = _w8_2d(4) + 2 * _w8_2d(5) + 2 * _w8_2d(8)
    assert abs(2 * W1 + 8 * W2 - 1.0) < 1e-15          # unit second moment of the weights
    Fx = F[0, 0].reshape(ny, nx)
    scale = -case.G12 * c1 * b
    want = {0: W1 + 2 * W2, 1: 2 * W1 + 6 * W2, 5: 1.0, nx - 2: 2 * W1 + 6 * W2, nx - 1: W1 + 2 * W2}
    for xx, factor in want.items():
        assert np.abs(Fx[:, xx] - scale * factor).max() < 1e-16, xx
    assert np.abs(F[0, 1]).max() < 1e-15                 # no y-force on a profile uniform in y
    assert np.abs(F[1]).max() < 1e-15                    # psi_1 uniform, ghosts included


def test_mirror_ghosts_carry_the_wall_flag():
    """The ghosts mirror the solid flag too: a channel whose walls run along x
    through an open face keeps its wall force translation invariant up to the
    face node, and no x-force appears there."""
    nx, ny = 10, 8
    N = nx * ny
    y = np.repeat(np.arange(ny), nx)
    solid = ((y == 0) | (y == ny - 1)).astype(np.uint8)
    rho = np.stack([np.full(N, 0.6), np.full(N, 0.4)])
    case = _box((nx, ny, 1), (False, False, True), rho, Gw=(0.05, -0.05))
    case.solid = solid
    s = oracle.Sim(case)
    _, _, F = s.moments()
    Fg = F.reshape(2, 3, ny, nx)
    assert np.abs(Fg[:, 1, 1:-1, :] - Fg[:, 1, 1:-1, nx // 2:nx // 2 + 1]).max() < 1e-16
    assert np.abs(Fg[:, 0]).max() < 1e-15
    assert np.abs(Fg[:, 1, 1, 0]).max() > 1e-3           # the wall force itself is not zero


# ------------------------------------------------------------ eq. 13 inlet

def _inlet_case(dim, alpha_on, x2_solid=False):
    n = (6, 3, 1) if dim == 2 else (6, 3, 3)
    N = int(np.prod(n))
    rho = np.stack([np.full(N, 0.7), np.full(N, 0.3)])
    c = _box(n, (False, True, True), rho)
    if x2_solid:
        sol = np.zeros(N, np.uint8)
        sol[np.arange(N) % n[0] == 1] = 1
        c.solid = sol
    rp, up = (0.55, 0.42), 0.013
    c.inlets = [cases.inlet(0, 0, (0, 0, 0), (1, n[1], n[2]), rp, up, alpha_on)]
    return c, rp, up


def _neq(e, rng):
    """A random non-equilibrium vector with no mass and no momentum."""
    v = rng.standard_normal(len(e)) * 1e-3
    A = np.vstack([np.ones(len(e)), e.T.astype(float)])
    return v - A.T @ np.linalg.lstsq(A.T, v, rcond=None)[0]


@pytest.mark.parametrize("dim", [2, 3])
def test_inlet_extrapolates_non_equilibrium_from_x2(dim):
    """eq. (13)/(14), alpha off: f_i(x1) = feq_i(rho^p, u^p) + f_i(x2) -
    feq_i(rho(x2), u(x2)) for the entering populations, with rho and u at x2
    from the streamed f and, for u, half of this step's force (reading A13).
    The node x2 carries a known non-equilibrium part; x1 carries a different
    one, so extrapolating from x1, dropping the half force or the NEQ part
    fails."""
    rng = np.random.default_rng(5)
    c, rp, up = _inlet_case(dim, alpha_on=False)
    s = oracle.Sim(c)
    e, _, _, _ = oracle.tables(dim)
    Q, N, nx = len(e), c.N, c.n[0]
    x = np.arange(N) % nx
    v = np.array([0.004, -0.002, 0.001 if dim == 3 else 0.0])
    F = np.zeros((2, 3, N))
    F[0, :, x == 1] = [2e-4, -1e-4, 5e-5 if dim == 3 else 0.0]
    F[1, :, x == 1] = [-5e-5, 3e-5, 0.0]
    r2 = (0.62, 0.35)
    fn = np.zeros((2, Q, N))
    neq = {}
    for n in range(N):
        for k in range(2):
            if x[n] == 1:
                neq[(k, n)] = _neq(e, rng)
                fn[k, :, n] = oracle.feq(dim, r2[k], v) + neq[(k, n)]
            else:
                fn[k, :, n] = oracle.feq(dim, 0.5, -v) + _neq(e, rng)
    s.set_next(fn)
    s.set_force(F)
    s.stage(7)
    out = s.get_next()
    u2 = v + 0.5 * F[:, :, x == 1].sum(0)[:, 0] / sum(r2)
    entering = e[:, 0] > 0
    worst = 0.0
    for n in np.nonzero(x == 0)[0]:
        for k in range(2):
            want = oracle.feq(dim, rp[k], [up, 0, 0]) + neq[(k, n + 1)] + oracle.feq(dim, r2[k], v) \
                - oracle.feq(dim, r2[k], u2)
            worst = max(worst, np.abs(out[k, entering, n] - want[entering]).max())
            assert np.array_equal(out[k, ~entering, n], fn[k, ~entering, n])
    assert worst < 1e-16


def test_inlet_with_solid_x2_imposes_equilibrium():
    """With no fluid node to extrapolate from, the non-equilibrium part is
    zero: the entering populations are feq(rho^p, u^p)."""
    c, rp, up = _inlet_case(2, alpha_on=False, x2_solid=True)
    s = oracle.Sim(c)
    e, _, _, _ = oracle.tables(2)
    fn = np.full((2, 9, c.N), 0.05)
    s.set_next(fn)
    s.set_force(np.zeros((2, 3, c.N)))
    s.stage(7)
    out = s.get_next()
    x = np.arange(c.N) % c.n[0]
    for n in np.nonzero(x == 0)[0]:
        for k in range(2):
            want = oracle.feq(2, rp[k], [up, 0, 0])
            assert np.abs(out[k, e[:, 0] > 0, n] - want[e[:, 0] > 0]).max() < 1e-17


# ------------------------------------------------------------ eq. 20 outlet

@pytest.mark.parametrize("dim", [2, 3])
def test_outflow_transmits_a_linear_travelling_profile(dim):
    """eqs. (20)-(21) discretise df/dt + U_c df/dn = 0 implicitly upwind, which
    transmits any profile g(s) = alpha + beta s travelling at U_c exactly.  The
    x' column is planted at equilibrium with normal velocity U (no force), so
    U_c = U; a population entering through the outlet with g(x_N at t) = prev
    and g(x' at t + 1) = f(x') must come out as g(x_N at t + 1) =
    f(x') + beta with beta = (prev - f(x')) / (1 + U).  Swapped weights give
    g at a node one spacing upstream instead."""
    rng = np.random.default_rng(9)
    n = (5, 3, 1) if dim == 2 else (5, 3, 3)
    N = int(np.prod(n))
    c = _box(n, (False, True, True), np.stack([np.full(N, 0.6), np.full(N, 0.4)]))
    c.outlet = cases.outlet(0, 1, (0, 0, 0), (1, n[1], n[2]))
    s = oracle.Sim(c)
    e, _, _, _ = oracle.tables(dim)
    Q = len(e)
    x = np.arange(N) % n[0]
    U = 0.037
    prev = 0.02 + 0.1 * rng.random((2, Q, N))
    s.set_f(prev)
    fn = np.zeros((2, Q, N))
    rp = (0.52, 0.31)
    for k in range(2):
        fn[k][:, x == n[0] - 2] = oracle.feq(dim, rp[k], [U, 0, 0])[:, None]
        fn[k][:, x != n[0] - 2] = 0.01
    s.set_next(fn)
    s.set_force(np.zeros((2, 3, N)))
    s.stage(8)
    d = s.diag()
    assert abs(d["u_conv"] - U) < 1e-16
    out = s.get_next()
    entering = e[:, 0] < 0
    last = np.nonzero(x == n[0] - 1)[0]
    fprime = fn[:, :, last - 1]
    beta = (prev[:, :, last] - fprime) / (1 + U)
    want = fprime + beta
    assert np.abs(out[:, entering][:, :, last] - want[:, entering]).max() < 1e-16
    assert np.array_equal(out[:, ~entering][:, :, last], fn[:, ~entering][:, :, last])


def test_outflow_backflow_is_clamped():
    """A column flowing back into the domain (U_c < 0) would make eq. (20)
    singular at U_c = -1; the reading clamps U_c at 0 and counts the clamp, so
    the entering populations keep their previous values."""
    n, N = (5, 3, 1), 15
    c = _box(n, (False, True, True), np.stack([np.full(N, 0.6), np.full(N, 0.4)]))
    c.outlet = cases.outlet(0, 1, (0, 0, 0), (1, 3, 1))
    s = oracle.Sim(c)
    e, _, _, _ = oracle.tables(2)
    x = np.arange(N) % 5
    prev = np.random.default_rng(2).random((2, 9, N))
    s.set_f(prev)
    fn = np.zeros((2, 9, N))
    for k in range(2):
        fn[k][:, x == 3] = oracle.feq(2, 0.5, [-0.02, 0, 0])[:, None]
    s.set_next(fn)
    s.set_force(np.zeros((2, 3, N)))
    s.stage(8)
    d = s.diag()
    assert d["u_conv"] == 0.0 and d["uc_clamps"] == 1
    out = s.get_next()
    last = np.nonzero(x == 4)[0]
    ent = e[:, 0] < 0
    assert np.array_equal(out[:, ent][:, :, last], prev[:, ent][:, :, last])
