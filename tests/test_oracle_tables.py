"""Pins of the FP64 oracle's building blocks against what the paper prints and
what the mathematics fixes (closed forms, exact rationals, special cases)."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_constants.json")))


def frac(s):
    return Fraction(s)


# ---------------------------------------------------------------- lattices

def test_d2q9_velocity_order_matches_unknown_sets():
    """The direction numbering is fixed by the sets of unknown populations of
    Sec. II B (eqs. 13, 14, 20) and the periodic sets of eq. (B2)."""
    e, w, _, _ = oracle.tables(2)
    u = GOLD["unknown_sets"]
    assert sorted(np.nonzero(e[:, 0] > 0)[0].tolist()) == u["left_inflow"]
    assert sorted(np.nonzero(e[:, 1] < 0)[0].tolist()) == u["top_inflow"]
    assert sorted(np.nonzero(e[:, 0] < 0)[0].tolist()) == u["right_outlet"]
    assert sorted(np.nonzero(e[:, 1] > 0)[0].tolist()) == u["B2c_up"]
    assert (e[0] == 0).all()
    # speeds: 1-4 axis-aligned, 5-8 diagonal
    r2 = (e ** 2).sum(1)
    assert r2.tolist() == [0, 1, 1, 1, 1, 2, 2, 2, 2]


def test_d2q9_weights_printed():
    _, w, _, _ = oracle.tables(2)
    want = [float(frac(s)) for s in GOLD["d2q9_weights"]["w"]]
    assert np.array_equal(w, np.array(want))


def test_d3q19_lattice():
    e, w, _, _ = oracle.tables(3)
    assert len(set(map(tuple, e.tolist()))) == 19
    r2 = (e ** 2).sum(1)
    assert sorted(r2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert abs(w.sum() - 1.0) < 1e-15
    # second moment isotropic with cs^2 = 1/3, fourth moment isotropic
    M2 = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(M2, np.eye(3) / 3, atol=1e-15)
    assert abs(np.sum(w * e[:, 0] ** 2 * e[:, 1] ** 2) - 1 / 9) < 1e-15
    assert abs(np.sum(w * e[:, 0] ** 4) - 1 / 3) < 1e-15


# ---------------------------------------------------------------- T matrix

def test_T_rows_0_2_equal_printed_eq3():
    _, _, T, _ = oracle.tables(2)
    assert np.array_equal(T[:3], np.array(GOLD["T_rows_0_2"]["rows"], dtype=float))


@pytest.mark.parametrize("dim,diag", [
    (2, [9, 36, 36, 6, 12, 6, 12, 4, 4]),
    (3, [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]),
])
def test_T_orthogonal_and_inverse(dim, diag):
    e, _, T, Ti = oracle.tables(dim)
    TT = T @ T.T
    assert np.array_equal(TT, np.diag(np.array(diag, dtype=float)))
    assert np.allclose(T @ Ti, np.eye(len(diag)), atol=1e-14)
    # integer entries
    assert np.array_equal(T, np.round(T))
    # conserved rows: density and the momentum components
    assert np.array_equal(T[0], np.ones(len(diag)))
    mom = [3, 5] if dim == 2 else [3, 5, 7]
    for a, r in enumerate(mom):
        assert np.array_equal(T[r], e[:, a].astype(float))


def test_printed_eq3_rows_3_8_not_orthogonal():
    """Why the oracle does not use the printed rows 3-8 of eq. (3): the printed
    matrix is not orthogonal (recorded so a change of reading is deliberate)."""
    printed = np.array([
        [1, 1, 1, 1, 1, 1, 1, 1, 1], [-4, -1, -1, -1, -1, 2, 2, 2, 2],
        [4, -2, -2, -2, -2, 1, 1, 1, 1], [0, 1, 0, -1, 0, 1, -1, 1, 1],
        [0, -1, 0, 2, 0, 1, -1, 1, -1], [0, 0, 1, 0, -1, 1, -1, -1, -1],
        [0, 0, -2, 0, 2, 1, -1, -1, 0], [0, 1, -1, 1, -1, 0, 0, 0, 1],
        [0, 0, 0, 0, 0, 1, 1, 1, 1]], dtype=float)
    G = printed @ printed.T
    assert np.abs(G - np.diag(np.diag(G))).max() >= 1


# ---------------------------------------------------------------- equilibrium

@pytest.mark.parametrize("dim", [2, 3])
def test_feq_moments(dim):
    """Sum feq = rho, sum e feq = rho u, sum e e feq = rho cs^2 I + rho u u."""
    rng = np.random.default_rng(1)
    e, _, _, _ = oracle.tables(dim)
    for _ in range(20):
        rho = rng.uniform(0.02, 1.2)
        u = np.zeros(3)
        u[:dim] = rng.uniform(-0.1, 0.1, dim)
        f = oracle.feq(dim, rho, u)
        assert abs(f.sum() - rho) < 1e-15
        assert np.allclose(e.T @ f, rho * u, atol=1e-16)
        P = np.einsum("i,ia,ib->ab", f, e, e)[:dim, :dim]
        want = rho * np.eye(dim) / 3 + rho * np.outer(u[:dim], u[:dim])
        assert np.allclose(P, want, atol=1e-15)


def test_printed_eq6_denominator_breaks_mass():
    """Reading of eq. (6): with the printed (e.u)^2/(2 cs^2) the zeroth moment
    is rho (1 - |u|^2) / ... != rho, so the cs^4 form is the consistent one."""
    e, w, _, _ = oracle.tables(2)
    rho, u = 1.0, np.array([0.05, -0.03, 0.0])
    eu = e @ u
    printed = rho * w * (1 + 3 * eu + eu ** 2 * 1.5 - 1.5 * (u @ u))
    assert abs(printed.sum() - rho) > 1e-3
    assert abs(oracle.feq(2, rho, u).sum() - rho) < 1e-15


# ---------------------------------------------------------------- forcing

@pytest.mark.parametrize("dim", [2, 3])
def test_forcing_moments(dim):
    """Sum Fbar = 0, sum e Fbar = F, sum e e Fbar = u F + F u (eq. 9)."""
    rng = np.random.default_rng(2)
    e, _, _, _ = oracle.tables(dim)
    for _ in range(20):
        u = np.zeros(3)
        F = np.zeros(3)
        u[:dim] = rng.uniform(-0.1, 0.1, dim)
        F[:dim] = rng.uniform(-1e-3, 1e-3, dim)
        Fb = oracle.forcing(dim, u, F)
        assert abs(Fb.sum()) < 1e-18
        assert np.allclose(e.T @ Fb, F, atol=1e-18)
        P = np.einsum("i,ia,ib->ab", Fb, e, e)
        assert np.allclose(P, np.outer(u, F) + np.outer(F, u), atol=1e-18)


# ---------------------------------------------------------------- collision

@pytest.mark.parametrize("dim", [2, 3])
def test_mrt_reduces_to_bgk(dim):
    """With every relaxation rate equal to 1/tau, eq. (1) is the BGK step
    f - (f - feq)/tau + (1 - 1/(2 tau)) Fbar."""
    rng = np.random.default_rng(3)
    q = oracle.Q(dim)
    for tau in (0.6, 1.0, 1.7):
        s = np.full(q, 1.0 / tau)
        u = np.zeros(3)
        F = np.zeros(3)
        u[:dim] = rng.uniform(-0.05, 0.05, dim)
        F[:dim] = rng.uniform(-1e-3, 1e-3, dim)
        rho = rng.uniform(0.05, 1.1)
        f = oracle.feq(dim, rho, u) * (1 + 0.05 * rng.standard_normal(q))
        got = oracle.collide_node(dim, s, f, rho, u, F)
        want = f - (f - oracle.feq(dim, rho, u)) / tau + (1 - 0.5 / tau) * oracle.forcing(dim, u, F)
        assert np.allclose(got, want, atol=1e-15, rtol=0)


def _case2(nu=(0.1, 0.4), s_q=1.2, policy=0, dim=2):
    class C:
        pass
    c = C()
    c.dim = dim
    c.n = (4, 4, 1 if dim == 2 else 4)
    c.periodic = (1, 1, 1)
    c.nu = nu
    c.s_q = s_q
    c.s_eps_policy = policy
    c.G12 = 0.0
    c.Gw = (0.0, 0.0)
    c.Fb = (0.0, 0.0, 0.0)
    c.inlets = []
    c.outlet = None
    return c


def test_relaxation_rates():
    """eq. (5): s_nu = 1/(3 nu + 1/2); s_eps from the most viscous phase;
    s_rho = s_j = 1 (eq. 4); the nu = 0.067 of Sec. III A gives the 1.43 of
    eq. (26)."""
    c = _case2(nu=(0.067, 0.067))
    s = oracle.relaxation(c, 0)
    printed = GOLD["laplace_relaxation"]["S"]
    for slot in (1, 2, 7, 8):
        assert abs(s[slot] - printed[slot]) < 5e-3
    for slot in (0, 3, 5):
        assert s[slot] == 1.0
    assert s[4] == s[6] == 1.2
    c = _case2(nu=(0.1, 0.4))
    s0, s1 = oracle.relaxation(c, 0), oracle.relaxation(c, 1)
    assert abs(s0[7] - 1 / (0.3 + 0.5)) < 1e-15 and abs(s1[7] - 1 / (1.2 + 0.5)) < 1e-15
    assert s0[2] == s1[2] == pytest.approx(1 / (1.2 + 0.5), abs=1e-15)
    c.s_eps_policy = 1
    assert oracle.relaxation(c, 0)[2] == pytest.approx(1 / 0.8, abs=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_collision_moments_closed_form(dim):
    """Moments of the post-collision state of eq. (1): mass kept, momentum
    becomes rho_k u + F/2 (s_j = 1), and the shear moments relax with s_nu:
    P*_ab = (1-s_nu) P_ab + s_nu rho u_a u_b + (1 - s_nu/2)(u_a F_b + F_a u_b)
    for a != b and for the normal-stress difference."""
    rng = np.random.default_rng(4)
    c = _case2(nu=(0.13, 0.05), dim=dim)
    e, _, _, _ = oracle.tables(dim)
    q = oracle.Q(dim)
    for k in (0, 1):
        s = oracle.relaxation(c, k)
        snu = 1 / (3 * c.nu[k] + 0.5)
        u = np.zeros(3)
        F = np.zeros(3)
        u[:dim] = rng.uniform(-0.05, 0.05, dim)
        F[:dim] = rng.uniform(-1e-3, 1e-3, dim)
        f = oracle.feq(dim, rng.uniform(0.05, 1.1), u * 0.7) * (1 + 0.05 * rng.standard_normal(q))
        rho = f.sum()
        fs = oracle.collide_node(dim, s, f, rho, u, F)
        assert abs(fs.sum() - f.sum()) < 1e-15
        assert np.allclose(e.T @ fs, rho * u + 0.5 * F, atol=1e-15)
        P = np.einsum("i,ia,ib->ab", f, e, e)
        Ps = np.einsum("i,ia,ib->ab", fs, e, e)
        UF = np.outer(u, F) + np.outer(F, u)
        uu = rho * np.outer(u, u)
        want = (1 - snu) * P + snu * uu + (1 - snu / 2) * UF
        assert abs(Ps[0, 1] - want[0, 1]) < 1e-15
        assert abs((Ps[0, 0] - Ps[1, 1]) - (want[0, 0] - want[1, 1])) < 1e-15
        if dim == 3:
            assert abs(Ps[1, 2] - want[1, 2]) < 1e-15
            assert abs(Ps[0, 2] - want[0, 2]) < 1e-15


# ---------------------------------------------------------------- stencil

def _iso_moments(off, w, dim):
    """Exact moments sum_w e_x^a e_y^b e_z^c of a stencil (Fractions)."""
    def mom(a, b, c=0):
        return sum(wj * (o[0] ** a) * (o[1] ** b) * (o[2] ** c) for o, wj in zip(off, w))
    return mom


def _e8_system(dim):
    """Normalisation and isotropy of the 8th-order stencil, solved exactly.

    For an isotropic rank-2n tensor the moments sum w e_x^a e_y^b e_z^c are in
    the ratio (a-1)!!(b-1)!!(c-1)!!.  Unknowns: one weight per shell."""
    shells = [1, 2, 4, 5, 8] if dim == 2 else [1, 2, 3, 4, 5, 6, 8]
    zr = 2 if dim == 3 else 0
    offs = [o for o in itertools.product(range(-2, 3), range(-2, 3), range(-zr, zr + 1))
            if sum(v * v for v in o) in shells]

    def row(a, b, c, a2, b2, c2, ratio):
        # sum_w (e^(a,b,c) - ratio * e^(a2,b2,c2)) = 0 per shell coefficient
        r = []
        for s in shells:
            r.append(sum(Fraction(o[0] ** a * o[1] ** b * o[2] ** c) - ratio * o[0] ** a2 * o[1] ** b2 * o[2] ** c2
                         for o in offs if sum(v * v for v in o) == s))
        return r

    rows, rhs = [], []
    rows.append([sum(Fraction(o[0] ** 2) for o in offs if sum(v * v for v in o) == s) for s in shells])
    rhs.append(Fraction(1))
    rows.append(row(4, 0, 0, 2, 2, 0, 3)); rhs.append(0)
    rows.append(row(6, 0, 0, 4, 2, 0, 5)); rhs.append(0)
    rows.append(row(8, 0, 0, 6, 2, 0, 7)); rhs.append(0)
    rows.append(row(6, 2, 0, 4, 4, 0, Fraction(5, 3))); rhs.append(0)
    if dim == 3:
        rows.append(row(4, 2, 0, 2, 2, 2, 3)); rhs.append(0)
        rows.append(row(4, 4, 0, 4, 2, 2, 3)); rhs.append(0)
    # exact Gaussian elimination
    n = len(shells)
    A = [r[:] + [Fraction(b)] for r, b in zip(rows, rhs)]
    for col in range(n):
        piv = next(i for i in range(col, n) if A[i][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        for i in range(n):
            if i != col and A[i][col] != 0:
                f = A[i][col] / A[col][col]
                A[i] = [x - f * y for x, y in zip(A[i], A[col])]
    return {s: A[i][n] / A[i][i] for i, s in enumerate(shells)}, offs


@pytest.mark.parametrize("dim,K", [(2, 24), (3, 92)])
def test_e8_stencil_unique_isotropic(dim, K):
    """The interaction weights are the unique solution of the 8th-order
    isotropy system on their shells; in 2-D they equal the printed values."""
    sol, offs = _e8_system(dim)
    off, w = oracle.stencil(dim)
    assert len(off) == K == len(offs)
    assert all(v > 0 for v in sol.values())
    for o, wj in zip(off, w):
        r2 = int((o ** 2).sum())
        assert wj == pytest.approx(float(sol[r2]), rel=1e-15, abs=0)
    if dim == 2:
        printed = {int(k): Fraction(v) for k, v in GOLD["e8_weights_2d"]["w_by_r2"].items()}
        assert printed == sol
    # odd moments vanish, E2 = 1 (exactly as floats summed)
    assert abs((w[:, None] * off).sum(0)).max() < 1e-16
    assert abs((w * off[:, 0] ** 2).sum() - 1.0) < 1e-15


# ---------------------------------------------------------------- alpha

def test_alpha_closed_form_left_inlet():
    """For the left inlet (unknowns 1, 5, 8) the correction of eqs. (15)-(19)
    is alpha_1 = 2 dJx/3, alpha_5 = dJx/6 + dJy/2, alpha_8 = dJx/6 - dJy/2,
    which moves the node momentum by exactly dJ."""
    e, w, _, _ = oracle.tables(2)
    U = [1, 5, 8]
    D = np.array([sum(w[j] * e[j, d] ** 2 for j in U) for d in range(2)])
    assert np.allclose(D, [1 / 6, 1 / 18], atol=1e-16)
    dJ = np.array([3e-4, -2e-4])
    alpha = {i: w[i] * (e[i, 0] * dJ[0] / D[0] + e[i, 1] * dJ[1] / D[1]) for i in U}
    assert alpha[1] == pytest.approx(2 * dJ[0] / 3, abs=1e-18)
    assert alpha[5] == pytest.approx(dJ[0] / 6 + dJ[1] / 2, abs=1e-18)
    assert alpha[8] == pytest.approx(dJ[0] / 6 - dJ[1] / 2, abs=1e-18)
    mom = sum(alpha[i] * e[i, :2] for i in U)
    assert np.allclose(mom, dJ, atol=1e-18)


def test_energy_moments_relax_with_s_e_and_s_eps():
    """D2Q9 rows 1 and 2 of eq. (3) (energy e and energy square eps) relax with
    s_e and s_eps towards rho(-2 + 3u^2) and rho(1 - 3u^2), with forcing
    moments 6 u.F and -6 u.F (closed forms of the equilibrium of eq. 6 and the
    forcing of eq. 9)."""
    rng = np.random.default_rng(5)
    e, _, _, _ = oracle.tables(2)
    e2 = (e ** 2).sum(1).astype(float)
    row_e = -4 + 3 * e2
    row_eps = 4 - 10.5 * e2 + 4.5 * e2 ** 2
    c = _case2(nu=(0.4, 0.06))
    for k in (0, 1):
        s = oracle.relaxation(c, k)
        u = np.array([0.03, -0.02, 0.0])
        F = np.array([2e-4, 1e-4, 0.0])
        f = oracle.feq(2, 0.8, u * 0.5) * (1 + 0.04 * rng.standard_normal(9))
        rho = f.sum()
        fs = oracle.collide_node(2, s, f, rho, u, F)
        uu, uF = u @ u, u @ F
        for row, slot, eq, fm in ((row_e, 1, rho * (-2 + 3 * uu), 6 * uF),
                                  (row_eps, 2, rho * (1 - 3 * uu), -6 * uF)):
            m, ms = row @ f, row @ fs
            want = m - s[slot] * (m - eq) + (1 - s[slot] / 2) * fm
            assert abs(ms - want) < 1e-15
