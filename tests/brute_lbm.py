"""Dense NumPy restatement of one step of the two-component pseudopotential
MRT lattice Boltzmann method with the corrected open boundaries
(arXiv:2512.12934), for tiny grids only.

It exists to catch implementation slips in the C oracle (an index, a loop
bound, a sign in a face rule), so it is written differently on purpose:
whole-array NumPy operations instead of node loops, streaming in the pull
form instead of the push form, ghost layers by ``numpy.pad`` (mode
"symmetric" is the mirror of eqs. 24-25, "wrap" the periodic image), and the
moment matrices built here from their polynomial rows.  It shares nothing
with ``oracle/`` or the HIP library; both only meet it through a case
object (geometry, parameters, initial fields).

The readings of the paper are the ones the oracle takes: eq. (3) rows as the
orthogonal polynomial basis, eq. (6) with (e.u)^2/(2 cs^4), eq. (10) with the
other component's psi, constant adhesion (eq. 11), s_e moving with s_eps,
alpha as a momentum correction (eqs. 15-19), U_c clamped at 0 (eqs. 20-21),
chi overriding the outlet column's normal velocity (eqs. 22-23).
"""
from fractions import Fraction

import numpy as np

CS2 = 1.0 / 3.0

E2D = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0],
                [1, 1, 0], [-1, 1, 0], [-1, -1, 0], [1, -1, 0]])
E3D = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
                [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])

# 8th-order isotropic interaction weights by squared offset length: the 2-D
# values printed in Sec. II A; the 3-D set solves the same conditions on the
# 5x5x5 cube (shells 1, 2, 3, 4, 5, 6, 8).
W8_2D = {1: Fraction(4, 21), 2: Fraction(4, 45), 4: Fraction(1, 60), 5: Fraction(2, 315), 8: Fraction(1, 5040)}
W8_3D = {1: Fraction(4, 45), 2: Fraction(1, 21), 3: Fraction(2, 105), 4: Fraction(5, 504),
         5: Fraction(1, 315), 6: Fraction(1, 630), 8: Fraction(1, 5040)}


def lattice(dim):
    e = E2D if dim == 2 else E3D
    e2 = (e * e).sum(1)
    if dim == 2:
        w = np.where(e2 == 0, 4 / 9, np.where(e2 == 1, 1 / 9, 1 / 36))
    else:
        w = np.where(e2 == 0, 1 / 3, np.where(e2 == 1, 1 / 18, 1 / 36))
    opp = np.array([int(np.nonzero((e == -e[i]).all(1))[0][0]) for i in range(len(e))])
    return e, w, opp


def moment_matrix(dim):
    e, _, _ = lattice(dim)
    x, y, z = (e[:, 0].astype(float), e[:, 1].astype(float), e[:, 2].astype(float))
    r2 = x * x + y * y + z * z
    if dim == 2:
        rows = [np.ones_like(x), 3 * r2 - 4, 4.5 * r2 ** 2 - 10.5 * r2 + 4, x, (3 * r2 - 5) * x,
                y, (3 * r2 - 5) * y, x * x - y * y, x * y]
    else:
        rows = [np.ones_like(x), 19 * r2 - 30, (21 * r2 ** 2 - 53 * r2 + 24) / 2,
                x, (5 * r2 - 9) * x, y, (5 * r2 - 9) * y, z, (5 * r2 - 9) * z,
                3 * x * x - r2, (3 * r2 - 5) * (3 * x * x - r2), y * y - z * z, (3 * r2 - 5) * (y * y - z * z),
                x * y, y * z, x * z, (y * y - z * z) * x, (z * z - x * x) * y, (x * x - y * y) * z]
    return np.array(rows)


def rates(case, k):
    nu = case.nu
    snu = 1.0 / (3 * nu[k] + 0.5)
    if case.s_eps_policy == 0:
        seps = 1.0 / (3 * max(nu) + 0.5)
        se = seps
    else:
        seps = se = snu
    sq = case.s_q
    if case.dim == 2:
        return np.array([1, se, seps, 1, sq, 1, sq, snu, snu], float)
    return np.array([1, se, seps, 1, sq, 1, sq, 1, sq, snu, snu, snu, snu, snu, snu, snu, sq, sq, sq], float)


def feq(e, w, rho, u):
    """rho [...], u [3, ...] -> [Q, ...]"""
    eu = np.einsum("id,d...->i...", e.astype(float), u)
    uu = (u * u).sum(0)
    return w.reshape((-1,) + (1,) * rho.ndim) * rho * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - uu / (2 * CS2))


def guo(e, w, u, F):
    """Forcing term of eq. (9): w_i [(e_i - u)/cs^2 + (e_i.u) e_i/cs^4] . F"""
    ef = e.astype(float)
    eu = np.einsum("id,d...->i...", ef, u)
    eF = np.einsum("id,d...->i...", ef, F)
    uF = (u * F).sum(0)
    return w.reshape((-1,) + (1,) * uF.ndim) * ((eF - uF) / CS2 + eu * eF / CS2 ** 2)


class Brute:
    """Grid arrays are [z, y, x] (2-D: [y, x]); populations [k, i, ...]."""

    def __init__(self, case):
        self.c = case
        self.dim = case.dim
        self.e, self.w, self.opp = lattice(self.dim)
        self.Q = len(self.w)
        nx, ny, nz = case.n
        self.shape = (ny, nx) if self.dim == 2 else (nz, ny, nx)
        self.solid = np.asarray(case.solid).reshape(self.shape).astype(bool)
        self.fluid = ~self.solid
        # axis a of the lattice (x, y, z) is array axis ax[a]
        self.ax = [self.dim - 1 - a for a in range(self.dim)]
        self.per = [bool(case.periodic[a]) for a in range(self.dim)]
        T = moment_matrix(self.dim)
        Ti = np.linalg.inv(T)
        self.A = [Ti @ np.diag(rates(case, k)) @ T for k in range(2)]
        self.B = [Ti @ np.diag(1 - rates(case, k) / 2) @ T for k in range(2)]
        W = W8_2D if self.dim == 2 else W8_3D
        r = range(-2, 3)
        offs = [(dx, dy, dz) for dz in (r if self.dim == 3 else [0]) for dy in r for dx in r]
        self.stencil = [(o, float(W[o[0] ** 2 + o[1] ** 2 + o[2] ** 2])) for o in offs
                        if o[0] ** 2 + o[1] ** 2 + o[2] ** 2 in W]
        uw = getattr(case, "wall_u", None)
        self.uw = None if uw is None else np.asarray(uw, float).reshape((3,) + self.shape)
        rho0 = np.asarray(case.rho0, float).reshape((2,) + self.shape)
        u0 = np.zeros((3,) + self.shape) if case.u0 is None else np.asarray(case.u0, float).reshape((3,) + self.shape)
        self.f = np.stack([feq(self.e, self.w, rho0[k], u0) for k in range(2)])
        self.f[:, :, self.solid] = 0.0
        self.faces = self._faces()

    # ----------------------------------------------------------- geometry
    def _grid(self):
        return np.stack(np.meshgrid(*[np.arange(s) for s in self.shape], indexing="ij"))

    def _faces(self):
        """Inlet ownership map (later patches win) and outlet mask."""
        c = self.c
        coord = self._grid()           # coord[j] is array axis j
        xyz = [coord[self.ax[a]] for a in range(self.dim)]
        owner = np.full(self.shape, -1)
        for p, inl in enumerate(c.inlets):
            m = self._patch(xyz, inl)
            owner[m & self.fluid] = p
        out = np.zeros(self.shape, bool)
        if c.outlet is not None:
            out = self._patch(xyz, c.outlet) & self.fluid
        return owner, out

    def _patch(self, xyz, p):
        a = p["axis"]
        layer = 0 if p["side"] == 0 else self.c.n[a] - 1
        m = xyz[a] == layer
        for b in range(self.dim):
            if b != a:
                m &= (xyz[b] >= p["lo"][b]) & (xyz[b] < p["hi"][b])
        return m

    def _shift(self, arr, off, fill):
        """out[x] = arr[x + off] (lattice offset off), periodic axes wrap,
        positions beyond a non-periodic face take ``fill``."""
        out = arr
        for a in range(self.dim):
            d = off[a]
            if d == 0:
                continue
            j = self.ax[a] + (arr.ndim - len(self.shape))
            if self.per[a]:
                out = np.roll(out, -d, axis=j)
            else:
                out = np.roll(out, -d, axis=j)
                n = arr.shape[j]
                idx = [slice(None)] * out.ndim
                idx[j] = slice(n - d, n) if d > 0 else slice(0, -d)
                out = out.copy()
                out[tuple(idx)] = fill
        return out

    def _ghost(self, arr):
        """Pad the grid axes by 2: wrap on periodic axes, mirror (eqs. 24-25)
        on the others."""
        lead = arr.ndim - len(self.shape)
        out = arr
        for a in range(self.dim):
            j = self.ax[a] + lead
            pad = [(0, 0)] * out.ndim
            pad[j] = (2, 2)
            out = np.pad(out, pad, mode="wrap" if self.per[a] else "symmetric")
        return out

    def _window(self, ext, off):
        """ext padded by 2 on every grid axis: the view at x + off."""
        lead = ext.ndim - len(self.shape)
        idx = [slice(None)] * ext.ndim
        for a in range(self.dim):
            j = self.ax[a] + lead
            idx[j] = slice(2 + off[a], 2 + off[a] + self.shape[j - lead])
        return ext[tuple(idx)]

    # ----------------------------------------------------------- one step
    def step(self):
        c, e, w, Q = self.c, self.e, self.w, self.Q
        ef = e.astype(float)
        fl = self.fluid
        f = self.f
        rho = f.sum(1) * fl
        psi = rho.copy()
        psi_x = self._ghost(psi)
        sol_x = self._ghost(self.solid.astype(float))
        gp = np.zeros((2, 3) + self.shape)
        gs = np.zeros((3,) + self.shape)
        for off, ww in self.stencil:
            o = np.array(off, float)[:, None]
            pv = self._window(psi_x, off)
            sv = self._window(sol_x, off)
            gp += ww * o.reshape((1, 3) + (1,) * len(self.shape)) * pv[:, None]
            gs += ww * o.reshape((3,) + (1,) * len(self.shape)) * sv
        rt = rho.sum(0)
        safe = np.where(fl, rt, 1.0)
        Fb = np.array(c.Fb, float).reshape((3,) + (1,) * len(self.shape))
        F = np.zeros((2, 3) + self.shape)
        for k in range(2):
            F[k] = (-c.G12 * psi[k] * gp[1 - k] - c.Gw[k] * psi[k] * gs + (rho[k] / safe) * Fb) * fl
        J = np.einsum("kin,id->dn", f.reshape(2, Q, -1), ef).reshape((3,) + self.shape)
        u = (J + 0.5 * F.sum(0)) / safe * fl

        owner, out = self.faces
        # stage 4: chi (eq. 23) and the outlet override (eq. 22)
        qin = 0.0
        for p, inl in enumerate(c.inlets):
            nv = np.zeros(3)
            nv[inl["axis"]] = 1 if inl["side"] == 0 else -1
            m = owner == p
            qin += (rt[m] * np.einsum("d,dn->n", nv, u[:, m])).sum()
        uc = u.copy()
        if c.outlet is not None:
            o = c.outlet
            no = np.zeros(3, int)
            no[o["axis"]] = 1 if o["side"] == 1 else -1
            back = tuple(-no)                       # x' = x_N - n_o
            rt_p = self._shift(rt, back, 0.0)
            u_p = self._shift(u, back, 0.0)
            fl_p = self._shift(fl, back, False)
            sel = out & fl_p
            qout = (rt_p[sel] * np.einsum("d,dn->n", no.astype(float), u_p[:, sel])).sum()
            chi = 1.0 if (abs(qout) < 1e-30 or qin * qout <= 0) else qin / qout
            if o.get("chi_on", 1):
                uc[o["axis"]][sel] = chi * u_p[o["axis"]][sel]
        # stages 5-6: collision, then pull streaming with bounce-back
        fs = np.zeros_like(f)
        for k in range(2):
            fe = feq(e, w, rho[k], uc)
            Fk = guo(e, w, uc, F[k])
            fs[k] = f[k] - np.einsum("ij,j...->i...", self.A[k], f[k] - fe) + np.einsum("ij,j...->i...", self.B[k], Fk)
        fn = np.full_like(f, np.nan)
        for i in range(Q):
            src = tuple(-e[i][:self.dim])
            src3 = tuple(list(src) + [0] * (3 - len(src)))
            pulled = self._shift(fs[:, i], src3, np.nan)
            src_solid = self._shift(self.solid, src3, False)
            src_out = self._shift(np.zeros(self.shape, bool), src3, True)
            bounced = fs[:, self.opp[i]]
            if self.uw is not None:
                # a moving wall at the source adds 2 w_i rho_k (e_i . u_w) / cs^2
                uws = self._shift(self.uw, src3, 0.0)
                bounced = bounced + 2 * w[i] * rho * np.einsum("d,d...->...", ef[i], uws)[None] / CS2
            v = np.where(src_solid & ~src_out, bounced, pulled)
            v = np.where(src_out, np.nan, v)
            fn[:, i] = np.where(fl, v, np.nan)
        # stage 7: inlets (eq. 13/14, then eqs. 15-19)
        for p, inl in enumerate(c.inlets):
            nv = np.zeros(3, int)
            nv[inl["axis"]] = 1 if inl["side"] == 0 else -1
            m = owner == p
            if not m.any():
                continue
            up = inl["u_n"] * nv.astype(float)
            f2 = self._shift(fn, tuple(nv), np.nan)[:, :, m]
            F2 = self._shift(F, tuple(nv), 0.0)[:, :, m]
            fl2 = self._shift(fl, tuple(nv), False)[m]
            r2 = f2.sum(1)
            J2 = np.einsum("kin,id->dn", f2, ef) + 0.5 * F2.sum(0)
            u2 = J2 / np.where(fl2, r2.sum(0), 1.0)
            entering = (e @ nv) > 0
            D = (w[entering, None] * ef[entering] ** 2).sum(0)
            for k in range(2):
                fp = feq(e, w, np.full(m.sum(), inl["rho"][k]), np.repeat(up[:, None], m.sum(), 1))
                f2e = feq(e, w, r2[k], u2)
                neq = np.where(fl2, f2[k] - f2e, 0.0)
                new = fn[k][:, m]
                new[entering] = fp[entering] + neq[entering]
                if inl.get("alpha_on", 1):
                    Jx = np.einsum("in,id->dn", new, ef) + 0.5 * F[k][:, m]
                    dJ = inl["rho"][k] * up[:, None] - Jx
                    corr = np.zeros_like(new)
                    for d in range(self.dim):
                        if D[d] > 0:
                            corr += w[:, None] * ef[:, d:d + 1] * dJ[d][None, :] / D[d]
                    new[entering] += corr[entering]
                fn[k][:, m] = new
        # stage 8: convective outflow (eqs. 20-21)
        if c.outlet is not None:
            fnp = self._shift(fn, back, np.nan)
            Fp = self._shift(F, back, 0.0)
            r = fnp.sum(1).sum(0)
            Jn = np.einsum("kin,i->n", fnp[:, :, sel], (ef @ no.astype(float))) + \
                0.5 * np.einsum("kdn,d->n", Fp[:, :, sel], no.astype(float))
            vel = Jn / r[sel]
            Uc = vel.mean() if vel.size else 0.0
            Uc = max(Uc, 0.0)
            entering = (e @ no) < 0
            for k in range(2):
                prev = f[k][:, out]
                nxt = np.where(sel[out][None, :], (prev + Uc * fnp[k][:, out]) / (1 + Uc), prev)
                cur = fn[k][:, out]
                cur[entering] = nxt[entering]
                fn[k][:, out] = cur
        fn[:, :, self.solid] = 0.0
        self.f = fn

    def f_nodes(self):
        """State as [2][Q][N] in x-fastest node order (solids zero)."""
        return self.f.reshape(2, self.Q, -1)
