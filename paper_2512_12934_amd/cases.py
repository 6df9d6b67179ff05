"""Seeded synthetic cases (geometry, parameters, initial fields).

This module describes inputs only: box sizes, solid masks, initial component
densities, inlet/outlet patches and the physical parameters of each workload.
It holds none of the method's arithmetic, so the FP64 oracle and the HIP
library can both be fed from it.

Node order is x fastest: ``n = x + nx*(y + ny*z)``.  Densities are
``rho0[k, n]`` for component k in {0, 1} (the paper's components 1 and 2).
"""
from __future__ import annotations

import copy
import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Case:
    name: str
    dim: int
    n: tuple
    periodic: tuple
    nu: tuple
    G12: float
    solid: np.ndarray
    rho0: np.ndarray
    u0: Optional[np.ndarray] = None
    s_q: float = 1.2
    s_eps_policy: int = 0          # 0: most-viscous phase (paper), 1: fixed = s_nu,k
    Gw: tuple = (0.0, 0.0)
    Fb: tuple = (0.0, 0.0, 0.0)
    inlets: list = dataclasses.field(default_factory=list)
    outlet: Optional[dict] = None
    wall_u: Optional[np.ndarray] = None   # [3, N] velocity of solid nodes (moving walls)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def fluid_nodes(self) -> int:
        return int((self.solid == 0).sum())

    def grid(self):
        """Return coordinate arrays (x, y, z), each of length N."""
        nx, ny, nz = self.n
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        return x.reshape(-1), y.reshape(-1), z.reshape(-1)

    def copy(self, **changes) -> "Case":
        c = copy.deepcopy(self)
        for k, v in changes.items():
            setattr(c, k, v)
        return c


# Bulk densities (phase-rich, dissolved) of the two coexisting phases at
# G12 = 0.9 for a total near 1.05: a flat interface of the oracle started from
# this pair in a 512-wide periodic box keeps it to 3e-3 over 40k steps, and it
# satisfies the leading-order coexistence condition
# c_s^2 ln(a/b) = G12 (a - b) to 1%.  Open-boundary cases feed both phases at
# these densities: with 1.0 / 0.03 the stream of the other phase is
# undersaturated (0.03 against ~0.09 dissolved) and dissolves the dispersed
# phase (the 3-D co-flow device then forms no droplets).
COEX_G09 = (0.96, 0.09)

# Adhesion strength that makes the dispersed phase non-wetting (contact angle
# ~180 degrees) at G12 = 0.9: from oracle sessile-drop runs on a 100 x 50
# channel (drop of radius 15, 6000 steps), the contact angle grows from ~85
# degrees at 0 to ~159 at 0.08 and the drop lifts off the wall at 0.1.
# tests/test_oracle_physics.py repeats the two end points.
GW_NONWETTING = 0.1


def sessile(g: float, nx: int = 100, ny: int = 50, R: float = 15.0, major: float = 1.0,
            minor: float = 0.03) -> Case:
    """Half-disc droplet of component 1 resting on the lower of two walls,
    periodic along x, adhesion +g (component 1) and -g (component 2)."""
    c = Case("sessile", 2, (nx, ny, 1), (True, False, True), (1.0 / 6.0, 1.0 / 6.0), 0.9,
             solid=None, rho0=None, Gw=(g, -g))
    x, y, _ = c.grid()
    c.solid = ((y == 0) | (y == ny - 1)).astype(np.uint8)
    inside = ((x - nx / 2) ** 2 + (y - 1) ** 2 < R * R) & (y >= 1)
    c.rho0 = _rho_from_mask(inside, major, minor)
    c.meta.update(R=R, major=major, minor=minor)
    return c


def _rho_from_mask(inside: np.ndarray, major: float, minor: float) -> np.ndarray:
    """Component 1 is ``major`` where ``inside``; component 2 is mirrored."""
    rho = np.empty((2, inside.size))
    rho[0] = np.where(inside, major, minor)
    rho[1] = np.where(inside, minor, major)
    return rho


def _plug(case: Case, regions) -> np.ndarray:
    """Initial velocity: uniform plug flow ``value`` along ``axis`` on each
    (mask, axis, value) region, zero on solids.  Starting open-boundary runs
    from the plug flow their inlets feed keeps the inlet and outlet mass flows
    comparable from the first step."""
    u0 = np.zeros((3, case.N))
    for mask, axis, value in regions:
        u0[axis][mask] = value
    u0[:, case.solid == 1] = 0.0
    return u0


def inlet(axis, side, lo, hi, rho, u_n, alpha_on=True):
    return {"axis": axis, "side": side, "lo": tuple(lo), "hi": tuple(hi),
            "rho": tuple(rho), "u_n": float(u_n), "alpha_on": int(bool(alpha_on))}


def outlet(axis, side, lo, hi, chi_on=True):
    return {"axis": axis, "side": side, "lo": tuple(lo), "hi": tuple(hi),
            "chi_on": int(bool(chi_on))}


# ---------------------------------------------------------------------------
# Laplace test: static droplet, fully periodic
# ---------------------------------------------------------------------------

def laplace(n: int = 64, R: float = 16.0, G12: float = 0.9, nu=(1.0 / 6.0, 1.0 / 6.0),
            major: float = 1.0, minor: float = 0.03, s_eps_policy: int = 0,
            dim: int = 2, center=None) -> Case:
    """Static droplet of radius R centred in an n^dim periodic box.

    Defaults: 64x64, R = 16, G12 = 0.9, relaxation time 1 for both components
    (nu = 1/6), droplet component density 1.0 inside / 0.03 outside and the
    other component mirrored, u = 0.  A node is inside when its distance to
    the centre is below R (sharp initial step)."""
    shape = (n, n, n if dim == 3 else 1)
    c = Case("laplace", dim, shape, (True, True, True), tuple(nu), G12,
             solid=np.zeros(int(np.prod(shape)), np.uint8), rho0=None,
             s_eps_policy=s_eps_policy)
    x, y, z = c.grid()
    cx = cy = cz = n / 2.0
    if center is not None:
        cx, cy = center[0], center[1]
        if dim == 3:
            cz = center[2]
    r2 = (x - cx) ** 2 + (y - cy) ** 2 + ((z - cz) ** 2 if dim == 3 else 0)
    c.rho0 = _rho_from_mask(r2 < R * R, major, minor)
    c.meta.update(R=R, major=major, minor=minor)
    return c


def drops(shape=(160, 64, 1), count: int = 7, seed: int = 5, r_range=(3.0, 9.0), G12: float = 0.9,
          nu=(1.0 / 6.0, 1.0 / 6.0), major: float = 1.0, minor: float = 0.03) -> Case:
    """Several droplets of seeded radii and centres in a periodic box (2-D when
    shape[2] == 1): a field with many components for the labelling checks."""
    dim = 2 if shape[2] == 1 else 3
    c = Case("drops", dim, tuple(shape), (True, True, True), tuple(nu), G12,
             solid=np.zeros(int(np.prod(shape)), np.uint8), rho0=None)
    rng = np.random.default_rng(seed)
    x, y, z = c.grid()
    inside = np.zeros(c.N, bool)
    for _ in range(count):
        R = rng.uniform(*r_range)
        cen = [rng.uniform(0, shape[a]) for a in range(3)]
        r2 = (x - cen[0]) ** 2 + (y - cen[1]) ** 2 + ((z - cen[2]) ** 2 if dim == 3 else 0)
        inside |= r2 < R * R
    c.rho0 = _rho_from_mask(inside, major, minor)
    c.meta.update(major=major, minor=minor)
    return c


# ---------------------------------------------------------------------------
# Random periodic / closed boxes (for invariants and parity at several tiles)
# ---------------------------------------------------------------------------

def random_box(shape, seed: int, dim: int = 2, periodic=(True, True, True),
               walls: bool = False, G12: float = 0.9, nu=(0.1, 0.3),
               amp: float = 0.02, Gw=(0.0, 0.0), Fb=(0.0, 0.0, 0.0),
               u_amp: float = 0.0) -> Case:
    """Smooth random two-component field in a box of the given shape.

    With ``walls`` every non-periodic axis gets a one-node solid shell and a
    few solid blocks are scattered inside."""
    rng = np.random.default_rng(seed)
    nx, ny = shape[0], shape[1]
    nz = shape[2] if dim == 3 else 1
    c = Case(f"random{dim}d", dim, (nx, ny, nz), tuple(periodic), tuple(nu), G12,
             solid=np.zeros(nx * ny * nz, np.uint8), rho0=None, Gw=tuple(Gw), Fb=tuple(Fb))
    x, y, z = c.grid()
    solid = np.zeros(c.N, bool)
    if walls:
        for a, (coord, size) in enumerate(((x, nx), (y, ny), (z, nz))):
            if a >= dim or periodic[a]:
                continue
            solid |= (coord == 0) | (coord == size - 1)
        for _ in range(3):
            bx, by = rng.integers(2, max(3, nx - 4)), rng.integers(2, max(3, ny - 4))
            blk = (x >= bx) & (x < bx + 2) & (y >= by) & (y < by + 2)
            if dim == 3:
                bz = rng.integers(2, max(3, nz - 4))
                blk &= (z >= bz) & (z < bz + 2)
            solid |= blk
    c.solid = solid.astype(np.uint8)
    # a smooth phase field: a few random Fourier modes
    phase = np.zeros(c.N)
    for _ in range(4):
        kx, ky, kz = rng.integers(1, 3, size=3)
        ph = rng.uniform(0, 2 * math.pi, size=3)
        phase += np.sin(2 * math.pi * kx * x / nx + ph[0]) * np.cos(2 * math.pi * ky * y / ny + ph[1]) \
            * (np.cos(2 * math.pi * kz * z / nz + ph[2]) if dim == 3 else 1.0)
    inside = phase > 0
    rho = _rho_from_mask(inside, 1.0, 0.05)
    rho *= 1.0 + amp * rng.standard_normal(rho.shape)
    c.rho0 = rho
    if u_amp > 0:
        u0 = np.zeros((3, c.N))
        u0[:dim] = u_amp * rng.standard_normal((dim, c.N))
        c.u0 = u0
    return c


# ---------------------------------------------------------------------------
# Two-phase Poiseuille flow between plates (periodic along x)
# ---------------------------------------------------------------------------

def poiseuille(M: float, Fb: float, width: int = 100, a: float = 25.0, nx: int = 4,
               nu2: float = 0.067, major: float = 1.02, minor: float = 0.03,
               G12: float = 0.9, u_init=None, dim: int = 2) -> Case:
    """Fluid 1 (viscosity M*nu2) in the core |y - yc| < a, fluid 2 outside, up
    to the walls; ``width`` fluid rows between two solid rows; body force Fb
    along x.  ``u_init`` optionally gives an initial u_x(y) profile (length
    width) applied to every column."""
    ny = width + 2
    nz = 1 if dim == 2 else 4
    c = Case("poiseuille", dim, (nx, ny, nz), (True, False, True), (M * nu2, nu2), G12,
             solid=None, rho0=None, Fb=(Fb, 0.0, 0.0))
    x, y, z = c.grid()
    c.solid = ((y == 0) | (y == ny - 1)).astype(np.uint8)
    yc = (ny - 1) / 2.0
    inside = np.abs(y - yc) < a
    c.rho0 = _rho_from_mask(inside, major, minor)
    if u_init is not None:
        u0 = np.zeros((3, c.N))
        prof = np.zeros(ny)
        prof[1:ny - 1] = u_init
        u0[0] = prof[y]
        u0[0][c.solid == 1] = 0.0
        c.u0 = u0
    c.meta.update(M=M, a=a, L=width / 2.0, yc=yc, major=major, minor=minor)
    return c


# ---------------------------------------------------------------------------
# Sheared layers between moving plates (Couette flow, Taylor deformation)
# ---------------------------------------------------------------------------

def _plates(c: Case, U_top: float, U_bot: float) -> None:
    """Solid rows y = 0 and y = n1 - 1, moving along x at U_bot and U_top."""
    x, y, z = c.grid()
    top, bot = y == c.n[1] - 1, y == 0
    c.solid = (top | bot).astype(np.uint8)
    uw = np.zeros((3, c.N))
    uw[0][top] = U_top
    uw[0][bot] = U_bot
    c.wall_u = uw


def couette(width: int = 20, nx: int = 6, U_top: float = 0.02, U_bot: float = -0.01, nu=(0.1, 0.1),
            rho=(0.4, 0.6), dim: int = 2, G12: float = 0.0) -> Case:
    """Uniform two-component mixture between plates moving along x (periodic
    along x, and z in 3-D): ``width`` fluid rows.  With no interaction the
    steady state is the linear Couette profile between the wall planes half
    a node outside the first and last fluid rows."""
    ny = width + 2
    nz = 1 if dim == 2 else 4
    N = nx * ny * nz
    c = Case("couette", dim, (nx, ny, nz), (True, False, True), tuple(nu), G12,
             solid=np.zeros(N, np.uint8), rho0=None)
    _plates(c, U_top, U_bot)
    c.rho0 = np.stack([np.full(N, rho[0]), np.full(N, rho[1])])
    c.meta.update(U_top=U_top, U_bot=U_bot, width=width)
    return c


def taylor(M: float, Ca: float, nx: int = 200, H: int = 100, R: float = 25.0, nu_c: float = 1.0 / 6.0,
           gamma: float = None, dim: int = 2, s_eps_policy: int = 0, G12: float = 0.9,
           major: float = COEX_G09[0], minor: float = COEX_G09[1]) -> Case:
    """Taylor deformation (Sec. III A, Fig. 4): a droplet of component 1
    (viscosity M nu_c) of radius R centred between two plates H fluid rows
    apart that move along x at +U (top) and -U (bottom); periodic along x
    (and z in 3-D, where the box is nx x (H+2) x nx/2... see ``nz``).  The
    plate speed follows the paper's capillary number Ca = U nu_c rho_c /
    gamma, with gamma the interfacial tension of G12 = 0.9 (GAMMA_G09)."""
    gamma = GAMMA_G09 if gamma is None else gamma
    ny = H + 2
    nz = 1 if dim == 2 else max(4, int(2 * R + 12))
    U = Ca * gamma / (nu_c * major)
    N = nx * ny * nz
    c = Case("taylor", dim, (nx, ny, nz), (True, False, True), (M * nu_c, nu_c), G12,
             solid=np.zeros(N, np.uint8), rho0=None, s_eps_policy=s_eps_policy)
    _plates(c, U, -U)
    x, y, z = c.grid()
    r2 = (x - nx / 2) ** 2 + (y - ny / 2) ** 2 + ((z - nz / 2) ** 2 if dim == 3 else 0)
    c.rho0 = _rho_from_mask(r2 < R * R, major, minor)
    # the initial velocity: the linear shear between the plates
    u0 = np.zeros((3, N))
    u0[0] = U * (2.0 * (y - 0.5) / H - 1.0)
    u0[:, c.solid == 1] = 0.0
    c.u0 = u0
    c.meta.update(M=M, Ca=Ca, U=U, H=H, R=R, major=major, minor=minor)
    return c


# ---------------------------------------------------------------------------
# Straight channel with inlet and outlet (2-D or 3-D)
# ---------------------------------------------------------------------------

def channel(length: int, width: int, u_in: float, nu=(0.067, 0.067), G12: float = 0.9,
            alpha_on=True, chi_on=True, droplet=None, major: float = 1.0,
            minor: float = 0.03, dim: int = 2, Gw=(0.0, 0.0)) -> Case:
    """Channel along x with walls on the other axes, inlet at x = 0 carrying
    the continuous phase (component 2), convective outlet at x = length-1.
    ``droplet=(cx, cy[, cz], R)`` places a component-1 droplet."""
    ny = width + 2
    nz = 1 if dim == 2 else width + 2
    c = Case("channel", dim, (length, ny, nz), (False, False, False), tuple(nu), G12,
             solid=None, rho0=None, Gw=tuple(Gw))
    x, y, z = c.grid()
    solid = (y == 0) | (y == ny - 1)
    if dim == 3:
        solid |= (z == 0) | (z == nz - 1)
    c.solid = solid.astype(np.uint8)
    inside = np.zeros(c.N, bool)
    if droplet is not None:
        if dim == 2:
            cx, cy, R = droplet
            inside = (x - cx) ** 2 + (y - cy) ** 2 < R * R
        else:
            cx, cy, cz, R = droplet
            inside = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 < R * R
    c.rho0 = _rho_from_mask(inside, major, minor)
    c.u0 = _plug(c, [(np.ones(c.N, bool), 0, u_in)])
    c.inlets = [inlet(0, 0, (0, 1, 1 if dim == 3 else 0), (1, ny - 1, nz - 1 if dim == 3 else 1),
                      (minor, major), u_in, alpha_on)]
    c.outlet = outlet(0, 1, (0, 1, 1 if dim == 3 else 0), (1, ny - 1, nz - 1 if dim == 3 else 1),
                      chi_on)
    c.meta.update(u_in=u_in, width=width)
    return c


# ---------------------------------------------------------------------------
# T-junction droplet generator (2-D)
# ---------------------------------------------------------------------------

def tjunction(W: int = 100, length: int = 800, x_side: int = 150, side_width: int = 100,
              side_len: int = 100, u_c: float = 0.01, u_d: float = 0.005,
              nu=(0.067, 0.067), G12: float = 0.9, Gw_mag: float = None,
              major: float = COEX_G09[0], minor: float = COEX_G09[1], alpha_on=True, chi_on=True) -> Case:
    """Main channel ``length`` x ``W`` fluid nodes between solid rows y = 0 and
    y = W+1, side channel of width ``side_width`` over x in
    [x_side, x_side+side_width) rising ``side_len`` rows above the main
    channel.  Continuous phase (component 2) enters at x = 0 with u_c;
    dispersed phase (component 1) enters through the top of the side channel
    with u_d (downwards); convective outlet at x = length-1.  Walls repel the
    dispersed phase with adhesion +Gw_mag and attract the continuous phase
    with -Gw_mag (default GW_NONWETTING: the dispersed phase does not wet the
    walls)."""
    if Gw_mag is None:
        Gw_mag = GW_NONWETTING
    nx = length
    ny = W + 2 + side_len
    c = Case("tjunction", 2, (nx, ny, 1), (False, False, False), tuple(nu), G12,
             solid=None, rho0=None, Gw=(Gw_mag, -Gw_mag))
    x, y, _ = c.grid()
    main = (y >= 1) & (y <= W)
    side = (x >= x_side) & (x < x_side + side_width) & (y > W)
    fluid = main | side
    c.solid = (~fluid).astype(np.uint8)
    c.rho0 = _rho_from_mask(side, major, minor)
    down = (x >= x_side) & main
    c.u0 = _plug(c, [(main & ~down, 0, u_c),
                     (down, 0, u_c + u_d * side_width / W),
                     (side, 1, -u_d)])
    c.inlets = [
        inlet(0, 0, (0, 1, 0), (1, W + 1, 1), (minor, major), u_c, alpha_on),
        inlet(1, 1, (x_side, 0, 0), (x_side + side_width, 1, 1), (major, minor), u_d, alpha_on),
    ]
    c.outlet = outlet(0, 1, (0, 1, 0), (1, W + 1, 1), chi_on)
    c.meta.update(W=W, u_c=u_c, u_d=u_d, x_side=x_side, side_width=side_width)
    return c


# ---------------------------------------------------------------------------
# 3-D co-flow device (square channel, coaxial dispersed-phase inlet)
# ---------------------------------------------------------------------------

def coflow3d(length: int = 600, width: int = 120, inner: int = 30, u_c: float = 0.02,
             u_d: float = 0.005, nu_c: float = 0.067, M: float = 5.0, G12: float = 0.9,
             Gw_mag: float = 0.0, major: float = COEX_G09[0], minor: float = COEX_G09[1],
             alpha_on=True, chi_on=True) -> Case:
    """Square channel of ``width`` x ``width`` fluid nodes (one-node solid
    shell, so the box is length x (width+2) x (width+2)).  The x = 0 face is
    the continuous-phase inlet (u_c); an ``inner`` x ``inner`` patch centred on
    it carries the dispersed phase (u_d).  Dispersed viscosity M * nu_c."""
    n1 = width + 2
    c = Case("coflow3d", 3, (length, n1, n1), (False, False, False), (M * nu_c, nu_c), G12,
             solid=None, rho0=None, Gw=(Gw_mag, -Gw_mag))
    x, y, z = c.grid()
    solid = (y == 0) | (y == n1 - 1) | (z == 0) | (z == n1 - 1)
    c.solid = solid.astype(np.uint8)
    c.rho0 = _rho_from_mask(np.zeros(c.N, bool), major, minor)
    lo = 1 + (width - inner) // 2
    hi = lo + inner
    u_mean = (u_c * (width * width - inner * inner) + u_d * inner * inner) / (width * width)
    c.u0 = _plug(c, [(np.ones(c.N, bool), 0, u_mean)])
    c.inlets = [
        inlet(0, 0, (0, 1, 1), (1, n1 - 1, n1 - 1), (minor, major), u_c, alpha_on),
        inlet(0, 0, (0, lo, lo), (1, hi, hi), (major, minor), u_d, alpha_on),
    ]
    c.outlet = outlet(0, 1, (0, 1, 1), (1, n1 - 1, n1 - 1), chi_on)
    c.meta.update(width=width, inner=inner, u_c=u_c, u_d=u_d, M=M)
    return c


def coflow3d_quarter(**kw) -> Case:
    """The 1/4-scale copy of the co-flow device: 150 x 30 x 30 fluid, 8 x 8 inner patch."""
    return coflow3d(length=150, width=30, inner=8, **kw)


def coflow_cylinder(length: int = 600, R: int = 60, r_in: int = 15, t_wall: int = 7, L_cap: int = 60,
                    focus=None, u_c: float = 0.02, u_d: float = 0.005, nu_c: float = 0.067, M: float = 5.0,
                    G12: float = 0.9, major: float = COEX_G09[0], minor: float = COEX_G09[1],
                    alpha_on=True, chi_on=True) -> Case:
    """Coaxial co-flow device built from the cylinder equation (eq. 28): the
    fluid domain of the outer tube is y'^2 + z'^2 <= R^2 (y', z' measured from
    the tube axis), 0 <= x < length.  An inner capillary of inner radius r_in
    and wall thickness t_wall runs from the inlet face to x = L_cap; its wall
    (r_in < r <= r_in + t_wall) is solid.  The dispersed phase (component 1,
    viscosity M nu_c) enters through the capillary at u_d, the continuous
    phase through the annulus around it at u_c, and leaves through the
    outlet face x = length - 1.

    ``focus = (x0, L, R_f)`` adds the focused structure: an orifice of radius
    R_f over x0 <= x < x0 + L downstream of the capillary tip, where the
    outer flow is squeezed through the narrower throat.

    The box is length x (2R + 3) x (2R + 3) with the tube axis at the centre
    node, so one solid layer at least surrounds the tube.  Both inlets are
    rectangles on the x = 0 face (later patches take precedence): the whole
    face for the continuous phase, and the square of side 2 r_in + 1 around
    the axis for the dispersed phase, which holds only capillary-interior
    fluid nodes when t_wall >= (sqrt(2) - 1) r_in (its corners fall on the
    capillary wall).  The initial state is the phase layout at the plug
    velocity that carries the inlets' total flow through each cross-section."""
    if t_wall < (math.sqrt(2.0) - 1.0) * r_in:
        raise ValueError("t_wall must be at least (sqrt(2) - 1) r_in so that the square inner inlet patch "
                         "holds only capillary-interior nodes")
    if not (0 < r_in and r_in + t_wall < R and 2 <= L_cap < length - 2):
        raise ValueError("the capillary must fit inside the tube and end inside the box")
    n1 = 2 * R + 3
    c0 = R + 1
    c = Case("coflow_cylinder", 3, (length, n1, n1), (False, False, False), (M * nu_c, nu_c), G12,
             solid=None, rho0=None)
    x, y, z = c.grid()
    r2 = (y - c0) ** 2 + (z - c0) ** 2
    R_x = np.full(length, float(R))
    if focus is not None:
        x0, L, R_f = focus
        if not (L_cap < x0 and x0 + L < length - 2 and 0 < R_f < R):
            raise ValueError("the orifice must sit between the capillary tip and the outlet, narrower than R")
        R_x[x0:x0 + L] = R_f
    tube = r2 <= R_x[x] ** 2
    cap_wall = (x < L_cap) & (r2 > r_in ** 2) & (r2 <= (r_in + t_wall) ** 2)
    core = (x < L_cap) & (r2 <= r_in ** 2)
    c.solid = (~tube | cap_wall).astype(np.uint8)
    c.rho0 = _rho_from_mask(core, major, minor)
    # plug velocity carrying the inlets' flow through each cross-section
    face0 = (x == 0) & (c.solid == 0)
    A_core = int((face0 & (r2 <= r_in ** 2)).sum())
    A_ann = int(face0.sum()) - A_core
    Q = u_c * A_ann + u_d * A_core
    area = np.bincount(x[c.solid == 0], minlength=length).astype(float)
    u0 = np.zeros((3, c.N))
    u0[0] = Q / np.maximum(area[x], 1.0)
    u0[:, c.solid == 1] = 0.0
    c.u0 = u0
    c.inlets = [
        inlet(0, 0, (0, 0, 0), (1, n1, n1), (minor, major), u_c, alpha_on),
        inlet(0, 0, (0, c0 - r_in, c0 - r_in), (1, c0 + r_in + 1, c0 + r_in + 1), (major, minor), u_d, alpha_on),
    ]
    c.outlet = outlet(0, 1, (0, 0, 0), (1, n1, n1), chi_on)
    c.meta.update(R=R, r_in=r_in, t_wall=t_wall, L_cap=L_cap, focus=focus, u_c=u_c, u_d=u_d, M=M,
                  A_core=A_core, A_annulus=A_ann, width=2 * R + 1, inner=2 * r_in + 1)
    return c


def transpose(case: Case, axes) -> Case:
    """The same case with its lattice axes reordered: axis a of the result is
    axis ``axes[a]`` of ``case`` (a 3-D permutation).  Arrays, patches, the
    body force and the initial velocity components move with the axes."""
    assert case.dim == 3 and sorted(axes) == [0, 1, 2]
    inv = [axes.index(a) for a in range(3)]
    nx, ny, nz = case.n
    n_new = tuple(case.n[a] for a in axes)

    def field(v):                       # [N] in x-fastest order -> permuted
        g = v.reshape(nz, ny, nx)      # index [z, y, x] = axis order (2, 1, 0)
        g = g.transpose([2 - axes[2], 2 - axes[1], 2 - axes[0]])
        return np.ascontiguousarray(g).reshape(-1)

    def face(p):
        q = dict(p)
        q["axis"] = inv[p["axis"]]
        q["lo"] = tuple(p["lo"][a] for a in axes)
        q["hi"] = tuple(p["hi"][a] for a in axes)
        return q

    c = case.copy()
    c.name = f"{case.name}_T{''.join(map(str, axes))}"
    c.n = n_new
    c.periodic = tuple(case.periodic[a] for a in axes)
    c.solid = field(case.solid)
    c.rho0 = np.stack([field(r) for r in case.rho0])
    if case.u0 is not None:
        c.u0 = np.stack([field(case.u0[a]) for a in axes])
    c.Fb = tuple(case.Fb[a] for a in axes)
    if case.wall_u is not None:
        c.wall_u = np.stack([field(case.wall_u[a]) for a in axes])
    c.inlets = [face(p) for p in case.inlets]
    c.outlet = face(case.outlet) if case.outlet is not None else None
    return c


# ---------------------------------------------------------------------------
# Batched sweep of T-junctions (uneven sizes and physics)
# ---------------------------------------------------------------------------

# Interfacial tension of the G12 = 0.9 interface in lattice units, from the
# slope of the oracle's Laplace sweep (dp against 1/R over R = 10..20 on the
# 64 x 64 box, 2000 steps): the scale that turns a capillary number into a
# viscosity.  tests/test_oracle_physics.py re-measures it.
GAMMA_G09 = 0.0438


def sweep_params(n: int = 256, seed: int = 12934, W_range=(32, 128)):
    """Draws (W, Ca, q, M) per instance in a fixed order: W uniform integer in
    [W_range[0], W_range[1]], log10 Ca ~ U(-3, -1), q ~ U(0.1, 2),
    log10 M ~ U(log10 0.5, 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        W = int(rng.integers(W_range[0], W_range[1] + 1))
        Ca = 10.0 ** rng.uniform(-3.0, -1.0)
        q = rng.uniform(0.1, 2.0)
        M = 10.0 ** rng.uniform(np.log10(0.5), 1.0)
        out.append((W, Ca, q, M))
    return out


def sweep_case(W: int, Ca: float, q: float, M: float, gamma: float = GAMMA_G09, u_c: float = 0.01,
               tau_range=(0.55, 3.0), nu_d_max: float = 1.5) -> Case:
    """One T-junction of the sweep: main channel 8W x W, side channel of width
    W entering at x = 1.5W and W long.  Ca = u_c rho_c nu_c / gamma sets
    nu_c; if its relaxation time leaves tau_range the inlet velocity u_c moves
    (within [0.002, 0.05]) instead.  nu_d = M nu_c (capped at nu_d_max),
    u_d = q u_c (equal channel widths).  meta records every adjustment."""
    nu_lo, nu_hi = (tau_range[0] - 0.5) / 3.0, (tau_range[1] - 0.5) / 3.0
    nu_c = Ca * gamma / u_c
    clamped = []
    if nu_c < nu_lo or nu_c > nu_hi:
        nu_c = min(max(nu_c, nu_lo), nu_hi)
        u_c = Ca * gamma / nu_c
        if not 0.002 <= u_c <= 0.05:
            u_c = min(max(u_c, 0.002), 0.05)
            clamped.append("u_c")
    nu_d = M * nu_c
    if nu_d > nu_d_max:
        nu_d = nu_d_max
        clamped.append("nu_d")
    c = tjunction(W=W, length=8 * W, x_side=int(1.5 * W), side_width=W, side_len=W, u_c=u_c, u_d=q * u_c,
                  nu=(nu_d, nu_c))
    c.name = f"sweep_W{W}"
    c.meta.update(Ca=Ca, q=q, M=M, nu_c=nu_c, nu_d=nu_d, clamped=clamped)
    return c


def sweep(n: int = 256, seed: int = 12934, W_range=(32, 128), **kw):
    """The batched-sweep workload: n uneven T-junction instances."""
    return [sweep_case(*p, **kw) for p in sweep_params(n, seed, W_range)]
