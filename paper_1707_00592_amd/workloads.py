"""Seeded synthetic inputs for the WENO-IS solver.

This module builds initial conditions only: it turns primitive fields
(rho, velocity, p, gamma, Pinf) into the conservative layout both the HIP
library and the oracle take, and it draws the random problems.  It holds
none of the finite-volume method's arithmetic and imports neither the
library nor the oracle, so both sides can use it.

Conservative layout: float64 array (nc, ncells), x fastest, with components
(rho, rho*u[, rho*v[, rho*w]], E, Gamma, Pi), Gamma = 1/(gamma-1),
Pi = gamma*Pinf/(gamma-1) and E = Gamma p + Pi + rho |u|^2 / 2, the
stiffened-gas equation of state of the paper's Sec. 2, eq. (2).

Problems (arXiv:1707.00592 and the workloads built on it):
  * gas-liquid shock tube, Sec. 5.2 eq. (36) in SI units (water 1000 kg/m^3,
    1 GPa, gamma 4.4, Pinf 0.6 GPa | air 50 kg/m^3, 0.1 MPa), t = 240 us
  * interface transport, Sec. 5.1 eq. (35)
  * 1D shock/bubble in liquid, Sec. 5.3 eq. (37)
  * 2D shock-bubble: air cylinder in water hit by a 1 GPa water shock
    (the water/air case of Sec. 6.2 and Table 2 with the water EOS of
    Sec. 5.2)
  * 3D shock-droplet: water sphere in air hit by a Mach 2.4 air shock
  * the paper's other workloads: the 1D shock/droplet of Sec. 5.4, the
    air-R22 and air-He cylinders of Sec. 6.1 (Table 1) and the air-water
    droplet and water-air bubble of Sec. 6.2 (Table 2)
  * a batch of uneven two-phase shock tubes drawn with SplitMix64
  * smooth entropy waves (the Euler analogue of the advection tests of
    Sec. 4) and random face stencils for parity checks
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

WATER = (4.4, 6.0e8)   # (gamma, Pinf) of water, Sec. 5.2 eq. (36) in SI
AIR = (1.4, 0.0)


@dataclass
class Problem:
    """A grid plus an initial conservative state."""
    U: np.ndarray                 # (nc, ncells) float64
    n: tuple                      # cells per axis, x first
    dx: tuple                     # cell size per axis
    bc_lo: tuple
    bc_hi: tuple
    t_end: float | None = None
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def ncells(self) -> int:
        return int(np.prod(self.n))


# ----------------------------------------------------------------- EOS form
def material(gamma, pinf):
    """(Gamma, Pi) = (1/(gamma-1), gamma Pinf/(gamma-1))."""
    gamma = np.asarray(gamma, dtype=np.float64)
    pinf = np.asarray(pinf, dtype=np.float64)
    return 1.0 / (gamma - 1.0), gamma * pinf / (gamma - 1.0)


def prim_to_cons(rho, vel, p, gamma, pinf) -> np.ndarray:
    """Conservative SoA state from primitive fields (all flattened, x fastest)."""
    rho = np.asarray(rho, dtype=np.float64).ravel()
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64).ravel(), rho.shape) for v in vel]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64).ravel(), rho.shape)
    G, P = material(np.broadcast_to(np.asarray(gamma, dtype=np.float64).ravel(), rho.shape),
                    np.broadcast_to(np.asarray(pinf, dtype=np.float64).ravel(), rho.shape))
    ke = np.zeros_like(rho)
    for v in vel:
        ke = ke + v * v
    E = G * p + P + 0.5 * rho * ke
    comps = [rho] + [rho * v for v in vel] + [E, G, P]
    return np.ascontiguousarray(np.stack(comps))


def cons_to_prim(U: np.ndarray, ndim: int) -> dict:
    """Inverse of prim_to_cons, for reporting and initial-condition checks."""
    rho = U[0]
    vel = [U[1 + a] / rho for a in range(ndim)]
    ke = sum(v * v for v in vel)
    E, G, P = U[1 + ndim], U[2 + ndim], U[3 + ndim]
    p = (E - 0.5 * rho * ke - P) / G
    gamma = 1.0 + 1.0 / G
    pinf = P * (gamma - 1.0) / gamma
    return {"rho": rho, "vel": vel, "p": p, "gamma": gamma, "pinf": pinf}


def cell_centres(n: int, lo: float, hi: float) -> np.ndarray:
    dx = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * dx


# ------------------------------------------------------- shock relations
def sg_shock_from_pressure(rho0, p0, gamma, pinf, p1):
    """Post-shock (rho1, u1, S) behind a right-moving shock running into a
    stiffened gas at rest, from the Rankine-Hugoniot conditions written in
    the shifted pressure p + Pinf."""
    pb0, pb1 = p0 + pinf, p1 + pinf
    g = gamma
    rho1 = rho0 * ((g + 1) * pb1 + (g - 1) * pb0) / ((g - 1) * pb1 + (g + 1) * pb0)
    m2 = (p1 - p0) / (1.0 / rho0 - 1.0 / rho1)
    S = math.sqrt(m2) / rho0
    u1 = S * (1.0 - rho0 / rho1)
    return rho1, u1, S


def ideal_shock_from_mach(rho0, p0, gamma, M):
    """Post-shock (rho1, u1, p1, S) of a right-moving normal shock of Mach M
    into an ideal gas at rest."""
    g = gamma
    c0 = math.sqrt(g * p0 / rho0)
    S = M * c0
    rho1 = rho0 * (g + 1) * M * M / ((g - 1) * M * M + 2)
    p1 = p0 * (1 + 2 * g / (g + 1) * (M * M - 1))
    u1 = S * (1 - rho0 / rho1)
    return rho1, u1, p1, S


# --------------------------------------------------------------- 1D cases
def sod_gas_liquid(n: int = 200) -> Problem:
    """Water (1000, 0, 1e9, 4.4, 6e8) | air (50, 0, 1e5, 1.4, 0) at x = 0.7
    on [0, 1], to t = 2.4e-4 s, transmissive ends."""
    x = cell_centres(n, 0.0, 1.0)
    left = x < 0.7
    WL = (1000.0, 0.0, 1.0e9, WATER[0], WATER[1])
    WR = (50.0, 0.0, 1.0e5, AIR[0], AIR[1])
    rho = np.where(left, WL[0], WR[0])
    u = np.where(left, WL[1], WR[1])
    p = np.where(left, WL[2], WR[2])
    ga = np.where(left, WL[3], WR[3])
    pi = np.where(left, WL[4], WR[4])
    U = prim_to_cons(rho, [u], p, ga, pi)
    return Problem(U, (n,), (1.0 / n,), (0,), (0,), t_end=2.4e-4, name="sod_gas_liquid",
                   extra={"WL": WL, "WR": WR, "x0": 0.7, "x": x})


def interface_transport(n: int = 200) -> Problem:
    """Sec. 5.1 eq. (35): (1, 100, 1, 7, 3000) | (0.001, 100, 1, 1.4, 0),
    interface at x = 2 on [0, 4], t = 0.01."""
    x = cell_centres(n, 0.0, 4.0)
    left = x < 2.0
    rho = np.where(left, 1.0, 0.001)
    ga = np.where(left, 7.0, 1.4)
    pi = np.where(left, 3000.0, 0.0)
    U = prim_to_cons(rho, [np.full(n, 100.0)], np.ones(n), ga, pi)
    return Problem(U, (n,), (4.0 / n,), (0,), (0,), t_end=0.01, name="interface_transport",
                   extra={"x": x, "u0": 100.0, "p0": 1.0})


def shock_bubble_1d(n: int = 200) -> Problem:
    """Sec. 5.3 eq. (37), four states on [0, 1].  The printed final time
    3.87 is read in units of 1e-3 (the shock then has crossed the bubble)."""
    x = cell_centres(n, 0.0, 1.0)
    rho = np.select([x < 0.25, x < 0.4, x < 0.6], [1.2199, 1.0, 1e-3], 1.0)
    u = np.select([x < 0.25], [42.455], 0.0)
    p = np.select([x < 0.25], [1e4], 1.0)
    ga = np.select([x < 0.4, x < 0.6], [7.0, 1.4], 7.0)
    pi = np.select([x < 0.4, x < 0.6], [3.31e3, 0.0], 3.31e3)
    U = prim_to_cons(rho, [u], p, ga, pi)
    return Problem(U, (n,), (1.0 / n,), (0,), (0,), t_end=3.87e-3, name="shock_bubble_1d",
                   extra={"x": x})


def shock_droplet_1d(n: int = 200) -> Problem:
    """Sec. 5.4 eq. (38): a Mach 2 air shock at x = 0.016 running right into
    air at rest and a liquid layer 0.0176 < x < 0.0224 (gamma 1.932, Pinf
    1.1645e4) on [0, 0.04], in the units of eq. (38).  The printed final
    time 333 is read in units of 1e-6 (3.33e-4: the reflected shock is then
    back near the left end, as eq. (37)'s 3.87 is read in units of 1e-3)."""
    x = cell_centres(n, 0.0, 0.04)
    rho = np.select([x < 0.016, x < 0.0176, x < 0.0224], [3.2e-3, 1.2e-3, 1.0], 1.2e-3)
    u = np.select([x < 0.016], [44.59], 0.0)
    p = np.select([x < 0.016], [4.5], 1.0)
    drop = (x >= 0.0176) & (x < 0.0224)
    ga = np.where(drop, 1.932, 1.4)
    pi = np.where(drop, 1.1645e4, 0.0)
    U = prim_to_cons(rho, [u], p, ga, pi)
    return Problem(U, (n,), (0.04 / n,), (0,), (0,), t_end=3.33e-4, name="shock_droplet_1d",
                   extra={"x": x})


def entropy_wave(n, ndim: int = 1, amp: float = 0.2, pulse: bool = False) -> Problem:
    """Smooth density wave advected by a uniform flow (u = 1 along every
    axis, p = 1, air) on the periodic unit box: the Euler analogue of the
    linear-advection convergence tests of Sec. 4.  Cell averages of
    rho = 1 + amp*sin(2 pi sum x) (or of the Gauss pulse of eqs. (33)-(34)
    when pulse=True) are taken with 8-point Gauss-Legendre per axis."""
    ns = (n,) * ndim if np.ndim(n) == 0 else tuple(n)
    rho = exact_entropy_average(ns, 0.0, amp, pulse)
    vel = [np.ones(int(np.prod(ns)))] * ndim
    U = prim_to_cons(rho, vel, 1.0, AIR[0], AIR[1])
    return Problem(U, ns, tuple(1.0 / s for s in ns), (1,) * ndim, (1,) * ndim,
                   name="entropy_wave", extra={"amp": amp, "pulse": pulse})


def _density_profile(xs, t, amp, pulse):
    s = sum(xs) - t * len(xs)
    if pulse:
        r2 = 0
        for x in xs:
            d = np.mod(x - t, 1.0) - 0.5
            r2 = r2 + d * d
        return 1.0 + amp * np.exp(-300.0 * r2)
    return 1.0 + amp * np.sin(2.0 * np.pi * s)


def exact_entropy_average(ns, t, amp=0.2, pulse=False) -> np.ndarray:
    """Exact cell averages (8-point Gauss-Legendre per axis) of the
    translated entropy wave at time t; flattened, x fastest."""
    ndim = len(ns)
    gx, gw = np.polynomial.legendre.leggauss(8)
    grids = []
    for a in range(ndim):
        h = 1.0 / ns[a]
        xc = cell_centres(ns[a], 0.0, 1.0)
        grids.append(((xc[:, None] + 0.5 * h * gx[None, :]), 0.5 * gw))
    if ndim == 1:
        (x, w), = grids
        return (_density_profile([x], t, amp, pulse) * w).sum(axis=1)
    if ndim == 2:
        (x, wx), (y, wy) = grids
        X = x[None, :, None, :]           # [j, i, gy, gx]
        Y = y[:, None, :, None]
        W = wy[None, None, :, None] * wx[None, None, None, :]
        return (_density_profile([X, Y], t, amp, pulse) * W).sum(axis=(2, 3)).ravel()
    (x, wx), (y, wy), (z, wz) = grids
    X = x[None, None, :, None, None, :]
    Y = y[None, :, None, None, :, None]
    Z = z[:, None, None, :, None, None]
    W = wz[None, None, None, :, None, None] * wy[None, None, None, None, :, None] * \
        wx[None, None, None, None, None, :]
    return (_density_profile([X, Y, Z], t, amp, pulse) * W).sum(axis=(3, 4, 5)).ravel()


# --------------------------------------------------------------- 2D / 3D
def shock_bubble_2d(nx: int = 1024, ny: int = 512, radius: float = 0.25,
                    centre=(0.9, 0.5), x_shock: float = 0.5) -> Problem:
    """Air cylinder (1, 0, 1e5, 1.4, 0) of radius 0.25 (a quarter of the
    height) at (0.9, 0.5) in water at rest (1000, 0, 1e5, 4.4, 6e8) on
    [0, 2] x [0, 1]; a planar right-moving water shock at x = 0.5 with
    post-shock pressure 1e9.  Transmissive boundaries; sharp interface
    (each cell takes the material of its centre)."""
    h = 1.0 / ny
    x = cell_centres(nx, 0.0, nx * h)
    y = cell_centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y)                       # [j, i]
    rho1, u1, S = sg_shock_from_pressure(1000.0, 1e5, WATER[0], WATER[1], 1e9)
    bubble = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 < radius ** 2
    post = X < x_shock
    rho = np.where(bubble, 1.0, np.where(post, rho1, 1000.0))
    u = np.where(post & ~bubble, u1, 0.0)
    p = np.where(post & ~bubble, 1e9, 1e5)
    ga = np.where(bubble, AIR[0], WATER[0])
    pi = np.where(bubble, AIR[1], WATER[1])
    U = prim_to_cons(rho, [u, np.zeros_like(u)], p, ga, pi)
    return Problem(U, (nx, ny), (h, h), (0, 0), (0, 0), name="shock_bubble_2d",
                   extra={"post_shock": (rho1, u1, 1e9), "shock_speed": S, "Lx": nx * h})


def _cylinder_problem(nx, ny, Lx, Ly, centre, radius, x_shock, pre, post, inside,
                      bc, name, t_end):
    """A gas or liquid cylinder in a channel, hit by a planar shock coming
    from the right (the post-shock state fills x > x_shock).  States are
    (rho, u, p, gamma, Pinf); sharp interface."""
    h = Lx / nx
    x = cell_centres(nx, 0.0, Lx)
    y = cell_centres(ny, 0.0, Ly)
    X, Y = np.meshgrid(x, y)                       # [j, i]
    cyl = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 < radius ** 2
    sh = (X > x_shock) & ~cyl
    f = [np.where(cyl, inside[k], np.where(sh, post[k], pre[k])) for k in range(5)]
    U = prim_to_cons(f[0], [f[1], np.zeros_like(f[1])], f[2], f[3], f[4])
    return Problem(U, (nx, ny), (h, Ly / ny), bc[0], bc[1], t_end=t_end, name=name,
                   extra={"pre": pre, "post": post, "inside": inside, "centre": centre,
                          "radius": radius, "x_shock": x_shock})


def shock_gas_cylinder_2d(gas: str = "R22", nx: int = 3000, ny: int = 1000) -> Problem:
    """Sec. 6.1, Table 1 and its figure: a 267 mm x 89 mm channel (SI
    units), a 50 mm cylinder of R22 (4.415, gamma 1.249) or He (0.255,
    gamma 1.648) centred 178 mm from the left end, in air (1.4, 0, 1e5,
    1.4) hit by the Ms = 1.22 shock whose post-shock air (1.927, -114.42,
    1.57e5) fills the last 64 mm.  Walls (reflective) at the top and bottom,
    transmissive ends; MOOD off in the paper.  The table's values are used
    as printed (its post-shock velocity is about 8% above the Rankine-
    Hugoniot value of the other entries).  t_end: the time of the paper's
    last comparison image for each gas (190 us for R22, 245 us for He)."""
    inside = {"R22": (4.415, 0.0, 1e5, 1.249, 0.0), "He": (0.255, 0.0, 1e5, 1.648, 0.0)}[gas]
    return _cylinder_problem(nx, ny, 0.267, 0.089, (0.178, 0.0445), 0.025, 0.203,
                             (1.4, 0.0, 1e5, 1.4, 0.0), (1.927, -114.42, 1.57e5, 1.4, 0.0),
                             inside, ((0, 2), (0, 2)), f"shock_{gas}_cylinder_2d",
                             190e-6 if gas == "R22" else 245e-6)


def air_water_2d(case: str = "droplet", n: int = 800) -> Problem:
    """Sec. 6.2, Table 2 and its figure: a 20 mm x 20 mm box (SI units),
    an 8 mm cylinder centred at (12, 10) mm, hit by a shock whose
    post-shock state fills x > 16 mm.  case "droplet": water (1000, 0, 1e5,
    4.34, 4.84e8) in air (1.2, 0, 1e5, 1.4) hit by an Ms = 2 air shock
    (3.2, -434, 4.56e5), MOOD off in the paper, up to 800 x 800 cells;
    case "bubble": air (1, 0, 1e5, 1.4) in water (1000, 0, 1e5, 7, 3.31e8)
    hit by a 1 GPa water shock (1219.9, -424.55, 1e9), MOOD on, up to
    1600 x 1600 cells.  Non-reflecting (zero-gradient) boundaries."""
    if case == "droplet":
        pre, post = (1.2, 0.0, 1e5, 1.4, 0.0), (3.2, -434.0, 4.56e5, 1.4, 0.0)
        inside = (1000.0, 0.0, 1e5, 4.34, 4.84e8)
    else:
        pre, post = (1000.0, 0.0, 1e5, 7.0, 3.31e8), (1219.9, -424.55, 1e9, 7.0, 3.31e8)
        inside = (1.0, 0.0, 1e5, 1.4, 0.0)
    return _cylinder_problem(n, n, 0.02, 0.02, (0.012, 0.010), 0.004, 0.016, pre, post,
                             inside, ((0, 0), (0, 0)), f"air_water_{case}_2d", None)


def shock_droplet_3d(n: int = 256, radius_cells: float = 32.0, x_shock: float = 0.3,
                     mach: float = 2.4) -> Problem:
    """Water sphere (1000, 0, 1e5, 4.4, 6e8) of radius 32 cells (at 256^3)
    centred in the unit cube, in air (1, 0, 1e5, 1.4, 0), struck by a
    Mach 2.4 air shock starting at x = 0.3.  Transmissive boundaries."""
    h = 1.0 / n
    r = radius_cells / 256.0
    c = cell_centres(n, 0.0, 1.0)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")  # [k, j, i]
    rho1, u1, p1, S = ideal_shock_from_mach(1.0, 1e5, AIR[0], mach)
    drop = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2 < r ** 2
    post = X < x_shock
    rho = np.where(drop, 1000.0, np.where(post, rho1, 1.0))
    u = np.where(post & ~drop, u1, 0.0)
    p = np.where(post & ~drop, p1, 1e5)
    ga = np.where(drop, WATER[0], AIR[0])
    pi = np.where(drop, WATER[1], AIR[1])
    zero = np.zeros_like(u)
    U = prim_to_cons(rho, [u, zero, zero], p, ga, pi)
    return Problem(U, (n, n, n), (h, h, h), (0, 0, 0), (0, 0, 0), name="shock_droplet_3d",
                   extra={"post_shock": (rho1, u1, p1), "shock_speed": S})


# ------------------------------------------------------------ SplitMix64
class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood 2014): state += 0x9E3779B97F4A7C15,
    then the two xor-shift-multiply mixing rounds."""
    MASK = (1 << 64) - 1

    def __init__(self, seed: int):
        self.state = seed & self.MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & self.MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def randint(self, lo: int, hi: int) -> int:
        """Integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1))


def _cavitates(WL, WR) -> bool:
    """True when the two rarefactions of the exact solution would drive the
    shifted pressure of a side to zero (the pressure-positivity condition of
    the exact Riemann problem written in p + Pinf)."""
    pmin = -min(WL[4], WR[4])
    total = WR[1] - WL[1]
    for (rho, u, p, g, pinf) in (WL, WR):
        c = math.sqrt(g * (p + pinf) / rho)
        ratio = (pmin + pinf) / (p + pinf)
        total += 2.0 * c / (g - 1.0) * (ratio ** ((g - 1.0) / (2.0 * g)) - 1.0)
    return total >= 0.0


def batch_riemann(nprob: int = 4096, seed: int = 1707, nmin: int = 128, nmax: int = 4096):
    """Independent two-phase shock tubes of uneven length.

    Per problem: N ~ U{nmin..nmax}; left and right states drawn
    independently with rho log-uniform in [1, 1000], p log-uniform in
    [1e5, 1e9], u uniform in [-100, 100], material water or air with
    probability 1/2; interface uniform in [0.3, 0.7] of the unit interval;
    dx = 1/N.  A draw whose exact solution would cavitate is redrawn.
    Returns dict(U (5, total), offsets (nprob+1,), dx (nprob,), states)."""
    rng = SplitMix64(seed)
    sizes, states, x0s = [], [], []
    for _ in range(nprob):
        n = rng.randint(nmin, nmax)
        while True:
            side = []
            for _s in range(2):
                rho = 10.0 ** (3.0 * rng.uniform())
                p = 10.0 ** (5.0 + 4.0 * rng.uniform())
                u = -100.0 + 200.0 * rng.uniform()
                mat = WATER if rng.uniform() < 0.5 else AIR
                side.append((rho, u, p, mat[0], mat[1]))
            x0 = 0.3 + 0.4 * rng.uniform()
            if not _cavitates(side[0], side[1]):
                break
        sizes.append(n); states.append(tuple(side)); x0s.append(x0)
    return batch_from_states(sizes, states, x0s)


def batch_from_states(sizes, states, x0s):
    """Shock tubes on [0, 1] stored back to back: problem k has sizes[k]
    cells (dx = 1/N), the states ((rho, u, p, gamma, pinf) left, right) =
    states[k] and its interface at x0s[k]."""
    nprob = len(sizes)
    offsets = np.zeros(nprob + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    rho = np.empty(total); u = np.empty(total); p = np.empty(total)
    ga = np.empty(total); pi = np.empty(total)
    for k, (n, (WL, WR), x0) in enumerate(zip(sizes, states, x0s)):
        x = cell_centres(n, 0.0, 1.0)
        sl = slice(offsets[k], offsets[k + 1])
        left = x < x0
        for arr, idx in ((rho, 0), (u, 1), (p, 2), (ga, 3), (pi, 4)):
            arr[sl] = np.where(left, WL[idx], WR[idx])
    U = prim_to_cons(rho, [u], p, ga, pi)
    dx = 1.0 / np.asarray(sizes, dtype=np.float64)
    return {"U": U, "offsets": offsets, "dx": dx, "states": list(states), "x0": np.asarray(x0s),
            "sizes": np.asarray(sizes)}


# ------------------------------------------------- random parity inputs
def random_two_phase(n, seed: int = 0, smooth: float = 0.5) -> Problem:
    """Random physical state on a grid of shape n (x first): water and air
    regions separated by a random interface, plus smooth perturbations and
    random jumps in rho, u, p.  Transmissive boundaries."""
    rs = np.random.default_rng(seed)
    ns = tuple(n)
    ndim = len(ns)
    coords = np.meshgrid(*[cell_centres(m, 0.0, 1.0) for m in ns[::-1]], indexing="ij")
    coords = coords[::-1]                      # x, y, z arrays shaped [k, j, i]
    phase = np.zeros(coords[0].shape)
    for a in range(ndim):
        phase = phase + rs.uniform(-1, 1) * np.sin(2 * np.pi * (rs.uniform(0.5, 2.0) * coords[a]
                                                                 + rs.uniform()))
    water = phase > 0
    pert = np.zeros_like(phase)
    for a in range(ndim):
        pert = pert + np.sin(2 * np.pi * rs.uniform(1, 3) * coords[a] + rs.uniform(0, 6))
    jump = np.where(coords[0] < rs.uniform(0.3, 0.7), 1.0, 0.0)
    rho = np.where(water, 1000.0 * (1 + 0.1 * smooth * pert + 0.2 * jump),
                   1.0 * (1 + 0.3 * smooth * pert + 1.0 * jump))
    p = 1e5 * (1 + 0.5 * smooth * pert ** 2 + 20.0 * jump)
    vel = [rs.uniform(-50, 50) + 30 * smooth * np.sin(2 * np.pi * coords[(a + 1) % ndim])
           + 50 * jump for a in range(ndim)]
    ga = np.where(water, WATER[0], AIR[0])
    pi = np.where(water, WATER[1], AIR[1])
    U = prim_to_cons(rho.ravel(), [v.ravel() for v in vel], p.ravel(), ga.ravel(), pi.ravel())
    return Problem(U, ns, tuple(1.0 / m for m in ns), (0,) * ndim, (0,) * ndim,
                   name="random_two_phase")
