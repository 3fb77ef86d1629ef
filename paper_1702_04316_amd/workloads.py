"""Seeded synthetic workloads for the HEVI step.

This module only builds inputs: grids, time-step sizes and initial states.
It holds none of the step's arithmetic; both the GPU library and the CPU
oracle receive the same float64 arrays from it.

The paper's own test cases (rising thermal bubbles, the acoustic wave on the
cubed sphere) are not reproduced; seeded boxes with the same structure stand
in for them: a hydrostatic, neutral background with theta0 = 300 K, smooth
potential-temperature bumps in hydrostatic pressure balance, LGL order 4 and
about ten vertical elements per column.

Two readings of the Courant numbers are provided (the literal boxes make the
explicit horizontal Courant number 15 or more, which no HEVI scheme can run):
  R1 (primary): keep the element counts, N, the height and the vertical
      Courant number; stretch the horizontal extent (and each bump's
      horizontal radius) by s so that the horizontal Courant number is 0.4.
  R2 (literal box): keep the box; dt from horizontal Courant number 0.4.
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np
from numpy.polynomial import legendre as _leg

# Physical constants of the synthetic atmosphere (passed to both sides).
CP = 1004.67
RGAS = 287.17
P00 = 1.0e5
GRAV = 9.80616
THETA0 = 300.0


@dataclass
class Grid:
    lx: float
    ly: float
    lz: float
    nex: int
    ney: int
    nez: int
    N: int
    zface: Optional[np.ndarray] = None

    @property
    def nx(self):
        return self.nex * self.N

    @property
    def ny(self):
        return self.ney * self.N

    @property
    def nz(self):
        return self.nez * self.N + 1

    @property
    def shape(self):
        return (5, self.nz, self.ny, self.nx)

    @property
    def n_unique(self):
        return self.nx * self.ny * self.nz

    @property
    def n_local(self):
        return self.nex * self.ney * self.nez * (self.N + 1) ** 3

    def faces(self):
        if self.zface is not None:
            return np.asarray(self.zface, dtype=np.float64)
        return self.lz * np.arange(self.nez + 1) / self.nez


@dataclass
class Background:
    theta0: float = THETA0
    p00: float = P00
    cp: float = CP
    rgas: float = RGAS
    grav: float = GRAV
    nbv: float = 0.0  # Brunt-Vaisala frequency [1/s]; 0: isentropic


@dataclass
class Workload:
    name: str
    grid: Grid
    dt: float
    nsteps: int
    seed: int
    nbumps: int
    amp: Tuple[float, float]
    radius: Tuple[float, float]
    stretch: float = 1.0
    background: Background = field(default_factory=Background)
    wind: Tuple[float, float] = (0.0, 0.0)  # uniform (u, v) of the initial state


def sound_speed(bg=None):
    bg = bg or Background()
    gamma = bg.cp / (bg.cp - bg.rgas)
    return float(np.sqrt(gamma * bg.rgas * bg.theta0))


def lgl_nodes(N):
    """LGL nodes on [-1, 1] from numpy's Legendre routines (input sampling only)."""
    inner = _leg.Legendre.basis(N).deriv().roots()
    return np.concatenate(([-1.0], np.sort(inner.real), [1.0]))


def node_coords(grid):
    """Unique-node coordinates x[nx], y[ny], z[nz] (x, y periodic: x = lx is node 0)."""
    xi = lgl_nodes(grid.N)
    hx = grid.lx / grid.nex
    hy = grid.ly / grid.ney
    x = np.array([ex * hx + (xi[a] + 1.0) * hx / 2.0 for ex in range(grid.nex) for a in range(grid.N)])
    y = np.array([ey * hy + (xi[b] + 1.0) * hy / 2.0 for ey in range(grid.ney) for b in range(grid.N)])
    zf = grid.faces()
    z = np.empty(grid.nz)
    for ez in range(grid.nez):
        for c in range(grid.N + 1):
            z[ez * grid.N + c] = zf[ez] + (xi[c] + 1.0) * (zf[ez + 1] - zf[ez]) / 2.0
    return x, y, z


def min_spacing_factor(N):
    """Smallest LGL spacing on [-1, 1], as a fraction of the element width."""
    xi = lgl_nodes(N)
    return float(np.min(np.diff(xi))) / 2.0


def dt_for_courant(grid, courant, axis, bg=None):
    """dt with C = c0 dt / dx_min (the Courant number of the introduction)."""
    c0 = sound_speed(bg)
    f = min_spacing_factor(grid.N)
    if axis == "z":
        h = float(np.min(np.diff(grid.faces())))
    elif axis == "x":
        h = grid.lx / grid.nex
    else:
        h = grid.ly / grid.ney
    return courant * f * h / c0


def _bumps(rng, nb, lx, ly, lz, amp, radius):
    out = []
    for _ in range(nb):
        fx, fy, fz = rng.uniform(0.0, 1.0), rng.uniform(0.0, 1.0), rng.uniform(0.0, 1.0)
        A = rng.uniform(amp[0], amp[1])
        r = rng.uniform(radius[0], radius[1])
        out.append((fx * lx, fy * ly, fz * lz, A, r))
    return out


def _theta_bumps(grid, bumps, stretch):
    x, y, z = node_coords(grid)
    th = np.zeros((grid.nz, grid.ny, grid.nx))
    X = x[None, None, :]
    Y = y[None, :, None]
    Z = z[:, None, None]
    for (xm, ym, zm, A, r) in bumps:
        rh = stretch * r
        dz = Z - zm
        # sum over periodic images so the field is smooth across x = 0 and y = 0
        gx = sum(np.exp(-((X - xm + m * grid.lx) / rh) ** 2) for m in range(-2, 3))
        gy = sum(np.exp(-((Y - ym + m * grid.ly) / rh) ** 2) for m in range(-2, 3))
        th = th + A * gx * gy * np.exp(-dz * dz / (r * r))
    return th


def hydrostatic_profile(z, bg=None):
    """theta0(z) and the hydrostatic density at heights z of the background
    the initial states are built on: theta0 constant (bg.nbv = 0) or
    theta0 exp(nbv^2 z/g), with d pi/dz = -g/(cp theta0) integrated in
    closed form and rho = p00 pi^(cv/R)/(R theta0)."""
    bg = bg or Background()
    z = np.asarray(z, dtype=np.float64)
    cv = bg.cp - bg.rgas
    if bg.nbv > 0.0:
        S = bg.nbv ** 2 / bg.grav
        th = bg.theta0 * np.exp(S * z)
        pi = 1.0 + bg.grav * np.expm1(-S * z) / (bg.cp * bg.theta0 * S)
    else:
        th = np.full_like(z, bg.theta0)
        pi = 1.0 - bg.grav * z / (bg.cp * bg.theta0)
    return th, bg.p00 * pi ** (cv / bg.rgas) / (bg.rgas * th)


def balanced_density(grid, theta_p, bg=None):
    """rho' that keeps the hydrostatic pressure unperturbed for a given theta'.

    Initial-condition recipe: with P held at its hydrostatic value, rho theta
    is unchanged, so rho' = -rho_hyd theta'/(theta0 + theta').
    """
    bg = bg or Background()
    _, _, z = node_coords(grid)
    th, rho_h = hydrostatic_profile(z, bg)
    return -rho_h[:, None, None] * theta_p / (th[:, None, None] + theta_p)


def make_initial_state(wl: Workload):
    """Seeded initial state (5, nz, ny, nx): theta' bumps, balanced rho', the
    workload's uniform wind (u, v), w = 0.

    Bump m: A_m exp(-((x-x_m)^2 + (y-y_m)^2)/(s r_m)^2 - (z-z_m)^2/r_m^2), summed
    over periodic images in x and y; centre drawn uniformly in the box, then
    A_m and r_m uniformly in their ranges (numpy PCG64, in that order)."""
    g = wl.grid
    rng = np.random.default_rng(wl.seed)
    bumps = _bumps(rng, wl.nbumps, g.lx, g.ly, g.lz, wl.amp, wl.radius)
    q = np.zeros(g.shape)
    q[4] = _theta_bumps(g, bumps, wl.stretch)
    q[0] = balanced_density(g, q[4], wl.background)
    q[1] = wl.wind[0]
    q[2] = wl.wind[1]
    return q


def make_random_state(grid, seed, wind=10.0, theta_amp=1.0, smooth=True):
    """A generic state for operator parity: theta' bumps, balanced-free rho',
    random winds; w vanishes on the bottom and top levels.

    smooth=False adds node-wise noise (parity of the discrete operators does
    not need smooth data)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = grid.nz, grid.ny, grid.nx
    x, y, z = node_coords(grid)
    X = x[None, None, :] / grid.lx
    Y = y[None, :, None] / grid.ly
    Z = z[:, None, None] / grid.lz
    q = np.zeros(grid.shape)

    def wave():
        kx, ky = rng.integers(0, 3, size=2)
        kz = rng.uniform(0.5, 2.0)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        return (np.cos(2 * np.pi * kx * X + ph[0]) * np.cos(2 * np.pi * ky * Y + ph[1])
                * np.cos(np.pi * kz * Z + ph[2]))

    q[0] = 1e-3 * wave()
    q[1] = wind * wave()
    q[2] = wind * wave()
    q[3] = 0.2 * wind * wave() * np.sin(np.pi * Z)
    q[4] = theta_amp * wave()
    if not smooth:
        noise = rng.standard_normal(grid.shape)
        q[0] += 1e-4 * noise[0]
        q[1] += 0.5 * noise[1]
        q[2] += 0.5 * noise[2]
        q[3] += 0.1 * noise[3]
        q[4] += 0.1 * noise[4]
    q[3, 0] = 0.0
    q[3, -1] = 0.0
    return q


def random_zface(nez, lz, seed):
    """Non-uniform element faces (heights between 0.5 and 1.5 of uniform)."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.5, 1.5, size=nez)
    zf = np.concatenate(([0.0], np.cumsum(h)))
    zf = zf * (lz / zf[-1])
    zf[-1] = lz
    return zf


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

C_VERT = 15.0
C_HORIZ = 0.4


def _stretch(lx, nex, lz, nez):
    # s * (lx/nex) = (C_VERT / C_HORIZ) * (lz/nez): horizontal Courant number 0.4
    return (C_VERT / C_HORIZ) * (lz / nez) * nex / lx


def box_small(reading="R1"):
    """4x4x4 elements, N=4, 1 km cube (literal), one 0.5 K bump of radius 250 m, 10 steps."""
    lx = ly = lz = 1000.0
    nex = ney = nez = 4
    s = _stretch(lx, nex, lz, nez) if reading == "R1" else 1.0
    g = Grid(lx * s, ly * s, lz, nex, ney, nez, 4)
    if reading == "R1":
        dt = dt_for_courant(g, C_VERT, "z")
    else:
        dt = dt_for_courant(g, C_HORIZ, "x")
    return Workload(f"box4x4x4_N4_{reading}", g, dt, 10, 1, 1, (0.5, 0.5), (250.0, 250.0), stretch=s)


def box_large(reading="R1", nex=64, ney=64):
    """64x64x10 elements, N=4, 20x20x10 km (literal), eight bumps 0.1-2 K,
    radius 0.5-2 km, 100 steps.  nex/ney may be reduced for a sub-box with
    the same element shape, order and dt."""
    lx = ly = 20000.0
    lz = 10000.0
    nez = 10
    s = _stretch(lx, 64, lz, nez) if reading == "R1" else 1.0
    hx = lx * s / 64
    g = Grid(hx * nex, hx * ney, lz, nex, ney, nez, 4)
    if reading == "R1":
        dt = dt_for_courant(g, C_VERT, "z")
    else:
        dt = dt_for_courant(g, C_HORIZ, "x")
    return Workload(f"box{nex}x{ney}x10_N4_{reading}", g, dt, 100, 2, 8, (0.1, 2.0), (500.0, 2000.0),
                    stretch=s)


def box_precision(size="small", reading="R1"):
    """Workloads of the precision form at N=7 (8x8x8 nodes per element):
    'small', 4x4x4 elements of the 1 km cube, one 0.5 K bump of radius
    250 m, for errors against the oracle; 'large', 28x28x28 elements
    (196x196x197 = 7,567,952 unique nodes, 11.2M element-local), eight
    bumps, for throughput.  Vertical Courant number 15; under R1 the
    horizontal extent is stretched to a horizontal Courant number of 0.4."""
    lx = ly = lz = 1000.0
    ne = 4 if size == "small" else 28
    s = _stretch(lx, ne, lz, ne) if reading == "R1" else 1.0
    g = Grid(lx * s, ly * s, lz, ne, ne, ne, 7)
    if reading == "R1":
        dt = dt_for_courant(g, C_VERT, "z")
    else:
        dt = dt_for_courant(g, C_HORIZ, "x")
    if size == "small":
        return Workload(f"box4x4x4_N7_{reading}", g, dt, 100, 1, 1, (0.5, 0.5), (250.0, 250.0), stretch=s)
    return Workload(f"box28x28x28_N7_{reading}", g, dt, 100, 3, 8, (0.1, 2.0), (50.0, 200.0), stretch=s)


NBV = 0.01  # Brunt-Vaisala frequency of the stratified workloads [1/s]


def box_stratified(size="small"):
    """The stratified-background workloads: the 4x4x4, N=4 box of
    box_small('R1') ('small') or the 64x64x10, N=4 box of box_large('R1')
    ('large') over theta0(z) = 300 K exp(Nb^2 z/g) with Nb = 0.01/s (a
    typical tropospheric stratification), same bumps, dt and steps."""
    wl = box_small("R1") if size == "small" else box_large("R1")
    bg = Background(nbv=NBV)
    name = wl.name.replace("_R1", "_strat")
    return Workload(name, wl.grid, wl.dt, wl.nsteps, wl.seed, wl.nbumps, wl.amp, wl.radius,
                    stretch=wl.stretch, background=bg, wind=wl.wind)


def ensemble_domains(seed=4, n=16):
    """An ensemble of n domains drawn per seed: square horizontal grids of
    16..64 elements per axis, 6..16 vertical elements, N in {3, 4, 5, 7},
    1..8 theta' bumps (0.1..2 K, 0.5..2 km), a uniform wind of 0..20 m/s in
    a random direction; the 20 x 20 x 10 km box of the 64x64x10 workload
    with vertical Courant number 15 and, under R1, the horizontal extent
    stretched so that the horizontal Courant number with c0 + |u| is 0.4."""
    rng = np.random.default_rng(seed)
    c0 = sound_speed()
    out = []
    for d in range(n):
        ne = int(rng.integers(16, 65))
        nez = int(rng.integers(6, 17))
        N = int(rng.choice([3, 4, 5, 7]))
        speed = float(rng.uniform(0.0, 20.0))
        ang = float(rng.uniform(0.0, 2.0 * np.pi))
        nb = int(rng.integers(1, 9))
        lx, lz = 20000.0, 10000.0
        s = _stretch(lx, ne, lz, nez) * (c0 + speed) / c0
        g = Grid(lx * s, lx * s, lz, ne, ne, nez, N)
        dt = dt_for_courant(g, C_VERT, "z")
        out.append(Workload(f"ens{d}_{ne}x{ne}x{nez}_N{N}", g, dt, 50, 100 * seed + d, nb, (0.1, 2.0),
                            (500.0, 2000.0), stretch=s, wind=(speed * np.cos(ang), speed * np.sin(ang))))
    return out


def ensemble_small_domains(seed=7):
    """One domain per order N in {3, 4, 5, 7} drawn like ensemble_domains
    (vertical elements spanning 6..16, a uniform wind of 0..20 m/s in a
    random direction, 1..3 theta' bumps, vertical Courant number 15 and the
    horizontal extent stretched to a horizontal Courant number of 0.4 with
    c0 + |u|), on 3..4 horizontal elements per axis so that the oracle can
    step every domain.  Bumps of 0.1..1 K with radii of 1..2 km: with the
    ensemble's 0.5..2 km radii some of these small periodic boxes sum the
    bump's images into a layer of theta' decreasing with height several
    kelvin deep, statically unstable over the neutral background, which
    convects within 50..70 steps (in the oracle as on the GPU) and turns
    rounding differences into exponentially growing ones."""
    rng = np.random.default_rng(seed)
    c0 = sound_speed()
    out = []
    for d, (N, nez) in enumerate(((3, 6), (4, 10), (5, 13), (7, 16))):
        ne = int(rng.integers(3, 5))
        speed = float(rng.uniform(0.0, 20.0))
        ang = float(rng.uniform(0.0, 2.0 * np.pi))
        nb = int(rng.integers(1, 4))
        lx, lz = 20000.0 * ne / 64, 10000.0
        s = _stretch(lx, ne, lz, nez) * (c0 + speed) / c0
        g = Grid(lx * s, lx * s, lz, ne, ne, nez, N)
        dt = dt_for_courant(g, C_VERT, "z")
        out.append(Workload(f"ens_small{d}_{ne}x{ne}x{nez}_N{N}", g, dt, 50, 100 * seed + d, nb, (0.1, 1.0),
                            (1000.0, 2000.0), stretch=s, wind=(speed * np.cos(ang), speed * np.sin(ang))))
    return out


IMEX3D_COURANT = 15.0
IMEX3D_TOL = 1e-8


def box_imex3d(size="full"):
    """Workloads of the 3D-IMEX step: N=5, elements of 625 x 625 x 1250 m
    (the 20 x 20 x 10 km box in 32 x 32 x 8 elements, literal, no
    stretching); dt at acoustic Courant number 15 on the smallest node
    spacing of any direction (here horizontal, so the horizontal acoustics
    are stiff as well, which HEVI cannot step).  'full': 32x32x8 elements
    (160x160x41 = 1,049,600 unique nodes), eight theta' bumps 0.1-2 K of
    radius 0.5-2 km; 'small': 4x4x2 elements (20x20x11 nodes), one 0.5 K
    bump of radius 500 m, for parity with the oracle."""
    ne, nez = (32, 8) if size == "full" else (4, 2)
    hx, hz = 20000.0 / 32, 10000.0 / 8
    g = Grid(hx * ne, hx * ne, hz * nez, ne, ne, nez, 5)
    dt = min(dt_for_courant(g, IMEX3D_COURANT, "x"), dt_for_courant(g, IMEX3D_COURANT, "z"))
    if size == "full":
        return Workload("box32x32x8_N5_3d", g, dt, 10, 5, 8, (0.1, 2.0), (500.0, 2000.0))
    return Workload("box4x4x2_N5_3d", g, dt, 10, 5, 1, (0.5, 0.5), (500.0, 500.0))
