"""Seeded synthetic scenario generators.

This module only draws random numbers and fills in problem data (mesh box,
per-cell material draws, boundary-condition and source descriptions).  It
contains none of the finite-element method's arithmetic, so both the GPU
library binding and the CPU oracle consume exactly the same arrays.

Conventions (shared vocabulary, not method):

* z points up; the top of the box is ``origin[2] + extent[2]``.
* Per-cell arrays are lexicographic with x fastest: ``c = i + nx*(j + ny*k)``.
* Node arrays (degree p) are lexicographic with x fastest over
  ``(p*nx+1) x (p*ny+1) x (p*nz+1)`` equispaced nodes.
* Faces are numbered 0..5 = x-, x+, y-, y+, z-, z+.
* Temperatures are in kelvin, pressures in pascal.

A *time function* is the 8-tuple ``(kind, c0, cx, cy, cz, amp, period, phase)``
whose value at point (x, y, z) and time t is
``c0 + cx*x + cy*y + cz*z + amp*w(t)`` with ``w = 0`` (kind 0),
``w = sin(2*pi*t/period + phase)`` (kind 1) or the square wave
``w = +1 if sin(2*pi*t/period + phase) >= 0 else -1`` (kind 2).

The concrete parameter choices follow the paper's workloads: layered soil
with per-layer material classes (Section 3.3, Table 3), a hydrostatic
pressure field plus a regional gradient (Section 3.3), energy piles on a
regular spacing with seasonal loading (Sections 3.2-3.3) and an injection
well (Section 2 benchmark, Table 1).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

PRESSURE = 0
TEMPERATURE = 1

DIRICHLET = 0
NEUMANN = 1

TF_CONST = 0
TF_SIN = 1
TF_SQUARE = 2

LINE_HEAT = 0   # rate in W per metre of line
LINE_WELL = 1   # rate in m^3/s for the whole screened interval

DAY = 86400.0
T15C = 288.15


def timefn(c0=0.0, cx=0.0, cy=0.0, cz=0.0, amp=0.0, period=1.0, phase=0.0,
           kind=TF_CONST) -> Tuple:
    return (int(kind), float(c0), float(cx), float(cy), float(cz),
            float(amp), float(period), float(phase))


@dataclass
class FaceBC:
    field: int
    face: int
    kind: int
    value: Tuple


@dataclass
class LineSource:
    x: float
    y: float
    z0: float
    z1: float
    kind: int
    rate: Tuple
    T_inj: float = 0.0


@dataclass
class DirColumn:
    field: int
    x: float
    y: float
    z0: float
    z1: float
    value: Tuple


@dataclass
class Scenario:
    name: str
    origin: Tuple[float, float, float]
    extent: Tuple[float, float, float]
    ncells: Tuple[int, int, int]
    degree: int
    permeability: Optional[np.ndarray]   # K_i [m^2], per cell (None: hydraulic_conductivity)
    porosity: Optional[np.ndarray]       # per cell (None: bulk thermal values given)
    lambda_solid: Optional[np.ndarray]   # W/m/K, per cell
    rhoc_solid: Optional[np.ndarray]     # J/m^3/K, per cell
    rho_w: float = 1000.0
    mu_w: float = 1.0e-3
    c_w: float = 4.18e6
    lambda_w: float = 0.6
    g: float = 9.81
    B_poro: float = 1.0e5             # <= 0 selects the steady pressure equation
    heat_source: Optional[np.ndarray] = None   # W/m^3 per cell
    # Site tables may give hydraulic conductivity K [m/s] and the bulk (soil +
    # water) conductivity and heat capacity directly; when set they are used
    # in place of permeability and the mixture of solid and water values.
    hydraulic_conductivity: Optional[np.ndarray] = None
    lambda_bulk: Optional[np.ndarray] = None
    rhoc_bulk: Optional[np.ndarray] = None
    # Graded (rectilinear) meshes: cell-edge coordinates per axis (ncells + 1
    # increasing values spanning the box); None = uniform spacing.
    edges: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None
    # General hexahedra of the box topology: coordinates of every node,
    # [nnode][3] with x fastest; None = box geometry.
    coords: Optional[np.ndarray] = None
    bcs: List[FaceBC] = field(default_factory=list)
    lines: List[LineSource] = field(default_factory=list)
    dir_columns: List[DirColumn] = field(default_factory=list)
    P0: Tuple = timefn()              # initial pressure (time function at t=0)
    T0: Tuple = timefn(T15C)          # initial temperature
    P0_steady: bool = False           # initial pressure = steady solution
    dt: float = DAY
    n_steps: int = 1
    t0: float = 0.0

    @property
    def ncell(self) -> int:
        nx, ny, nz = self.ncells
        return nx * ny * nz

    @property
    def nodes_per_dim(self) -> Tuple[int, int, int]:
        p = self.degree
        return tuple(p * n + 1 for n in self.ncells)

    @property
    def nnode(self) -> int:
        a, b, c = self.nodes_per_dim
        return a * b * c

    def replace(self, **kw) -> "Scenario":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------- helpers
def hydrostatic(s_top_z: float, p_top: float, rho_w: float, g: float,
                grad_x: float = 0.0, x_ref: float = 0.0) -> Tuple:
    """p = p_top + rho*g*(z_top - z) + rho*g*grad_x*(x_ref - x)."""
    rg = rho_w * g
    return timefn(c0=p_top + rg * s_top_z + rg * grad_x * x_ref,
                  cx=-rg * grad_x, cz=-rg)


def _cell_centres_z(origin, extent, ncells):
    nz = ncells[2]
    hz = extent[2] / nz
    return origin[2] + (np.arange(nz) + 0.5) * hz


def layered_lognormal(rng, origin, extent, ncells, n_layers, mean_lo=-12.0,
                      mean_hi=-10.0, sd=0.5, phi_lo=0.2, phi_hi=0.35):
    """Horizontal layers with per-layer mean log10 permeability and i.i.d.
    per-cell lognormal scatter; porosity uniform per cell."""
    nx, ny, nz = ncells
    zc = _cell_centres_z(origin, extent, ncells) - origin[2]
    layer_h = extent[2] / n_layers
    layer = np.minimum((zc / layer_h).astype(np.int64), n_layers - 1)
    means = rng.uniform(mean_lo, mean_hi, size=n_layers)
    logk = means[layer][:, None, None] + sd * rng.standard_normal((nz, ny, nx))
    perm = np.power(10.0, logk).reshape(-1)
    phi = rng.uniform(phi_lo, phi_hi, size=nx * ny * nz)
    return perm, phi


def _uniform(nc, v):
    return np.full(nc, float(v))


def graded_edges(lo: float, hi: float, n: int, fine=(), ratio: float = 3.0,
                 blend: float = 0.1) -> np.ndarray:
    """n + 1 cell edges on [lo, hi], cells about `ratio` times smaller inside
    the intervals `fine` (list of (a, b)) than elsewhere, with smooth
    transitions `blend` * (hi - lo) wide: the edges are equal quantiles of the
    mesh density 1 + (ratio - 1) * window(x)."""
    xs = np.linspace(lo, hi, 20001)
    rho = np.ones_like(xs)
    w = max(blend * (hi - lo), 1e-12)
    for a, b in fine:
        up = 0.5 * (1.0 + np.tanh((xs - a) / (0.25 * w)))
        down = 0.5 * (1.0 - np.tanh((xs - b) / (0.25 * w)))
        rho += (ratio - 1.0) * up * down
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (rho[1:] + rho[:-1]) * np.diff(xs))])
    cdf /= cdf[-1]
    e = np.interp(np.linspace(0.0, 1.0, n + 1), cdf, xs)
    e[0], e[-1] = lo, hi
    return e


# ----------------------------------------------------------------- configs
def config1(seed: int = 1) -> Scenario:
    """100 m cube, 16^3 Q1, homogeneous medium, steady Darcy pressure with a
    1e4 Pa drop across x, ten daily heat steps with a random 2x2x2-cell heat
    source block and 15 C Dirichlet on every face."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = (16, 16, 16)
    origin, extent = (0.0, 0.0, 0.0), (100.0, 100.0, 100.0)
    nc = n[0] * n[1] * n[2]
    s = Scenario("c1", origin, extent, n, 1,
                 permeability=_uniform(nc, 1e-12), porosity=_uniform(nc, 0.3),
                 lambda_solid=_uniform(nc, 2.5), rhoc_solid=_uniform(nc, 2.0e6),
                 B_poro=0.0, dt=DAY, n_steps=10)
    p_hyd = hydrostatic(100.0, 1.0e5, s.rho_w, s.g)
    p_hi = (p_hyd[0], p_hyd[1] + 1.0e4) + p_hyd[2:]
    s.bcs = [FaceBC(PRESSURE, 0, DIRICHLET, p_hi),
             FaceBC(PRESSURE, 1, DIRICHLET, p_hyd)]
    s.bcs += [FaceBC(TEMPERATURE, f, DIRICHLET, timefn(T15C)) for f in range(6)]
    o = rng.integers(0, 15, size=3)
    mag = rng.uniform(10.0, 50.0)
    src = np.zeros((n[2], n[1], n[0]))
    src[o[2]:o[2] + 2, o[1]:o[1] + 2, o[0]:o[0] + 2] = mag
    s.heat_source = src.reshape(-1)
    s.P0 = p_hyd
    s.P0_steady = True
    s.T0 = timefn(T15C)
    return s


def config2(seed: int = 2, ncells=(128, 128, 64), n_steps: int = 100) -> Scenario:
    """500 x 500 x 100 m layered aquifer with an injection/extraction well
    pair (+-0.01 m^3/s, injected water at 40 C), transient pressure."""
    rng = np.random.Generator(np.random.PCG64(seed))
    origin, extent = (0.0, 0.0, 0.0), (500.0, 500.0, 100.0)
    perm, phi = layered_lognormal(rng, origin, extent, ncells, 5)
    nc = perm.size
    s = Scenario("c2", origin, extent, tuple(ncells), 1, permeability=perm,
                 porosity=phi, lambda_solid=_uniform(nc, 2.5),
                 rhoc_solid=_uniform(nc, 2.0e6), B_poro=1.0e5, dt=DAY,
                 n_steps=n_steps)
    p_hyd = hydrostatic(100.0, 1.0e5, s.rho_w, s.g)
    s.bcs = [FaceBC(PRESSURE, f, DIRICHLET, p_hyd) for f in range(4)]
    s.bcs += [FaceBC(TEMPERATURE, f, DIRICHLET, timefn(T15C)) for f in range(6)]
    s.lines = [LineSource(150.0, 250.0, 0.0, 100.0, LINE_WELL, timefn(0.01),
                          T_inj=313.15),
               LineSource(350.0, 250.0, 0.0, 100.0, LINE_WELL, timefn(-0.01),
                          T_inj=0.0)]
    s.P0 = p_hyd
    s.T0 = timefn(T15C)
    return s


def terrain_coords(origin, extent, ncells, top_amp=8.0, bottom_amp=5.0, shear=0.03):
    """Node coordinates of a terrain-following hexahedral mesh of the box
    topology: every node column keeps its (i, j) but its node planes are
    stretched between a curved bottom and a curved top surface (sigma
    layers), and the interior is sheared horizontally (the shear vanishes on
    the four side faces, which stay planar).  Cells are general hexahedra:
    non-parallel, non-planar faces.  Returns [nnode][3], x fastest."""
    (x0, y0, z0), (Lx, Ly, Lz) = origin, extent
    nx, ny, nz = ncells
    x = x0 + Lx * np.arange(nx + 1) / nx
    y = y0 + Ly * np.arange(ny + 1) / ny
    s = np.arange(nz + 1) / nz
    Z3, Y3, X3 = np.meshgrid(s, y, x, indexing="ij")
    u, v = (X3 - x0) / Lx, (Y3 - y0) / Ly
    top = z0 + Lz + top_amp * np.sin(2.0 * np.pi * u) * np.sin(np.pi * v)
    bot = z0 + bottom_amp * np.cos(np.pi * u) * np.cos(2.0 * np.pi * v)
    zz = bot + Z3 * (top - bot)
    xx = X3 + shear * Lx * (Z3 - 0.5) * np.sin(np.pi * u) * np.sin(np.pi * v)
    yy = Y3 + shear * Ly * np.sin(2.0 * np.pi * u) * np.sin(np.pi * v) * (1.0 - Z3)
    return np.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)], axis=1)


def aquifer_hex(seed: int = 7, ncells=(128, 128, 64), n_steps: int = 10) -> Scenario:
    """The 500 x 500 x 100 m layered aquifer on a terrain-following mesh of
    general hexahedra (terrain_coords): layered lognormal permeability by
    cell layer, transient pressure with a regional hydraulic gradient of
    0.005 along x (hydrostatic plus gradient on the x faces), a heated zone
    (50 W/m^3 in a block of cells) in a 15 C ground held at 15 C on the side
    and top faces."""
    rng = np.random.Generator(np.random.PCG64(seed))
    origin, extent = (0.0, 0.0, 0.0), (500.0, 500.0, 100.0)
    perm, phi = layered_lognormal(rng, origin, extent, ncells, 5)
    nc = perm.size
    s = Scenario("aquifer_hex", origin, extent, tuple(ncells), 1, permeability=perm,
                 porosity=phi, lambda_solid=_uniform(nc, 2.5),
                 rhoc_solid=_uniform(nc, 2.0e6), B_poro=1.0e5, dt=DAY,
                 n_steps=n_steps)
    s.coords = terrain_coords(origin, extent, ncells)
    p_g = hydrostatic(100.0, 1.0e5, s.rho_w, s.g, grad_x=0.005, x_ref=500.0)
    s.bcs = [FaceBC(PRESSURE, 0, DIRICHLET, p_g), FaceBC(PRESSURE, 1, DIRICHLET, p_g)]
    s.bcs += [FaceBC(TEMPERATURE, f, DIRICHLET, timefn(T15C)) for f in (0, 1, 2, 3, 5)]
    nx, ny, nz = ncells
    q = np.zeros((nz, ny, nx))
    q[nz // 4:nz // 2, 3 * ny // 8:5 * ny // 8, nx // 4:3 * nx // 8] = 50.0
    s.heat_source = q.reshape(-1)
    s.P0 = p_g
    s.T0 = timefn(T15C)
    return s


def config3(seed: int = 3, degree: int = 1, ncells=None, n_steps: int = 365) -> Scenario:
    """1 x 1 x 0.2 km energy-pile field: 400 piles on a 20 x 20 grid at 25 m
    spacing, each a 30 m line heat source with a seasonal 50 W/m sine of
    seeded phase; regional hydraulic gradient 0.001 along x."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if ncells is None:
        ncells = (256, 256, 128) if degree == 1 else (128, 128, 64)
    origin, extent = (0.0, 0.0, 0.0), (1000.0, 1000.0, 200.0)
    perm, phi = layered_lognormal(rng, origin, extent, ncells, 5)
    nc = perm.size
    s = Scenario("c3q%d" % degree, origin, extent, tuple(ncells), degree,
                 permeability=perm, porosity=phi,
                 lambda_solid=_uniform(nc, 2.5), rhoc_solid=_uniform(nc, 2.0e6),
                 B_poro=1.0e5, dt=DAY, n_steps=n_steps)
    p_g = hydrostatic(200.0, 1.0e5, s.rho_w, s.g, grad_x=0.001, x_ref=1000.0)
    s.bcs = [FaceBC(PRESSURE, 0, DIRICHLET, p_g), FaceBC(PRESSURE, 1, DIRICHLET, p_g)]
    s.bcs += [FaceBC(TEMPERATURE, f, DIRICHLET, timefn(T15C)) for f in range(6)]
    phases = rng.uniform(0.0, 2.0 * np.pi, size=400)
    xs = 262.5 + 25.0 * np.arange(20)
    k = 0
    for jy in range(20):
        for ix in range(20):
            s.lines.append(LineSource(xs[ix], xs[jy], 170.0, 200.0, LINE_HEAT,
                                      timefn(amp=50.0, period=365.0 * DAY,
                                             phase=phases[k], kind=TF_SIN)))
            k += 1
    s.P0 = p_g
    s.P0_steady = True
    s.T0 = timefn(T15C)
    return s


def config4_instance(i: int, n_override: Optional[int] = None,
                     n_steps: int = 50) -> Scenario:
    """One design scenario of the batched set: n^3 Q1 cells on a 200 m cube,
    layered lognormal permeability, 10-200 energy piles as Dirichlet
    temperature columns on a 10 m lattice at a seeded 30-50 C."""
    rng = np.random.Generator(np.random.PCG64(4000 + i))
    n = int(rng.integers(32, 97))
    if n_override is not None:
        n = int(n_override)
    ncells = (n, n, n)
    origin, extent = (0.0, 0.0, 0.0), (200.0, 200.0, 200.0)
    perm, phi = layered_lognormal(rng, origin, extent, ncells, 5)
    nc = perm.size
    s = Scenario("c4_%d" % i, origin, extent, ncells, 1, permeability=perm,
                 porosity=phi, lambda_solid=_uniform(nc, 2.5),
                 rhoc_solid=_uniform(nc, 2.0e6), B_poro=1.0e5, dt=DAY,
                 n_steps=n_steps)
    p_g = hydrostatic(200.0, 1.0e5, s.rho_w, s.g, grad_x=0.001, x_ref=200.0)
    s.bcs = [FaceBC(PRESSURE, 0, DIRICHLET, p_g), FaceBC(PRESSURE, 1, DIRICHLET, p_g)]
    s.bcs += [FaceBC(TEMPERATURE, f, DIRICHLET, timefn(T15C)) for f in range(6)]
    n_piles = int(rng.integers(10, 201))
    lattice = [(10.0 * (a + 1), 10.0 * (b + 1)) for b in range(19) for a in range(19)]
    pick = rng.choice(len(lattice), size=n_piles, replace=False)
    T_inj = rng.uniform(303.15, 323.15)
    for q in sorted(pick.tolist()):
        x, y = lattice[q]
        s.dir_columns.append(DirColumn(TEMPERATURE, x, y, 170.0, 200.0, timefn(T_inj)))
    s.P0 = p_g
    s.P0_steady = True
    s.T0 = timefn(T15C)
    return s


def config5(seed: int, ncells=(128, 128, 64), n_steps: int = 100) -> Scenario:
    """The layered-aquifer setup with permeability/porosity re-drawn per seed
    (training seeds 5000-5019, test seeds 5100-5109)."""
    s = config2(seed=seed, ncells=ncells, n_steps=n_steps)
    s.name = "c5_%d" % seed
    return s


# Soil and rock classes of the island site (Table 3): hydraulic conductivity
# [m/s], bulk volumetric heat capacity [J/m^3/K], bulk thermal conductivity
# [W/m/K], and the depth [m] below the surface where the class ends (the
# bedrock top is drawn per scenario between 70 and 80 m, Section 3.3).
ISLAND_LAYERS = (
    ("fill", 1.1e-5, 2.5e6, 2.2, 8.0),
    ("shoal", 3.5e-5, 2.5e6, 2.2, 12.0),
    ("young bay mud", 1.7e-9, 3.5e6, 1.5, 30.0),
    ("old bay mud", 1.7e-9, 3.5e6, 1.7, None),
    ("franciscan bedrock", 1.0e-6, 2.0e6, 2.97, float("inf")),
)
T_SEA = 287.45        # K, mean of the site record and the sea temperature


def island(seed: int = 6, ncells=(256, 160, 64), n_steps: int = 365,
           degree: int = 1, graded: bool = False) -> Scenario:
    """Island-style pile field on a 640 x 400 x 100 m box (Section 3.3 on a
    structured mesh): the five soil/rock classes of Table 3 with bulk thermal
    values and a seeded scatter of hydraulic conductivity, the bedrock top on
    a seeded plane between 70 and 80 m depth; a seasonal surface temperature
    (a sinusoid about 287.45 K that starts at 287.65 K, standing in for the
    monthly record), a geothermal inflow of 0.0891 W/m^2 through the bottom,
    lateral temperatures held at the initial 0.03 K/m geotherm; pressure
    hydrostatic on the left face and 5 Pa/m higher across the box on the
    right, no flow elsewhere, starting from the steady solution; energy piles
    60 m long on a 20 m lattice under seeded building footprints, held at
    288.55 +- 13 K as a square wave of one year (summer half first).
    graded=True refines the mesh three times around the building footprints
    and over the pile depth (the paper's site mesh is refined around the
    piles, Fig. 10b)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    origin, extent = (0.0, 0.0, 0.0), (640.0, 400.0, 100.0)
    nx, ny, nz = ncells
    nc = nx * ny * nz
    z_top = origin[2] + extent[2]
    a, b = rng.uniform(-1.0, 1.0, size=2)
    piles = set()
    for _ in range(8):
        w, d = rng.uniform(60.0, 160.0), rng.uniform(40.0, 100.0)
        x0 = rng.uniform(60.0, extent[0] - 60.0 - w)
        y0 = rng.uniform(60.0, extent[1] - 60.0 - d)
        for i in range(int(np.ceil(x0 / 20.0)), int(np.floor((x0 + w) / 20.0)) + 1):
            for j in range(int(np.ceil(y0 / 20.0)), int(np.floor((y0 + d) / 20.0)) + 1):
                piles.add((i, j))
    edges = None
    if graded:
        px = [20.0 * i for i, _ in piles] or [0.5 * extent[0]]
        py = [20.0 * j for _, j in piles] or [0.5 * extent[1]]
        edges = (graded_edges(origin[0], origin[0] + extent[0], nx,
                              [(min(px) - 20.0, max(px) + 20.0)]),
                 graded_edges(origin[1], origin[1] + extent[1], ny,
                              [(min(py) - 20.0, max(py) + 20.0)]),
                 graded_edges(origin[2], z_top, nz, [(z_top - 70.0, z_top)]))
        xc, yc = 0.5 * (edges[0][1:] + edges[0][:-1]), 0.5 * (edges[1][1:] + edges[1][:-1])
        depth = z_top - 0.5 * (edges[2][1:] + edges[2][:-1])
    else:
        xc = origin[0] + (np.arange(nx) + 0.5) * extent[0] / nx
        yc = origin[1] + (np.arange(ny) + 0.5) * extent[1] / ny
        depth = z_top - _cell_centres_z(origin, extent, ncells)
    plane = (a * (xc[None, :] / extent[0] - 0.5) + b * (yc[:, None] / extent[1] - 0.5))
    d_rock = 75.0 + 5.0 * plane / max(1e-12, 0.5 * (abs(a) + abs(b)))   # [ny, nx] in [70, 80]
    cls = np.zeros((nz, ny, nx), dtype=np.int64)
    for q, (_, _, _, _, d_end) in enumerate(ISLAND_LAYERS[:3]):
        cls[depth >= d_end] = q + 1
    cls[(cls == 3) & (depth[:, None, None] >= d_rock[None, :, :])] = 4
    cls = cls.reshape(-1)
    logK = np.log10([r[1] for r in ISLAND_LAYERS])[cls] + 0.2 * rng.standard_normal(nc)
    s = Scenario("island", origin, extent, tuple(ncells), degree,
                 permeability=None, porosity=None, lambda_solid=None, rhoc_solid=None,
                 hydraulic_conductivity=np.power(10.0, logK),
                 lambda_bulk=np.array([r[3] for r in ISLAND_LAYERS])[cls],
                 rhoc_bulk=np.array([r[2] for r in ISLAND_LAYERS])[cls],
                 B_poro=1.0e5, dt=DAY, n_steps=n_steps, edges=edges)
    p_left = hydrostatic(z_top, 1.0e5, s.rho_w, s.g)
    p_right = (p_left[0], p_left[1] + 5.0 * extent[0]) + p_left[2:]
    s.bcs = [FaceBC(PRESSURE, 0, DIRICHLET, p_left), FaceBC(PRESSURE, 1, DIRICHLET, p_right)]
    geotherm = timefn(c0=T_SEA + 0.03 * z_top, cz=-0.03)
    s.bcs += [FaceBC(TEMPERATURE, f, DIRICHLET, geotherm) for f in range(4)]
    s.bcs += [FaceBC(TEMPERATURE, 4, NEUMANN, timefn(-0.0891)),
              FaceBC(TEMPERATURE, 5, DIRICHLET,
                     timefn(c0=T_SEA, amp=3.5, period=365.0 * DAY,
                            phase=float(np.arcsin(0.2 / 3.5)), kind=TF_SIN))]
    for i, j in sorted(piles):
        s.dir_columns.append(DirColumn(TEMPERATURE, origin[0] + 20.0 * i, origin[1] + 20.0 * j,
                                       z_top - 60.0, z_top,
                                       timefn(c0=288.55, amp=13.0, period=365.0 * DAY,
                                              kind=TF_SQUARE)))
    s.P0 = p_left
    s.P0_steady = True
    s.T0 = geotherm
    return s


def ates(ncells=(64, 64, 240), n_steps: int = 180, degree: int = 1,
         r_well: float = 0.1) -> Scenario:
    """Three-dimensional analogue of the hot-water injection benchmark
    (Section 2, Table 1, Fig. 2): a 40 x 40 x 300 m column with a caprock
    (depth 0-100 m), an aquifer (100-200 m, hydraulic conductivity 1e-6 m/s)
    and a basement (200-300 m, 1e-10 m/s); bulk c_T 1.2e6 J/m^3/K and
    lambda 1.2 W/m/K everywhere, water heat capacity 1e6 J/m^3/K, storage
    modulus 1e5 Pa.  A wellbore on the column axis injects an outward flux of
    0.001 m/s through its surface over the aquifer (a line source of
    0.001 * 2 pi r_well m^3/s per metre) at 288.15 K, and holds the aquifer
    section of the axis at 288.15 K.  Surface 278.15 K, 0.05 K/m geotherm
    (held on the lateral faces; the matching 0.06 W/m^2 enters through the
    bottom), pressure hydrostatic from 0.1 MPa at the surface on the lateral
    faces, no flow through top and bottom.  180 daily steps (six months)."""
    origin, extent = (0.0, 0.0, 0.0), (40.0, 40.0, 300.0)
    nx, ny, nz = ncells
    nc = nx * ny * nz
    z_top = extent[2]
    depth = z_top - _cell_centres_z(origin, extent, ncells)
    aquifer = (depth >= 100.0) & (depth < 200.0)
    K = np.where(aquifer, 1.0e-6, 1.0e-10)[:, None, None] * np.ones((nz, ny, nx))
    s = Scenario("ates", origin, extent, tuple(ncells), degree,
                 permeability=None, porosity=None, lambda_solid=None, rhoc_solid=None,
                 hydraulic_conductivity=K.reshape(-1), lambda_bulk=np.full(nc, 1.2),
                 rhoc_bulk=np.full(nc, 1.2e6), c_w=1.0e6, B_poro=1.0e5, dt=DAY,
                 n_steps=n_steps)
    p_hyd = hydrostatic(z_top, 1.0e5, s.rho_w, s.g)
    s.bcs = [FaceBC(PRESSURE, f, DIRICHLET, p_hyd) for f in range(4)]
    geotherm = timefn(c0=278.15 + 0.05 * z_top, cz=-0.05)
    s.bcs += [FaceBC(TEMPERATURE, f, DIRICHLET, geotherm) for f in range(4)]
    s.bcs += [FaceBC(TEMPERATURE, 4, NEUMANN, timefn(-1.2 * 0.05)),
              FaceBC(TEMPERATURE, 5, DIRICHLET, timefn(278.15))]
    xc, yc = origin[0] + 0.5 * extent[0], origin[1] + 0.5 * extent[1]
    rate = 0.001 * 2.0 * np.pi * r_well * 100.0
    s.lines = [LineSource(xc, yc, z_top - 200.0, z_top - 100.0, LINE_WELL, timefn(rate),
                          T_inj=288.15)]
    s.dir_columns = [DirColumn(TEMPERATURE, xc, yc, z_top - 200.0, z_top - 100.0,
                               timefn(288.15))]
    s.P0 = p_hyd
    s.T0 = geotherm
    return s


def random_field(seed: int, n: int, kind: str = "normal") -> np.ndarray:
    """Seeded random vector for operator-apply tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "normal":
        return rng.standard_normal(n)
    return rng.uniform(-1.0, 1.0, n)
