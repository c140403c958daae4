"""Seeded synthetic inputs: grids, fluids and initial primitive fields.

This module holds no arithmetic of the numerical method.  It only lays out
initial conditions in primitive variables V = (a1r1, a2r2, u, [v], p, a1)
(SoA ``[nvar][ny][nx]``), cell-centred at x_i = x0 + (i + 1/2) dx, and the
boundary kinds, for the test problems of the paper's Sec. 6 and for the
benchmark workloads.  Converting V to conservative W is done separately by the
code under test and by the reference implementation.

Readings (where the paper fixes nothing):
  * sharp initial conditions are sampled at cell centres, no smoothing;
  * the absent phase of a pure cell gets a partial density of 1e-8 kg/m^3 and
    the volume-fraction floor ``eps`` of the workload;
  * post-shock water states come from the stiffened-gas Rankine-Hugoniot
    relations for a shock running into water at rest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# fluid properties [Table 1]: phase 1 liquid water, phase 2 air
GAMMA = (6.12, 1.4)
PINF = (3.43e8, 0.0)

BC_PERIODIC, BC_EXTRAP, BC_REFLECT, BC_DIRICHLET = 0, 1, 2, 3
ABSENT_PARTIAL_DENSITY = 1e-8


@dataclass
class ProblemSpec:
    name: str
    ndim: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float = 0.0
    y1: float = 1.0
    bc: tuple = (BC_EXTRAP,) * 4       # x-lo, x-hi, y-lo, y-hi
    prim: np.ndarray = None            # [nvar][ny][nx] float64
    t_end: float = 0.0
    dt_fixed: float = 0.0              # > 0: constant time step
    cfl: float = 0.5
    dirichlet_prim: list = field(default_factory=lambda: [None] * 4)
    gamma: tuple = GAMMA
    pinf: tuple = PINF
    nz: int = 1                        # 3D only; bc then has 6 entries
    z0: float = 0.0
    z1: float = 1.0

    @property
    def nvar(self) -> int:
        return {1: 5, 2: 6, 3: 7}[self.ndim]

    @property
    def dz(self) -> float:
        return (self.z1 - self.z0) / self.nz if self.ndim == 3 else 1.0

    def centres3(self):
        """cell-centre grids X, Y, Z of shape [nz][ny][nx] (3D)."""
        x = self.x0 + (np.arange(self.nx) + 0.5) * self.dx
        y = self.y0 + (np.arange(self.ny) + 0.5) * self.dy
        z = self.z0 + (np.arange(self.nz) + 0.5) * self.dz
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return X, Y, Z

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ny if self.ndim >= 2 else 1.0

    def centres(self):
        x = self.x0 + (np.arange(self.nx) + 0.5) * self.dx
        if self.ndim == 1:
            return x, None
        y = self.y0 + (np.arange(self.ny) + 0.5) * self.dy
        return x, y


def _fill(nvar, shape, state):
    """Primitive field filled with one state tuple (len nvar)."""
    V = np.empty((nvar,) + shape)
    for k in range(nvar):
        V[k] = state[k]
    return V


def _water(p, u=0.0, v=None, rho=1000.0, eps=1e-8):
    st = [rho, ABSENT_PARTIAL_DENSITY, u]
    if v is not None:
        st.append(v)
    st += [p, 1.0 - eps]
    return st


def _gas(p, rho, u=0.0, v=None, eps=1e-8):
    st = [ABSENT_PARTIAL_DENSITY, rho, u]
    if v is not None:
        st.append(v)
    st += [p, eps]
    return st


def _set(V, mask, state):
    for k in range(V.shape[0]):
        V[k][mask] = state[k]


# ------------------------------------------------------------------ 1D cases
def water_air_shock_tube(n: int = 400, eps: float = 1e-8) -> ProblemSpec:
    """1D water-air shock tube on [0,1], interface at x = 0.7: water at 1e9 Pa
    on the left, air (rho 50) at 1e5 Pa on the right, constant extrapolation,
    CFL 0.5, t_end = 2.4e-4 s."""
    s = ProblemSpec("water_air_shock_tube", 1, n, 1, 0.0, 1.0, bc=(BC_EXTRAP,) * 4,
                    t_end=2.4e-4, cfl=0.5)
    x, _ = s.centres()
    V = _fill(5, (1, n), _gas(1e5, 50.0, eps=eps))
    _set(V, (x < 0.7)[None, :], _water(1e9, eps=eps))
    s.prim = V
    return s


def interface_advection(n: int = 200) -> ProblemSpec:
    """Two material interfaces advected one period [Sec. 6.2]."""
    s = ProblemSpec("interface_advection", 1, n, 1, 0.0, 1.0, bc=(BC_PERIODIC,) * 4,
                    t_end=0.01, dt_fixed=1.25e-6)
    x, _ = s.centres()
    V = _fill(5, (1, n), _gas(101325.0, 1.204, u=100.0))
    _set(V, ((x >= 0.25) & (x < 0.75))[None, :], _water(101325.0, u=100.0))
    s.prim = V
    return s


def gas_liquid_sod(n: int = 200) -> ProblemSpec:
    """Gas/liquid Sod shock tube [Sec. 6.3]."""
    s = ProblemSpec("gas_liquid_sod", 1, n, 1, 0.0, 1.5, bc=(BC_EXTRAP,) * 4,
                    t_end=3e-4, dt_fixed=1.25e-6)
    x, _ = s.centres()
    V = _fill(5, (1, n), _gas(1e5, 20.0))
    _set(V, (x < 0.8)[None, :], _water(1e9))
    s.prim = V
    return s


def sedov_multimaterial(n: int = 401) -> ProblemSpec:
    """Planar multi-material Sedov blast [Sec. 6.4]: water at -3e7 Pa with a
    single air cell at 1.28e6/dx Pa in the middle."""
    s = ProblemSpec("sedov_multimaterial", 1, n, 1, 0.0, 4.0, bc=(BC_EXTRAP,) * 4,
                    t_end=1e-3, dt_fixed=2.5e-7)
    x, _ = s.centres()
    dx = s.dx
    V = _fill(5, (1, n), _water(-3.0e7))
    mid = (x >= 2.0 - 0.5 * dx) & (x <= 2.0 + 0.5 * dx)
    _set(V, mid[None, :], _gas(1.28e6 / dx, 1.0))
    s.prim = V
    return s


def single_phase_shock_tube(n: int, left=(1500.0, 0.0, 2e9), right=(1000.0, 0.0, 1e5),
                            x_int: float = 0.5, eps: float = 1e-8) -> ProblemSpec:
    """Water/water Riemann problem (single stiffened gas), extrapolation BCs."""
    s = ProblemSpec("single_phase_shock_tube", 1, n, 1, 0.0, 1.0, bc=(BC_EXTRAP,) * 4)
    x, _ = s.centres()
    V = _fill(5, (1, n), _water(right[2], u=right[1], rho=right[0], eps=eps))
    _set(V, (x < x_int)[None, :], _water(left[2], u=left[1], rho=left[0], eps=eps))
    s.prim = V
    return s


# ------------------------------------------------------------------ 2D cases
def convergence_advection(N: int) -> ProblemSpec:
    """2D periodic volume-fraction wave [Sec. 6.1]: rho1 = 1000, rho2 = 1,
    u = v = 10, p = 101325, a1 = 0.5 + 0.25 sin(pi (x + y)) on [-1,1)^2,
    t = 1e-4 s, dt/dx = 4e-5 s/m."""
    s = ProblemSpec("convergence_advection", 2, N, N, -1.0, 1.0, -1.0, 1.0,
                    bc=(BC_PERIODIC,) * 4, t_end=1e-4)
    s.dt_fixed = 4e-5 * s.dx
    x, y = s.centres()
    X, Y = np.meshgrid(x, y)
    a1 = 0.5 + 0.25 * np.sin(np.pi * (X + Y))
    V = np.empty((6, N, N))
    V[0] = 1000.0 * a1
    V[1] = 1.0 * (1.0 - a1)
    V[2] = 10.0
    V[3] = 10.0
    V[4] = 101325.0
    V[5] = a1
    s.prim = V
    return s


def convergence_exact_alpha(s: ProblemSpec, t: float) -> np.ndarray:
    """Exact volume fraction of the convergence problem at time t."""
    x, y = s.centres()
    X, Y = np.meshgrid(x, y)
    return 0.5 + 0.25 * np.sin(np.pi * (X + Y - 20.0 * t))


def rankine_hugoniot_water(p0: float, rho0: float, p1: float):
    """Post-shock (rho1, u1) and shock speed for a right-running shock into
    still water (stiffened gas, Table 1)."""
    g, pinf = GAMMA[0], PINF[0]
    a0, a1 = p0 + pinf, p1 + pinf
    rho1 = rho0 * ((g + 1.0) * a1 + (g - 1.0) * a0) / ((g - 1.0) * a1 + (g + 1.0) * a0)
    S = math.sqrt((p1 - p0) / (rho0 * (1.0 - rho0 / rho1)))
    u1 = S * (1.0 - rho0 / rho1)
    return rho1, u1, S


def shock_bubble(n: int = 1024, eps: float = 1e-6) -> ProblemSpec:
    """2D shock-bubble interaction on [0,2]^2: air bubble (r 0.2, rho 1,
    p 1e5) centred at (1,1) in water (rho 1000, p 1e5), hit by a planar water
    shock (post-shock p = 1e9) starting at x = 0.6.  x-boundaries outflow,
    y-boundaries reflective."""
    s = ProblemSpec("shock_bubble", 2, n, n, 0.0, 2.0, 0.0, 2.0,
                    bc=(BC_EXTRAP, BC_EXTRAP, BC_REFLECT, BC_REFLECT), cfl=0.5)
    x, y = s.centres()
    X, Y = np.meshgrid(x, y)
    rho1, u1, _ = rankine_hugoniot_water(1e5, 1000.0, 1e9)
    V = _fill(6, (n, n), _water(1e5, 0.0, 0.0, eps=eps))
    _set(V, X < 0.6, _water(1e9, u1, 0.0, rho=rho1, eps=eps))
    _set(V, (X - 1.0) ** 2 + (Y - 1.0) ** 2 < 0.2 ** 2, _gas(1e5, 1.0, 0.0, 0.0, eps=eps))
    s.prim = V
    return s


def underwater_explosion(n: int = 2048, eps: float = 1e-6) -> ProblemSpec:
    """2D underwater explosion near a wall on [-2,2]x[0,4]: gas bubble
    (r 0.12 at (0,1), rho 1270, p 8.29e8) in water (rho 1000, p 1e5); wall
    (reflective) at y = 0, outflow elsewhere; t_end = 2e-4 s."""
    s = ProblemSpec("underwater_explosion", 2, n, n, -2.0, 2.0, 0.0, 4.0,
                    bc=(BC_EXTRAP, BC_EXTRAP, BC_REFLECT, BC_EXTRAP), t_end=2e-4)
    x, y = s.centres()
    X, Y = np.meshgrid(x, y)
    V = _fill(6, (n, n), _water(1e5, 0.0, 0.0, eps=eps))
    _set(V, X ** 2 + (Y - 1.0) ** 2 < 0.12 ** 2, _gas(8.29e8, 1270.0, 0.0, 0.0, eps=eps))
    s.prim = V
    return s


def mach10_cylinder(nx: int = 1152, ny: int = 768) -> ProblemSpec:
    """Mach 10 air shock hitting a water cylinder [Sec. 6.6]: domain
    [0, 30L] x [-10L, 10L] with L = 1 mm, cylinder of diameter 8L centred at
    (13L, 0), constant extrapolation on every side; pre-shock air (1.2, 1e5),
    post-shock air (6.8571, u = 2817.9, 1.165e7), water (1000, 1e5), all with
    the 1e-8 floors of the paper's table.  The shock starts at x = 9L, the
    upstream edge of the cylinder (schematic of Sec. 6.6).  Runs to 16 us."""
    L = 1e-3
    s = ProblemSpec("mach10_cylinder", 2, nx, ny, 0.0, 30 * L, -10 * L, 10 * L,
                    bc=(BC_EXTRAP,) * 4, t_end=16e-6, cfl=0.5)
    x, y = s.centres()
    X, Y = np.meshgrid(x, y)
    V = _fill(6, (ny, nx), _gas(1.0e5, 1.2, 0.0, 0.0))
    _set(V, X < 9 * L, _gas(1.165e7, 6.8571, 2.8179e3, 0.0))
    _set(V, (X - 13 * L) ** 2 + Y ** 2 < (4 * L) ** 2, _water(1.0e5, 0.0, 0.0))
    s.prim = V
    return s


def mach100_jet(nx: int = 1024, ny: int = 512) -> ProblemSpec:
    """Mach 100 water jet entering air [Sec. 6.7]: domain [0, L] x
    [-0.25L, 0.25L] with L = 1 m, ambient air (1, 1e5) at rest; the left side
    is a Dirichlet boundary whose rows with |y| <= 0.05L carry water (1000,
    u = 1.5e5, 1e5) and the others the ambient air; constant extrapolation
    on the other three sides.  Runs to 4 us."""
    s = ProblemSpec("mach100_jet", 2, nx, ny, 0.0, 1.0, -0.25, 0.25,
                    bc=(BC_DIRICHLET, BC_EXTRAP, BC_EXTRAP, BC_EXTRAP), t_end=4e-6, cfl=0.5)
    _, y = s.centres()
    air = _gas(1.0e5, 1.0, 0.0, 0.0)
    s.prim = _fill(6, (ny, nx), air)
    rows = np.empty((ny, 6))
    rows[:] = air
    rows[np.abs(y) <= 0.05] = _water(1.0e5, 1.5e5, 0.0)
    s.dirichlet_prim = [rows, None, None, None]
    return s


# ------------------------------------------------------------------ 3D cases
def random_smooth_state_3d(nx: int, ny: int, nz: int, seed: int, with_bubble: bool = True,
                           with_shock: bool = True, eps: float = 1e-6) -> ProblemSpec:
    """3D parity input: water with smooth random perturbations of p, u, v, w
    and rho (random Fourier modes), an air sphere and a water shock; the
    sides are extrapolated, reflective or periodic."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = ProblemSpec(f"random_smooth3d_{seed}", 3, nx, ny, 0.0, 1.0, 0.0, ny / nx,
                    bc=(BC_EXTRAP, BC_REFLECT, BC_PERIODIC, BC_PERIODIC, BC_REFLECT, BC_EXTRAP),
                    nz=nz, z0=0.0, z1=nz / nx)
    X, Y, Z = s.centres3()

    def modes(amp):
        f = np.zeros_like(X)
        for _ in range(3):
            kx, ky, kz = rng.integers(1, 4, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            f += amp * rng.uniform(0.3, 1.0) * np.sin(2 * np.pi * (kx * X + ky * Y + kz * Z) + ph)
        return f

    V = np.empty((7,) + X.shape)
    V[0] = 1000.0 + modes(20.0)
    V[1] = ABSENT_PARTIAL_DENSITY
    V[2] = modes(30.0)
    V[3] = modes(30.0)
    V[4] = modes(30.0)
    V[5] = 2e5 + modes(5e4)
    V[6] = 1.0 - eps
    if with_shock:
        _set(V, X < 0.25, [1214.6, ABSENT_PARTIAL_DENSITY, 420.0, 0.0, 0.0, 1e9, 1.0 - eps])
    if with_bubble:
        cy, cz = 0.5 * (s.y1 - s.y0), 0.5 * (s.z1 - s.z0)
        m = (X - 0.55) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2 < 0.12 ** 2
        _set(V, m, [ABSENT_PARTIAL_DENSITY, 1.0, 0.0, 0.0, 0.0, 1e5, eps])
    s.prim = V
    return s


def underwater_explosion_3d(n: int = 256, eps: float = 1e-6) -> ProblemSpec:
    """3D underwater explosion near a wall on [-1,1]x[-1,1]x[0,2]: gas sphere
    (r 0.12 at (0,0,0.5), rho 1270, p 8.29e8) in water (rho 1000, p 1e5); wall
    (reflective) at z = 0, outflow elsewhere (the 2D workload's 3D form)."""
    s = ProblemSpec("underwater_explosion_3d", 3, n, n, -1.0, 1.0, -1.0, 1.0,
                    bc=(BC_EXTRAP, BC_EXTRAP, BC_EXTRAP, BC_EXTRAP, BC_REFLECT, BC_EXTRAP),
                    nz=n, z0=0.0, z1=2.0)
    X, Y, Z = s.centres3()
    V = np.empty((7,) + X.shape)
    for k, x in enumerate([1000.0, ABSENT_PARTIAL_DENSITY, 0.0, 0.0, 0.0, 1e5, 1.0 - eps]):
        V[k] = x
    _set(V, X ** 2 + Y ** 2 + (Z - 0.5) ** 2 < 0.12 ** 2,
         [ABSENT_PARTIAL_DENSITY, 1270.0, 0.0, 0.0, 0.0, 8.29e8, eps])
    s.prim = V
    return s


def sedov_blast_3d(n: int = 24) -> ProblemSpec:
    """3D multi-material blast in the style of Sec. 6.4: water at -3e7 Pa on
    [0,1]^3 with a 2x2x2 block of air at 1.28e6/dx Pa in the middle; the
    limiters act on many faces from the first step."""
    s = ProblemSpec("sedov_blast_3d", 3, n, n, 0.0, 1.0, 0.0, 1.0, bc=(BC_EXTRAP,) * 6,
                    nz=n, z0=0.0, z1=1.0)
    V = np.empty((7, n, n, n))
    for k, x in enumerate([1000.0, 1e-8, 0.0, 0.0, 0.0, -3.0e7, 1.0 - 1e-8]):
        V[k] = x
    c = n // 2 - 1
    blk = (slice(c, c + 2),) * 3
    for k, x in enumerate([1e-8, 1.0, 0.0, 0.0, 0.0, 1.28e6 / s.dx, 1e-8]):
        V[k][blk] = x
    s.prim = V
    return s


BATCH_SIDES = (64, 96, 128, 192, 256, 384, 512)


def random_instance(i: int, base_seed: int = 20210210, eps: float = 1e-6) -> ProblemSpec:
    """One seeded random 2D water/air instance of the batched workload:
    side uniform in BATCH_SIDES; half planar Riemann problems, half gas
    bubbles; pressure ratio log-uniform in [1e1, 1e4] over 1e5 Pa; bubble
    radius uniform in [0.05, 0.3] of the side; water/gas density ratio
    uniform in [20, 1000] with water at 1000."""
    rng = np.random.Generator(np.random.PCG64(base_seed + i))
    n = int(rng.choice(BATCH_SIDES))
    kind = int(rng.integers(0, 2))
    ratio = 10.0 ** rng.uniform(1.0, 4.0)
    radius = rng.uniform(0.05, 0.3)
    dens_ratio = rng.uniform(20.0, 1000.0)
    p_lo, p_hi = 1e5, 1e5 * ratio
    rho_g = 1000.0 / dens_ratio
    s = ProblemSpec(f"instance_{i}", 2, n, n, 0.0, 1.0, 0.0, 1.0,
                    bc=(BC_EXTRAP, BC_EXTRAP, BC_REFLECT, BC_REFLECT))
    x, y = s.centres()
    X, Y = np.meshgrid(x, y)
    if kind == 0:     # planar Riemann problem: high-pressure water | gas
        V = _fill(6, (n, n), _gas(p_lo, rho_g, 0.0, 0.0, eps=eps))
        _set(V, X < 0.5, _water(p_hi, 0.0, 0.0, eps=eps))
    else:             # high-pressure gas bubble in still water
        V = _fill(6, (n, n), _water(p_lo, 0.0, 0.0, eps=eps))
        _set(V, (X - 0.5) ** 2 + (Y - 0.5) ** 2 < radius ** 2,
             _gas(p_hi, rho_g, 0.0, 0.0, eps=eps))
    s.prim = V
    return s


def random_smooth_state(nx: int, ny: int, seed: int, ndim: int = 2,
                        with_bubble: bool = True, with_shock: bool = True,
                        eps: float = 1e-6) -> ProblemSpec:
    """Water with smooth random perturbations of p, u, v (a few random Fourier
    modes), optionally an air bubble (material interface) and a water shock.
    Used as a parity input that exercises smooth regions, interfaces and
    shocks; boundaries cycle through all kinds."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if ndim == 1:
        s = ProblemSpec(f"random_smooth_{seed}", 1, nx, 1, 0.0, 1.0,
                        bc=(BC_EXTRAP, BC_REFLECT, BC_EXTRAP, BC_EXTRAP))
    else:
        s = ProblemSpec(f"random_smooth_{seed}", 2, nx, ny, 0.0, 1.0, 0.0, ny / nx,
                        bc=(BC_EXTRAP, BC_REFLECT, BC_PERIODIC, BC_PERIODIC))
    x, y = s.centres()
    if ndim == 1:
        X = x[None, :]
        Y = np.zeros_like(X)
    else:
        X, Y = np.meshgrid(x, y)

    def modes(amp):
        f = np.zeros_like(X)
        for _ in range(3):
            kx, ky = rng.integers(1, 4, size=2)
            ph = rng.uniform(0, 2 * np.pi)
            f += amp * rng.uniform(0.3, 1.0) * np.sin(2 * np.pi * (kx * X + ky * Y) + ph)
        return f

    p = 2e5 + modes(5e4)
    u = modes(30.0)
    v = modes(30.0)
    rho = 1000.0 + modes(20.0)
    nv = 5 if ndim == 1 else 6
    V = np.empty((nv,) + X.shape)
    V[0] = rho
    V[1] = ABSENT_PARTIAL_DENSITY
    V[2] = u
    if ndim == 2:
        V[3] = v
    V[nv - 2] = p
    V[nv - 1] = 1.0 - eps
    if with_shock:
        m = X < 0.25
        st = _water(1e9, 420.0, 0.0 if ndim == 2 else None, rho=1214.6, eps=eps)
        _set(V, m, st)
    if with_bubble:
        r = 0.12 if ndim == 2 else 0.1
        cx, cy = 0.55, (0.5 * (s.y1 - s.y0) if ndim == 2 else 0.0)
        m = (X - cx) ** 2 + (Y - cy) ** 2 < r ** 2
        st = _gas(1e5, 1.2, 0.0, 0.0 if ndim == 2 else None, eps=eps)
        _set(V, m, st)
    s.prim = V
    return s


# ------------------------------------------------------------ serving trace
@dataclass
class Request:
    rid: int
    arrival: float
    ndim: int
    n: int
    steps: int
    fp32: bool
    seed: int


def serving_trace(n_requests: int = 2000, rate: float = 200.0, seed: int = 4):
    """Poisson arrivals at `rate` req/s; half 1D (cells log-uniform in
    [200, 2e4]), half 2D (side log-uniform in [64, 1024]); steps log-uniform
    in [100, 2000]; FP64 or FP32 with equal odds."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    reqs = []
    for k in range(n_requests):
        ndim = 1 if rng.uniform() < 0.5 else 2
        if ndim == 1:
            n = int(round(10 ** rng.uniform(math.log10(200), math.log10(2e4))))
        else:
            n = int(round(10 ** rng.uniform(math.log10(64), math.log10(1024))))
        steps = int(round(10 ** rng.uniform(2.0, math.log10(2000))))
        reqs.append(Request(k, float(t[k]), ndim, n, steps, bool(rng.uniform() < 0.5),
                            int(rng.integers(0, 2**31))))
    return reqs


def request_problem(r: Request) -> ProblemSpec:
    """Initial condition of one serving request: a seeded shock tube (1D) or a
    seeded random 2D instance resized to the request's side."""
    rng = np.random.Generator(np.random.PCG64(r.seed))
    if r.ndim == 1:
        ratio = 10.0 ** rng.uniform(1.0, 4.0)
        rho_g = 1000.0 / rng.uniform(20.0, 1000.0)
        x_int = rng.uniform(0.3, 0.7)
        s = ProblemSpec(f"req_{r.rid}", 1, r.n, 1, 0.0, 1.0, bc=(BC_EXTRAP,) * 4)
        x, _ = s.centres()
        V = _fill(5, (1, r.n), _gas(1e5, rho_g))
        _set(V, (x < x_int)[None, :], _water(1e5 * ratio))
        s.prim = V
        return s
    base = random_instance(r.seed % 100000)
    s = ProblemSpec(f"req_{r.rid}", 2, r.n, r.n, 0.0, 1.0, 0.0, 1.0, bc=base.bc)
    # resample the instance's geometry at the request's resolution
    src = base.prim
    idx = ((np.arange(r.n) + 0.5) * base.nx / r.n).astype(int)
    s.prim = np.ascontiguousarray(src[:, idx][:, :, idx])
    return s
