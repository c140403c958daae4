"""Pins of the oracle's three-dimensional extension (Sec. 2: the system
extends directly to 3D; one more momentum component and a z-sweep).

The 3D code is pinned to the 2D oracle (itself pinned by the paper's
convergence table and the other tests in test_oracle_pins.py) and to
properties the mathematics fixes:
  * dimensional reduction, exact: a state constant along one axis with no
    velocity along it gives, on every slab, the 2D RHS of that slab, for
    each of the three axis pairs (this fixes the sweeps, the rotation of
    the three momenta, the line addressing and the order L_x + L_y + L_z);
  * discrete conservation on a periodic grid with the limiters active;
  * equivariance under a permutation of the axes (grid sizes, spacings and
    state permuted together);
  * positivity and boundedness on every stage of a 3D blast, and the
    failure of the same run without the limiters.
"""
from __future__ import annotations

import numpy as np
import pytest

from helpers import oracle_setup, oracle_W, orc, pb

# axis pair of the 2D problem inside the 3D grid: (2D x -> 3D axis, 2D y -> 3D axis)
PAIRS = [(0, 1), (1, 2), (0, 2)]


def _setup3(nx, ny, nz, dx, dy, dz, bc6, **kw):
    return orc.Setup(ndim=3, nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, bc=tuple(bc6), **kw)


def _extrude(spec, pair, n_ext):
    """3D primitive state [7][nz][ny][nx] constant along the third axis, with
    the 2D problem's (x, y) mapped to the axes in `pair`."""
    ax, ay = pair
    ext = 3 - ax - ay
    V2 = spec.prim                                   # [6][ny2][nx2]
    shape = [0, 0, 0]
    shape[ax], shape[ay], shape[ext] = spec.nx, spec.ny, n_ext
    nx, ny, nz = shape
    V3 = np.zeros((7, nz, ny, nx))
    # 2D field f[j2][i2] -> 3D array indexed [k][j][i]
    def place(f):
        g = np.zeros((nx, ny, nz))                   # index by (i, j, k)
        idx = [slice(None)] * 3
        src = f.T                                    # [i2][j2]
        # broadcast over the extruded axis
        order = [ax, ay, ext]
        g_view = np.moveaxis(g, order, [0, 1, 2])
        g_view[...] = src[:, :, None]
        return np.transpose(g, (2, 1, 0))
    V3[0] = place(V2[0])
    V3[1] = place(V2[1])
    vel2 = (V2[2], V2[3])
    V3[2 + ax] = place(vel2[0])
    V3[2 + ay] = place(vel2[1])
    V3[5] = place(V2[4])
    V3[6] = place(V2[5])
    h = [0.0, 0.0, 0.0]
    h[ax], h[ay], h[ext] = spec.dx, spec.dy, 1.7e-3
    bc6 = [pb.BC_PERIODIC] * 6
    bc6[2 * ax], bc6[2 * ax + 1] = spec.bc[0], spec.bc[1]
    bc6[2 * ay], bc6[2 * ay + 1] = spec.bc[2], spec.bc[3]
    return V3, (nx, ny, nz), h, bc6


def _slab_2d(L3, pair, comp_map, k_ext):
    """The 2D-ordered RHS of one slab of a 3D RHS."""
    ax, ay = pair
    ext = 3 - ax - ay
    out = []
    for c3 in comp_map:
        f = np.transpose(L3[c3], (2, 1, 0))          # (i, j, k)
        f = np.moveaxis(f, [ax, ay, ext], [0, 1, 2])[:, :, k_ext]   # [i2][j2]
        out.append(f.T)
    return np.array(out)


@pytest.mark.parametrize("pair", PAIRS)
def test_3d_reduces_to_2d_exactly(pair):
    spec = pb.random_smooth_state(23, 17, seed=31)
    s2 = oracle_setup(spec, flux_limiter=False)
    W2 = oracle_W(spec, s2)
    dt = 1e-7
    L2 = orc.rhs(s2, W2, dt)
    V3, (nx, ny, nz), h, bc6 = _extrude(spec, pair, 5)
    s3 = _setup3(nx, ny, nz, *h, bc6, flux_limiter=False)
    W3 = orc.prim_to_cons(s3, V3)
    L3 = orc.rhs(s3, W3, dt)
    ax, ay = pair
    ext = 3 - ax - ay
    comp_map = [0, 1, 2 + ax, 2 + ay, 5, 6]
    for k in range(V3.shape[1 + (2 - ext)]):
        got = _slab_2d(L3, pair, comp_map, k)
        assert np.array_equal(got, L2), (pair, k, np.abs(got - L2).max())
    # no momentum appears along the extruded axis
    assert np.all(L3[2 + ext] == 0.0)


def _blast3(n=12, h=(1e-3, 1.3e-3, 0.8e-3), shape=None):
    """Water at -3e7 Pa with a 2x2x2 air block at high pressure (Sec. 6.4 in
    3D), small random velocities."""
    nx, ny, nz = shape or (n, n, n)
    rng = np.random.Generator(np.random.PCG64(5))
    V = np.empty((7, nz, ny, nx))
    V[0], V[1], V[5], V[6] = 1000.0, 1e-8, -3e7, 1 - 1e-8
    V[2:5] = rng.uniform(-5, 5, size=(3, nz, ny, nx))
    c = (nz // 2 - 1, ny // 2 - 1, nx // 2 - 1)
    blk = (slice(c[0], c[0] + 2), slice(c[1], c[1] + 2), slice(c[2], c[2] + 2))
    for v, x in zip((0, 1, 5, 6), (1e-8, 1.0, 1.28e6 / h[0], 1e-8)):
        V[v][blk] = x
    return V


def test_3d_conservation_periodic_with_limiters():
    h = (1e-3, 1.3e-3, 0.8e-3)
    V = _blast3(10, h)
    s = _setup3(10, 10, 10, *h, [pb.BC_PERIODIC] * 6)
    W = orc.prim_to_cons(s, V)
    dt = orc.cfl_dt(s, W)
    L = orc.rhs(s, W, dt)
    _, _, th = orc.faces(s, W, 0, dt)
    assert (th < 1).sum() > 0, "the flux limiter must act"
    for v in range(6):   # conservative components (a1 is not conserved)
        tot = np.abs(L[v]).sum()
        assert abs(L[v].sum()) <= 1e-12 * tot, (v, L[v].sum(), tot)


def test_3d_axis_permutation_equivariance():
    """(x, y, z) -> (y, z, x): grid sizes, spacings, BCs and the state permuted
    together give the permuted RHS (to round-off of the summation order)."""
    nx, ny, nz = 9, 7, 6
    h = (1e-3, 1.3e-3, 0.8e-3)
    V = _blast3(shape=(nx, ny, nz), h=h)
    bc = [pb.BC_EXTRAP, pb.BC_REFLECT, pb.BC_PERIODIC, pb.BC_PERIODIC, pb.BC_REFLECT, pb.BC_EXTRAP]
    s = _setup3(nx, ny, nz, *h, bc)
    W = orc.prim_to_cons(s, V)
    dt = orc.cfl_dt(s, W)
    L = orc.rhs(s, W, dt)
    # new axes: x' = y, y' = z, z' = x; arrays [k'][j'][i'] = [x][z][y]
    Vp = np.transpose(V, (0, 3, 1, 2)).copy()
    Vp[2], Vp[3], Vp[4] = V[3].transpose(2, 0, 1), V[4].transpose(2, 0, 1), V[2].transpose(2, 0, 1)
    sp = _setup3(ny, nz, nx, h[1], h[2], h[0], bc[2:4] + bc[4:6] + bc[0:2])
    Wp = orc.prim_to_cons(sp, Vp)
    assert orc.cfl_dt(sp, Wp) == pytest.approx(dt, rel=1e-15)
    Lp = orc.rhs(sp, Wp, dt)
    back = np.transpose(Lp, (0, 2, 3, 1))               # [v][z][y][x]
    perm = [0, 1, 4, 2, 3, 5, 6]                        # rho u <- x'' slot etc.
    for v in range(7):
        want = L[v]
        got = back[perm[v]]
        M = np.abs(want).max()
        assert np.abs(got - want).max() <= 1e-12 * M, (v, np.abs(got - want).max(), M)


def test_3d_cfl_reduces_to_2d():
    spec = pb.random_smooth_state(16, 12, seed=32)
    s2 = oracle_setup(spec)
    W2 = oracle_W(spec, s2)
    V3, (nx, ny, nz), h, bc6 = _extrude(spec, (0, 1), 3)
    h[2] = 1e30                                       # the z term vanishes
    s3 = _setup3(nx, ny, nz, *h, bc6)
    W3 = orc.prim_to_cons(s3, V3)
    assert orc.cfl_dt(s3, W3) == orc.cfl_dt(s2, W2)
    a3, a2 = orc.max_wavespeed(s3, W3), orc.max_wavespeed(s2, W2)
    assert a3[0] == a2[0] and a3[1] == a2[1]


def test_3d_blast_stays_admissible_and_fails_without_limiters():
    h = (1e-3, 1e-3, 1e-3)
    V = _blast3(10, h)
    bc = [pb.BC_EXTRAP] * 6
    s = _setup3(10, 10, 10, *h, bc)
    W = orc.prim_to_cons(s, V)
    dt = 0.25 * orc.cfl_dt(s, W)
    W1, steps, t = orc.run(s, W, 30 * dt, dt)
    assert steps == 30 and orc.count_inadmissible(s, W1) == 0
    s_off = _setup3(10, 10, 10, *h, bc, interp_limiter=False, flux_limiter=False)
    with pytest.raises(FloatingPointError):
        orc.run(s_off, W, 30 * dt, dt)


def test_3d_uniform_state_zero_rhs():
    V = np.empty((7, 5, 6, 7))
    V[:] = np.array([1000.0, 1e-8, 30.0, -20.0, 10.0, 2e5, 1 - 1e-8])[:, None, None, None]
    s = _setup3(7, 6, 5, 1e-3, 1e-3, 1e-3, [pb.BC_PERIODIC] * 6)
    L = orc.rhs(s, orc.prim_to_cons(s, V), 1e-8)
    assert np.all(L == 0.0)


def test_3d_rhs_cells_matches_rhs():
    h = (1e-3, 1.3e-3, 0.8e-3)
    V = _blast3(shape=(9, 7, 6), h=h)
    s = _setup3(9, 7, 6, *h, [pb.BC_EXTRAP, pb.BC_REFLECT] * 3)
    W = orc.prim_to_cons(s, V)
    dt = orc.cfl_dt(s, W)
    L = orc.rhs(s, W, dt)
    cells = np.arange(0, 9 * 7 * 6, 7)
    got = orc.rhs_cells(s, W, dt, cells)
    want = L.reshape(7, -1)[:, cells].T
    assert np.array_equal(got, want)
