"""3D form on the GPU against the 3D oracle, element by element, through the
C ABI (the direct extension of Sec. 2: seven components, x/y/z sweeps).

Tolerance as for 2D: 1e-12 per cell scaled by the variable's maximum after
one RHS or one step (in practice the results are bit-identical).
"""
from __future__ import annotations

import numpy as np
import pytest

from helpers import oracle_setup, oracle_W, orc, pb
from test_gpu_parity import assert_parity, dev, host, rhs_case, solver_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("shape,seed", [((40, 33, 21), 1), ((64, 5, 70), 2), ((7, 9, 130), 3),
                                        ((130, 66, 9), 4)])
def test_rhs_3d_random_states(shape, seed):
    rhs_case(pb.random_smooth_state_3d(*shape, seed=seed))


@pytest.mark.parametrize("shape,bc", [
    ((61, 13, 8), (pb.BC_PERIODIC,) * 2 + (pb.BC_REFLECT, pb.BC_EXTRAP) + (pb.BC_EXTRAP, pb.BC_REFLECT)),
    ((62, 15, 31), (pb.BC_REFLECT,) * 2 + (pb.BC_PERIODIC,) * 2 + (pb.BC_PERIODIC,) * 2),
    ((97, 12, 6), (pb.BC_EXTRAP,) * 4 + (pb.BC_REFLECT,) * 2)])
def test_rhs_3d_lds_windows_and_tiles(shape, bc):
    """x pass with LDS windows (rows of 61 cells and more, tiles crossing row
    and slab ends) under every x side kind; strided passes whose lines end
    inside a staged tile (ragged last tile) or fill whole tiles."""
    spec = pb.random_smooth_state_3d(*shape, seed=sum(shape))
    spec.bc = bc
    rhs_case(spec)


def test_rhs_3d_degenerate_shapes():
    """one cell along an axis (periodic there) and short lines"""
    for shape in ((17, 9, 1), (1, 20, 30), (33, 1, 12), (3, 3, 3)):
        spec = pb.random_smooth_state_3d(*shape, seed=9, with_shock=False)
        spec.bc = (pb.BC_PERIODIC,) * 2 + (pb.BC_EXTRAP,) * 2 + (pb.BC_PERIODIC,) * 2
        rhs_case(spec)


def test_rhs_3d_schemes_and_limiter_switches():
    spec = pb.random_smooth_state_3d(36, 29, 23, seed=5)
    rhs_case(spec, scheme=1)
    rhs_case(spec, interp_limiter=False)
    rhs_case(spec, flux_limiter=False, interp_limiter=False)


def test_rhs_3d_limiters_active_blast():
    """3D Sedov-style blast after one oracle step, where the flux limiter
    acts on faces of every direction: RHS and three device-CFL steps."""
    spec = pb.sedov_blast_3d(24)
    s = oracle_setup(spec)
    W, _, bad = orc.ssprk3_step(s, oracle_W(spec, s))
    assert bad == 0
    dt = orc.cfl_dt(s, W)
    for d in range(3):
        _, _, th = orc.faces(s, W, d, dt)
        assert (th < 1).sum() > 10, d
    sol = solver_for(spec)
    assert_parity(host(sol.rhs(dev(W), dt=dt)), orc.rhs(s, W, dt), what="blast3d rhs")
    Wd = dev(W)
    for k in range(3):
        sol.step(Wd, 0.0)
        W, _, bad = orc.ssprk3_step(s, W)
        assert bad == 0 and sol.count_inadmissible(Wd) == 0
        assert_parity(host(Wd), W, what=f"blast3d step {k + 1}")


def test_ssprk3_step_3d_and_dt():
    spec = pb.random_smooth_state_3d(45, 38, 27, seed=6)
    s = oracle_setup(spec)
    W = oracle_W(spec, s)
    ref, dt_ref, bad = orc.ssprk3_step(s, W)
    assert bad == 0
    sol = solver_for(spec)
    Wd = dev(W)
    dtu = torch.zeros(1, dtype=torch.float64, device="cuda")
    sol.step(Wd, 0.0, dt_used=dtu)
    assert host(dtu)[0] == dt_ref
    assert_parity(host(Wd), ref, what="3d step")
    a = host(sol.max_wavespeed(dev(W)))
    assert np.array_equal(a, orc.max_wavespeed(s, W))


def test_prim_to_cons_and_admissible_3d():
    spec = pb.random_smooth_state_3d(31, 17, 11, seed=7)
    s = oracle_setup(spec)
    sol = solver_for(spec)
    Wd = sol.prim_to_cons(dev(spec.prim))
    W = orc.prim_to_cons(s, spec.prim)
    assert np.array_equal(host(Wd), W)
    assert sol.count_inadmissible(Wd) == 0
    W[1, 3, 4, 5] = -1.0
    W[6, 0, 0, 0] = 1.5
    assert sol.count_inadmissible(dev(W)) == orc.count_inadmissible(s, W) == 2


def test_advance_3d_matches_oracle_time_loop():
    spec = pb.sedov_blast_3d(16)
    s = oracle_setup(spec)
    W0 = oracle_W(spec, s)
    t_end = 12 * orc.cfl_dt(s, W0)
    ref, steps, t_ref = orc.run(s, W0, t_end)
    sol = solver_for(spec)
    Wd = dev(W0)
    n, t = sol.advance(Wd, t_end, chunk=4)
    assert n == steps and t == t_ref
    assert_parity(host(Wd), ref, what="advance 3d")


def test_underwater_explosion_3d_full_size_sampled():
    """256^3 (16.8 M cells): RHS at cells sampled around the gas sphere and
    across the grid against the oracle cell by cell; 20 device-CFL steps stay
    admissible; sampled RHS again from there."""
    spec = pb.underwater_explosion_3d(256)
    s = oracle_setup(spec)
    W = oracle_W(spec, s)
    rng = np.random.Generator(np.random.PCG64(11))
    n = spec.nx
    near = []
    for _ in range(1500):        # cells within 0.2 of the sphere centre (0, 0, 0.5)
        p = rng.normal(size=3)
        p = p / np.linalg.norm(p) * rng.uniform(0.0, 0.2)
        i = int((p[0] + 1.0) / spec.dx)
        j = int((p[1] + 1.0) / spec.dy)
        k = int((p[2] + 0.5 - spec.z0) / spec.dz)
        near.append((k * n + j) * n + i)
    cells = np.unique(np.concatenate([np.array(near, dtype=np.int64),
                                      rng.integers(0, n ** 3, size=500)]))
    sol = solver_for(spec)
    for phase in range(2):
        dt = orc.cfl_dt(s, W)
        got = host(sol.rhs(dev(W), dt=dt)).reshape(7, -1)[:, cells].T
        want = orc.rhs_cells(s, W, dt, cells)
        assert_parity(got.T.copy(), want.T.copy(), what=f"uwe3d phase {phase}")
        if phase == 0:
            Wd = dev(W)
            for _ in range(20):
                sol.step(Wd, 0.0)
            assert sol.count_inadmissible(Wd) == 0
            W = host(Wd)
            del Wd
