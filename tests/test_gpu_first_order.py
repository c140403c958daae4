"""The first-order HLLC scheme (the paper's comparison scheme, Sec. 3) in 2D
runs as one pass per SSP-RK3 stage (k_fo_stage: 62-column strips marching
down row blocks sized so the grid fills the GPU once).  Its results must be the oracle's bit for bit: grids
whose width and height leave ragged last strips and row blocks, single
rows and columns, every side kind (periodic, extrapolated, reflective,
per-row Dirichlet), RHS calls, multi-step calls (the wave-speed maxima of a
step's last stage give the next step's time step), the device time loop, and
the full-size shock-bubble."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import oracle_setup, oracle_W, orc, pb
from test_gpu_parity import assert_parity, dev, host, solver_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rows(rng, n, nvar=6):
    """n admissible primitive states (water or air) for Dirichlet rows."""
    out = np.empty((n, nvar))
    for k in range(n):
        if rng.uniform() < 0.5:
            out[k] = (1000.0, 1e-6, rng.uniform(-50, 50), rng.uniform(-50, 50), rng.uniform(1e5, 1e8), 1 - 1e-6)
        else:
            out[k] = (1e-6, 1.2, rng.uniform(-50, 50), rng.uniform(-50, 50), rng.uniform(1e5, 1e6), 1e-6)
    return out


def _cases():
    out = []
    for (nx, ny, seed) in ((61, 9, 1), (62, 8, 2), (63, 17, 3), (124, 16, 4), (125, 1, 5),
                           (1, 40, 6), (130, 33, 7), (200, 3, 8)):
        sp = pb.random_smooth_state(nx, ny, seed)
        if nx < 3:   # a reflective side needs three cells
            sp.bc = (pb.BC_PERIODIC, pb.BC_PERIODIC, pb.BC_EXTRAP, pb.BC_EXTRAP)
        out.append(sp)
    refl = pb.random_smooth_state(70, 45, 9)
    refl.bc = (pb.BC_REFLECT, pb.BC_REFLECT, pb.BC_REFLECT, pb.BC_REFLECT)
    out.append(refl)
    tiny = pb.random_smooth_state(3, 3, 10)
    tiny.bc = (pb.BC_REFLECT, pb.BC_EXTRAP, pb.BC_PERIODIC, pb.BC_PERIODIC)
    out.append(tiny)
    rng = np.random.Generator(np.random.PCG64(12))
    diri = pb.random_smooth_state(93, 27, 11)
    diri.bc = (pb.BC_DIRICHLET, pb.BC_EXTRAP, pb.BC_REFLECT, pb.BC_DIRICHLET)
    diri.dirichlet_prim = [_rows(rng, 27), None, None, _rows(rng, 93)]
    out.append(diri)
    # several rows per wave task (the row blocks are sized to the GPU)
    out.append(pb.random_smooth_state(600, 700, 13))
    big = pb.random_smooth_state(1000, 500, 14)
    big.bc = (pb.BC_DIRICHLET, pb.BC_EXTRAP, pb.BC_REFLECT, pb.BC_REFLECT)
    big.dirichlet_prim = [_rows(rng, 500), None, None, None]
    out.append(big)
    return out


@pytest.mark.parametrize("k", range(13))
def test_first_order_pass_rhs_and_steps_equal_the_oracle(k):
    spec = _cases()[k]
    print(f"  first order {spec.nx}x{spec.ny} bc {spec.bc}", flush=True)
    s = oracle_setup(spec, scheme=1)
    W = oracle_W(spec, s)
    dt = orc.cfl_dt(s, W)
    sol = solver_for(spec, scheme=1)
    assert_parity(host(sol.rhs(dev(W), dt=dt)), orc.rhs(s, W, dt), what="fo rhs")
    ref = W
    dts = []
    for _ in range(4):
        ref, d, bad = orc.ssprk3_step(s, ref)
        assert bad == 0
        dts.append(d)
    Wd = dev(W)
    got_dt = torch.zeros(4, dtype=torch.float64, device="cuda")
    sol.steps(Wd, 4, 0.0, dts=got_dt)
    assert host(got_dt).tolist() == dts
    assert np.array_equal(host(Wd), ref)
    assert sol.violations() == 0


def test_first_order_full_size_shock_bubble():
    """The default workload at full size in first-order mode: 3 steps in one
    call and the device time loop over 5 more, bit for bit the oracle's."""
    spec = pb.shock_bubble(1024)
    s = oracle_setup(spec, scheme=1)
    W = oracle_W(spec, s)
    sol = solver_for(spec, scheme=1)
    Wd = dev(W)
    sol.steps(Wd, 3, 0.0)
    ref = W
    for _ in range(3):
        ref, _, bad = orc.ssprk3_step(s, ref)
        assert bad == 0
    assert np.array_equal(host(Wd), ref)
    t_end = 5 * orc.cfl_dt(s, ref) * 0.999
    ref2, steps, t_ref = orc.run(s, ref, t_end)
    n, t = sol.advance(Wd, t_end, chunk=4)
    assert n == steps and t == t_ref
    assert_parity(host(Wd), ref2, what="fo 1024 advance")
    assert np.array_equal(host(Wd), ref2)
    assert sol.violations() == 0
