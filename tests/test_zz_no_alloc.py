"""The allocation-free right-hand side (wcns_rhs_noalloc), called through the
C ABI, against the context path (wcns_rhs) on the same inputs: bit for bit,
on two calls in a row, the second on a smaller grid (the static scratch
keeps the first call's contents), in 2D and 1D, in both precisions, and at
the largest grid class it accepts (1024^2); grids past its scratch are
refused before any device work."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from helpers import oracle_setup, oracle_W, orc, pb

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2102_05287_amd import wcns  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def noalloc_rhs(spec, W, dt, precision=wcns.FP64, **params):
    """wcns_rhs_noalloc through ctypes on the current torch stream."""
    g = wcns.grid_of(spec)
    e = wcns._Eos()
    e.gamma[0], e.gamma[1] = spec.gamma
    e.pinf[0], e.pinf[1] = spec.pinf
    p = wcns.default_params(cfl=spec.cfl, **params)
    out = torch.empty_like(W)
    rc = wcns.lib().wcns_rhs_noalloc(C.byref(g), C.byref(e), C.byref(p), int(precision),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                     C.c_void_p(W.data_ptr()), C.c_void_p(out.data_ptr()), float(dt))
    return rc, out


def context_rhs(spec, W, dt, precision=wcns.FP64, **params):
    sol = wcns.Solver.from_spec(spec, precision=precision, **params)
    out = sol.rhs(W, dt=dt)
    torch.cuda.synchronize()
    sol.close()
    return out


@pytest.mark.parametrize("precision", [wcns.FP64, wcns.FP32_BULK])
def test_noalloc_rhs_equals_rhs_twice_second_smaller(precision):
    specs = [pb.random_smooth_state(150, 97, seed=31), pb.random_smooth_state(70, 45, seed=32),
             pb.water_air_shock_tube(400), pb.water_air_shock_tube(130)]
    for spec in specs:
        s = oracle_setup(spec)
        W = dev(oracle_W(spec, s))
        dt = orc.cfl_dt(s, oracle_W(spec, s))
        print(f"  noalloc {spec.name} {spec.nx}x{spec.ny} precision {precision}", flush=True)
        rc, got = noalloc_rhs(spec, W, dt, precision)
        assert rc == 0, rc
        ref = context_rhs(spec, W, dt, precision)
        assert torch.equal(got, ref), spec.name
        if precision == wcns.FP64:
            assert np.array_equal(got.cpu().numpy(), orc.rhs(s, oracle_W(spec, s), dt))


def test_noalloc_rhs_first_order_pass_twice_second_smaller():
    """The first-order scheme in 2D (its one-pass stage, whose idle lanes
    store to a sink carved from the scratch): two grids in a row, the second
    smaller, equal to the context path and to the oracle."""
    for spec in (pb.random_smooth_state(200, 130, seed=35), pb.random_smooth_state(63, 17, seed=36)):
        s = oracle_setup(spec, scheme=1)
        Wh = oracle_W(spec, s)
        W = dev(Wh)
        dt = orc.cfl_dt(s, Wh)
        print(f"  noalloc first order {spec.nx}x{spec.ny}", flush=True)
        rc, got = noalloc_rhs(spec, W, dt, scheme=1)
        assert rc == 0, rc
        assert torch.equal(got, context_rhs(spec, W, dt, scheme=1))
        assert np.array_equal(got.cpu().numpy(), orc.rhs(s, Wh, dt))


def test_noalloc_rhs_full_size_shock_bubble():
    """The 1024^2 shock-bubble (the largest grid class the scratch holds)
    twice in a row, then a smaller random state with an air bubble and a
    water shock."""
    spec = pb.shock_bubble(1024)
    V = torch.from_numpy(spec.prim).cuda()
    spec.prim = None
    W = wcns.prim_to_cons(V, 2)
    del V
    dt = 1e-8
    print("  noalloc shock_bubble 1024x1024 fp64", flush=True)
    ref = context_rhs(spec, W, dt)
    for _ in range(2):
        rc, got = noalloc_rhs(spec, W, dt)
        assert rc == 0 and torch.equal(got, ref)
    blast = pb.random_smooth_state(96, 64, seed=33)
    s = oracle_setup(blast)
    Wb = dev(oracle_W(blast, s))
    dtb = orc.cfl_dt(s, oracle_W(blast, s))
    rc, got = noalloc_rhs(blast, Wb, dtb)
    assert rc == 0 and torch.equal(got, context_rhs(blast, Wb, dtb))


def test_noalloc_rhs_refuses_grids_past_its_scratch_and_dirichlet_sides():
    spec = pb.random_smooth_state(40, 30, seed=34)
    W = dev(oracle_W(spec, oracle_setup(spec)))
    big = pb.random_smooth_state(8, 8, seed=1)
    big.nx, big.ny = 2048, 2048
    rc, _ = noalloc_rhs(big, W, 1e-9)
    assert rc == -7
    diri = pb.random_smooth_state(40, 30, seed=34)
    diri.bc = (pb.BC_DIRICHLET, pb.BC_EXTRAP, pb.BC_PERIODIC, pb.BC_PERIODIC)
    diri.dirichlet_prim = [diri.prim[:, :, 0].T.copy(), None, None, None]
    rc, _ = noalloc_rhs(diri, W, 1e-9)
    assert rc == -1
