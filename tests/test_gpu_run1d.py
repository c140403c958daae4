"""Whole 1D runs with the time loop on the device (wcns_run, one workgroup)
against the oracle's time loop and against stepping with wcns_ssprk3_step.

The run executes the same arithmetic per stage as the multi-kernel path, so
final states, step counts and final times are compared exactly."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import oracle_setup, oracle_W, orc, pb
from test_gpu_parity import assert_parity, dev, host, solver_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2102_05287_amd import wcns  # noqa: E402


@pytest.mark.parametrize("name", ["water_air_tube", "sedov", "interface_advection", "sod"])
def test_run_matches_oracle_time_loop(name):
    spec = {"water_air_tube": lambda: pb.water_air_shock_tube(400),
            "sedov": lambda: pb.sedov_multimaterial(401),
            "interface_advection": lambda: pb.interface_advection(200),
            "sod": lambda: pb.gas_liquid_sod(200)}[name]()
    s = oracle_setup(spec)
    W0 = oracle_W(spec, s)
    ref, steps, t_ref = orc.run(s, W0, spec.t_end, spec.dt_fixed)
    sol = solver_for(spec)
    Wd = dev(W0)
    n, t = sol.run(Wd, spec.t_end, dt_fixed=spec.dt_fixed)
    print(f"  {name}: {n} steps to t = {t!r}", flush=True)
    assert n == steps and t == t_ref
    got = host(Wd)
    assert_parity(got, ref, what=name)
    assert np.array_equal(got, ref), np.abs(got - ref).max()
    assert sol.count_inadmissible(Wd) == 0


@pytest.mark.parametrize("precision", [wcns.FP64, wcns.FP32_BULK])
def test_run_equals_eager_steps(precision):
    """Same bits as wcns_ssprk3_step step by step, with the per-step dt
    record, for both precisions and with Dirichlet sides."""
    spec = pb.water_air_shock_tube(333)
    spec.bc = (pb.BC_DIRICHLET, pb.BC_EXTRAP, pb.BC_EXTRAP, pb.BC_EXTRAP)
    spec.dirichlet_prim = [spec.prim[:, 0, 0].copy(), None, None, None]
    s = oracle_setup(spec)
    W0 = oracle_W(spec, s)
    sol = solver_for(spec, precision=precision)
    We, Wr = dev(W0), dev(W0)
    ebuf = torch.zeros(40, dtype=torch.float64, device="cuda")
    rbuf = torch.zeros(40, dtype=torch.float64, device="cuda")
    for k in range(40):
        sol.step(We, 0.0, dt_used=ebuf[k:k + 1])
    n, t = sol.run(Wr, 1.0, max_steps=40, dts=rbuf)
    assert n == 40
    assert torch.equal(We, Wr)
    assert torch.equal(ebuf, rbuf)
    assert t == sum(host(ebuf).tolist()) or abs(t - host(ebuf).sum()) <= 1e-18


def test_run_edge_cases():
    spec = pb.water_air_shock_tube(64)
    s = oracle_setup(spec)
    W0 = oracle_W(spec, s)
    sol = solver_for(spec)
    Wd = dev(W0)
    assert sol.run(Wd, spec.t_end, max_steps=0) == (0, 0.0)
    assert np.array_equal(host(Wd), W0)
    assert sol.run(Wd, 0.0) == (0, 0.0)               # already at t_end
    n, t = sol.run(Wd, 1e-6, t=1e-6 - 1e-9)           # one short step (two if t + dt rounds low)
    assert n in (1, 2) and t == 1e-6
    with pytest.raises(wcns.WcnsError):
        sol.run(Wd, 1.0, dt_fixed=-1.0)
    sol2 = solver_for(pb.random_smooth_state(16, 16, 1))   # 2D: not available
    with pytest.raises(wcns.WcnsError):
        sol2.run(dev(oracle_W(pb.random_smooth_state(16, 16, 1))), 1e-6)


@pytest.mark.parametrize("nsteps", [3999, 2048])
def test_run_counts_inadmissible_cells_like_stepping(nsteps):
    """The whole-run kernel counts the cells outside G exactly as the
    multi-kernel steps do (the run's input, every stage result): Sedov with
    both limiters off, 3999 fixed steps (three full launches of 1024 steps
    and a partial one) or 2048 (ending on a launch boundary), against
    wcns_ssprk3_steps on a fresh context.  The final states agree bit for
    bit (NaNs in the same places)."""
    spec = pb.sedov_multimaterial(401)
    s = oracle_setup(spec)
    W0 = oracle_W(spec, s)
    sol_r = solver_for(spec, interp_limiter=False, flux_limiter=False)
    sol_s = solver_for(spec, interp_limiter=False, flux_limiter=False)
    Wr, Ws = dev(W0), dev(W0)
    n, t = sol_r.run(Wr, 1.0, dt_fixed=spec.dt_fixed, max_steps=nsteps)
    assert n == nsteps
    sol_s.steps(Ws, nsteps, spec.dt_fixed)
    vr, vs = sol_r.violations(clear=True), sol_s.violations(clear=True)
    print(f"  limiters off, {nsteps} steps: run counted {vr}, steps counted {vs}", flush=True)
    assert vr == vs > 0
    assert np.array_equal(host(Wr), host(Ws), equal_nan=True)


def test_run_and_advance_stop_when_a_step_would_not_advance_the_time():
    """A step too small to change t (here dt = 1e-300 at t = 1; an infinite
    wave speed gives the same) ends the device time loop instead of leaving
    it running in place: wcns_run returns WCNS_ERR_CFL and the device loop
    of Solver.advance skips the step, which raises; the state is untouched."""
    spec = pb.water_air_shock_tube(64)
    s = oracle_setup(spec)
    W0 = oracle_W(spec, s)
    sol = solver_for(spec)
    Wd = dev(W0)
    with pytest.raises(wcns.WcnsError) as e:
        sol.run(Wd, 2.0, t=1.0, dt_fixed=1e-300)
    assert e.value.code == -6
    with pytest.raises(wcns.WcnsError) as e:
        sol.advance(Wd, 2.0, t=1.0, dt=1e-300, chunk=8)
    assert e.value.code == -6
    assert np.array_equal(host(Wd), W0)
    assert sol.violations() == 0
    n, t = sol.run(Wd, spec.t_end, dt_fixed=spec.dt_fixed)   # the context still runs
    assert n > 0 and t == spec.t_end
