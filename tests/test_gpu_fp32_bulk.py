"""Precision form: FP32 bulk (interpolation, midpoint flux, HCS) with FP64
primitive recovery, limiters and fallback flux, checked against the FP64
oracle.  Accuracy is stated as relative L1 per variable; positivity and
boundedness must hold exactly (no inadmissible cell after any step)."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from helpers import oracle_setup, oracle_W, orc, pb

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2102_05287_amd import wcns  # noqa: E402

FP32 = wcns.FP32_BULK


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l1(g, r):
    return [float(np.abs(g[v] - r[v]).sum() / max(np.abs(r[v]).sum(), 1e-300)) for v in range(r.shape[0])]


def step_error(spec, s, W, dt, got, ref):
    """Per-variable error of one Euler step dt*L relative to the state scale
    (|W_v|; rho*c for the momenta, whose state can be identically zero)."""
    V, c = orc.cons_to_prim(s, W)
    rho = W[0] + W[1]
    out = []
    for v in range(W.shape[0]):
        mom = v in (2, 3) if spec.ndim == 2 else v == 2
        scale = np.abs(rho * c).sum() if mom else np.abs(W[v]).sum()
        out.append(float(dt * np.abs(got[v] - ref[v]).sum() / scale))
    return out


def test_fp32_bulk_rhs_close_to_oracle_on_smooth_data():
    """Smooth data (no limiter activity): one FP32-bulk RHS is within FP32
    round-off of the oracle.  (At material interfaces the limiters divide by
    differences of ~1e-8, so FP32 rounding moves their theta at O(1); there
    the meaningful comparison is the final-time L1 below.)"""
    specs = [pb.random_smooth_state(96, 70, 3, with_bubble=False, with_shock=False),
             pb.convergence_advection(64)]
    for spec in specs:
        s = oracle_setup(spec)
        W = oracle_W(spec, s)
        dt = orc.cfl_dt(s, W)
        ref = orc.rhs(s, W, dt)
        sol = wcns.Solver.from_spec(spec, precision=FP32)
        got = host(sol.rhs(dev(W), dt=dt))
        errs = step_error(spec, s, W, dt, got, ref)
        print(f"  fp32 rhs {spec.name}: per-step relative error {['%.1e' % e for e in errs]}", flush=True)
        assert max(errs) < 1e-6, errs


def run_gpu(sol, W0, t_end, cfl, dx, dy):
    Wd = dev(W0)
    t, n = 0.0, 0
    while t < t_end:
        a = host(sol.max_wavespeed(Wd))
        dt = cfl / (a[0] / dx + a[1] / dy)
        if t + dt > t_end:
            dt = t_end - t
        sol.step(Wd, dt)
        t += dt
        n += 1
        assert sol.count_inadmissible(Wd) == 0, n
    return host(Wd), n


def test_fp32_bulk_underwater_explosion_256_l1():
    """Underwater explosion at 256^2 to t = 2e-4 s: FP32-bulk GPU against the
    FP64 oracle (and the FP64 GPU path), relative L1 per variable."""
    spec = pb.underwater_explosion(256)
    s = oracle_setup(spec)
    W0 = oracle_W(spec, s)
    ref, steps, _ = orc.run(s, W0, spec.t_end)
    sol32 = wcns.Solver.from_spec(spec, precision=FP32)
    got32, n32 = run_gpu(sol32, W0, spec.t_end, spec.cfl, spec.dx, spec.dy)
    sol64 = wcns.Solver.from_spec(spec)
    got64, n64 = run_gpu(sol64, W0, spec.t_end, spec.cfl, spec.dx, spec.dy)
    e32 = rel_l1(got32, ref)
    e64 = rel_l1(got64, ref)
    print("  underwater 256 steps oracle/fp64/fp32:", steps, n64, n32, flush=True)
    print("  rel L1 fp32 vs oracle:", ["%.2e" % e for e in e32], flush=True)
    print("  rel L1 fp64 vs oracle:", ["%.2e" % e for e in e64], flush=True)
    assert max(e64) <= 1e-9
    assert max(e32) < 2e-3, e32


def test_fp32_bulk_full_size_2048_against_fp64_gpu():
    """The precision form at its full size (2048^2 underwater explosion, the
    bench's launch configuration): 10 steps of the FP32-bulk path against
    the FP64 path on the same GPU, both with the FP64 path's CFL time step,
    relative L1 per variable below 1e-2 (measured 1e-7 .. 4e-3, largest for
    the momenta, which start at zero) and no inadmissible cell."""
    spec = pb.underwater_explosion(2048)
    V = torch.from_numpy(spec.prim).cuda()
    spec.prim = None
    sol64 = wcns.Solver.from_spec(spec)
    sol32 = wcns.Solver.from_spec(spec, precision=FP32)
    W64 = sol64.prim_to_cons(V)
    W32 = W64.clone()
    del V
    dtu = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(10):
        sol64.step(W64, 0.0, dt_used=dtu)
        sol32.step(W32, float(dtu.item()))
    assert sol32.count_inadmissible(W32) == 0 and sol64.count_inadmissible(W64) == 0
    e = [float((W32[v] - W64[v]).abs().sum() / W64[v].abs().sum()) for v in range(6)]
    print("  2048^2 rel L1 fp32-bulk vs fp64:", ["%.2e" % x for x in e], flush=True)
    assert max(e) < 1e-2, e


def test_first_order_scheme_is_fp64_in_both_precisions():
    """The first-order HLLC mode has no interpolation, midpoint flux or HCS,
    the parts the precision form runs in FP32, so its FP32-bulk solve is
    the FP64 one: steps of a random 2D state (periodic and Dirichlet sides,
    several y-tiles) and of a 1D tube, bit for bit in both precisions and
    against the oracle."""
    cases = [pb.random_smooth_state(70, 45, 21), pb.water_air_shock_tube(200)]
    dirichlet = pb.random_smooth_state(66, 37, 22)
    dirichlet.bc = (pb.BC_DIRICHLET, pb.BC_EXTRAP, pb.BC_PERIODIC, pb.BC_PERIODIC)
    dirichlet.dirichlet_prim = [dirichlet.prim[:, :, 0].T.copy(), None, None, None]
    cases.append(dirichlet)
    for spec in cases:
        s = oracle_setup(spec, scheme=1)
        W = oracle_W(spec, s)
        ref = W
        for _ in range(3):
            ref, dt, bad = orc.ssprk3_step(s, ref)
            assert bad == 0
        out = []
        for prec in (wcns.FP64, FP32):
            sol = wcns.Solver.from_spec(spec, precision=prec, scheme=1)
            Wd = dev(W)
            sol.steps(Wd, 3, 0.0)
            out.append(host(Wd))
            sol.close()
        print(f"  hllc1 {spec.name}: fp64 == fp32-bulk == oracle", flush=True)
        assert np.array_equal(out[0], out[1]), spec.name
        assert np.array_equal(out[0], ref), spec.name
