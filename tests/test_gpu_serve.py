"""Serving form: continuous batching of mixed 1D/2D, FP64/FP32-bulk solves.
Each served result must equal the same solve run alone, bit for bit (the
batched kernels run the single-solve arithmetic per tile); every FP64 served
result must equal the oracle's solve bit for bit, and every FP32-bulk one
must stay within the precision form's stated L1 bound of it; admission must
respect the HBM budget, and every solve must get exactly its own steps."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import oracle_setup, orc, pb

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2102_05287_amd import serve, wcns  # noqa: E402


def small_trace(k=14, seed=7):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for rid in range(k):
        t += rng.exponential(0.02)
        ndim = 1 if rng.uniform() < 0.5 else 2
        n = int(rng.integers(100, 400)) if ndim == 1 else int(rng.integers(16, 48))
        r = pb.Request(rid, t, ndim, n, int(rng.integers(3, 30)), bool(rng.uniform() < 0.5),
                       int(rng.integers(0, 2**31)))
        out.append(serve.Solve(rid, t, pb.request_problem(r), r.steps, r.fp32))
    return out


def alone(s):
    sp = s.spec
    sol = wcns.Solver.from_spec(sp, precision=wcns.FP32_BULK if s.fp32 else wcns.FP64)
    V = torch.from_numpy(np.ascontiguousarray(sp.prim)).cuda()
    W = wcns.prim_to_cons(V, sp.ndim)
    for _ in range(s.steps):
        sol.step(W, 0.0)
    torch.cuda.synchronize()
    return W.cpu().numpy()


def oracle_solve(s):
    """The request run by the oracle: the same CFL SSP-RK3 steps."""
    sp = s.spec
    st = oracle_setup(sp)
    W = orc.prim_to_cons(st, sp.prim)
    for _ in range(s.steps):
        W, _, bad = orc.ssprk3_step(st, W)
        assert bad == 0, s.rid
    return st, W


def fp32_error(st, got, ref):
    """Relative L1 error per variable (momenta against the sum of rho*c,
    since their own sum can be near zero)."""
    V, c = orc.cons_to_prim(st, ref)
    rho = ref[0] + ref[1]
    out = []
    for v in range(ref.shape[0]):
        mom = v == 2 or (ref.shape[0] == 6 and v == 3)
        scale = np.abs(rho * c).sum() if mom else np.abs(ref[v]).sum()
        out.append(float(np.abs(got[v] - ref[v]).sum() / scale))
    return out


def test_served_results_equal_solo_results():
    solves = small_trace()
    biggest = max(serve.footprint_bytes(s.spec.ndim, s.spec.nx, s.spec.ny) for s in solves)
    budget = 3 * biggest           # forces queueing: not everything fits at once
    srv = serve.Server(hbm_budget=budget, max_slots=6, chunk=4, keep_results=True)
    done, summary = srv.run(solves, realtime=True)
    assert summary["requests"] == len(solves)
    assert srv.peak_used <= budget
    assert srv.used == 0 and srv.active == 0
    assert summary["failed"] == 0
    worst32 = 0.0
    for s in done:
        assert s.taken == s.steps and not s.failed
        ref = alone(s)
        assert np.array_equal(s.result, ref), s.rid
        st, orc_ref = oracle_solve(s)
        got = s.result.reshape(orc_ref.shape)
        if s.fp32:
            e = fp32_error(st, got, orc_ref)
            worst32 = max(worst32, max(e))
            assert max(e) < 2e-3, (s.rid, e)
        else:
            assert np.array_equal(got, orc_ref), s.rid
    print(f"  served FP64 results == oracle; FP32-bulk worst relative L1 {worst32:.2e}", flush=True)
    print("  serve summary:", summary, flush=True)


def test_server_retires_a_failing_solve():
    """A request whose initial state has a cell outside the admissible set
    (a1 = 1.5) is retired as failed after the tick that found it; the
    others complete and equal their solo solves."""
    solves = small_trace(6, seed=11)
    bad = solves[2]
    bad.spec.prim = np.array(bad.spec.prim)
    bad.spec.prim[-1].flat[bad.spec.prim[-1].size // 2] = 1.5
    srv = serve.Server(hbm_budget=1 << 30, max_slots=8, chunk=3, keep_results=True)
    done, summary = srv.run(solves, realtime=False)
    assert summary["requests"] == len(solves) and summary["failed"] == 1
    for s in done:
        if s.rid == bad.rid:
            assert s.failed and s.bad_cells >= 1
            continue
        assert not s.failed and s.taken == s.steps
        assert np.array_equal(s.result, alone(s)), s.rid


def test_server_rejects_a_request_larger_than_the_budget():
    solves = small_trace(3)
    srv = serve.Server(hbm_budget=1024, max_slots=4, chunk=2)
    with pytest.raises(RuntimeError):
        srv.run(solves, realtime=False)
