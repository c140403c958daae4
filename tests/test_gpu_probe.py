"""The measurement aids behind the roofline: the FP64 issue-cost probe
that weights divides and square roots (its timings scale with the work and
its ratios fall in the range the instruction sequences allow: an IEEE
divide is 11 VALU instructions on gfx950, one of them a quarter-rate
reciprocal; a square root 19), and the per-class launch profile."""
from __future__ import annotations

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2102_05287_amd import wcns  # noqa: E402


def test_issue_probe_scales_and_weights_are_plausible():
    wcns.issue_probe("fma", 64)
    t1 = wcns.issue_probe("fma", 512)
    t2 = wcns.issue_probe("fma", 2048)
    assert 0 < t1 < t2 and 2.5 < t2 / t1 < 5.5        # linear in the work
    w = wcns.issue_weights(1024)["weights"]
    assert 0.8 < w["fma"] < 1.25                   # FMA over the FMA run before it
    assert 0.5 < w["add"] < 1.5 and 0.5 < w["mul"] < 1.5
    assert 8.0 < w["div"] < 20.0
    assert 6.0 < w["div_core"] < w["div"] * 1.2
    assert 10.0 < w["sqrt"] < 30.0
    # FP32 without packed math issues at the FP64 rate; the quotient is a
    # quarter-rate reciprocal and a product
    assert 0.8 < w["fma_f32"] < 1.25
    assert 2.0 < w["div_f32"] < 8.0
    assert 1.0 < w["sqrt_f32"] < 20.0


def test_profile_counts_the_launches_of_a_multi_step_call():
    """The per-class launch counts the roofline reads (wcns_profile): n steps
    in one 2D call run the node primitives once and, per stage, one
    finalize, one x-sweep, one y-sweep and one fixup; an RHS evaluation
    runs the node primitives again.  The times are positive."""
    import numpy as np
    from paper_2102_05287_amd import problems as pb
    spec = pb.random_smooth_state(96, 70, 5)          # 71 face rows: 5 y-tile rows, a fixup
    sol = wcns.Solver.from_spec(spec)
    W = sol.prim_to_cons(torch.from_numpy(np.ascontiguousarray(spec.prim)).cuda())
    sol.profile(True)
    n = 4
    sol.steps(W, n, 0.0)
    prof = sol.profile_read(reset=True)
    assert prof["node"][1] == 1
    for k in ("finalize", "sweep_x", "sweep_y", "fixup_y"):
        assert prof[k][1] == 3 * n, (k, prof[k])
        assert prof[k][0] > 0.0
    sol.rhs(W, dt=1e-9)
    prof = sol.profile_read(reset=True)
    assert prof["node"][1] == 1 and prof["sweep_y"][1] == 1 and prof["finalize"][1] == 1
    sol.profile(False)
    sol.close()


def test_profile_survives_a_stream_switch():
    """Switching the context's stream with profiling on folds the timings
    recorded on the old stream first: the launch counts of steps taken on
    two streams add up and every class has a positive time."""
    import numpy as np
    from paper_2102_05287_amd import problems as pb
    spec = pb.random_smooth_state(96, 70, 6)
    sol = wcns.Solver.from_spec(spec)
    W = sol.prim_to_cons(torch.from_numpy(np.ascontiguousarray(spec.prim)).cuda())
    torch.cuda.synchronize()
    sol.profile(True)
    sol.steps(W, 2, 0.0)
    other = torch.cuda.Stream()
    other.wait_stream(torch.cuda.current_stream())
    sol.set_stream(other.cuda_stream)
    sol.steps(W, 3, 0.0)
    prof = sol.profile_read(reset=True)
    sol.set_stream(torch.cuda.current_stream().cuda_stream)
    torch.cuda.current_stream().wait_stream(other)
    assert prof["node"][1] == 2                      # the first stage of each call
    for k in ("finalize", "sweep_x", "sweep_y", "fixup_y"):
        assert prof[k][1] == 3 * 5, (k, prof[k])
        assert prof[k][0] > 0.0
    sol.profile(False)
    sol.close()
