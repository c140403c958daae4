"""The FP64 issue-cost probe that weights divides and square roots in the
roofline: its timings scale with the work and its ratios fall in the range
the instruction sequences allow (an IEEE divide is 11 VALU instructions on
gfx950, one of them a quarter-rate reciprocal; a square root 19)."""
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
