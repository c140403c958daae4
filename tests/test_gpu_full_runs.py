"""Whole solves of the full-size 2D workloads held to the oracle bit for
bit: the shock-bubble interaction at 1024^2 over 1000 CFL steps (one
multi-step call), the underwater explosion near a wall at 2048^2 in FP64 to
its final time t = 2e-4 s and the Mach 100 jet with its per-row Dirichlet
inflow to t = 4e-6 s (the device time loop, last step shortened on the
device), and the 3D underwater explosion at 256^3 over 20 CFL steps.  The oracle's final states take over an hour of CPU on 8 cores, so
they are kept as SHA-256 digests with the step counts and final times
(tests/golden/full_runs.json, written from the oracle alone by
tests/golden/write_full_runs.py); the device's state must hash the same."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import pytest

from helpers import oracle_setup, oracle_W, pb
from test_gpu_parity import dev, host, solver_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_runs.json")) as _f:
    GOLD = json.load(_f)["runs"]


def digest(W: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(W, dtype="<f8").tobytes()).hexdigest()


def test_shock_bubble_1000_steps_is_the_oracles_bit_for_bit():
    g = GOLD["shock_bubble_1024_1000_steps"]
    spec = pb.shock_bubble(1024)
    Wd = dev(oracle_W(spec, oracle_setup(spec)))
    sol = solver_for(spec)
    dts = torch.zeros(1000, dtype=torch.float64, device="cuda")
    sol.steps(Wd, 1000, 0.0, dts=dts)
    W = host(Wd)
    t = 0.0
    for d in host(dts).tolist():
        t += d
    print(f"  shock-bubble 1000 steps: t = {t!r} (oracle {g['t']!r})", flush=True)
    assert t == g["t"]
    assert digest(W) == g["sha256"]
    assert sol.violations() == 0
    sol.close()


@pytest.mark.parametrize("key", ["underwater_explosion_2048_to_t_end", "mach100_jet_to_t_end"])
def test_solve_to_final_time_is_the_oracles_bit_for_bit(key):
    g = GOLD[key]
    spec = pb.underwater_explosion(2048) if key.startswith("underwater") else pb.mach100_jet()
    Wd = dev(oracle_W(spec, oracle_setup(spec)))
    sol = solver_for(spec)
    n, t = sol.advance(Wd, spec.t_end, chunk=128)
    print(f"  {key}: {n} steps, t = {t!r} (oracle {g['steps']}, {g['t']!r})",
          flush=True)
    assert n == g["steps"] and t == g["t"]
    assert digest(host(Wd)) == g["sha256"]
    assert sol.violations() == 0
    sol.close()


def test_3d_underwater_explosion_20_steps_is_the_oracles_bit_for_bit():
    g = GOLD["underwater_explosion_3d_256_20_steps"]
    spec = pb.underwater_explosion_3d(256)
    Wd = dev(oracle_W(spec, oracle_setup(spec)))
    spec.prim = None
    sol = solver_for(spec)
    dts = torch.zeros(20, dtype=torch.float64, device="cuda")
    sol.steps(Wd, 20, 0.0, dts=dts)
    t = 0.0
    for d in host(dts).tolist():
        t += d
    print(f"  3D 256^3 20 steps: t = {t!r} (oracle {g['t']!r})", flush=True)
    assert t == g["t"]
    assert digest(host(Wd)) == g["sha256"]
    assert sol.violations() == 0
    sol.close()
