"""Write tests/golden/full_runs.json: the oracle's whole solves of the two
full-size 2D workloads, kept as the SHA-256 of the final state's bytes (and
a few readable figures), so that a GPU test can hold the device's whole solve
to the oracle bit for bit without the oracle's hours of CPU time:

  * the shock-bubble interaction at 1024^2, 1000 CFL-0.5 SSP-RK3 steps;
  * the underwater explosion near a wall at 2048^2 (FP64) to its final time
    t = 2e-4 s, the last step shortened to land on it;
  * the Mach 100 water jet at 1024 x 512 (per-row Dirichlet inflow) to its
    final time 4e-6 s;
  * the 3D underwater explosion near a wall at 256^3, 20 CFL steps.

Calls only the oracle (its OpenMP build, bit-identical to the serial one;
about 14, 60, 20 and 10 minutes on 8 cores).  Run from the repository root,
naming the runs to (re)compute (default: all); the others are kept:
    python tests/golden/write_full_runs.py [shock_bubble underwater jet 3d]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
from helpers import oracle_setup, oracle_W  # noqa: E402
from helpers import orc, pb  # noqa: E402


def digest(W: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(W, dtype="<f8").tobytes()).hexdigest()


def record(name, spec, W, steps, t, secs):
    s = oracle_setup(spec)
    return {
        "workload": name,
        "grid": [spec.nx, spec.ny] + ([spec.nz] if spec.ndim == 3 else []),
        "steps": steps,
        "t": t,
        "t_hex": float(t).hex(),
        "sha256": digest(W),
        "component_sums": [float(np.sum(W[k])) for k in range(W.shape[0])],
        "alpha1_min_max": [float(W[-1].min()), float(W[-1].max())],
        "inadmissible": orc.count_inadmissible(s, W),
        "oracle_seconds": round(secs, 1),
    }


def main(which):
    path = os.path.join(HERE, "full_runs.json")
    out = {"note": "final states of whole oracle solves (oracle/oracle.py run_parallel), "
                   "written by tests/golden/write_full_runs.py; sha256 of the state as "
                   "[nvar][ny][nx] little-endian float64",
           "runs": {}}
    if os.path.exists(path):
        with open(path) as f:
            out["runs"] = json.load(f)["runs"]

    def solve(key, name, spec, t_end, max_steps=10**9):
        s = oracle_setup(spec)
        t0 = time.time()
        W, steps, t = orc.run_parallel(s, oracle_W(spec, s), t_end, 0.0, max_steps)
        out["runs"][key] = record(name, spec, W, steps, t, time.time() - t0)
        print(json.dumps(out["runs"][key]), flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)

    if "shock_bubble" in which:
        solve("shock_bubble_1024_1000_steps", "2D shock-bubble 1024x1024, 1000 SSP-RK3 steps at CFL 0.5",
              pb.shock_bubble(1024), float("inf"), 1000)
    if "underwater" in which:
        ue = pb.underwater_explosion(2048)
        solve("underwater_explosion_2048_to_t_end",
              f"2D underwater explosion near a wall 2048x2048, FP64, to t = {ue.t_end} s", ue, ue.t_end)
    if "jet" in which:
        jet = pb.mach100_jet()
        solve("mach100_jet_to_t_end",
              f"2D Mach 100 water jet 1024x512 (per-row Dirichlet inflow) to t = {jet.t_end} s", jet,
              jet.t_end)
    if "3d" in which:
        solve("underwater_explosion_3d_256_20_steps",
              "3D underwater explosion near a wall 256^3, 20 SSP-RK3 steps at CFL 0.5",
              pb.underwater_explosion_3d(256), float("inf"), 20)


if __name__ == "__main__":
    main(sys.argv[1:] or ["shock_bubble", "underwater", "jet", "3d"])
