"""Write tests/golden/full_runs.json: the oracle's whole solves of the two
full-size 2D workloads, kept as the SHA-256 of the final state's bytes (and
a few readable figures), so that a GPU test can hold the device's whole solve
to the oracle bit for bit without the oracle's hours of CPU time:

  * the shock-bubble interaction at 1024^2, 1000 CFL-0.5 SSP-RK3 steps;
  * the underwater explosion near a wall at 2048^2 (FP64) to its final time
    t = 2e-4 s, the last step shortened to land on it.

Calls only the oracle (its OpenMP build, bit-identical to the serial one;
about 25 minutes on 8 cores).  Run from the repository root:
    python tests/golden/write_full_runs.py
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
        "grid": [spec.nx, spec.ny],
        "steps": steps,
        "t": t,
        "t_hex": float(t).hex(),
        "sha256": digest(W),
        "component_sums": [float(np.sum(W[k])) for k in range(W.shape[0])],
        "alpha1_min_max": [float(W[5].min()), float(W[5].max())],
        "inadmissible": orc.count_inadmissible(s, W),
        "oracle_seconds": round(secs, 1),
    }


def main():
    out = {"note": "final states of whole oracle solves (oracle/oracle.py run_parallel), "
                   "written by tests/golden/write_full_runs.py; sha256 of the state as "
                   "[6][ny][nx] little-endian float64",
           "runs": {}}
    sb = pb.shock_bubble(1024)
    s = oracle_setup(sb)
    t0 = time.time()
    W, steps, t = orc.run_parallel(s, oracle_W(sb, s), float("inf"), 0.0, 1000)
    out["runs"]["shock_bubble_1024_1000_steps"] = record(
        "2D shock-bubble 1024x1024, 1000 SSP-RK3 steps at CFL 0.5", sb, W, steps, t, time.time() - t0)
    print(json.dumps(out["runs"]["shock_bubble_1024_1000_steps"]), flush=True)
    del W
    ue = pb.underwater_explosion(2048)
    s = oracle_setup(ue)
    t0 = time.time()
    W, steps, t = orc.run_parallel(s, oracle_W(ue, s), ue.t_end)
    out["runs"]["underwater_explosion_2048_to_t_end"] = record(
        f"2D underwater explosion near a wall 2048x2048, FP64, to t = {ue.t_end} s", ue, W, steps, t,
        time.time() - t0)
    print(json.dumps(out["runs"]["underwater_explosion_2048_to_t_end"]), flush=True)
    with open(os.path.join(HERE, "full_runs.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
