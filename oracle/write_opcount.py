"""Write tests/golden/opcount.json: the oracle's algorithmic operation counts
per node and per face on the common path (smooth data, no limiter branch
taken), used to price the ALU roofline.  Calls only the oracle."""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
from oracle import oracle as orc  # noqa: E402


def main():
    out = {"source": "oracle/wcns_oracle.cpp instantiated with the counting scalar",
           "state": "2D water/air mixture, alpha = 0.5 + 0.25 sin(pi(x+y)), u=v=10, "
                    "p=101325 (paper Sec. 6.1 convergence problem), N=16, face between "
                    "cells 2 and 3 of row 3; no limiter branch taken",
           "counts": {}}
    for scheme, name in ((0, "ppwcnsis"), (1, "hllc1")):
        s = orc.Setup(ndim=2, nx=16, ny=16, dx=2.0 / 16, dy=2.0 / 16, scheme=scheme)
        x = -1.0 + (np.arange(16) + 0.5) * 2.0 / 16
        X, Y = np.meshgrid(x, x)
        a1 = 0.5 + 0.25 * np.sin(np.pi * (X + Y))
        V = np.stack([1000.0 * a1, 1.0 - a1, 10 + 0 * a1, 10 + 0 * a1, 101325 + 0 * a1, a1])
        W = orc.prim_to_cons(s, V)
        st = np.array([[W[v, 3, i] for v in range(6)] for i in range(6)])
        out["counts"][name] = orc.opcount_face(s, st, 1e-6)
    # 3D face: the same mixture extruded in z with w = 10 (7 components)
    s3 = orc.Setup(ndim=3, nx=16, ny=16, nz=4, dx=2.0 / 16, dy=2.0 / 16, dz=2.0 / 16)
    x = -1.0 + (np.arange(16) + 0.5) * 2.0 / 16
    X, Y = np.meshgrid(x, x)
    a1 = 0.5 + 0.25 * np.sin(np.pi * (X + Y))
    V = np.stack([1000.0 * a1, 1.0 - a1, 10 + 0 * a1, 10 + 0 * a1, 10 + 0 * a1,
                  101325 + 0 * a1, a1])
    V3 = np.repeat(V[:, None], 4, axis=1)
    W3 = orc.prim_to_cons(s3, V3)
    st3 = np.array([[W3[v, 0, 3, i] for v in range(7)] for i in range(6)])
    out["counts"]["ppwcnsis_3d"] = orc.opcount_face(s3, st3, 1e-6)
    out["state_3d"] = "the same mixture extruded along z with w = 10, 16x16x4, x-face"
    path = os.path.join(os.path.dirname(HERE), "tests", "golden", "opcount.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
