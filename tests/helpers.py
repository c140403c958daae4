"""Test helpers: build oracle setups from the seeded problem specs."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2102_05287_amd import problems as pb  # noqa: E402


def oracle_setup(spec: pb.ProblemSpec, **kw) -> orc.Setup:
    s = orc.Setup(ndim=spec.ndim, nx=spec.nx, ny=spec.ny, dx=spec.dx, dy=spec.dy,
                  bc=tuple(spec.bc), gamma=spec.gamma, pinf=spec.pinf, cfl=spec.cfl,
                  dirichlet_prim=list(spec.dirichlet_prim), nz=spec.nz, dz=spec.dz)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def oracle_W(spec: pb.ProblemSpec, s: orc.Setup | None = None) -> np.ndarray:
    s = s or oracle_setup(spec)
    return orc.prim_to_cons(s, spec.prim)


def l2_alpha_error(spec, W, t):
    """L2 error of alpha_1 against the exact convergence solution [Sec. 6.1]."""
    ex = pb.convergence_exact_alpha(spec, t)
    a = W[5]
    return float(np.sqrt(np.sum(spec.dx * spec.dy * (a - ex) ** 2) / np.sum(spec.dx * spec.dy * np.ones_like(a))))
