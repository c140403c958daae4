"""Exact Riemann solver for two stiffened gases (textbook two-shock /
two-rarefaction construction with p -> p + p_inf on each side).

Used only to pin the reference implementation on shock tubes: the left and
right states may have different (gamma, p_inf).  Solution is sampled at
x/t.  Pure-python + numpy; scipy's brentq finds the star pressure.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


class Side:
    def __init__(self, rho, u, p, gamma, pinf):
        self.rho, self.u, self.p, self.g, self.pinf = rho, u, p, gamma, pinf
        self.c = math.sqrt(gamma * (p + pinf) / rho)

    def f(self, p):
        """Velocity jump across the wave connecting this side to pressure p."""
        g, pb, pK = self.g, p + self.pinf, self.p + self.pinf
        if p > self.p:   # shock
            A = 2.0 / ((g + 1.0) * self.rho)
            B = (g - 1.0) / (g + 1.0) * pK
            return (p - self.p) * math.sqrt(A / (pb + B))
        return 2.0 * self.c / (g - 1.0) * ((pb / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(L: Side, R: Side):
    fun = lambda p: L.f(p) + R.f(p) + R.u - L.u
    lo = -min(L.pinf, R.pinf) + 1e-9 * max(L.p + L.pinf, R.p + R.pinf)
    hi = 10.0 * max(L.p + L.pinf, R.p + R.pinf)
    ps = brentq(fun, lo, hi, xtol=1e-12, rtol=1e-15, maxiter=500)
    us = 0.5 * (L.u + R.u) + 0.5 * (R.f(ps) - L.f(ps))
    return ps, us


def _side_sample(K: Side, ps, us, xi, left: bool):
    """Sample (rho, u, p) at similarity coordinate xi on one side of the contact."""
    g, pinf = K.g, K.pinf
    sgn = -1.0 if left else 1.0
    pK, pS = K.p + pinf, ps + pinf
    if ps > K.p:  # shock
        rho_s = K.rho * ((pS / pK + (g - 1.0) / (g + 1.0)) / ((g - 1.0) / (g + 1.0) * pS / pK + 1.0))
        S = K.u + sgn * K.c * math.sqrt((g + 1.0) / (2.0 * g) * pS / pK + (g - 1.0) / (2.0 * g))
        if (left and xi < S) or (not left and xi > S):
            return K.rho, K.u, K.p
        return rho_s, us, ps
    # rarefaction
    rho_s = K.rho * (pS / pK) ** (1.0 / g)
    c_s = K.c * (pS / pK) ** ((g - 1.0) / (2.0 * g))
    head = K.u + sgn * K.c
    tail = us + sgn * c_s
    if (left and xi < head) or (not left and xi > head):
        return K.rho, K.u, K.p
    if (left and xi > tail) or (not left and xi < tail):
        return rho_s, us, ps
    # inside the fan
    if left:
        c = 2.0 / (g + 1.0) * (K.c + (g - 1.0) / 2.0 * (K.u - xi))
        u = 2.0 / (g + 1.0) * (K.c + (g - 1.0) / 2.0 * K.u + xi)
    else:
        c = 2.0 / (g + 1.0) * (K.c - (g - 1.0) / 2.0 * (K.u - xi))
        u = 2.0 / (g + 1.0) * (-K.c + (g - 1.0) / 2.0 * K.u + xi)
    rho = K.rho * (c / K.c) ** (2.0 / (g - 1.0))
    p = pK * (c / K.c) ** (2.0 * g / (g - 1.0)) - pinf
    return rho, u, p


def sample(L: Side, R: Side, x: np.ndarray, x0: float, t: float):
    """(rho, u, p, side) arrays at positions x, time t; side 0 left material."""
    ps, us = star_state(L, R)
    out = np.zeros((4, x.size))
    for k, xv in enumerate(x):
        xi = (xv - x0) / t
        if xi < us:
            out[:3, k] = _side_sample(L, ps, us, xi, True)
            out[3, k] = 0
        else:
            out[:3, k] = _side_sample(R, ps, us, xi, False)
            out[3, k] = 1
    return out
