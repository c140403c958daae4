"""Pins of the reference implementation (oracle) to what the paper and the
mathematics fix, independently of the oracle's own formulas.

Each test names the passage it checks.  CPU only.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

from helpers import oracle_setup, oracle_W, l2_alpha_error, orc, pb
import exact_riemann as er

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_table():
    rows = []
    with open(os.path.join(GOLDEN, "convergence_table.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, h, w = line.split()
                rows.append((int(n), float(h), float(w)))
    return rows


def _s2d(**kw):
    return orc.Setup(ndim=2, nx=1, ny=1, **kw)


def _cons(s, prim_rows):
    """prim rows (a1r1, a2r2, u, v, p, a1) -> conservative rows, via the oracle."""
    V = np.ascontiguousarray(np.array(prim_rows, dtype=float).T)
    return orc.prim_to_cons(s, V).T.copy()


# --------------------------------------------------------------------------
# Sec. 6.1 convergence table: the strongest end-to-end pin (no free constant
# for HLLC; the WENO epsilon reading for PP-WCNS-IS).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [8, 16, 32, 64])
def test_convergence_table_hllc(N):
    row = {r[0]: r for r in _golden_table()}[N]
    spec = pb.convergence_advection(N)
    s = oracle_setup(spec, scheme=1)
    W, steps, t = orc.run(s, oracle_W(spec, s), spec.t_end, spec.dt_fixed)
    assert abs(t - 1e-4) < 1e-15
    err = l2_alpha_error(spec, W, t)
    assert abs(err - row[1]) / row[1] < 1.5e-3, (err, row[1])


@pytest.mark.parametrize("N", [8, 16, 32, 64])
def test_convergence_table_ppwcnsis(N):
    row = {r[0]: r for r in _golden_table()}[N]
    spec = pb.convergence_advection(N)
    s = oracle_setup(spec, scheme=0)
    W, steps, t = orc.run(s, oracle_W(spec, s), spec.t_end, spec.dt_fixed)
    err = l2_alpha_error(spec, W, t)
    # the table prints 4 significant digits
    assert abs(err - row[2]) / row[2] < 1.5e-3, (err, row[2])


@pytest.mark.slow
@pytest.mark.parametrize("N", [128, 256])
def test_convergence_table_large(N):
    row = {r[0]: r for r in _golden_table()}[N]
    spec = pb.convergence_advection(N)
    for scheme, col in ((1, 1), (0, 2)):
        s = oracle_setup(spec, scheme=scheme)
        W, steps, t = orc.run(s, oracle_W(spec, s), spec.t_end, spec.dt_fixed)
        err = l2_alpha_error(spec, W, t)
        assert abs(err - row[col]) / row[col] < 5e-3, (scheme, err, row[col])


# --------------------------------------------------------------------------
# IS-WENO interpolation [Sec. 4.3; App. B]
# --------------------------------------------------------------------------
def test_weno_linear_limit_is_printed_s5():
    """With an enormous epsilon the IS weights reduce to d_k, so the value must
    equal the printed expanded 5-point interpolation (3,-20,90,60,-5)/128."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b, c, d, e = rng.normal(size=5) * 10 ** rng.uniform(-3, 3)
        got = orc.weno_is(a, b, c, d, e, eps=1e300)
        want = (3 * a - 20 * b + 90 * c + 60 * d - 5 * e) / 128.0
        assert abs(got - want) <= 1e-13 * (abs(a) + abs(b) + abs(c) + abs(d) + abs(e))


def test_weno_exact_for_quadratics():
    """Quadratic data: tau_5 vanishes, the weights are linear and the 5-point
    interpolation is exact [Sec. 4.3]."""
    for (A, B, Cc) in [(3, 2, 1), (-1, 5, 7), (0.5, -0.25, 2.0)]:
        f = lambda x: A * x * x + B * x + Cc
        vals = [f(x) for x in (-2, -1, 0, 1, 2)]
        got = orc.weno_is(*vals)
        assert abs(got - f(0.5)) <= 1e-14 * max(1.0, abs(f(0.5)))


def test_weno_fifth_order_smooth():
    """Away from critical points the nonlinear interpolation is fifth order
    [App. B]: error ratio ~ 2^5 under halving."""
    x0 = 0.3
    errs = []
    for h in (0.2, 0.1, 0.05, 0.025):
        xs = x0 + h * np.arange(-2, 3)
        got = orc.weno_is(*np.sin(xs + 0.4))
        errs.append(abs(got - math.sin(x0 + 0.5 * h + 0.4)))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(3)]
    assert min(rates[1:]) > 4.6, rates


def test_weno_picks_smooth_side_of_a_jump():
    """Step between u_i and u_{i+1}: the left-biased value uses the smooth
    two-point stencils and returns u_i (ENO property, Sec. 4.3)."""
    got = orc.weno_is(0.0, 0.0, 0.0, 1.0, 1.0)
    assert abs(got) < 1e-20
    got = orc.weno_is(1.0, 1.0, 1.0, 0.0, 0.0)
    assert abs(got - 1.0) < 1e-15


def test_weno_odd_symmetry():
    rng = np.random.default_rng(2)
    for _ in range(50):
        v = rng.normal(size=5)
        assert orc.weno_is(*(-v)) == -orc.weno_is(*v)


# --------------------------------------------------------------------------
# HCS explicit midpoint-and-node scheme [Sec. 4.1]
# --------------------------------------------------------------------------
def _hcs_derivative(G, Gt, h, i):
    # flux difference (Ghat_{i+1/2} - Ghat_{i-1/2})/h with Ghat from the oracle
    hp = orc.hcs(Gt(i + 0.5), G(i - 2), G(i - 1), G(i), G(i + 1), G(i + 2), G(i + 3))
    hm = orc.hcs(Gt(i - 0.5), G(i - 3), G(i - 2), G(i - 1), G(i), G(i + 1), G(i + 2))
    return (hp - hm) / h


def test_hcs_matches_printed_derivative_form():
    """The implied reconstructed flux must reproduce the printed HCS
    derivative with psi = 256/175 for arbitrary node/midpoint data."""
    rng = np.random.default_rng(3)
    psi = 256.0 / 175.0
    for _ in range(50):
        node = {k: rng.normal() for k in range(-3, 4)}
        mid = {k + 0.5: rng.normal() for k in (-1, 0)}
        G = lambda k: node[k]
        Gt = lambda k: mid[k]
        got = _hcs_derivative(G, Gt, 1.0, 0)
        want = (psi * (mid[0.5] - mid[-0.5])
                - (175 * psi - 192) / 256 * (node[1] - node[-1])
                + (35 * psi - 48) / 320 * (node[2] - node[-2])
                - (45 * psi - 64) / 3840 * (node[3] - node[-3]))
        assert abs(got - want) < 1e-13


def test_hcs_eighth_order_leading_error():
    """With exact midpoint fluxes the HCS derivative error is
    -(1/40320) G^(9) dx^8 + O(dx^10)  [Sec. 4.1]."""
    k, x0 = 1.0, 0.37
    for h in (0.4, 0.3):
        G = lambda m: math.sin(k * (x0 + m * h))
        got = _hcs_derivative(G, G, h, 0)
        err = got - k * math.cos(k * x0)
        lead = -(1.0 / 40320.0) * (k ** 9) * math.cos(k * x0) * h ** 8
        assert abs(err / lead - 1.0) < 0.05 * (h / 0.3) ** 2 + 0.02, (h, err, lead)


# --------------------------------------------------------------------------
# Characteristic decomposition [App. A]
# --------------------------------------------------------------------------
def test_projection_is_eigendecomposition_of_A():
    """Extract R^{-1} and R from the oracle's projection/back-projection and
    check R R^{-1} = I and R diag(-c,0,0,0,0,c) R^{-1} = A - u I with A the
    printed quasi-linear matrix at the face averages."""
    s = _s2d()
    rng = np.random.default_rng(4)
    for trial in range(5):
        pl = [800 + 200 * rng.uniform(), 0.5 + rng.uniform(), 10 * rng.normal(), 5 * rng.normal(),
              1e5 * (1 + 10 * rng.uniform()), 0.3 + 0.4 * rng.uniform()]
        pr = [800 + 200 * rng.uniform(), 0.5 + rng.uniform(), 10 * rng.normal(), 5 * rng.normal(),
              1e5 * (1 + 10 * rng.uniform()), 0.3 + 0.4 * rng.uniform()]
        XL, XR = _cons(s, [pl, pr])
        nl, nr = orc.node(s, XL), orc.node(s, XR)
        a1 = 0.5 * (XL[0] + XR[0]); a2 = 0.5 * (XL[1] + XR[1])
        rho = 0.5 * (nl[0] + nr[0]); c = 0.5 * (nl[4] + nr[4])
        base = np.array([900.0, 1.0, 3.0, -2.0, 3e5, 0.5])
        scale = np.array([50.0, 0.2, 2.0, 2.0, 5e4, 0.1])
        Vs = np.array([base + scale * (np.arange(6) == k) * (1 + k) for k in range(6)])
        Xs = _cons(s, Vs)
        Vx = np.array([[X[0], X[1], *orc.node(s, X)[1:4], X[5]] for X in Xs])  # exact V of X
        Us = np.array([orc.project(s, XL, XR, X) for X in Xs])
        Rinv = Us.T @ np.linalg.inv(Vx.T)
        Wb = np.array([orc.back_project(s, XL, XR, U) for U in Us])
        Vb = np.array([[X[0], X[1], *orc.node(s, X)[1:4], X[5]] for X in Wb])
        R = Vb.T @ np.linalg.inv(Us.T)
        D = np.diag(1.0 / scale)
        assert np.allclose(D @ R @ Rinv @ np.linalg.inv(D), np.eye(6), atol=1e-9)
        A = np.zeros((6, 6))
        A[0, 2] = a1; A[1, 2] = a2; A[2, 4] = 1.0 / rho; A[4, 2] = rho * c * c
        got = R @ np.diag([-c, 0, 0, 0, 0, c]) @ Rinv
        Sc = np.diag(scale)
        assert np.allclose(np.linalg.inv(Sc) @ got @ Sc, np.linalg.inv(Sc) @ A @ Sc,
                           rtol=1e-8, atol=1e-8 * np.abs(np.linalg.inv(Sc) @ A @ Sc).max())


# --------------------------------------------------------------------------
# Equation of state and admissible set [Sec. 2]
# --------------------------------------------------------------------------
def test_single_phase_limits_of_mixture_eos():
    """alpha_1 = 1 (0) must recover the stiffened-gas (ideal-gas) relation of
    one phase: rho e = (p + gamma pinf)/(gamma - 1)."""
    s = _s2d()
    for a1, g, pinf in ((1.0, 6.12, 3.43e8), (0.0, 1.4, 0.0)):
        rho, u, v, p = 900.0, 12.0, -4.0, 3e6
        E = (p + g * pinf) / (g - 1.0) + 0.5 * rho * (u * u + v * v)
        X = [rho * a1, rho * (1 - a1), rho * u, rho * v, E, a1]
        nd = orc.node(s, X)
        assert abs(nd[3] - p) < 1e-9 * (p + pinf)
        assert abs(nd[4] - math.sqrt(g * (p + pinf) / rho)) < 1e-12 * nd[4]


def test_sound_speed_two_forms():
    """rho c^2 = gbar (p + pbar_inf) = gbar (gbar - 1)(rho e - pbar_inf)."""
    s = _s2d()
    rng = np.random.default_rng(5)
    for _ in range(100):
        a1 = rng.uniform()
        X = _cons(s, [[1000 * a1 + 1e-8, 1.2 * (1 - a1) + 1e-8, rng.normal() * 50,
                       rng.normal() * 50, 10 ** rng.uniform(4, 9), a1]])[0]
        nd = orc.node(s, X)
        gbar = 1.0 + 1.0 / (a1 / 5.12 + (1 - a1) / 0.4)
        h = orc.rhoc2_tilde(s, X)
        assert abs(nd[0] * nd[4] ** 2 - gbar * (gbar - 1) * h) < 1e-9 * nd[0] * nd[4] ** 2


def _hessian_scaled(f, x, steps):
    n = len(x)
    H = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            def ev(di, dj):
                y = np.array(x, dtype=float)
                y[i] += di * steps[i]
                y[j] += dj * steps[j]
                return f(y)
            H[i, j] = (ev(1, 1) - ev(1, -1) - ev(-1, 1) + ev(-1, -1)) / 4.0
    return H


def test_lemma1_concavity():
    """Lemma 1: rho e - pbar_inf is concave in W when the gas has pinf = 0
    and gamma_liquid >= gamma_gas; with gamma_gas > gamma_liquid it is not."""
    good = _s2d()
    rng = np.random.default_rng(6)
    for _ in range(20):
        a1 = rng.uniform(0.05, 0.95)
        X = _cons(good, [[1000 * a1, 1.2 * (1 - a1), 20 * rng.normal(), 20 * rng.normal(), 1e6, a1]])[0]
        steps = np.array([5.0, 0.05, 5.0, 5.0, 1e4, 2e-3])
        H = _hessian_scaled(lambda y: orc.rhoc2_tilde(good, y), X, steps)
        ev = np.linalg.eigvalsh(0.5 * (H + H.T))
        assert ev.max() <= 1e-6 * np.abs(ev).max(), ev
    bad = _s2d(gamma=(1.2, 1.67), pinf=(3.43e8, 0.0))
    assert not orc.eos_valid(bad)
    found = False
    for a1 in np.linspace(0.05, 0.95, 19):
        X = _cons(bad, [[1000 * a1, 1.2 * (1 - a1), 0.0, 0.0, 1e6, a1]])[0]
        steps = np.array([5.0, 0.05, 5.0, 5.0, 1e4, 2e-3])
        H = _hessian_scaled(lambda y: orc.rhoc2_tilde(bad, y), X, steps)
        if np.linalg.eigvalsh(0.5 * (H + H.T)).max() > 0:
            found = True
    assert found
    assert orc.eos_valid(good)
    assert not orc.eos_valid(_s2d(pinf=(3.43e8, 1e5)))


# --------------------------------------------------------------------------
# HLLC [Sec. 3]
# --------------------------------------------------------------------------
def _random_admissible(s, rng, n):
    rows = []
    for _ in range(n):
        water = rng.uniform() < 0.5
        eps = 10 ** rng.uniform(-8, -2)
        a1 = 1 - eps if water else eps
        rho = 10 ** rng.uniform(2.7, 3.2) if water else 10 ** rng.uniform(-1, 2)
        p = 10 ** rng.uniform(3, 9.5)
        if water and rng.uniform() < 0.3:
            p = -rng.uniform(0, 2e8)        # tension in the liquid (Sec. 6.4)
        rows.append([rho * a1 if water else 1e-8, 1e-8 if water else rho * (1 - a1),
                     rng.normal() * 300, rng.normal() * 300, p, a1])
    return _cons(s, rows)


def test_hllc_consistency():
    s = _s2d()
    rng = np.random.default_rng(7)
    for X in _random_admissible(s, rng, 50):
        F, fa, ss = orc.hllc(s, X, X)
        rho, un, ut, p, c, h = orc.node(s, X)
        want = [X[0] * un, X[1] * un, X[2] * un + p, X[3] * un, (X[4] + p) * un]
        sc = np.abs(want).max() + abs(p)
        assert np.abs(np.array(F) - want).max() <= 1e-12 * sc
        assert abs(ss - un) <= 1e-10 * (abs(un) + c)
        assert abs(fa - X[5] * un) <= 1e-10 * (abs(un) + c)


def test_hllc_contact_is_preserved():
    """Equal p and u on both sides: the contact moves at u (s* = u) and the
    momentum flux carries exactly the pressure [Sec. 3.1]."""
    s = _s2d()
    for u in (-40.0, 0.0, 75.0):
        XL, XR = _cons(s, [[1000.0, 1e-8, u, 3.0, 2e5, 1 - 1e-8], [1e-8, 1.2, u, 3.0, 2e5, 1e-8]])
        F, fa, ss = orc.hllc(s, XL, XR)
        assert abs(ss - u) < 1e-11 * (abs(u) + 1.0)
        rho_up = (XL if u >= 0 else XR)
        if u != 0:
            assert abs(F[2] - (rho_up[2] * u + 2e5)) < 1e-9 * 2e5


def test_first_order_half_cell_states_admissible():
    """Sec. 3.3: with lambda max(|u|+c) <= 1/2 the first-order half-cell
    states W_i - 2 lambda (G^-_{HLLC} - F_i), W_{i+1} + 2 lambda (G^+ - F) lie
    in G, for arbitrary admissible pairs (water/air, tension, large jumps)."""
    s = _s2d()
    rng = np.random.default_rng(8)
    Xs = _random_admissible(s, rng, 400)
    for k in range(0, 400, 2):
        XL, XR = Xs[k], Xs[k + 1]
        nl, nr = orc.node(s, XL), orc.node(s, XR)
        amax = max(abs(nl[1]) + nl[4], abs(nr[1]) + nr[4])
        lam = 0.5 / amax
        F, fa, ss = orc.hllc(s, XL, XR)
        Hm = np.array([*F, fa - XL[5] * ss])
        Hp = np.array([*F, fa - XR[5] * ss])
        FL = np.array([XL[0] * nl[1], XL[1] * nl[1], XL[2] * nl[1] + nl[3], XL[3] * nl[1], (XL[4] + nl[3]) * nl[1], 0.0])
        FR = np.array([XR[0] * nr[1], XR[1] * nr[1], XR[2] * nr[1] + nr[3], XR[3] * nr[1], (XR[4] + nr[3]) * nr[1], 0.0])
        P = XL - 2 * lam * (Hm - FL)
        M = XR + 2 * lam * (Hp - FR)
        for Y, ref in ((P, XL), (M, XR)):
            assert Y[0] >= -1e-12 * abs(ref[0]) - 1e-300
            assert Y[1] >= -1e-12 * abs(ref[1]) - 1e-300
            assert -1e-12 <= Y[5] <= 1 + 1e-12
            assert orc.rhoc2_tilde(s, Y) > 0


def test_hllc_sgn_zero_is_continuous():
    """The flux weights (1 +- sgn s*)/2 switch sides at s* = 0; both one-sided
    forms agree there, so the flux is continuous across s* = 0 (symmetric
    collision gives s* = 0 exactly and zero mass flux)."""
    s = _s2d()
    for w in (0.0, 30.0):
        XL, XR = _cons(s, [[1000.0, 1e-8, w, 0.0, 2e5, 1 - 1e-8], [1000.0, 1e-8, -w, 0.0, 2e5, 1 - 1e-8]])
        F0, fa0, ss0 = orc.hllc(s, XL, XR)
        assert ss0 == 0.0 and F0[0] == 0.0 and F0[1] == 0.0
    XL, XR = _cons(s, [[1000.0, 1e-8, 0.0, 0.0, 2e5, 1 - 1e-8], [1e-8, 1.2, 0.0, 0.0, 2e5, 1e-8]])
    F0, fa0, ss0 = orc.hllc(s, XL, XR)
    for du in (1e-9, -1e-9):
        XLp, XRp = _cons(s, [[1000.0, 1e-8, du, 0.0, 2e5, 1 - 1e-8], [1e-8, 1.2, du, 0.0, 2e5, 1e-8]])
        F1, fa1, ss1 = orc.hllc(s, XLp, XRp)
        assert np.abs(np.array(F1) - F0).max() < 1e-3 * 2e5
        assert abs(fa1 - fa0) < 1e-6


# --------------------------------------------------------------------------
# Limiters [Sec. 5]
# --------------------------------------------------------------------------
def test_interp_limiter_leaves_admissible_states():
    s = _s2d()
    A, B = _cons(s, [[1000.0, 1e-8, 3.0, 1.0, 2e5, 1 - 1e-8], [990.0, 2e-8, 3.5, 1.0, 2.1e5, 1 - 2e-8]])
    assert np.array_equal(orc.interp_limit(s, A, B), B)


def test_interp_limiter_partial_density_solves_theta():
    """Alg. 1: theta solves (1-theta) q(A) + theta q(B) = eps."""
    s = _s2d()
    A = _cons(s, [[1000.0, 1e-8, 3.0, 1.0, 2e5, 1 - 1e-8]])[0]
    B = A.copy(); B[1] = -5e-8
    out = orc.interp_limit(s, A, B)
    assert abs(out[1] - s.eps_arho) < 1e-22
    th = (A[1] - s.eps_arho) / (A[1] - B[1])
    assert np.allclose(out, (1 - th) * A + th * B, rtol=1e-14, atol=1e-300)


def test_interp_limiter_sound_speed_jensen_bound():
    """Alg. 3: after limiting, rho*ctilde^2 >= eps (Jensen, concavity of
    Lemma 1) even though theta comes from a linear formula."""
    s = _s2d()
    rng = np.random.default_rng(9)
    for _ in range(200):
        A = _random_admissible(s, rng, 1)[0]
        B = A.copy()
        B[4] = A[4] - rng.uniform(1.0, 3.0) * (orc.rhoc2_tilde(s, A) + 1.0)  # push E below pinf
        B[2] += rng.normal() * abs(A[2] + 1)
        out = orc.interp_limit(s, A, B)
        h = orc.rhoc2_tilde(s, out)
        assert h >= s.hs_rhoc2 or np.array_equal(out, A)
        assert out[0] >= s.hs_arho and out[1] >= s.hs_arho or np.array_equal(out, A)


def test_interp_limiter_volume_fraction_bounds():
    s = _s2d()
    A = _cons(s, [[1000.0 * 0.9, 1.2 * 0.1, 3.0, 1.0, 2e5, 0.9]])[0]
    B = A.copy(); B[5] = 1.3
    out = orc.interp_limit(s, A, B)
    assert s.eps_alpha - 1e-16 <= out[5] <= 1 - s.eps_alpha + 1e-16


def test_flux_limiter_identity_and_bounds():
    s = _s2d()
    rng = np.random.default_rng(10)
    Xs = _random_admissible(s, rng, 200)
    for k in range(0, 200, 2):
        XL, XR = Xs[k], Xs[k + 1]
        nl, nr = orc.node(s, XL), orc.node(s, XR)
        lam = 0.5 / max(abs(nl[1]) + nl[4], abs(nr[1]) + nr[4])
        F, fa, ss = orc.hllc(s, XL, XR)
        Hm = np.array([*F, fa - XL[5] * ss]); Hp = np.array([*F, fa - XR[5] * ss])
        Gm, Gp, th = orc.flux_limit_face(s, XL, XR, lam, Hm, Hp, Hm, Hp)
        assert np.array_equal(Gm, Hm) and np.array_equal(Gp, Hp)
        # a wild high-order flux gets pulled back into G
        pert = rng.normal(size=6) * (np.abs(Hm) + 1.0) * 50
        Gm, Gp, th = orc.flux_limit_face(s, XL, XR, lam, Hm, Hp, Hm + pert, Hp + pert)
        FL = np.array([XL[0] * nl[1], XL[1] * nl[1], XL[2] * nl[1] + nl[3], XL[3] * nl[1], (XL[4] + nl[3]) * nl[1], 0.0])
        FR = np.array([XR[0] * nr[1], XR[1] * nr[1], XR[2] * nr[1] + nr[3], XR[3] * nr[1], (XR[4] + nr[3]) * nr[1], 0.0])
        P = XL - 2 * lam * (Gm - FL)
        M = XR + 2 * lam * (Gp - FR)
        for Y in (P, M):
            assert Y[0] >= 0 and Y[1] >= 0 and 0 <= Y[5] <= 1
            assert orc.rhoc2_tilde(s, Y) > 0
        # conservative components of G^- and G^+ stay identical (Sec. 5.2)
        assert np.array_equal(Gm[:5], Gp[:5])


# --------------------------------------------------------------------------
# Whole-grid properties
# --------------------------------------------------------------------------
def test_conservation_periodic():
    """Flux-difference form on a periodic grid: the conservative components
    of the RHS sum to zero up to round-off [Sec. 4.1]."""
    spec = pb.random_smooth_state(48, 40, seed=11)
    spec.bc = (pb.BC_PERIODIC,) * 4
    s = oracle_setup(spec)
    W = oracle_W(spec, s)
    L = orc.rhs(s, W, 2e-8)
    for v in range(5):
        tot = L[v].sum()
        assert abs(tot) <= 1e-12 * np.abs(L[v]).sum(), (v, tot)
    W1, dt, bad = orc.ssprk3_step(s, W)
    assert bad == 0
    for v in range(5):
        assert abs(W1[v].sum() - W[v].sum()) <= 1e-13 * np.abs(W[v]).sum()


def test_first_order_alpha_update_matches_sec31():
    """HLLC scheme: the alpha RHS equals the printed first-order advection
    update -[u+_{i-1/2}(a_i - a_{i-1}) + u-_{i+1/2}(a_{i+1} - a_i)]/dx."""
    spec = pb.random_smooth_state(64, 1, seed=12, ndim=1)
    spec.bc = (pb.BC_PERIODIC,) * 4
    s = oracle_setup(spec, scheme=1)
    W = oracle_W(spec, s)
    L = orc.rhs(s, W, 1e-8)
    n = spec.nx
    X = lambda i: np.array([W[0, 0, i % n], W[1, 0, i % n], W[2, 0, i % n], 0.0, W[3, 0, i % n], W[4, 0, i % n]])
    a = W[4, 0]
    for i in range(n):
        _, _, s_lo = orc.hllc(s, X(i - 1), X(i))
        _, _, s_hi = orc.hllc(s, X(i), X(i + 1))
        want = -(max(0.0, s_lo) * (a[i] - a[(i - 1) % n]) + min(0.0, s_hi) * (a[(i + 1) % n] - a[i])) / spec.dx
        assert abs(L[4, 0, i] - want) <= 1e-10 * (abs(want) + 1e-3)


def test_limiters_inactive_on_smooth_data():
    """Smooth admissible data: both limiters leave the scheme untouched,
    bit for bit (theta = 1 everywhere)."""
    spec = pb.convergence_advection(32)
    s_on = oracle_setup(spec)
    s_off = oracle_setup(spec, interp_limiter=False, flux_limiter=False)
    W = oracle_W(spec, s_on)
    assert np.array_equal(orc.rhs(s_on, W, spec.dt_fixed), orc.rhs(s_off, W, spec.dt_fixed))


def test_mirror_and_transpose_symmetry():
    spec = pb.random_smooth_state(40, 40, seed=13)
    spec.bc = (pb.BC_PERIODIC,) * 4
    s = oracle_setup(spec)
    W = oracle_W(spec, s)
    L = orc.rhs(s, W, 1e-8)
    # mirror in x
    Wm = W[:, :, ::-1].copy(); Wm[2] *= -1
    Lm = orc.rhs(s, Wm, 1e-8)
    Lm_back = Lm[:, :, ::-1].copy(); Lm_back[2] *= -1
    for v in range(6):
        assert np.abs(Lm_back[v] - L[v]).max() <= 1e-11 * np.abs(L[v]).max()
    # swap x and y
    Wt = W.transpose(0, 2, 1)[[0, 1, 3, 2, 4, 5]].copy()
    Lt = orc.rhs(s, Wt, 1e-8)
    Lt_back = Lt.transpose(0, 2, 1)[[0, 1, 3, 2, 4, 5]]
    for v in range(6):
        assert np.abs(Lt_back[v] - L[v]).max() <= 1e-11 * np.abs(L[v]).max()


def test_rhs_cells_equals_full_rhs():
    spec = pb.random_smooth_state(30, 22, seed=14)
    s = oracle_setup(spec)
    W = oracle_W(spec, s)
    L = orc.rhs(s, W, 3e-8)
    cells = np.array([0, 5, 29, 30, 31, 300, 659, 640, 333])
    got = orc.rhs_cells(s, W, 3e-8, cells)
    for q, c in enumerate(cells):
        assert np.array_equal(got[q], L[:, c // 30, c % 30])


def test_interface_advection_keeps_p_u_equilibrium():
    """Sec. 6.2: two interfaces advected one period keep u and p uniform
    (exact in exact arithmetic) and alpha bounded."""
    spec = pb.interface_advection(200)
    s = oracle_setup(spec)
    W, steps, t = orc.run(s, oracle_W(spec, s), spec.t_end, spec.dt_fixed)
    assert steps == 8000
    V, c = orc.cons_to_prim(s, W)
    assert np.abs(V[2] / 100.0 - 1.0).max() < 1e-7
    assert np.abs(V[3] / 101325.0 - 1.0).max() < 1e-7
    assert W[4].min() >= 0 and W[4].max() <= 1
    # the profile has come back to its place: the interfaces are still sharp
    x, _ = spec.centres()
    inside = (x > 0.3) & (x < 0.7)
    outside = (x < 0.2) | (x > 0.8)
    assert W[4, 0, inside].min() > 0.99 and W[4, 0, outside].max() < 0.01


def test_shock_tubes_converge_to_exact_solution():
    """First-order L1 convergence to the exact Riemann solution for a
    single-phase stiffened-gas tube and the water-air tube."""
    cases = [
        (lambda n: pb.single_phase_shock_tube(n), er.Side(1500.0, 0.0, 2e9, 6.12, 3.43e8),
         er.Side(1000.0, 0.0, 1e5, 6.12, 3.43e8), 0.5, 1e-4),
        (lambda n: pb.water_air_shock_tube(n), er.Side(1000.0, 0.0, 1e9, 6.12, 3.43e8),
         er.Side(50.0, 0.0, 1e5, 1.4, 0.0), 0.7, 2.4e-4),
    ]
    for mk, L, R, x0, tend in cases:
        errs = []
        for n in (100, 200, 400):
            spec = mk(n)
            s = oracle_setup(spec)
            W, steps, t = orc.run(s, oracle_W(spec, s), tend)
            x, _ = spec.centres()
            ex = er.sample(L, R, x, x0, t)
            V, c = orc.cons_to_prim(s, W)
            errs.append([np.mean(np.abs(W[0, 0] + W[1, 0] - ex[0])) / np.mean(ex[0]),
                         np.mean(np.abs(V[3, 0] - ex[2])) / np.mean(np.abs(ex[2]))])
        errs = np.array(errs)
        assert np.all(errs[1] < errs[0]) and np.all(errs[2] < 0.75 * errs[1]), errs
        assert errs[2].max() < 0.03


def test_positivity_every_stage_sedov_and_water_air():
    """Sec. 6.4 (liquid under tension, strong blast) and the water-air tube:
    no stage ever leaves the admissible set."""
    spec = pb.sedov_multimaterial(401)
    s = oracle_setup(spec)
    W, steps, t = orc.run(s, oracle_W(spec, s), spec.t_end, spec.dt_fixed)
    assert steps == 4000 and orc.count_inadmissible(s, W) == 0
    spec = pb.water_air_shock_tube(400)
    s = oracle_setup(spec)
    W, steps, t = orc.run(s, oracle_W(spec, s), spec.t_end)
    assert orc.count_inadmissible(s, W) == 0 and abs(t - spec.t_end) < 1e-18


def test_limiters_are_needed_on_sedov():
    """Negative control: without the two limiters the same Sedov run leaves
    the admissible set (Sec. 5 motivation)."""
    spec = pb.sedov_multimaterial(401)
    s = oracle_setup(spec, interp_limiter=False, flux_limiter=False)
    with pytest.raises(FloatingPointError):
        orc.run(s, oracle_W(spec, s), spec.t_end, spec.dt_fixed)


def test_cfl_time_step_and_lambda():
    spec = pb.shock_bubble(64)
    s = oracle_setup(spec)
    W = oracle_W(spec, s)
    a = orc.max_wavespeed(s, W)
    dt = orc.cfl_dt(s, W)
    assert abs(dt * (a[0] / spec.dx + a[1] / spec.dy) - 0.5) < 1e-15
    lam = orc.stage_lambda(s, W, dt)
    # lambda_x = CFL / max(|u|+c) when dt is the CFL step (Sec. 3.3)
    assert abs(lam[0] * a[0] - 0.5) < 1e-14 and abs(lam[1] * a[1] - 0.5) < 1e-14


def test_opcount_is_plausible():
    spec = pb.convergence_advection(16)
    s = oracle_setup(spec)
    W = oracle_W(spec, s)
    st = np.array([[W[v, 3, i] for v in range(6)] for i in range(6)])
    oc = orc.opcount_face(s, st, 1e-6)
    assert oc["node"]["div"] == 4 and oc["node"]["sqrt"] == 1
    assert 100 <= oc["face"]["div"] <= 140
    assert oc["face"]["sqrt"] == 2


# --------------------------------------------------------------------------
# Dirichlet sides with one ghost state per boundary row (the jet inflow of
# Sec. 6.7) and their place in the CFL maxima (Sec. 3.3).
# --------------------------------------------------------------------------
def _banded_state(nx, ny):
    """x-uniform state with water/air bands in y at one pressure, u = 30."""
    V = np.empty((6, ny, nx))
    for j in range(ny):
        st = (1000.0, 1e-8, 30.0, 0.0, 1e5, 1 - 1e-8) if (j // 3) % 2 == 0 else \
             (1e-8, 1.2, 30.0, 0.0, 1e5, 1e-8)
        V[:, j, :] = np.array(st)[:, None]
    return V


def test_dirichlet_rows_follow_their_row():
    """Each x-lo ghost row equal to its interior row: every x-face of a row
    sees six identical states, so all n+1 faces of the row carry the same
    split fluxes, the boundary faces included.  Reversing the profile makes
    the boundary faces of the rows whose band changes differ."""
    nx, ny = 9, 12
    V = _banded_state(nx, ny)
    rows = np.ascontiguousarray(V[:, :, 0].T)
    s = orc.Setup(ndim=2, nx=nx, ny=ny, dx=1e-3, dy=1e-3,
                  bc=(orc.BC_DIRICHLET, orc.BC_EXTRAP, orc.BC_EXTRAP, orc.BC_EXTRAP),
                  dirichlet_prim=[rows, None, None, None])
    W = orc.prim_to_cons(s, V)
    Gm, Gp, _ = orc.faces(s, W, 0, 1e-9)
    for j in range(ny):
        assert np.array_equal(Gm[j], np.broadcast_to(Gm[j, -1], Gm[j].shape)), j
        assert np.array_equal(Gp[j], np.broadcast_to(Gp[j, -1], Gp[j].shape)), j
    s.dirichlet_prim = [np.ascontiguousarray(rows[::-1]), None, None, None]
    Gm2, _, _ = orc.faces(s, W, 0, 1e-9)
    changed = [j for j in range(ny) if (j // 3) % 2 != ((ny - 1 - j) // 3) % 2]
    assert changed
    for j in range(ny):
        differs = not np.array_equal(Gm2[j, 0], Gm2[j, -1])
        assert differs == (j in changed), j


def test_dirichlet_supersonic_inflow_face_flux():
    """1D supersonic inflow (water at 3000 m/s into air at 1000 m/s, both
    faster than sound): the first-order HLLC flux of the inflow face is the
    physical flux of the ghost state (Sec. 3.2, upwind case)."""
    n = 8
    ghost = (1000.0, 1e-8, 3000.0, 2e5, 1 - 1e-8)
    V = np.empty((5, 1, n))
    V[:, 0, :] = np.array((1e-8, 1.2, 1000.0, 1e5, 1e-8))[:, None]
    s = orc.Setup(ndim=1, nx=n, dx=1e-3,
                  bc=(orc.BC_DIRICHLET, orc.BC_EXTRAP, orc.BC_PERIODIC, orc.BC_PERIODIC),
                  dirichlet_prim=[ghost, None, None, None], scheme=1)
    W = orc.prim_to_cons(s, V)
    Gm, Gp, _ = orc.faces(s, W, 0, 1e-9)
    a1r1, a2r2, u, p, _ = ghost
    rho = a1r1 + a2r2
    want = (a1r1 * u, a2r2 * u, rho * u * u + p)
    for k in range(3):
        assert math.isclose(Gm[0, 0, k], want[k], rel_tol=1e-14), (k, Gm[0, 0, k], want[k])
        assert math.isclose(Gp[0, 0, k], want[k], rel_tol=1e-14), k


def test_dirichlet_ghosts_enter_the_cfl_maxima():
    """Air at rest with a 1.5e5 m/s water inflow row (Sec. 6.7): the x
    maximum is the inflow's |u| + c (c of water at 1e5 Pa about 1449 m/s),
    the y maximum only sees the interior air."""
    nx, ny = 16, 8
    V = np.empty((6, ny, nx))
    V[:] = np.array((1e-8, 1.0, 0.0, 0.0, 1e5, 1e-8))[:, None, None]
    rows = np.tile(np.array((1e-8, 1.0, 0.0, 0.0, 1e5, 1e-8)), (ny, 1))
    rows[3:5] = (1000.0, 1e-8, 1.5e5, 0.0, 1e5, 1 - 1e-8)
    s = orc.Setup(ndim=2, nx=nx, ny=ny, dx=1e-3, dy=1e-3,
                  bc=(orc.BC_DIRICHLET, orc.BC_EXTRAP, orc.BC_EXTRAP, orc.BC_EXTRAP),
                  dirichlet_prim=[rows, None, None, None])
    a = orc.max_wavespeed(s, orc.prim_to_cons(s, V))
    assert 1.5e5 + 1440.0 < a[0] < 1.5e5 + 1460.0, a
    assert 370.0 < a[1] < 380.0, a


def test_openmp_build_of_the_oracle_is_bitwise_identical():
    """The all-cores CPU baseline: the same oracle source built with OpenMP
    over grid rows (3D: grid lines) gives the serial build's RHS bit for bit
    (2D with every side kind, 1D, a limiter-active state, 3D)."""
    cases = [pb.random_smooth_state(96, 70, seed=41), pb.water_air_shock_tube(400),
             pb.shock_bubble(64), pb.random_smooth_state_3d(20, 17, 13, seed=42)]
    for spec in cases:
        s = oracle_setup(spec)
        W = oracle_W(spec, s)
        dt = orc.cfl_dt(s, W)
        a = orc.rhs(s, W, dt)
        b = orc.rhs_parallel(s, W, dt)
        assert np.array_equal(a, b), spec.name
