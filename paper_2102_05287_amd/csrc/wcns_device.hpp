// Device-side arithmetic of the PP-WCNS-IS right-hand side on gfx950.
//
// Everything here is per-thread scalar code, FP64 except the precision
// form's FP32 routines (marked below): the method is stencil and
// Riemann-solver arithmetic with no dense contraction, so there is no MFMA
// use.  Each routine cites the passage of the paper that defines it.
//
// Sweeps work on a 6-component state rotated into the sweep direction,
//   X = (a1r1, a2r2, m_n, m_t, E, a1),
// with m_n the normal and m_t the tangential momentum.  The 1D system (no
// m_t) is the HAS_T = false instantiation: every tangential term is dropped
// at compile time.
//
// Every FP64 expression is evaluated in the order the serial reference
// writes it, with FMA contraction switched off and IEEE-rounded divides and
// square roots, so results are bit-identical to it: the liquid pressure
// recovery at low pressure cancels ~4 decimal digits and the limiters divide
// by differences of order 1e-8, so any extra or different rounding shows.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace wcns {

// Mixture EOS constants [Sec. 2]: g_k = 1/(gamma_k - 1),
// q_k = gamma_k pinf_k/(gamma_k - 1).
struct EosC {
  double g1, g2, q1, q2;
};

struct Tol {
  double eps_arho, eps_alpha, eps_rhoc2;   // Sec. 5.1 limiter tolerances
  double hs_arho, hs_alpha, hs_rhoc2;      // hard-switch tolerances
  double weno_eps;                         // IS-weight epsilon (Sec. 4.3)
};

// Node quantities in the rotated frame: the state and its primitive
// recovery (u_n, u_t, p, c, rho*ctilde^2).
struct NodeQ {
  double w[6];
  double un, ut, p, c, h;
};

// ---------------------------------------------------------------- division
// IEEE-754 double division without the range-scaling steps.  gfx950's
// correctly rounded divide is: div_scale(den), rcp, div_scale(num), two
// Newton steps (4 FMA), mul, residual FMA, div_fmas, div_fixup.  When
// neither operand needs exponent scaling (|a|, |b| in roughly
// [1e-290, 1e300], quotient normal) and no operand is 0/inf/NaN in the
// denominator, div_scale returns its input, div_fmas is a plain FMA and
// div_fixup returns the quotient unchanged, so the 8-instruction core below
// yields the same bits (sign of a zero quotient aside).  Every division of
// the face pipeline has such operands (positive densities, Gamma, sound
// speeds, beta + eps >= eps, strictly negative HLLC denominators, ...);
// wcns_selftest_division checks the identity on the device.
__device__ __forceinline__ double ddiv(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  double q = a * r;
  double rem = __builtin_fma(-b, q, a);
  return __builtin_fma(rem, r, q);
}

// a/b for a divisor whose correctly rounded reciprocal y = RN(1/b) is
// accurate to 2^-55 relative or better: q0 = a*y is then within one ulp of
// a/b, the residual a - b*q0 is exact (FMA), and one correction q0 + r*y
// rounds to the IEEE quotient (Markstein's theorem); 3 VALU instructions.
// 1/2100 (HCS) is accurate to 2^-60; grid spacings are checked on the host,
// which passes y = 0 when the check fails (hdiv then uses ddiv).
__device__ __forceinline__ double cdiv(double a, double b, double y) {
  double q = a * y;
  double r = __builtin_fma(-b, q, a);
  return __builtin_fma(r, y, q);
}
constexpr double R2100 = 1.0 / 2100.0;

// division by a grid spacing h with its checked reciprocal y (0: none)
__device__ __forceinline__ double hdiv(double a, double h, double y) {
  return y != 0.0 ? cdiv(a, h, y) : ddiv(a, h);
}

// ---------------------------------------------------------------- EOS
__device__ __forceinline__ double mix_gamma(const EosC& e, double a1) {
#pragma clang fp contract(off)
  double a2 = 1.0 - a1;
  return a1 * e.g1 + a2 * e.g2;
}
__device__ __forceinline__ double mix_pi(const EosC& e, double a1) {
#pragma clang fp contract(off)
  double a2 = 1.0 - a1;
  return a1 * e.q1 + a2 * e.q2;
}

// Primitive recovery and mixture sound speed of one state [Sec. 2]:
// p = (rho e - Pi)/Gamma, pbar_inf = Pi/(1+Gamma), gbar = 1 + 1/Gamma,
// c^2 = gbar (p + pbar_inf)/rho, h = rho e - pbar_inf.
template <bool HAS_T>
__device__ __forceinline__ void recover(const EosC& e, const double X[6], double& un, double& ut,
                                        double& p, double& c, double& h) {
#pragma clang fp contract(off)
  double rho = X[0] + X[1];
  double irho = ddiv(1.0, rho);
  un = X[2] * irho;
  double ke;
  if (HAS_T) {
    ut = X[3] * irho;
    ke = X[2] * un + X[3] * ut;
  } else {
    ut = 0.0;
    ke = X[2] * un;
  }
  double rhoe = X[4] - 0.5 * ke;
  double Gam = mix_gamma(e, X[5]);
  double Pi = mix_pi(e, X[5]);
  p = ddiv(rhoe - Pi, Gam);
  double pinf_bar = ddiv(Pi, 1.0 + Gam);
  double gbar = 1.0 + ddiv(1.0, Gam);
  double c2 = gbar * (p + pinf_bar) * irho;
  c = sqrt(c2);
  h = rhoe - pinf_bar;
}

// rho*ctilde^2 = rho e - pbar_inf of a state [Sec. 5.1]
template <bool HAS_T>
__device__ __forceinline__ double rhoc2_tilde(const EosC& e, const double X[6]) {
#pragma clang fp contract(off)
  double rho = X[0] + X[1];
  double irho = ddiv(1.0, rho);
  double un = X[2] * irho;
  double ke;
  if (HAS_T) {
    double ut = X[3] * irho;
    ke = X[2] * un + X[3] * ut;
  } else {
    ke = X[2] * un;
  }
  double rhoe = X[4] - 0.5 * ke;
  double Gam = mix_gamma(e, X[5]);
  double Pi = mix_pi(e, X[5]);
  return rhoe - ddiv(Pi, 1.0 + Gam);
}

// Node flux G = F + (0,...,0, a1 u_n) [Sec. 3.2 flux-source form]
template <bool HAS_T>
__device__ __forceinline__ void node_flux(const NodeQ& n, double g[6]) {
#pragma clang fp contract(off)
  g[0] = n.w[0] * n.un;
  g[1] = n.w[1] * n.un;
  g[2] = n.w[2] * n.un + n.p;
  g[3] = HAS_T ? n.w[3] * n.un : 0.0;
  g[4] = (n.w[4] + n.p) * n.un;
  g[5] = n.w[5] * n.un;
}

// ---------------------------------------------------------------- HLLC
// [Sec. 3.1 star states with Einfeldt speeds and Batten's contact speed;
// Sec. 3.2 conservative flux, f_alpha and u* = s*]
struct HllcOut {
  double F[5];
  double fa, ss;
};

template <bool HAS_T>
__device__ __forceinline__ void hllc(const NodeQ& L, const NodeQ& R, HllcOut& o) {
#pragma clang fp contract(off)
  double rhoL = L.w[0] + L.w[1], rhoR = R.w[0] + R.w[1];
  double ubar = 0.5 * (L.un + R.un);
  double cbar = 0.5 * (L.c + R.c);
  double aL = ubar - cbar, bL = L.un - L.c;
  double sL = (bL < aL) ? bL : aL;
  double aR = ubar + cbar, bR = R.un + R.c;
  double sR = (aR < bR) ? bR : aR;
  double num = R.p - L.p + rhoL * L.un * (sL - L.un) - rhoR * R.un * (sR - R.un);
  double den = rhoL * (sL - L.un) - rhoR * (sR - R.un);
  double ss = ddiv(num, den);
  o.ss = ss;
  double sm = (sL < 0.0) ? sL : 0.0;
  double sp = (0.0 < sR) ? sR : 0.0;
  // sgn(s*) with sgn(0) = 0: weights (1 +- sgn)/2
  double sg = (ss > 0.0) ? 1.0 : ((ss < 0.0) ? -1.0 : 0.0);
  double wl = (1.0 + sg) * 0.5;
  double wr = (1.0 - sg) * 0.5;
  double fl[5], fr[5];
  {
    double chi = ddiv(sL - L.un, sL - ss);
    double g[6];
    node_flux<HAS_T>(L, g);
    double ws[5];
    ws[0] = chi * L.w[0];
    ws[1] = chi * L.w[1];
    ws[2] = chi * rhoL * ss;
    ws[3] = HAS_T ? chi * rhoL * L.ut : 0.0;
    ws[4] = chi * (L.w[4] + (ss - L.un) * (rhoL * ss + ddiv(L.p, sL - L.un)));
#pragma unroll
    for (int v = 0; v < 5; ++v) fl[v] = g[v] + sm * (ws[v] - L.w[v]);
  }
  {
    double chi = ddiv(sR - R.un, sR - ss);
    double g[6];
    node_flux<HAS_T>(R, g);
    double ws[5];
    ws[0] = chi * R.w[0];
    ws[1] = chi * R.w[1];
    ws[2] = chi * rhoR * ss;
    ws[3] = HAS_T ? chi * rhoR * R.ut : 0.0;
    ws[4] = chi * (R.w[4] + (ss - R.un) * (rhoR * ss + ddiv(R.p, sR - R.un)));
#pragma unroll
    for (int v = 0; v < 5; ++v) fr[v] = g[v] + sp * (ws[v] - R.w[v]);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) o.F[v] = wl * fl[v] + wr * fr[v];
  o.fa = wl * (L.w[5] * ss) + wr * (R.w[5] * ss);
}

// ---------------------------------------------------------------- WENO-IS
// Incremental-stencil nonlinear interpolation [Sec. 4.3], left-biased on
// (a,b,c,d,e) = (u_{i-2},...,u_{i+2}); right-biased = flipped stencil.
// Sub-stencils S0..S3, indicators beta_0, beta_1, beta_01, beta_2, beta_3,
// reference indicator tau_5 and the IS weights eta_k/sum(eta), every
// operation rounded as written (IEEE divides, no contraction).
__device__ __forceinline__ double weno_is(double a, double b, double c, double d, double e,
                                          double eps) {
#pragma clang fp contract(off)
  double u0 = 0.5 * (c + d);
  double u1 = 0.5 * (-b + 3.0 * c);
  double u2 = 0.125 * (3.0 * c + 6.0 * d - e);
  double u3 = 0.125 * (3.0 * a - 10.0 * b + 15.0 * c);
  double b0 = (c - d) * (c - d);
  double b1 = (b - c) * (b - c);
  double t01a = b - 2.0 * c + d, t01b = b - d;
  double b01 = (13.0 / 12.0) * t01a * t01a + 0.25 * t01b * t01b;
  double t2a = c - 2.0 * d + e, t2b = 3.0 * c - 4.0 * d + e;
  double b2 = (13.0 / 12.0) * t2a * t2a + 0.25 * t2b * t2b;
  double t3a = a - 2.0 * b + c, t3b = a - 4.0 * b + 3.0 * c;
  double b3 = (13.0 / 12.0) * t3a * t3a + 0.25 * t3b * t3b;
  double t5a = e - 4.0 * d + 6.0 * c - 4.0 * b + a;
  double t5b = e - 2.0 * d + 2.0 * b - a;
  double tau5 = (13.0 / 12.0) * t5a * t5a + 0.25 * t5b * t5b;
  double r01 = ddiv(tau5, b01 + eps);
  double eta0 = (15.0 / 32.0) * (1.0 + ddiv(tau5, b0 + eps) * r01);
  double eta1 = (5.0 / 32.0) * (1.0 + ddiv(tau5, b1 + eps) * r01);
  double eta2 = (5.0 / 16.0) * (1.0 + ddiv(tau5, b2 + eps));
  double eta3 = (1.0 / 16.0) * (1.0 + ddiv(tau5, b3 + eps));
  double sum = eta0 + eta1 + eta2 + eta3;
  return ddiv(eta0 * u0 + eta1 * u1 + eta2 * u2 + eta3 * u3, sum);
}

// ---------------------------------------------------------------- FP32 bulk
// The precision form evaluates the characteristic interpolation, the
// midpoint HLLC flux and the HCS reconstruction in FP32; the primitive
// recovery (p, c^2), the limiters' states and theta solves and the
// first-order HLLC fallback flux stay FP64 (their positivity argument needs
// it).  FP32 quotients use the hardware reciprocal (~1 ulp).
__device__ __forceinline__ float fdivf(float a, float b) {
#pragma clang fp contract(fast)
  return a * __builtin_amdgcn_rcpf(b);
}

struct NodeQf {
  float w[6];
  float un, ut, p, c;
};

struct HllcOutF {
  float F[5];
  float fa, ss;
};

// HLLC flux [Sec. 3.1-3.2] in FP32 (same formulas as hllc()).
template <bool HAS_T>
__device__ __forceinline__ void hllc_f(const NodeQf& L, const NodeQf& R, HllcOutF& o) {
#pragma clang fp contract(fast)
  float rhoL = L.w[0] + L.w[1], rhoR = R.w[0] + R.w[1];
  float ubar = 0.5f * (L.un + R.un);
  float cbar = 0.5f * (L.c + R.c);
  float sL = fminf(ubar - cbar, L.un - L.c);
  float sR = fmaxf(ubar + cbar, R.un + R.c);
  float num = R.p - L.p + rhoL * L.un * (sL - L.un) - rhoR * R.un * (sR - R.un);
  float den = rhoL * (sL - L.un) - rhoR * (sR - R.un);
  float ss = fdivf(num, den);
  o.ss = ss;
  float sm = fminf(sL, 0.0f);
  float sp = fmaxf(sR, 0.0f);
  float sg = (ss > 0.0f) ? 1.0f : ((ss < 0.0f) ? -1.0f : 0.0f);
  float wl = (1.0f + sg) * 0.5f;
  float wr = (1.0f - sg) * 0.5f;
  float fl[5], fr[5];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const NodeQf& K = side == 0 ? L : R;
    float rho = side == 0 ? rhoL : rhoR;
    float sK = side == 0 ? sL : sR;
    float sE = side == 0 ? sm : sp;
    float chi = fdivf(sK - K.un, sK - ss);
    float g[5] = {K.w[0] * K.un, K.w[1] * K.un, K.w[2] * K.un + K.p, HAS_T ? K.w[3] * K.un : 0.0f,
                  (K.w[4] + K.p) * K.un};
    float ws[5];
    ws[0] = chi * K.w[0];
    ws[1] = chi * K.w[1];
    ws[2] = chi * rho * ss;
    ws[3] = HAS_T ? chi * rho * K.ut : 0.0f;
    ws[4] = chi * (K.w[4] + (ss - K.un) * (rho * ss + fdivf(K.p, sK - K.un)));
    float* f = side == 0 ? fl : fr;
#pragma unroll
    for (int v = 0; v < 5; ++v) f[v] = g[v] + sE * (ws[v] - K.w[v]);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) o.F[v] = wl * fl[v] + wr * fr[v];
  o.fa = wl * (L.w[5] * ss) + wr * (R.w[5] * ss);
}

// IS-WENO interpolation [Sec. 4.3] in FP32.  Guard for the FP32 range:
// eps is raised to 1e-30 (1e-40 is subnormal in FP32) and each ratio
// tau_5/(beta + eps) is capped at 1e15 so the products of two ratios stay
// finite; a capped weight still exceeds the others by ~1e15, far beyond FP32
// resolution, so the selected stencils are unchanged.
__device__ __forceinline__ float weno_is_f(float a, float b, float c, float d, float e, float eps) {
#pragma clang fp contract(fast)
  const float cap = 1e15f;
  float u0 = 0.5f * (c + d);
  float u1 = 0.5f * (-b + 3.0f * c);
  float u2 = 0.125f * (3.0f * c + 6.0f * d - e);
  float u3 = 0.125f * (3.0f * a - 10.0f * b + 15.0f * c);
  float b0 = (c - d) * (c - d);
  float b1 = (b - c) * (b - c);
  float t01a = b - 2.0f * c + d, t01b = b - d;
  float b01 = (13.0f / 12.0f) * t01a * t01a + 0.25f * t01b * t01b;
  float t2a = c - 2.0f * d + e, t2b = 3.0f * c - 4.0f * d + e;
  float b2 = (13.0f / 12.0f) * t2a * t2a + 0.25f * t2b * t2b;
  float t3a = a - 2.0f * b + c, t3b = a - 4.0f * b + 3.0f * c;
  float b3 = (13.0f / 12.0f) * t3a * t3a + 0.25f * t3b * t3b;
  float t5a = e - 4.0f * d + 6.0f * c - 4.0f * b + a;
  float t5b = e - 2.0f * d + 2.0f * b - a;
  float tau5 = (13.0f / 12.0f) * t5a * t5a + 0.25f * t5b * t5b;
  float r01 = fminf(fdivf(tau5, b01 + eps), cap);
  float eta0 = (15.0f / 32.0f) * (1.0f + fminf(fdivf(tau5, b0 + eps), cap) * r01);
  float eta1 = (5.0f / 32.0f) * (1.0f + fminf(fdivf(tau5, b1 + eps), cap) * r01);
  float eta2 = (5.0f / 16.0f) * (1.0f + fminf(fdivf(tau5, b2 + eps), cap));
  float eta3 = (1.0f / 16.0f) * (1.0f + fminf(fdivf(tau5, b3 + eps), cap));
  float sum = eta0 + eta1 + eta2 + eta3;
  return fdivf(eta0 * u0 + eta1 * u1 + eta2 * u2 + eta3 * u3, sum);
}

// Compiler-only barrier between phases of the face pipeline: node values
// are re-read (from L1/L2) after it instead of being held in registers.
// (A scheduling barrier as well was measured to be slower: the scheduler's
// overlap of neighbouring phases pays for the registers it costs.)
__device__ __forceinline__ void phase_barrier() { asm volatile("" ::: "memory"); }

// ---------------------------------------------------------------- limiters
// theta of the convex blend (1-theta) A + theta B for one test function
// [Algorithms 1-6]: 0 if q(A) < eps, the root of the linear blend if
// q(B) < eps, else 1.
__device__ __forceinline__ double limiter_theta(double qA, double qB, double eps) {
#pragma clang fp contract(off)
  if (qA < eps) return 0.0;
  if (qB < eps) return ddiv(qA - eps, qA - qB);
  return 1.0;
}

// test function k: 0 a1r1, 1 a2r2, 2 a1, 3 1-a1, 4 rho*ctilde^2
template <bool HAS_T>
__device__ __forceinline__ double test_fn(const EosC& e, int k, const double X[6]) {
#pragma clang fp contract(off)
  switch (k) {
    case 0: return X[0];
    case 1: return X[1];
    case 2: return X[5];
    case 3: return 1.0 - X[5];
    default: return rhoc2_tilde<HAS_T>(e, X);
  }
}

__device__ __forceinline__ double tol_of(const Tol& t, int k) {
  return k < 2 ? t.eps_arho : (k < 4 ? t.eps_alpha : t.eps_rhoc2);
}

template <bool HAS_T>
__device__ __forceinline__ bool hard_switch_fails(const EosC& e, const Tol& t, const double X[6]) {
#pragma clang fp contract(off)
  if (X[0] < t.hs_arho) return true;
  if (X[1] < t.hs_arho) return true;
  if (X[5] < t.hs_alpha) return true;
  if (1.0 - X[5] < t.hs_alpha) return true;
  if (rhoc2_tilde<HAS_T>(e, X) < t.hs_rhoc2) return true;
  return false;
}

// Interpolation limiter, Algorithms 1-3 and the hard switch [Sec. 5.1].
// A: node state on the side of the interpolated value (W_i for the
// left-biased value, W_{i+1} for the right-biased one), hA = its
// rho*ctilde^2; B: interpolated state, limited in place.  A blend with
// theta = 1 is the identity, so it is skipped; the hard switch reuses the
// last rho*ctilde^2 of B when B has not changed since it was evaluated.
template <bool HAS_T>
__device__ __forceinline__ void interp_limit(const EosC& e, const Tol& t, const double A[6],
                                             double hA, double B[6]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double qA = test_fn<HAS_T>(e, k, A);
    double eps = tol_of(t, k);
    double qB = test_fn<HAS_T>(e, k, B);
    if (qA < eps) {
#pragma unroll
      for (int v = 0; v < 6; ++v) B[v] = A[v];   // theta = 0
    } else if (qB < eps) {
      double th = ddiv(qA - eps, qA - qB);
#pragma unroll
      for (int v = 0; v < 6; ++v) B[v] = (1.0 - th) * A[v] + th * B[v];
    }
  }
  double hB = rhoc2_tilde<HAS_T>(e, B);
  if (hA < t.eps_rhoc2) {
#pragma unroll
    for (int v = 0; v < 6; ++v) B[v] = A[v];
    hB = hA;
  } else if (hB < t.eps_rhoc2) {
    double th = ddiv(hA - t.eps_rhoc2, hA - hB);
#pragma unroll
    for (int v = 0; v < 6; ++v) B[v] = (1.0 - th) * A[v] + th * B[v];
    hB = rhoc2_tilde<HAS_T>(e, B);
  }
  bool fail = B[0] < t.hs_arho || B[1] < t.hs_arho || B[5] < t.hs_alpha ||
              1.0 - B[5] < t.hs_alpha || hB < t.hs_rhoc2;
  if (fail) {
#pragma unroll
    for (int v = 0; v < 6; ++v) B[v] = A[v];
  }
}

// Half-cell state component v of the flux limiter [Sec. 5.2]:
//   side 0: W_i - 2 lam (G^- - F_i),  side 1: W_{i+1} + 2 lam (G^+ - F_{i+1})
__device__ __forceinline__ double half_state(int side, double w, double lam, double g, double f) {
  return side == 0 ? w - 2.0 * lam * (g - f) : w + 2.0 * lam * (g - f);
}

// Flux limiter, Algorithms 4-6 and the hard switch [Sec. 5.2].
// Half-cell states P(G) = W_i - 2 lam (G^- - F_i), M(G) = W_{i+1} +
// 2 lam (G^+ - F_{i+1}); theta = min(theta+, theta-) per test; both fluxes
// blended toward the first-order HLLC ones (Hm, Hp).  The states are formed
// on demand from (W, F, G) instead of being stored.  Returns the smallest
// theta applied (0 if the hard switch fired).
template <bool HAS_T>
__device__ __forceinline__ double flux_limit(const EosC& e, const Tol& t, const double Wl[6],
                                             const double Wr[6], const double Fl[6],
                                             const double Fr[6], double lam, const double Hm[6],
                                             const double Hp[6], double Gm[6], double Gp[6]) {
  double thmin = 1.0;
  double hPG = 0.0, hMG = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double eps = tol_of(t, k);
    double qPH, qPG, qMH, qMG;
    if (k < 4) {
      // a1r1, a2r2, a1 or 1-a1 of the four half-cell states
      const int v = k == 0 ? 0 : (k == 1 ? 1 : 5);
      qPH = half_state(0, Wl[v], lam, Hm[v], Fl[v]);
      qPG = half_state(0, Wl[v], lam, Gm[v], Fl[v]);
      qMH = half_state(1, Wr[v], lam, Hp[v], Fr[v]);
      qMG = half_state(1, Wr[v], lam, Gp[v], Fr[v]);
      if (k == 3) { qPH = 1.0 - qPH; qPG = 1.0 - qPG; qMH = 1.0 - qMH; qMG = 1.0 - qMG; }
    } else {
      double X[6];
#pragma unroll
      for (int v = 0; v < 6; ++v) X[v] = half_state(0, Wl[v], lam, Hm[v], Fl[v]);
      qPH = rhoc2_tilde<HAS_T>(e, X);
#pragma unroll
      for (int v = 0; v < 6; ++v) X[v] = half_state(0, Wl[v], lam, Gm[v], Fl[v]);
      qPG = rhoc2_tilde<HAS_T>(e, X);
#pragma unroll
      for (int v = 0; v < 6; ++v) X[v] = half_state(1, Wr[v], lam, Hp[v], Fr[v]);
      qMH = rhoc2_tilde<HAS_T>(e, X);
#pragma unroll
      for (int v = 0; v < 6; ++v) X[v] = half_state(1, Wr[v], lam, Gp[v], Fr[v]);
      qMG = rhoc2_tilde<HAS_T>(e, X);
      hPG = qPG;
      hMG = qMG;
    }
    double thp = limiter_theta(qPH, qPG, eps);
    double thm = limiter_theta(qMH, qMG, eps);
    double th = (thm < thp) ? thm : thp;
    if (th != 1.0) {
#pragma unroll
      for (int v = 0; v < 6; ++v) {
        Gp[v] = (1.0 - th) * Hp[v] + th * Gp[v];
        Gm[v] = (1.0 - th) * Hm[v] + th * Gm[v];
      }
      thmin = (th < thmin) ? th : thmin;
      if (k == 4) {
        double X[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) X[v] = half_state(0, Wl[v], lam, Gm[v], Fl[v]);
        hPG = rhoc2_tilde<HAS_T>(e, X);
#pragma unroll
        for (int v = 0; v < 6; ++v) X[v] = half_state(1, Wr[v], lam, Gp[v], Fr[v]);
        hMG = rhoc2_tilde<HAS_T>(e, X);
      }
    }
  }
  // hard switch on the final half-cell states
  bool fail = false;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const double* Wx = side == 0 ? Wl : Wr;
    const double* Fx = side == 0 ? Fl : Fr;
    const double* Gx = side == 0 ? Gm : Gp;
    double x0 = half_state(side, Wx[0], lam, Gx[0], Fx[0]);
    double x1 = half_state(side, Wx[1], lam, Gx[1], Fx[1]);
    double x5 = half_state(side, Wx[5], lam, Gx[5], Fx[5]);
    double hx = side == 0 ? hPG : hMG;
    fail = fail || x0 < t.hs_arho || x1 < t.hs_arho || x5 < t.hs_alpha || 1.0 - x5 < t.hs_alpha ||
           hx < t.hs_rhoc2;
  }
  if (fail) {
#pragma unroll
    for (int v = 0; v < 6; ++v) { Gm[v] = Hm[v]; Gp[v] = Hp[v]; }
    thmin = 0.0;
  }
  return thmin;
}

// HCS implied reconstructed flux with psi = 256/175 [Sec. 4.1]:
// [3072 gt - 505 (g_i + g_{i+1}) + 20 (g_{i-1} + g_{i+2}) - (g_{i-2} + g_{i+3})]/2100
__device__ __forceinline__ double hcs(double gt, double s01, double s12, double s03) {
#pragma clang fp contract(off)
  return cdiv(3072.0 * gt - 505.0 * s01 + 20.0 * s12 - s03, 2100.0, R2100);
}

}  // namespace wcns
