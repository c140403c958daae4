// ============================================================================
// Reference ("oracle") implementation of the PP-WCNS-IS right-hand side for
// Allaire's five-equation two-phase model (Wong, Angel, Barad & Kiris,
// "A positivity-preserving high-order weighted compact nonlinear scheme for
// compressible gas-liquid flows", arXiv 2102.05287).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, serial FP64 CPU
// statement of what the method computes.  It is used by the test-suite, by
// the package smoke check and by the CPU-baseline leg of the benchmark, and by
// nothing else.  It shares no code, header, constant table or helper with the
// GPU library, and it never loads it.
//
// Build: g++ -std=c++17 -O2 -ffp-contract=off -shared -fPIC (no fast-math, no
// FMA contraction) so that every operation is rounded once, in source order.
//
// Every arithmetic routine is a template on the scalar type T so the same
// source, instantiated with an operation-counting scalar, yields the
// algorithmic operation count of one cell update (used for the roofline).
//
// State layout (SoA): W[v][k][j][i], v over
//   3D: (a1r1, a2r2, rho*u, rho*v, rho*w, E, a1)   (the direct 3D extension)
//   2D: (a1r1, a2r2, rho*u, rho*v, E, a1)     (paper Sec. 3, conservative W)
//   1D: (a1r1, a2r2, rho*u, E, a1)             (rho*v dropped, Sec. 2)
// Internally every sweep works on a 6-component state rotated into the sweep
// direction: (a1r1, a2r2, m_n, m_t, E, a1) with m_n the normal momentum and
// m_t the tangential one (m_t = 0 in 1D, which reproduces the 1D system
// exactly because every m_t/u_t term is then an exact zero).
//
// Readings of points the paper leaves open are marked "Reading:" below.
// ============================================================================
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

namespace {

// ---------------------------------------------------------------------------
// Parameters (C layout shared with the Python ctypes binding of this oracle).
// ---------------------------------------------------------------------------
struct Problem {
  int32_t ndim, nx, ny, pad0;
  double dx, dy;
  int32_t bc[4];            // x-lo, x-hi, y-lo, y-hi: 0 periodic, 1 constant
                            // extrapolation, 2 reflective wall, 3 Dirichlet
  const double* dirichlet_rows[4];  // Dirichlet sides: conservative ghost state
                            // of each boundary row (x sides, ny rows) or
                            // column (y sides, nx columns), nvar values each
                            // in state order; a side's three ghost layers
                            // share their row's state
  double gamma[2], pinf[2]; // phase 1 (liquid), phase 2 (gas)  [Table 1]
  double eps_arho, eps_alpha, eps_rhoc2;   // limiter tolerances  [Sec. 5.1]
  double hs_arho, hs_alpha, hs_rhoc2;      // hard-switch tolerances
  double weno_eps;                         // epsilon of the IS weights
  double cfl;
  int32_t interp_limiter, flux_limiter, scheme;  // scheme 0 PP-WCNS-IS, 1 HLLC1
  int32_t pad1;
  int32_t nz;               // 1 unless ndim = 3
  int32_t bcz[2];           // z-lo, z-hi (3D; Dirichlet not supported there)
  int32_t pad2;
  double dz;
};

enum { BC_PERIODIC = 0, BC_EXTRAP = 1, BC_REFLECT = 2, BC_DIRICHLET = 3 };

// ---------------------------------------------------------------------------
// Operation-counting scalar.  Each +,-,*,/,sqrt and each comparison (min,
// max, sign tests, limiter tests) increments a counter.  Conversions from
// double literals are free (they are constants).
// ---------------------------------------------------------------------------
struct OpCounts { long long add, mul, div, sqrt, cmp; };
static OpCounts g_ops;

// The counts are also filed by step of the face pipeline (the phase set by
// count_phase; bookkeeping only, no arithmetic): the precision form runs
// some steps in FP32, so its roofline prices each step at its own precision.
enum {
  PH_FIRST_ORDER,   // first-order HLLC flux at the face [Sec. 3.2]
  PH_PROJECT,       // face averages and U = R^{-1} V [Sec. 4.2, App. A]
  PH_WENO,          // IS-WENO interpolation [Sec. 4.3]
  PH_BACK_V,        // V = R U [App. A]
  PH_TO_W,          // V -> W [Sec. 2]
  PH_INTERP_LIMIT,  // Algorithms 1-3 [Sec. 5.1]
  PH_MID_RECOVER,   // primitives of the limited midpoint states [Sec. 2]
  PH_MID_HLLC,      // midpoint HLLC flux [Sec. 3.1-3.2]
  PH_HCS,           // HCS flux and velocity [Sec. 4.1]
  PH_SPLIT_LIMIT,   // split fluxes G^{+-} and Algorithms 4-6 [Sec. 3.2, 5.2]
  NPHASE
};
static OpCounts g_phase_ops[NPHASE];
static int g_phase = 0;

struct Cnt {
  double v;
  Cnt() : v(0) {}
  Cnt(double x) : v(x) {}
};
inline void tick(long long OpCounts::*f) {
  g_ops.*f += 1;
  g_phase_ops[g_phase].*f += 1;
}
inline Cnt operator+(Cnt a, Cnt b) { tick(&OpCounts::add); return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { tick(&OpCounts::add); return Cnt(a.v - b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }  // sign flip: free
inline Cnt operator*(Cnt a, Cnt b) { tick(&OpCounts::mul); return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { tick(&OpCounts::div); return Cnt(a.v / b.v); }
inline bool operator<(Cnt a, Cnt b) { tick(&OpCounts::cmp); return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { tick(&OpCounts::cmp); return a.v > b.v; }
inline bool operator==(Cnt a, Cnt b) { tick(&OpCounts::cmp); return a.v == b.v; }
inline Cnt sqrt(Cnt a) { tick(&OpCounts::sqrt); return Cnt(std::sqrt(a.v)); }
// the step the next operations belong to (counting scalar only)
inline void count_phase(const Cnt&, int ph) { g_phase = ph; }
inline void count_phase(const double&, int) {}
inline double val(Cnt a) { return a.v; }
inline double val(double a) { return a; }
using std::sqrt;

template <class T> inline T tmin(T a, T b) { return (b < a) ? b : a; }
template <class T> inline T tmax(T a, T b) { return (a < b) ? b : a; }
// sgn with sgn(0) = 0.  Reading: the HLLC flux weights (1 +/- sgn s*)/2
// average the two sides when s* = 0 [Sec. 3.2, HLLC flux].
template <class T> inline T tsgn(T a) {
  if (a > T(0.0)) return T(1.0);
  if (a < T(0.0)) return T(-1.0);
  return T(0.0);
}

// ---------------------------------------------------------------------------
// Equation of state [Sec. 2, stiffened gas per phase and mixture rules]
//   1/(gbar-1) = sum_k alpha_k/(gamma_k-1)                      =: Gamma
//   gbar*pbar_inf/(gbar-1) = sum_k alpha_k gamma_k pinf_k/(gamma_k-1) =: Pi
//   p/(gbar-1) + gbar*pbar_inf/(gbar-1) = rho*e   =>  p = (rho e - Pi)/Gamma
//   pbar_inf = Pi/(1+Gamma),  gbar = 1 + 1/Gamma,
//   rho c^2 = gbar (p + pbar_inf)                   [Sec. 2, mixture c]
// ---------------------------------------------------------------------------
struct Eos { double g1, g2, q1, q2; };  // g_k = 1/(gamma_k-1), q_k = gamma_k pinf_k/(gamma_k-1)

inline Eos make_eos(const Problem& P) {
  Eos e;
  e.g1 = 1.0 / (P.gamma[0] - 1.0);
  e.g2 = 1.0 / (P.gamma[1] - 1.0);
  e.q1 = P.gamma[0] * P.pinf[0] / (P.gamma[0] - 1.0);
  e.q2 = P.gamma[1] * P.pinf[1] / (P.gamma[1] - 1.0);
  return e;
}

template <class T> inline T mix_Gamma(const Eos& e, T a1) {
  T a2 = T(1.0) - a1;
  return a1 * T(e.g1) + a2 * T(e.g2);
}
template <class T> inline T mix_Pi(const Eos& e, T a1) {
  T a2 = T(1.0) - a1;
  return a1 * T(e.q1) + a2 * T(e.q2);
}

// Rotated states have NR = 6 components (1D, 2D) or NR = 7 (3D):
//   X = (a1r1, a2r2, m_n, m_t, [m_s,] E, a1)
// with m_n the normal and m_t (m_s) the tangential momenta.  In 3D the second
// tangential momentum is one more passive component (Sec. 2: the extension of
// the system to three dimensions is direct).  E sits at NR-2, a1 at NR-1.
template <int NR> struct Lay {
  static_assert(NR == 6 || NR == 7, "rotated states have 6 or 7 components");
  static constexpr int IE = NR - 2, IA = NR - 1;
};

// Node quantities of a rotated state
template <class T, int NR = 6> struct Node {
  T w[NR];
  T rho, un, ut, us, p, c, h;   // us: second tangential velocity (0 unless NR = 7)
                                // h = rho*ctilde^2 = rho e - pbar_inf  [Sec. 5.1]
  T g[NR];                      // flux G = F + (0,..,0, a1 u)  [Sec. 3.2]
};

// rho*ctilde^2 of a state (the third limiter test function) [Sec. 5.1]
template <int NR = 6, class T> inline T rhoc2_tilde(const Eos& e, const T* X) {
  constexpr int IE = Lay<NR>::IE, IA = Lay<NR>::IA;
  T rho = X[0] + X[1];
  T irho = T(1.0) / rho;
  T un = X[2] * irho;
  T ut = X[3] * irho;
  T ke = X[2] * un + X[3] * ut;
  if (NR == 7) ke = ke + X[4] * (X[4] * irho);
  T rhoe = X[IE] - T(0.5) * ke;
  T Gam = mix_Gamma(e, X[IA]);
  T Pi = mix_Pi(e, X[IA]);
  T pinf_bar = Pi / (T(1.0) + Gam);
  return rhoe - pinf_bar;
}

// Conservative -> primitive, sound speed and node flux [Sec. 2; Sec. 3.2
// flux-source form; WCNS steps 1 and 7].
template <int NR = 6, class T> inline Node<T, NR> node_from_w(const Eos& e, const T* X) {
  constexpr int IE = Lay<NR>::IE, IA = Lay<NR>::IA;
  Node<T, NR> n;
  for (int v = 0; v < NR; ++v) n.w[v] = X[v];
  n.rho = X[0] + X[1];
  T irho = T(1.0) / n.rho;
  n.un = X[2] * irho;
  n.ut = X[3] * irho;
  n.us = NR == 7 ? X[4] * irho : T(0.0);
  T ke = X[2] * n.un + X[3] * n.ut;
  if (NR == 7) ke = ke + X[4] * n.us;
  T rhoe = X[IE] - T(0.5) * ke;
  T Gam = mix_Gamma(e, X[IA]);
  T Pi = mix_Pi(e, X[IA]);
  n.p = (rhoe - Pi) / Gam;
  T pinf_bar = Pi / (T(1.0) + Gam);
  T gbar = T(1.0) + T(1.0) / Gam;
  T c2 = gbar * (n.p + pinf_bar) * irho;
  n.c = sqrt(c2);
  n.h = rhoe - pinf_bar;
  n.g[0] = X[0] * n.un;
  n.g[1] = X[1] * n.un;
  n.g[2] = X[2] * n.un + n.p;
  n.g[3] = X[3] * n.un;
  if (NR == 7) n.g[4] = X[4] * n.un;
  n.g[IE] = (X[IE] + n.p) * n.un;
  n.g[IA] = X[IA] * n.un;
  return n;
}

// ---------------------------------------------------------------------------
// HLLC approximate Riemann solver [Sec. 3.1 star states, Einfeldt speeds,
// Batten contact speed; Sec. 3.2 conservative flux, u* and f_alpha].
// Outputs F (the NR-1 conservative components), f_alpha and s*.
// ---------------------------------------------------------------------------
template <class T, int NR>
inline void hllc(const Node<T, NR>& L, const Node<T, NR>& R, T* F, T& falpha, T& sstar) {
  constexpr int IE = Lay<NR>::IE, IA = Lay<NR>::IA;
  T ubar = T(0.5) * (L.un + R.un);
  T cbar = T(0.5) * (L.c + R.c);
  T sL = tmin(ubar - cbar, L.un - L.c);
  T sR = tmax(ubar + cbar, R.un + R.c);
  T num = R.p - L.p + L.rho * L.un * (sL - L.un) - R.rho * R.un * (sR - R.un);
  T den = L.rho * (sL - L.un) - R.rho * (sR - R.un);
  T ss = num / den;
  sstar = ss;
  // star states W*_K
  T chiL = (sL - L.un) / (sL - ss);
  T chiR = (sR - R.un) / (sR - ss);
  T WsL[NR - 1], WsR[NR - 1];
  WsL[0] = chiL * L.w[0];
  WsL[1] = chiL * L.w[1];
  WsL[2] = chiL * L.rho * ss;
  WsL[3] = chiL * L.rho * L.ut;
  if (NR == 7) WsL[4] = chiL * L.rho * L.us;
  WsL[IE] = chiL * (L.w[IE] + (ss - L.un) * (L.rho * ss + L.p / (sL - L.un)));
  WsR[0] = chiR * R.w[0];
  WsR[1] = chiR * R.w[1];
  WsR[2] = chiR * R.rho * ss;
  WsR[3] = chiR * R.rho * R.ut;
  if (NR == 7) WsR[4] = chiR * R.rho * R.us;
  WsR[IE] = chiR * (R.w[IE] + (ss - R.un) * (R.rho * ss + R.p / (sR - R.un)));
  T sm = tmin(T(0.0), sL);
  T sp = tmax(T(0.0), sR);
  T sg = tsgn(ss);
  T wl = (T(1.0) + sg) * T(0.5);
  T wr = (T(1.0) - sg) * T(0.5);
  // F_K is the conservative flux: the node flux g without its alpha part
  for (int v = 0; v < NR - 1; ++v) {
    T fl = L.g[v] + sm * (WsL[v] - L.w[v]);
    T fr = R.g[v] + sp * (WsR[v] - R.w[v]);
    F[v] = wl * fl + wr * fr;
  }
  falpha = wl * (L.w[IA] * ss) + wr * (R.w[IA] * ss);
}

// ---------------------------------------------------------------------------
// Incremental-stencil WENO interpolation to the midpoint [Sec. 4.3].
// Left-biased form on (a,b,c,d,e) = (u_{i-2}, u_{i-1}, u_i, u_{i+1}, u_{i+2});
// the right-biased value is the same routine on the flipped stencil.
// ---------------------------------------------------------------------------
template <class T>
inline T weno_is(T a, T b, T c, T d, T e, double eps) {
  // sub-stencil interpolations S0..S3
  // (the factors 1/2 and 1/8 are exact powers of two: multiplying is
  // bit-identical to dividing)
  T u0 = T(0.5) * (c + d);
  T u1 = T(0.5) * (-b + T(3.0) * c);
  T u2 = T(0.125) * (T(3.0) * c + T(6.0) * d - e);
  T u3 = T(0.125) * (T(3.0) * a - T(10.0) * b + T(15.0) * c);
  // smoothness indicators
  T b0 = (c - d) * (c - d);
  T b1 = (b - c) * (b - c);
  T t01a = b - T(2.0) * c + d, t01b = b - d;
  T b01 = T(13.0 / 12.0) * t01a * t01a + T(0.25) * t01b * t01b;
  T t2a = c - T(2.0) * d + e, t2b = T(3.0) * c - T(4.0) * d + e;
  T b2 = T(13.0 / 12.0) * t2a * t2a + T(0.25) * t2b * t2b;
  T t3a = a - T(2.0) * b + c, t3b = a - T(4.0) * b + T(3.0) * c;
  T b3 = T(13.0 / 12.0) * t3a * t3a + T(0.25) * t3b * t3b;
  // reference indicator tau_5
  T t5a = e - T(4.0) * d + T(6.0) * c - T(4.0) * b + a;
  T t5b = e - T(2.0) * d + T(2.0) * b - a;
  T tau5 = T(13.0 / 12.0) * t5a * t5a + T(0.25) * t5b * t5b;
  // nonlinear weights
  T E(eps);
  T r01 = tau5 / (b01 + E);
  T eta0 = T(15.0 / 32.0) * (T(1.0) + tau5 / (b0 + E) * r01);
  T eta1 = T(5.0 / 32.0) * (T(1.0) + tau5 / (b1 + E) * r01);
  T eta2 = T(5.0 / 16.0) * (T(1.0) + tau5 / (b2 + E));
  T eta3 = T(1.0 / 16.0) * (T(1.0) + tau5 / (b3 + E));
  T sum = eta0 + eta1 + eta2 + eta3;
  return (eta0 * u0 + eta1 * u1 + eta2 * u2 + eta3 * u3) / sum;
}

// ---------------------------------------------------------------------------
// Limiter building block: one test function q and one tolerance; returns the
// theta of a convex blend (1-theta) A + theta B  [Algorithms 1-6].
// Reading: comparisons are strict "<", as printed.
// ---------------------------------------------------------------------------
template <class T> inline T limiter_theta(T qA, T qB, double eps) {
  if (qA < T(eps)) return T(0.0);
  if (qB < T(eps)) return (qA - T(eps)) / (qA - qB);
  return T(1.0);
}

// Test function k of a rotated state: 0 a1r1, 1 a2r2, 2 a1, 3 a2 = 1-a1,
// 4 rho*ctilde^2.
template <int NR = 6, class T> inline T test_fn(const Eos& e, int k, const T* X) {
  constexpr int IA = Lay<NR>::IA;
  switch (k) {
    case 0: return X[0];
    case 1: return X[1];
    case 2: return X[IA];
    case 3: return T(1.0) - X[IA];
    default: return rhoc2_tilde<NR>(e, X);
  }
}

// true when a state fails the hard-switch tolerances [Sec. 5.1, 5.2]
template <int NR = 6, class T>
inline bool hard_switch_fails(const Eos& e, const Problem& P, const T* X) {
  constexpr int IA = Lay<NR>::IA;
  if (X[0] < T(P.hs_arho)) return true;
  if (X[1] < T(P.hs_arho)) return true;
  if (X[IA] < T(P.hs_alpha)) return true;
  if (T(1.0) - X[IA] < T(P.hs_alpha)) return true;
  if (rhoc2_tilde<NR>(e, X) < T(P.hs_rhoc2)) return true;
  return false;
}

inline double tol_of(const Problem& P, int k) {
  return k < 2 ? P.eps_arho : (k < 4 ? P.eps_alpha : P.eps_rhoc2);
}

// Interpolation limiter, Algorithms 1-3 plus the hard switch [Sec. 5.1]:
// B (the WENO-interpolated state) is pulled toward A (the node state on its
// side: W_i for the left-biased value, W_{i+1} for the right-biased one).
template <int NR = 6, class T>
inline void interp_limit(const Eos& e, const Problem& P, const T* A, T* B) {
  for (int k = 0; k < 5; ++k) {
    T th = limiter_theta(test_fn<NR>(e, k, A), test_fn<NR>(e, k, B), tol_of(P, k));
    // the blend with theta = 1 is the identity: only a theta < 1 changes B
    if (val(th) != 1.0)
      for (int v = 0; v < NR; ++v) B[v] = (T(1.0) - th) * A[v] + th * B[v];
  }
  if (hard_switch_fails<NR>(e, P, B))
    for (int v = 0; v < NR; ++v) B[v] = A[v];
}

// Flux limiter, Algorithms 4-6 plus the hard switch [Sec. 5.2].
// Gm/Gp: high-order G^-_{i+1/2}, G^+_{i+1/2}; Hm/Hp: first-order HLLC ones.
// Wl/Wr: node states W_i, W_{i+1}; Fl/Fr: their conservative fluxes F (alpha
// component 0).  lam = dt/(dx*sigma).  Returns the last theta used (1 when
// no limiting happened, 0 when the hard switch fired).
template <int NR = 6, class T>
inline T flux_limit(const Eos& e, const Problem& P, const T* Wl, const T* Wr,
                    const T* Fl, const T* Fr, T lam, const T* Hm, const T* Hp,
                    T* Gm, T* Gp) {
  T PH[NR], MH[NR], PG[NR], MG[NR];
  // half-cell states W_i^{+} = W_i - 2 lam (G^- - F_i),
  //                 W_{i+1}^{-} = W_{i+1} + 2 lam (G^+ - F_{i+1})
  auto states = [&](const T* gm, const T* gp, T* Ps, T* Ms) {
    for (int v = 0; v < NR; ++v) {
      Ps[v] = Wl[v] - T(2.0) * lam * (gm[v] - Fl[v]);
      Ms[v] = Wr[v] + T(2.0) * lam * (gp[v] - Fr[v]);
    }
  };
  states(Hm, Hp, PH, MH);
  states(Gm, Gp, PG, MG);
  T thmin = T(1.0);
  for (int k = 0; k < 5; ++k) {
    double eps = tol_of(P, k);
    T thp = limiter_theta(test_fn<NR>(e, k, PH), test_fn<NR>(e, k, PG), eps);
    T thm = limiter_theta(test_fn<NR>(e, k, MH), test_fn<NR>(e, k, MG), eps);
    T th = tmin(thp, thm);
    if (val(th) != 1.0) {   // theta = 1 leaves both fluxes unchanged
      for (int v = 0; v < NR; ++v) {
        Gp[v] = (T(1.0) - th) * Hp[v] + th * Gp[v];
        Gm[v] = (T(1.0) - th) * Hm[v] + th * Gm[v];
      }
      // Reading: the half-cell states of the next test are recomputed from
      // the blended fluxes (equal, in exact arithmetic, to blending states).
      states(Gm, Gp, PG, MG);
      thmin = tmin(thmin, th);
    }
  }
  if (hard_switch_fails<NR>(e, P, PG) || hard_switch_fails<NR>(e, P, MG)) {
    for (int v = 0; v < NR; ++v) { Gm[v] = Hm[v]; Gp[v] = Hp[v]; }
    thmin = T(0.0);
  }
  return thmin;
}

// Characteristic projection built from face averages [App. A, R_A and
// R_A^{-1}; Sec. 4.2]: the plain means of the two nodes' partial
// densities, total density and sound speed.
template <class T> struct FaceAvg { T a1, a2, rho, c, k1, k2; };

template <class T, int NR>
inline FaceAvg<T> face_avg(const Node<T, NR>& L, const Node<T, NR>& R) {
  FaceAvg<T> f;
  f.a1 = T(0.5) * (L.w[0] + R.w[0]);
  f.a2 = T(0.5) * (L.w[1] + R.w[1]);
  f.rho = T(0.5) * (L.rho + R.rho);
  f.c = T(0.5) * (L.c + R.c);
  f.k1 = T(1.0) / (f.rho * f.c);
  f.k2 = T(1.0) / (f.rho * f.c * f.c);
  return f;
}

// U = R^{-1} V with V = (a1r1, a2r2, u_n, u_t, [u_s,] p, a1); the fields are
// (u_n - p/(rho c), a1r1 - a1 p/(rho c^2), a2r2 - a2 p/(rho c^2), u_t,
// [u_s,] a1, u_n + p/(rho c))
template <class T, int NR>
inline void project(const FaceAvg<T>& f, const Node<T, NR>& n, T* U) {
  U[0] = n.un - n.p * f.k1;
  U[1] = n.w[0] - f.a1 * n.p * f.k2;
  U[2] = n.w[1] - f.a2 * n.p * f.k2;
  U[3] = n.ut;
  if (NR == 7) U[4] = n.us;
  U[NR - 2] = n.w[Lay<NR>::IA];
  U[NR - 1] = n.un + n.p * f.k1;
}

// V = R U, then V -> W  [App. A; Sec. 2 mixture EOS for E]
template <int NR = 6, class T>
inline void back_project_to_w(const Eos& e, const FaceAvg<T>& f, const T* U, T* X) {
  constexpr int IE = Lay<NR>::IE, IA = Lay<NR>::IA;
  const T& Uplus = U[NR - 1];
  T a1r1 = U[1] + f.a1 * (Uplus - U[0]) / (T(2.0) * f.c);
  T a2r2 = U[2] + f.a2 * (Uplus - U[0]) / (T(2.0) * f.c);
  T un = T(0.5) * (U[0] + Uplus);
  T ut = U[3];
  T us = NR == 7 ? U[4] : T(0.0);
  T p = T(0.5) * f.rho * f.c * (Uplus - U[0]);
  T a1 = U[NR - 2];
  count_phase(a1, PH_TO_W);
  T rho = a1r1 + a2r2;
  X[0] = a1r1;
  X[1] = a2r2;
  X[2] = rho * un;
  X[3] = rho * ut;
  if (NR == 7) X[4] = rho * us;
  T ke = un * un + ut * ut;
  if (NR == 7) ke = ke + us * us;
  X[IE] = mix_Gamma(e, a1) * p + mix_Pi(e, a1) + T(0.5) * rho * ke;
  X[IA] = a1;
}

// HCS implied reconstructed flux, psi = 256/175  [Sec. 4.1]:
// ghat = [3072 gt - 505 (g_i + g_{i+1}) + 20 (g_{i-1} + g_{i+2})
//         - (g_{i-2} + g_{i+3})] / 2100
template <class T>
inline T hcs(T gt, T gm2, T gm1, T g0, T gp1, T gp2, T gp3) {
  return (T(3072.0) * gt - T(505.0) * (g0 + gp1) + T(20.0) * (gm1 + gp2) - (gm2 + gp3)) /
         T(2100.0);
}

// ---------------------------------------------------------------------------
// One face i+1/2 of one sweep: the nine WCNS steps [Sec. 4.2] with the
// interpolation limiter [Sec. 5.1] and the flux limiter [Sec. 5.2].
// nd[0..5] are the node quantities of nodes i-2 .. i+3 (rotated frame).
// Outputs G^-_{i+1/2} and G^+_{i+1/2} (NR components each).
// ---------------------------------------------------------------------------
template <class T, int NR>
inline T face_flux(const Eos& e, const Problem& P, const Node<T, NR> nd[6], T lam, T* Gm,
                   T* Gp) {
  constexpr int IA = Lay<NR>::IA;
  const Node<T, NR>& nl = nd[2];
  const Node<T, NR>& nr = nd[3];
  // first-order HLLC at the face from W_i, W_{i+1}  [Sec. 3.2]
  count_phase(lam, PH_FIRST_ORDER);
  T Fh[NR - 1], fah, ush;
  hllc(nl, nr, Fh, fah, ush);
  T Hm[NR], Hp[NR];
  for (int v = 0; v < NR - 1; ++v) { Hm[v] = Fh[v]; Hp[v] = Fh[v]; }
  Hm[IA] = fah - nl.w[IA] * ush;   // G^{-}: alpha of cell i      [Sec. 3.2]
  Hp[IA] = fah - nr.w[IA] * ush;   // G^{+}: alpha of cell i+1
  if (P.scheme == 1) {             // first-order HLLC scheme (theta = 0)
    for (int v = 0; v < NR; ++v) { Gm[v] = Hm[v]; Gp[v] = Hp[v]; }
    return T(0.0);
  }
  // step 2: characteristic projection of the stencil nodes
  count_phase(lam, PH_PROJECT);
  FaceAvg<T> fa = face_avg(nl, nr);
  T U[6][NR];
  for (int m = 0; m < 6; ++m) project(fa, nd[m], U[m]);
  // step 3: left- and right-biased IS-WENO interpolation per field
  count_phase(lam, PH_WENO);
  T UL[NR], UR[NR];
  for (int k = 0; k < NR; ++k) {
    UL[k] = weno_is(U[0][k], U[1][k], U[2][k], U[3][k], U[4][k], P.weno_eps);
    UR[k] = weno_is(U[5][k], U[4][k], U[3][k], U[2][k], U[1][k], P.weno_eps);
  }
  // steps 4-5: back to primitive, then conservative
  T WL[NR], WR[NR];
  count_phase(lam, PH_BACK_V);
  back_project_to_w<NR>(e, fa, UL, WL);
  count_phase(lam, PH_BACK_V);
  back_project_to_w<NR>(e, fa, UR, WR);
  // interpolation limiter toward W_i (left) and W_{i+1} (right)
  count_phase(lam, PH_INTERP_LIMIT);
  if (P.interp_limiter) {
    interp_limit<NR>(e, P, nl.w, WL);
    interp_limit<NR>(e, P, nr.w, WR);
  }
  // step 6: high-order midpoint flux and velocity from the Riemann solver
  count_phase(lam, PH_MID_RECOVER);
  Node<T, NR> tl = node_from_w<NR>(e, WL);
  Node<T, NR> tr = node_from_w<NR>(e, WR);
  count_phase(lam, PH_MID_HLLC);
  T Ft[NR - 1], fat, ust;
  hllc(tl, tr, Ft, fat, ust);
  T gt[NR];
  for (int v = 0; v < NR - 1; ++v) gt[v] = Ft[v];
  gt[IA] = fat;
  // steps 7-8: node fluxes and HCS reconstruction of the flux and velocity
  count_phase(lam, PH_HCS);
  T Gh[NR];
  for (int v = 0; v < NR; ++v)
    Gh[v] = hcs(gt[v], nd[0].g[v], nd[1].g[v], nd[2].g[v], nd[3].g[v], nd[4].g[v], nd[5].g[v]);
  T uh = hcs(ust, nd[0].un, nd[1].un, nd[2].un, nd[3].un, nd[4].un, nd[5].un);
  // step 9: non-conservative split fluxes G^{+-}
  count_phase(lam, PH_SPLIT_LIMIT);
  for (int v = 0; v < NR - 1; ++v) { Gm[v] = Gh[v]; Gp[v] = Gh[v]; }
  Gm[IA] = Gh[IA] - nl.w[IA] * uh;
  Gp[IA] = Gh[IA] - nr.w[IA] * uh;
  // flux limiter toward the first-order HLLC fluxes
  if (P.flux_limiter) {
    T Fl[NR], Fr[NR];
    for (int v = 0; v < NR - 1; ++v) { Fl[v] = nl.g[v]; Fr[v] = nr.g[v]; }
    Fl[IA] = T(0.0);
    Fr[IA] = T(0.0);
    return flux_limit<NR>(e, P, nl.w, nr.w, Fl, Fr, lam, Hm, Hp, Gm, Gp);
  }
  return T(1.0);
}

// ---------------------------------------------------------------------------
// Grid plumbing: ghost cells, rotation, sweeps.
// ---------------------------------------------------------------------------
inline int nvar_of(const Problem& P) { return P.ndim == 1 ? 5 : (P.ndim == 2 ? 6 : 7); }
inline long ncell_of(const Problem& P) {
  return (long)P.nx * P.ny * (P.ndim == 3 ? P.nz : 1);
}

// full 6-component state of cell (i,j) in the unrotated frame
inline void load_cell(const Problem& P, const double* W, int i, int j, double X[6]) {
  const long n = (long)P.nx * P.ny;
  const long o = (long)j * P.nx + i;
  if (P.ndim == 1) {
    X[0] = W[0 * n + o]; X[1] = W[1 * n + o]; X[2] = W[2 * n + o];
    X[3] = 0.0;          X[4] = W[3 * n + o]; X[5] = W[4 * n + o];
  } else {
    for (int v = 0; v < 6; ++v) X[v] = W[v * n + o];
  }
}

// index of the interior cell that supplies ghost index g along a line of n
// cells, and whether the normal momentum flips sign; returns -1 for Dirichlet
inline int ghost_source(int bc_lo, int bc_hi, int g, int n, bool& flip) {
  flip = false;
  if (g >= 0 && g < n) return g;
  int bc = g < 0 ? bc_lo : bc_hi;
  switch (bc) {
    case BC_PERIODIC: return ((g % n) + n) % n;
    case BC_EXTRAP: return g < 0 ? 0 : n - 1;
    case BC_REFLECT: flip = true; return g < 0 ? -1 - g : 2 * n - 1 - g;
    default: return -1;
  }
}

// 6-state of (possibly ghost) node at position g along a line, rotated frame.
// dir 0: line along x at row j; dir 1: line along y at column i.
inline void load_rotated(const Problem& P, const double* W, int dir, int line, int g,
                         double X[6]) {
  const int n = dir == 0 ? P.nx : P.ny;
  const int lo = dir == 0 ? P.bc[0] : P.bc[2];
  const int hi = dir == 0 ? P.bc[1] : P.bc[3];
  bool flip;
  int s = ghost_source(lo, hi, g, n, flip);
  double Y[6];
  if (s < 0) {
    const int nv = P.ndim == 1 ? 5 : 6;
    const double* d = P.dirichlet_rows[dir * 2 + (g < 0 ? 0 : 1)] + (size_t)line * nv;
    if (P.ndim == 1) { Y[0] = d[0]; Y[1] = d[1]; Y[2] = d[2]; Y[3] = 0.0; Y[4] = d[3]; Y[5] = d[4]; }
    else for (int v = 0; v < 6; ++v) Y[v] = d[v];
  } else if (dir == 0) {
    load_cell(P, W, s, line, Y);
  } else {
    load_cell(P, W, line, s, Y);
  }
  // reflective wall: mirror the state and negate the wall-normal momentum
  if (flip) { if (dir == 0) Y[2] = -Y[2]; else Y[3] = -Y[3]; }
  // rotate into (a1r1, a2r2, m_n, m_t, E, a1)
  X[0] = Y[0]; X[1] = Y[1]; X[4] = Y[4]; X[5] = Y[5];
  if (dir == 0) { X[2] = Y[2]; X[3] = Y[3]; }
  else { X[2] = Y[3]; X[3] = Y[2]; }
}

// rotated flux components back to the unrotated variable order (6 comps)
inline void unrotate(int dir, const double R[6], double X[6]) {
  X[0] = R[0]; X[1] = R[1]; X[4] = R[4]; X[5] = R[5];
  if (dir == 0) { X[2] = R[2]; X[3] = R[3]; }
  else { X[2] = R[3]; X[3] = R[2]; }
}

// Max wave speeds max(|u|+c), max(|v|+c) [Sec. 3.3] over every state a face
// flux of that direction sees: the interior cells and, on a Dirichlet side,
// its ghost states (the other ghost kinds copy interior states).  Reading:
// the CFL bound behind sigma and lambda must hold at the boundary faces too,
// where an inflow state can be much faster than the interior (Sec. 6.7).
void max_wavespeed(const Problem& P, const double* W, double amax[2]) {
  Eos e = make_eos(P);
  amax[0] = 0.0; amax[1] = 0.0;
  for (int j = 0; j < P.ny; ++j)
    for (int i = 0; i < P.nx; ++i) {
      double X[6];
      load_cell(P, W, i, j, X);
      Node<double> n = node_from_w(e, X);   // frame x: un = u, ut = v
      amax[0] = std::max(amax[0], std::fabs(n.un) + n.c);
      amax[1] = std::max(amax[1], std::fabs(n.ut) + n.c);
    }
  for (int side = 0; side < (P.ndim == 1 ? 2 : 4); ++side) {
    if (P.bc[side] != BC_DIRICHLET) continue;
    const int dir = side / 2;
    const int nline = dir == 0 ? P.ny : P.nx;
    const int g = (side & 1) ? (dir == 0 ? P.nx : P.ny) : -1;
    for (int l = 0; l < nline; ++l) {
      double X[6];
      load_rotated(P, W, dir, l, g, X);
      Node<double> n = node_from_w(e, X);   // rotated frame: un normal to the side
      amax[dir] = std::max(amax[dir], std::fabs(n.un) + n.c);
    }
  }
}

// Directional split sigma and lambda = dt/(dx sigma) [Sec. 3.3]; 1D: dt/dx.
// Reading: sigma is taken from the state the Euler stage is applied to.
void stage_lambda(const Problem& P, const double* W, double dt, double lam[2]) {
  double a[2];
  max_wavespeed(P, W, a);
  if (P.ndim == 1) { lam[0] = dt / P.dx; lam[1] = 0.0; return; }
  double tx = a[0] / P.dx, ty = a[1] / P.dy;
  double sx = tx / (tx + ty), sy = ty / (tx + ty);
  lam[0] = dt / (P.dx * sx);
  lam[1] = dt / (P.dy * sy);
}

// Faces of one line: face k (k = 0..n) sits between cells k-1 and k.
// Gm[k], Gp[k] in the rotated frame; theta[k] optional.
void sweep_line(const Problem& P, const double* W, int dir, int line, double lam,
                std::vector<double>& Gm, std::vector<double>& Gp, double* theta_out) {
  Eos e = make_eos(P);
  const int n = dir == 0 ? P.nx : P.ny;
  // node quantities for cells -3 .. n+2 (3 ghost layers each side)
  std::vector<Node<double>> nodes(n + 6);
  for (int g = -3; g < n + 3; ++g) {
    double X[6];
    load_rotated(P, W, dir, line, g, X);
    nodes[g + 3] = node_from_w(e, X);
  }
  Gm.assign((size_t)(n + 1) * 6, 0.0);
  Gp.assign((size_t)(n + 1) * 6, 0.0);
  for (int k = 0; k <= n; ++k) {
    // stencil nodes k-3 .. k+2  ->  padded indices k .. k+5
    double th = face_flux(e, P, &nodes[k], lam, &Gm[(size_t)k * 6], &Gp[(size_t)k * 6]);
    if (theta_out) theta_out[k] = th;
  }
}

void rhs3(const Problem& P, const double* W, double* L, double dt);
// Semi-discrete RHS L(W) [Sec. 4.1, flux-difference form with G^{+-}].
void rhs(const Problem& P, const double* W, double* L, double dt) {
  if (P.ndim == 3) { rhs3(P, W, L, dt); return; }
  const int nv = nvar_of(P);
  const long ncell = (long)P.nx * P.ny;
  double lam[2];
  stage_lambda(P, W, dt, lam);
  std::vector<double> Lx((size_t)ncell * 6, 0.0);
  // Rows (and below, columns) are independent: the OpenMP build of this file
  // (the all-cores CPU baseline) splits them over threads, each writing its
  // own rows, so its results are those of the serial build bit for bit.
#pragma omp parallel for schedule(dynamic, 2)
  for (int j = 0; j < P.ny; ++j) {
    std::vector<double> Gm, Gp;
    sweep_line(P, W, 0, j, lam[0], Gm, Gp, nullptr);
    for (int i = 0; i < P.nx; ++i) {
      double Rm[6], Rp[6], Xm[6], Xp[6];
      for (int v = 0; v < 6; ++v) { Rm[v] = Gm[(size_t)(i + 1) * 6 + v]; Rp[v] = Gp[(size_t)i * 6 + v]; }
      unrotate(0, Rm, Xm); unrotate(0, Rp, Xp);
      for (int v = 0; v < 6; ++v) Lx[((size_t)j * P.nx + i) * 6 + v] = -(Xm[v] - Xp[v]) / P.dx;
    }
  }
  std::vector<double> Ly((size_t)ncell * 6, 0.0);
  if (P.ndim == 2) {
#pragma omp parallel for schedule(dynamic, 2)
    for (int i = 0; i < P.nx; ++i) {
      std::vector<double> Gm, Gp;
      sweep_line(P, W, 1, i, lam[1], Gm, Gp, nullptr);
      for (int j = 0; j < P.ny; ++j) {
        double Rm[6], Rp[6], Xm[6], Xp[6];
        for (int v = 0; v < 6; ++v) { Rm[v] = Gm[(size_t)(j + 1) * 6 + v]; Rp[v] = Gp[(size_t)j * 6 + v]; }
        unrotate(1, Rm, Xm); unrotate(1, Rp, Xp);
        for (int v = 0; v < 6; ++v) Ly[((size_t)j * P.nx + i) * 6 + v] = -(Xm[v] - Xp[v]) / P.dy;
      }
    }
  }
  for (long c = 0; c < ncell; ++c) {
    if (P.ndim == 1) {
      const int map[5] = {0, 1, 2, 4, 5};
      for (int v = 0; v < 5; ++v) L[(long)v * ncell + c] = Lx[(size_t)c * 6 + map[v]];
    } else {
      for (int v = 0; v < 6; ++v) L[(long)v * ncell + c] = Lx[(size_t)c * 6 + v] + Ly[(size_t)c * 6 + v];
    }
  }
  (void)nv;
}

// Same RHS restricted to a list of cells (for sampled comparisons on large
// grids).  Each cell evaluates its own faces from its own stencil.
void rhs_cells(const Problem& P, const double* W, double dt, const int64_t* cells, long nc,
               double* out) {
  Eos e = make_eos(P);
  const int nv = nvar_of(P);
  double lam[2];
  stage_lambda(P, W, dt, lam);
  for (long q = 0; q < nc; ++q) {
    const int i = (int)(cells[q] % P.nx), j = (int)(cells[q] / P.nx);
    double Lsum[6] = {0, 0, 0, 0, 0, 0};
    for (int dir = 0; dir < P.ndim; ++dir) {
      const int line = dir == 0 ? j : i, pos = dir == 0 ? i : j;
      Node<double> nodes[7];   // cells pos-3 .. pos+3
      for (int g = 0; g < 7; ++g) {
        double X[6];
        load_rotated(P, W, dir, line, pos - 3 + g, X);
        nodes[g] = node_from_w(e, X);
      }
      double Gm_lo[6], Gp_lo[6], Gm_hi[6], Gp_hi[6];
      face_flux(e, P, &nodes[0], lam[dir], Gm_lo, Gp_lo);  // face pos-1/2
      face_flux(e, P, &nodes[1], lam[dir], Gm_hi, Gp_hi);  // face pos+1/2
      double Xm[6], Xp[6];
      unrotate(dir, Gm_hi, Xm); unrotate(dir, Gp_lo, Xp);
      const double d = dir == 0 ? P.dx : P.dy;
      for (int v = 0; v < 6; ++v) {
        double part = -(Xm[v] - Xp[v]) / d;
        Lsum[v] = dir == 0 ? part : Lsum[v] + part;   // L = L_x + L_y, as in rhs()
      }
    }
    if (P.ndim == 1) {
      const int map[5] = {0, 1, 2, 4, 5};
      for (int v = 0; v < 5; ++v) out[q * nv + v] = Lsum[map[v]];
    } else {
      for (int v = 0; v < 6; ++v) out[q * nv + v] = Lsum[v];
    }
  }
}

// Admissible set G [Sec. 2]: 0 <= a1 <= 1, a_k r_k >= 0, rho e - pbar_inf > 0.
long count_inadmissible3(const Problem& P, const double* W);
long count_inadmissible(const Problem& P, const double* W) {
  if (P.ndim == 3) return count_inadmissible3(P, W);
  Eos e = make_eos(P);
  long bad = 0;
  for (int j = 0; j < P.ny; ++j)
    for (int i = 0; i < P.nx; ++i) {
      double X[6];
      load_cell(P, W, i, j, X);
      double h = rhoc2_tilde(e, X);
      bool ok = X[5] >= 0.0 && X[5] <= 1.0 && X[0] >= 0.0 && X[1] >= 0.0 && h > 0.0;
      if (!ok) ++bad;
    }
  return bad;
}

// ---------------------------------------------------------------------------
// Three dimensions (the direct extension of Sec. 2): W[7][nz][ny][nx] =
// (a1r1, a2r2, rho u, rho v, rho w, E, a1).  Rotated frames, with the two
// tangential momenta passive:
//   x: (m_n, m_t, m_s) = (rho u, rho v, rho w)
//   y: (rho v, rho u, rho w)
//   z: (rho w, rho u, rho v)
// A line in direction d is addressed by the two other cell indices (a, b):
// x (j, k), y (i, k), z (i, j).  Periodic, extrapolation and reflective
// sides only.
// ---------------------------------------------------------------------------
inline int len3(const Problem& P, int d) { return d == 0 ? P.nx : (d == 1 ? P.ny : P.nz); }
inline double h3(const Problem& P, int d) { return d == 0 ? P.dx : (d == 1 ? P.dy : P.dz); }
inline int bc3(const Problem& P, int side) { return side < 4 ? P.bc[side] : P.bcz[side - 4]; }
inline long cell3(const Problem& P, int i, int j, int k) {
  return ((long)k * P.ny + j) * P.nx + i;
}
inline long line_cell3(const Problem& P, int d, int a, int b, int pos) {
  return d == 0 ? cell3(P, pos, a, b) : (d == 1 ? cell3(P, a, pos, b) : cell3(P, a, b, pos));
}

inline void load_cell3(const Problem& P, const double* W, long o, double X[7]) {
  const long n = ncell_of(P);
  for (int v = 0; v < 7; ++v) X[v] = W[v * n + o];
}

// Node quantities of a cell for a sweep in direction d.  Reading (3D
// primitive recovery): the recovery runs once per cell on the unrotated
// state, so its kinetic energy is (rho u u + rho v v) + rho w w for every
// sweep (with three momenta the rotated order would round differently per
// direction); the velocities and momenta are then permuted into the
// direction's frame and the node flux formed there [Sec. 2; Sec. 3.2].
inline Node<double, 7> node_rotated3(const Eos& e, const double Y[7], int d) {
  Node<double, 7> c = node_from_w<7>(e, Y);   // x frame: un = u, ut = v, us = w
  Node<double, 7> n = c;
  const double vel[3] = {c.un, c.ut, c.us};
  n.w[0] = Y[0]; n.w[1] = Y[1]; n.w[5] = Y[5]; n.w[6] = Y[6];
  if (d == 0) return c;
  if (d == 1) {
    n.w[2] = Y[3]; n.w[3] = Y[2]; n.w[4] = Y[4];
    n.un = vel[1]; n.ut = vel[0]; n.us = vel[2];
  } else {
    n.w[2] = Y[4]; n.w[3] = Y[2]; n.w[4] = Y[3];
    n.un = vel[2]; n.ut = vel[0]; n.us = vel[1];
  }
  n.g[0] = n.w[0] * n.un;
  n.g[1] = n.w[1] * n.un;
  n.g[2] = n.w[2] * n.un + n.p;
  n.g[3] = n.w[3] * n.un;
  n.g[4] = n.w[4] * n.un;
  n.g[5] = (n.w[5] + n.p) * n.un;
  n.g[6] = n.w[6] * n.un;
  return n;
}

// the unrotated state of the (possibly ghost) node g of a line, reflective
// ghosts mirrored with the wall-normal momentum negated
inline void load_line3(const Problem& P, const double* W, int d, int a, int b, int g,
                       double Y[7]) {
  bool flip;
  int s = ghost_source(bc3(P, 2 * d), bc3(P, 2 * d + 1), g, len3(P, d), flip);
  load_cell3(P, W, line_cell3(P, d, a, b, s), Y);
  if (flip) Y[2 + d] = -Y[2 + d];
}

inline void unrotate3(int d, const double R[7], double X[7]) {
  X[0] = R[0]; X[1] = R[1]; X[5] = R[5]; X[6] = R[6];
  if (d == 0) { X[2] = R[2]; X[3] = R[3]; X[4] = R[4]; }
  else if (d == 1) { X[3] = R[2]; X[2] = R[3]; X[4] = R[4]; }
  else { X[4] = R[2]; X[2] = R[3]; X[3] = R[4]; }
}

// max(|u|+c), max(|v|+c), max(|w|+c) over the cells [Sec. 3.3]
void max_wavespeed3(const Problem& P, const double* W, double amax[3]) {
  Eos e = make_eos(P);
  amax[0] = amax[1] = amax[2] = 0.0;
  const long n = ncell_of(P);
  for (long o = 0; o < n; ++o) {
    double X[7];
    load_cell3(P, W, o, X);
    Node<double, 7> nd = node_from_w<7>(e, X);   // x frame: un = u, ut = v, us = w
    amax[0] = std::max(amax[0], std::fabs(nd.un) + nd.c);
    amax[1] = std::max(amax[1], std::fabs(nd.ut) + nd.c);
    amax[2] = std::max(amax[2], std::fabs(nd.us) + nd.c);
  }
}

// Reading (3D split of Sec. 3.3): sigma_d = tau_d/(tau_x + tau_y + tau_z),
// tau_d = max(|u_d|+c)/h_d, lambda_d = dt/(h_d sigma_d).
void stage_lambda3(const Problem& P, const double* W, double dt, double lam[3]) {
  double a[3];
  max_wavespeed3(P, W, a);
  double t[3] = {a[0] / P.dx, a[1] / P.dy, a[2] / P.dz};
  double tot = t[0] + t[1] + t[2];
  for (int d = 0; d < 3; ++d) lam[d] = dt / (h3(P, d) * (t[d] / tot));
}

double cfl_dt3(const Problem& P, const double* W) {
  double a[3];
  max_wavespeed3(P, W, a);
  return P.cfl / (a[0] / P.dx + a[1] / P.dy + a[2] / P.dz);
}

void sweep_line3(const Problem& P, const double* W, int d, int a, int b, double lam,
                 std::vector<double>& Gm, std::vector<double>& Gp, double* theta_out) {
  Eos e = make_eos(P);
  const int n = len3(P, d);
  std::vector<Node<double, 7>> nodes(n + 6);
  for (int g = -3; g < n + 3; ++g) {
    double Y[7];
    load_line3(P, W, d, a, b, g, Y);
    nodes[g + 3] = node_rotated3(e, Y, d);
  }
  Gm.assign((size_t)(n + 1) * 7, 0.0);
  Gp.assign((size_t)(n + 1) * 7, 0.0);
  for (int f = 0; f <= n; ++f) {
    double th = face_flux(e, P, &nodes[f], lam, &Gm[(size_t)f * 7], &Gp[(size_t)f * 7]);
    if (theta_out) theta_out[f] = th;
  }
}

// L = (L_x + L_y) + L_z, each -(G^-_{i+1/2} - G^+_{i-1/2})/h  [Sec. 4.1]
void rhs3(const Problem& P, const double* W, double* L, double dt) {
  const long n = ncell_of(P);
  double lam[3];
  stage_lambda3(P, W, dt, lam);
  std::vector<double> Ld[3];
  for (int d = 0; d < 3; ++d) {
    Ld[d].assign((size_t)n * 7, 0.0);
    const int na = d == 0 ? P.ny : P.nx, nb = d == 2 ? P.ny : P.nz;
    // Lines are independent (each cell lies on one line per direction): the
    // OpenMP build splits them over threads, the same bits as the serial one.
#pragma omp parallel for schedule(dynamic, 4)
    for (long l = 0; l < (long)na * nb; ++l) {
      const int b = (int)(l / na), a = (int)(l % na);
      std::vector<double> Gm, Gp;
      sweep_line3(P, W, d, a, b, lam[d], Gm, Gp, nullptr);
      for (int pos = 0; pos < len3(P, d); ++pos) {
        double Xm[7], Xp[7];
        unrotate3(d, &Gm[(size_t)(pos + 1) * 7], Xm);
        unrotate3(d, &Gp[(size_t)pos * 7], Xp);
        const long o = line_cell3(P, d, a, b, pos);
        for (int v = 0; v < 7; ++v) Ld[d][(size_t)o * 7 + v] = -(Xm[v] - Xp[v]) / h3(P, d);
      }
    }
  }
  for (long o = 0; o < n; ++o)
    for (int v = 0; v < 7; ++v)
      L[(long)v * n + o] = Ld[0][(size_t)o * 7 + v] + Ld[1][(size_t)o * 7 + v] +
                           Ld[2][(size_t)o * 7 + v];
}

// the same RHS on a list of cells, each from its own stencils
void rhs_cells3(const Problem& P, const double* W, double dt, const int64_t* cells, long nc,
                double* out) {
  Eos e = make_eos(P);
  double lam[3];
  stage_lambda3(P, W, dt, lam);
  for (long q = 0; q < nc; ++q) {
    const int i = (int)(cells[q] % P.nx), j = (int)((cells[q] / P.nx) % P.ny);
    const int k = (int)(cells[q] / ((long)P.nx * P.ny));
    double Lsum[7];
    for (int d = 0; d < 3; ++d) {
      const int a = d == 0 ? j : i, b = d == 2 ? j : k, pos = d == 0 ? i : (d == 1 ? j : k);
      Node<double, 7> nodes[7];
      for (int g = 0; g < 7; ++g) {
        double Y[7];
        load_line3(P, W, d, a, b, pos - 3 + g, Y);
        nodes[g] = node_rotated3(e, Y, d);
      }
      double Gm_lo[7], Gp_lo[7], Gm_hi[7], Gp_hi[7], Xm[7], Xp[7];
      face_flux(e, P, &nodes[0], lam[d], Gm_lo, Gp_lo);
      face_flux(e, P, &nodes[1], lam[d], Gm_hi, Gp_hi);
      unrotate3(d, Gm_hi, Xm);
      unrotate3(d, Gp_lo, Xp);
      for (int v = 0; v < 7; ++v) {
        double part = -(Xm[v] - Xp[v]) / h3(P, d);
        Lsum[v] = d == 0 ? part : Lsum[v] + part;
      }
    }
    for (int v = 0; v < 7; ++v) out[q * 7 + v] = Lsum[v];
  }
}

long count_inadmissible3(const Problem& P, const double* W) {
  Eos e = make_eos(P);
  long bad = 0;
  const long n = ncell_of(P);
  for (long o = 0; o < n; ++o) {
    double X[7];
    load_cell3(P, W, o, X);
    double h = rhoc2_tilde<7>(e, X);
    bool ok = X[6] >= 0.0 && X[6] <= 1.0 && X[0] >= 0.0 && X[1] >= 0.0 && h > 0.0;
    if (!ok) ++bad;
  }
  return bad;
}

// Three-stage SSP Runge-Kutta (TVD-RK3, Shu-Osher form) [Sec. 5.3, Sec. 6].
// Returns the number of inadmissible cells seen after any stage.
long ssprk3_step(const Problem& P, double* W, double dt) {
  const long n = (long)nvar_of(P) * ncell_of(P);
  std::vector<double> W0(W, W + n), W1(n), L(n);
  long bad = 0;
  rhs(P, W, L.data(), dt);
  for (long q = 0; q < n; ++q) W1[q] = W0[q] + dt * L[q];
  bad += count_inadmissible(P, W1.data());
  rhs(P, W1.data(), L.data(), dt);
  for (long q = 0; q < n; ++q) W1[q] = 0.75 * W0[q] + 0.25 * (W1[q] + dt * L[q]);
  bad += count_inadmissible(P, W1.data());
  rhs(P, W1.data(), L.data(), dt);
  for (long q = 0; q < n; ++q) W[q] = (1.0 / 3.0) * W0[q] + (2.0 / 3.0) * (W1[q] + dt * L[q]);
  bad += count_inadmissible(P, W);
  return bad;
}

// CFL time step from the state at the start of the step [Sec. 3.3]:
// dt = CFL/(tau_x + tau_y), tau = max(|u|+c)/dx.
double cfl_dt(const Problem& P, const double* W) {
  if (P.ndim == 3) return cfl_dt3(P, W);
  double a[2];
  max_wavespeed(P, W, a);
  if (P.ndim == 1) return P.cfl * P.dx / a[0];
  return P.cfl / (a[0] / P.dx + a[1] / P.dy);
}

bool eos_valid(const Problem& P) {
  // Lemma 1 / Theorem 1: exactly one ideal-gas phase (pinf = 0), the other
  // phase's gamma must be at least the gas gamma; all gamma > 1, pinf >= 0.
  if (!(P.gamma[0] > 1.0 && P.gamma[1] > 1.0)) return false;
  if (P.pinf[0] < 0.0 || P.pinf[1] < 0.0) return false;
  if (P.pinf[1] == 0.0) return P.gamma[0] >= P.gamma[1];
  if (P.pinf[0] == 0.0) return P.gamma[1] >= P.gamma[0];
  return false;
}

}  // namespace

// ============================================================================
// C entry points (ctypes).  Return codes: 0 ok, -1 bad argument, -2 EOS
// violates Lemma 1, -5 inadmissible state encountered.
// ============================================================================
extern "C" {

int oracle_eos_valid(const Problem* P) { return eos_valid(*P) ? 1 : 0; }

// primitive (a1r1, a2r2, u, [v, [w,]] p, a1) -> conservative, SoA [nv][n]
int oracle_prim_to_cons(const Problem* P, const double* V, double* W, long n) {
  Eos e = make_eos(*P);
  const int nv = nvar_of(*P);
  for (long q = 0; q < n; ++q) {
    double a1r1 = V[0 * n + q], a2r2 = V[1 * n + q], u = V[2 * n + q];
    double v = nv >= 6 ? V[3 * n + q] : 0.0;
    double w = nv == 7 ? V[4 * n + q] : 0.0;
    double p = V[(nv - 2) * n + q], a1 = V[(nv - 1) * n + q];
    double rho = a1r1 + a2r2;
    W[0 * n + q] = a1r1;
    W[1 * n + q] = a2r2;
    W[2 * n + q] = rho * u;
    if (nv >= 6) W[3 * n + q] = rho * v;
    if (nv == 7) W[4 * n + q] = rho * w;
    double ke = u * u + v * v;
    if (nv == 7) ke = ke + w * w;
    W[(nv - 2) * n + q] = mix_Gamma(e, a1) * p + mix_Pi(e, a1) + 0.5 * rho * ke;
    W[(nv - 1) * n + q] = a1;
  }
  return 0;
}

// conservative -> primitive (a1r1, a2r2, u, [v, [w,]] p, a1) plus c, SoA
int oracle_cons_to_prim(const Problem* P, const double* W, double* V, double* c, long n) {
  Eos e = make_eos(*P);
  const int nv = nvar_of(*P);
  if (nv == 7) {
    for (long q = 0; q < n; ++q) {
      double X[7];
      for (int v = 0; v < 7; ++v) X[v] = W[v * n + q];
      Node<double, 7> nd = node_from_w<7>(e, X);
      V[0 * n + q] = X[0]; V[1 * n + q] = X[1];
      V[2 * n + q] = nd.un; V[3 * n + q] = nd.ut; V[4 * n + q] = nd.us;
      V[5 * n + q] = nd.p; V[6 * n + q] = X[6];
      if (c) c[q] = nd.c;
    }
    return 0;
  }
  for (long q = 0; q < n; ++q) {
    double X[6];
    X[0] = W[0 * n + q]; X[1] = W[1 * n + q]; X[2] = W[2 * n + q];
    X[3] = nv == 6 ? W[3 * n + q] : 0.0;
    X[4] = W[(nv - 2) * n + q]; X[5] = W[(nv - 1) * n + q];
    Node<double> nd = node_from_w(e, X);
    V[0 * n + q] = X[0]; V[1 * n + q] = X[1]; V[2 * n + q] = nd.un;
    if (nv == 6) V[3 * n + q] = nd.ut;
    V[(nv - 2) * n + q] = nd.p; V[(nv - 1) * n + q] = X[5];
    if (c) c[q] = nd.c;
  }
  return 0;
}

// grid checks shared by the entry points: sizes, and no Dirichlet side in 3D
static bool grid_ok(const Problem* P) {
  if (P->nx < 1 || P->ny < 1 || (P->ndim == 3 && P->nz < 1)) return false;
  if (P->ndim == 3)
    for (int s = 0; s < 6; ++s)
      if (bc3(*P, s) == BC_DIRICHLET) return false;
  return true;
}

int oracle_rhs(const Problem* P, const double* W, double* L, double dt) {
  if (!eos_valid(*P)) return -2;
  if (!grid_ok(P)) return -1;
  rhs(*P, W, L, dt);
  return 0;
}

int oracle_rhs_cells(const Problem* P, const double* W, double dt, const int64_t* cells,
                     long nc, double* out) {
  if (!eos_valid(*P)) return -2;
  if (!grid_ok(P)) return -1;
  if (P->ndim == 3) rhs_cells3(*P, W, dt, cells, nc, out);
  else rhs_cells(*P, W, dt, cells, nc, out);
  return 0;
}

// Flux of every face of every line in one direction, before (ho) and after
// limiting, plus theta: arrays [nline][n+1][6] in the rotated frame.
int oracle_faces(const Problem* P, const double* W, int dir, double dt, double* Gm, double* Gp,
                 double* theta) {
  if (!eos_valid(*P)) return -2;
  if (!grid_ok(P)) return -1;
  if (P->ndim == 3) {
    // lines ordered by (b, a): x (k, j), y (k, i), z (j, i); [nline][n+1][7]
    double lam3[3];
    stage_lambda3(*P, W, dt, lam3);
    const int n = len3(*P, dir);
    const int na = dir == 0 ? P->ny : P->nx, nb = dir == 2 ? P->ny : P->nz;
    std::vector<double> gm, gp;
    for (int b = 0; b < nb; ++b)
      for (int a = 0; a < na; ++a) {
        const long l = (long)b * na + a;
        sweep_line3(*P, W, dir, a, b, lam3[dir], gm, gp, theta ? theta + l * (n + 1) : nullptr);
        std::memcpy(Gm + l * (n + 1) * 7, gm.data(), sizeof(double) * (n + 1) * 7);
        std::memcpy(Gp + l * (n + 1) * 7, gp.data(), sizeof(double) * (n + 1) * 7);
      }
    return 0;
  }
  double lam[2];
  stage_lambda(*P, W, dt, lam);
  const int nline = dir == 0 ? P->ny : P->nx;
  const int n = dir == 0 ? P->nx : P->ny;
  std::vector<double> gm, gp;
  for (int l = 0; l < nline; ++l) {
    sweep_line(*P, W, dir, l, lam[dir], gm, gp, theta ? theta + (long)l * (n + 1) : nullptr);
    std::memcpy(Gm + (long)l * (n + 1) * 6, gm.data(), sizeof(double) * (n + 1) * 6);
    std::memcpy(Gp + (long)l * (n + 1) * 6, gp.data(), sizeof(double) * (n + 1) * 6);
  }
  return 0;
}

// Stand-alone flux limiter on one face [Algorithms 4-6], rotated frame,
// 6-component states: used to pin the limiter in isolation.
double oracle_flux_limit_face(const Problem* P, const double* Wl, const double* Wr,
                              double lam, const double* Hm, const double* Hp, double* Gm,
                              double* Gp) {
  Eos e = make_eos(*P);
  Node<double> nl = node_from_w(e, Wl), nr = node_from_w(e, Wr);
  double Fl[6] = {nl.g[0], nl.g[1], nl.g[2], nl.g[3], nl.g[4], 0.0};
  double Fr[6] = {nr.g[0], nr.g[1], nr.g[2], nr.g[3], nr.g[4], 0.0};
  return flux_limit(e, *P, Wl, Wr, Fl, Fr, lam, Hm, Hp, Gm, Gp);
}

void oracle_interp_limit(const Problem* P, const double* A, double* B) {
  Eos e = make_eos(*P);
  interp_limit(e, *P, A, B);
}

double oracle_weno_is(double a, double b, double c, double d, double e, double eps) {
  return weno_is<double>(a, b, c, d, e, eps);
}

double oracle_hcs(double gt, double gm2, double gm1, double g0, double gp1, double gp2,
                  double gp3) {
  return hcs<double>(gt, gm2, gm1, g0, gp1, gp2, gp3);
}

// HLLC on two rotated 6-states: F[5], f_alpha, s*, and the two star states
void oracle_hllc(const Problem* P, const double* WL, const double* WR, double* F,
                 double* falpha, double* sstar) {
  Eos e = make_eos(*P);
  Node<double> L = node_from_w(e, WL), R = node_from_w(e, WR);
  hllc(L, R, F, *falpha, *sstar);
}

// node quantities of a rotated 6-state: rho, un, ut, p, c, h
void oracle_node(const Problem* P, const double* X, double* out6) {
  Eos e = make_eos(*P);
  Node<double> n = node_from_w(e, X);
  out6[0] = n.rho; out6[1] = n.un; out6[2] = n.ut; out6[3] = n.p; out6[4] = n.c; out6[5] = n.h;
}

double oracle_rhoc2_tilde(const Problem* P, const double* X) {
  Eos e = make_eos(*P);
  return rhoc2_tilde(e, X);
}

// projection with the face averages of nodes (L, R): U = R^{-1} V(X), and the
// back-projection of U to a conservative state
void oracle_project(const Problem* P, const double* XL, const double* XR, const double* X,
                    double* U) {
  Eos e = make_eos(*P);
  Node<double> L = node_from_w(e, XL), R = node_from_w(e, XR), N = node_from_w(e, X);
  FaceAvg<double> f = face_avg(L, R);
  project(f, N, U);
}
void oracle_back_project(const Problem* P, const double* XL, const double* XR, const double* U,
                         double* X) {
  Eos e = make_eos(*P);
  Node<double> L = node_from_w(e, XL), R = node_from_w(e, XR);
  FaceAvg<double> f = face_avg(L, R);
  back_project_to_w(e, f, U, X);
}

// amax: 2 values (1D/2D) or 3 (3D)
void oracle_max_wavespeed(const Problem* P, const double* W, double* amax) {
  if (P->ndim == 3) max_wavespeed3(*P, W, amax);
  else max_wavespeed(*P, W, amax);
}

void oracle_stage_lambda(const Problem* P, const double* W, double dt, double* lam) {
  if (P->ndim == 3) stage_lambda3(*P, W, dt, lam);
  else stage_lambda(*P, W, dt, lam);
}

long oracle_count_inadmissible(const Problem* P, const double* W) {
  return count_inadmissible(*P, W);
}

double oracle_cfl_dt(const Problem* P, const double* W) { return cfl_dt(*P, W); }

// One SSP-RK3 step; dt <= 0 selects the CFL time step. Returns the number of
// inadmissible cells seen after any stage (0 expected); *dt_used receives dt.
long oracle_ssprk3_step(const Problem* P, double* W, double dt, double* dt_used) {
  if (!grid_ok(P)) return -1;
  if (dt <= 0.0) dt = cfl_dt(*P, W);
  if (dt_used) *dt_used = dt;
  return ssprk3_step(*P, W, dt);
}

// Run to t_end.  dt_fixed > 0: constant step (the last one clipped to hit
// t_end); otherwise CFL steps.  Returns steps taken, or -5 if any stage left
// an inadmissible cell (the state at that point is returned in W).
long oracle_run(const Problem* P, double* W, double t_end, double dt_fixed, long max_steps,
                double* t_out) {
  if (!eos_valid(*P)) return -2;
  if (!grid_ok(P)) return -1;
  double t = 0.0;
  long steps = 0;
  while (t < t_end && steps < max_steps) {
    double dt = dt_fixed > 0.0 ? dt_fixed : cfl_dt(*P, W);
    // Reading: the last step is shortened to land on t_end
    if (t + dt > t_end) dt = t_end - t;
    long bad = ssprk3_step(*P, W, dt);
    t += dt;
    ++steps;
    if (bad) { if (t_out) *t_out = t; return -5; }
  }
  if (t_out) *t_out = t;
  return steps;
}

// Algorithmic operation counts of one face of a given stencil (rotated frame,
// 6 nodes x 6 components), split into the per-node part (one node: primitive
// recovery, sound speed, node flux) and the per-face part (everything else).
// out: [node add, mul, div, sqrt, cmp, face add, mul, div, sqrt, cmp]
void oracle_opcount_face(const Problem* P, const double* stencil /* [6][6] */, double lam,
                         long long* out) {
  Eos e = make_eos(*P);
  Node<Cnt> nd[6];
  g_ops = OpCounts{0, 0, 0, 0, 0};
  for (int m = 0; m < 6; ++m) {
    Cnt X[6];
    for (int v = 0; v < 6; ++v) X[v] = Cnt(stencil[m * 6 + v]);
    nd[m] = node_from_w(e, X);
  }
  OpCounts six = g_ops;
  g_ops = OpCounts{0, 0, 0, 0, 0};
  for (int k = 0; k < NPHASE; ++k) g_phase_ops[k] = OpCounts{0, 0, 0, 0, 0};
  Cnt Gm[6], Gp[6];
  face_flux(e, *P, nd, Cnt(lam), Gm, Gp);
  OpCounts f = g_ops;
  g_phase = 0;
  out[0] = six.add / 6; out[1] = six.mul / 6; out[2] = six.div / 6;
  out[3] = six.sqrt / 6; out[4] = six.cmp / 6;
  out[5] = f.add; out[6] = f.mul; out[7] = f.div; out[8] = f.sqrt; out[9] = f.cmp;
}

// The face part of the last oracle_opcount_face by step of the pipeline:
// out[5 k .. 5 k + 4] = (add, mul, div, sqrt, cmp) of phase k < NPHASE
// (the PH_ order above); returns NPHASE.
int oracle_opcount_phases(long long* out) {
  for (int k = 0; k < NPHASE; ++k) {
    const OpCounts& c = g_phase_ops[k];
    out[5 * k] = c.add; out[5 * k + 1] = c.mul; out[5 * k + 2] = c.div;
    out[5 * k + 3] = c.sqrt; out[5 * k + 4] = c.cmp;
  }
  return NPHASE;
}

// The same for a 3D face (rotated frame, 6 nodes x 7 components).
void oracle_opcount_face3(const Problem* P, const double* stencil /* [6][7] */, double lam,
                          long long* out) {
  Eos e = make_eos(*P);
  Node<Cnt, 7> nd[6];
  g_ops = OpCounts{0, 0, 0, 0, 0};
  for (int m = 0; m < 6; ++m) {
    Cnt X[7];
    for (int v = 0; v < 7; ++v) X[v] = Cnt(stencil[m * 7 + v]);
    nd[m] = node_from_w<7>(e, X);
  }
  OpCounts six = g_ops;
  g_ops = OpCounts{0, 0, 0, 0, 0};
  Cnt Gm[7], Gp[7];
  face_flux(e, *P, nd, Cnt(lam), Gm, Gp);
  OpCounts f = g_ops;
  out[0] = six.add / 6; out[1] = six.mul / 6; out[2] = six.div / 6;
  out[3] = six.sqrt / 6; out[4] = six.cmp / 6;
  out[5] = f.add; out[6] = f.mul; out[7] = f.div; out[8] = f.sqrt; out[9] = f.cmp;
}

}  // extern "C"
