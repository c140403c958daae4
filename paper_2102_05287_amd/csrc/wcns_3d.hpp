// Three-dimensional form of the PP-WCNS-IS right-hand side: the direct
// extension of Sec. 2 (a third momentum component, a z-sweep), with every
// step of the 2D pipeline unchanged per face.
//
// State [7][nz][ny][nx] = (a1r1, a2r2, rho u, rho v, rho w, E, a1).  Node
// primitives P [6][nz][ny][nx] = (u, v, w, p, c, rho ctilde^2) are recovered
// once per cell in the unrotated frame, kinetic energy (rho u u + rho v v) +
// rho w w.  Rotated frames (normal, tangential, second tangential momentum):
//   x (rho u, rho v, rho w), y (rho v, rho u, rho w), z (rho w, rho u, rho v).
// The two tangential momenta are passive components of the characteristic
// projection (App. A extended by one field), of HLLC and of the limiters.
//
//   k3_node      primitives + block maxima of |u|+c, |v|+c, |w|+c
//   k3_finalize  dt and the three-way split sigma, lambda (Sec. 3.3)
//   k3_sweep_xl  x pass, one wave per flattened tile of 62 cells with its
//                stencil window in LDS: L_x (k3_sweep_x, global loads, for
//                rows narrower than 61 cells)
//   k3_sweep_l   y-lines (per z slab) or z-lines: one block over 32
//                consecutive columns x 16 face rows (8 waves), stencil rows
//                staged in LDS; the y pass adds L_y to L in place, the z
//                pass finishes L = (L_x + L_y) + L_z and applies the SSP-RK3
//                stage combination
//   k3_fixup     the cell rows between two tiles of a strided pass
#pragma once
#include "wcns_kernels.hpp"

#pragma clang fp contract(off)

namespace wcns {

// Strided-pass tiles: 32 columns x 16 face rows (8 waves, 59 KB of LDS, two
// blocks per CU; against 8-row tiles the passes run ~1% slower but the
// fixups have half the rows: 1.008x per RHS at 256^3).
constexpr int YW3 = 16;   // face rows per tile
constexpr int L3_THREADS = 32 * YW3;   // 8 waves: each covers two face rows

struct K3Args {
  int32_t nx, ny, nz, tile_x;
  double dx, dy, dz;
  double rdx, rdy, rdz;       // checked reciprocals of the spacings (0: divide)
  int32_t bc[6];              // x-lo, x-hi, y-lo, y-hi, z-lo, z-hi
  int32_t interp_limiter, flux_limiter, scheme, out_mode;
  int32_t nbr, last;          // strided pass: tile rows; 1 when it finishes the cell
  EosC eos;
  Tol tol;
  const double* W;            // state differentiated [7][N]
  const double* Wc[7];        // its component bases
  const double* Pc[6];        // node primitives u, v, w, p, c, h
  const double* step;         // [0] dt, [1..3] lambda, [4..6] maxima
  const double* Lin;          // L accumulated so far (strided passes)
  double* Lout;               // x pass: L_x
  double* out;                // y pass: L_x + L_y; z pass: L or next stage
  const double* Un;           // state at the start of the step
  double* edge;               // strided-pass tile edges [nslab][nbr][14][ncol]
  double ca, cb;              // RK: out = ca*Un + cb*(W + dt*L)
  // lazy admissibility report, as in KArgs: stage results (and k3_node's
  // input with check_in) outside G counted into *viol, flag *vflag raised;
  // node_skip: a k3_node launch inside a step (returns when it is skipped)
  unsigned long long* viol;
  int32_t* vflag;
  int32_t check_in, node_skip;
};

struct NodeQ3 {
  double w[7];
  double un, ut, us, p, c, h;
};

// Primitive recovery of a state in the given frame [Sec. 2]
__device__ __forceinline__ void recover3(const EosC& e, const double X[7], double& un,
                                         double& ut, double& us, double& p, double& c,
                                         double& h) {
  double rho = X[0] + X[1];
  double irho = ddiv(1.0, rho);
  un = X[2] * irho;
  ut = X[3] * irho;
  us = X[4] * irho;
  double ke = X[2] * un + X[3] * ut;
  ke = ke + X[4] * us;
  double rhoe = X[5] - 0.5 * ke;
  double Gam = mix_gamma(e, X[6]);
  double Pi = mix_pi(e, X[6]);
  p = ddiv(rhoe - Pi, Gam);
  double pinf_bar = ddiv(Pi, 1.0 + Gam);
  double gbar = 1.0 + ddiv(1.0, Gam);
  double c2 = gbar * (p + pinf_bar) * irho;
  c = sqrt(c2);
  h = rhoe - pinf_bar;
}

__device__ __forceinline__ double rhoc2_tilde3(const EosC& e, const double X[7]) {
  double rho = X[0] + X[1];
  double irho = ddiv(1.0, rho);
  double un = X[2] * irho;
  double ut = X[3] * irho;
  double ke = X[2] * un + X[3] * ut;
  ke = ke + X[4] * (X[4] * irho);
  double rhoe = X[5] - 0.5 * ke;
  double Gam = mix_gamma(e, X[6]);
  double Pi = mix_pi(e, X[6]);
  return rhoe - ddiv(Pi, 1.0 + Gam);
}

// node flux G = F + (0,...,0, a1 u_n) [Sec. 3.2]
__device__ __forceinline__ void node_flux3(const NodeQ3& n, double g[7]) {
  g[0] = n.w[0] * n.un;
  g[1] = n.w[1] * n.un;
  g[2] = n.w[2] * n.un + n.p;
  g[3] = n.w[3] * n.un;
  g[4] = n.w[4] * n.un;
  g[5] = (n.w[5] + n.p) * n.un;
  g[6] = n.w[6] * n.un;
}

struct HllcOut3 {
  double F[6];
  double fa, ss;
};

// HLLC [Sec. 3.1 star states, Einfeldt speeds, Batten contact speed; Sec. 3.2]
__device__ __forceinline__ void hllc3(const NodeQ3& L, const NodeQ3& R, HllcOut3& o) {
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
  double sg = (ss > 0.0) ? 1.0 : ((ss < 0.0) ? -1.0 : 0.0);
  double wl = (1.0 + sg) * 0.5;
  double wr = (1.0 - sg) * 0.5;
  double fl[6], fr[6];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const NodeQ3& K = side == 0 ? L : R;
    const double sK = side == 0 ? sL : sR;
    const double rhoK = side == 0 ? rhoL : rhoR;
    const double sE = side == 0 ? sm : sp;
    double chi = ddiv(sK - K.un, sK - ss);
    double g[7];
    node_flux3(K, g);
    double ws[6];
    ws[0] = chi * K.w[0];
    ws[1] = chi * K.w[1];
    ws[2] = chi * rhoK * ss;
    ws[3] = chi * rhoK * K.ut;
    ws[4] = chi * rhoK * K.us;
    ws[5] = chi * (K.w[5] + (ss - K.un) * (rhoK * ss + ddiv(K.p, sK - K.un)));
    double* f = side == 0 ? fl : fr;
#pragma unroll
    for (int v = 0; v < 6; ++v) f[v] = g[v] + sE * (ws[v] - K.w[v]);
  }
#pragma unroll
  for (int v = 0; v < 6; ++v) o.F[v] = wl * fl[v] + wr * fr[v];
  o.fa = wl * (L.w[6] * ss) + wr * (R.w[6] * ss);
}

// limiter test functions: 0 a1r1, 1 a2r2, 2 a1, 3 1-a1, 4 rho*ctilde^2
__device__ __forceinline__ double test_fn3(const EosC& e, int k, const double X[7]) {
  switch (k) {
    case 0: return X[0];
    case 1: return X[1];
    case 2: return X[6];
    case 3: return 1.0 - X[6];
    default: return rhoc2_tilde3(e, X);
  }
}

// Interpolation limiter, Algorithms 1-3 and the hard switch [Sec. 5.1]
__device__ __forceinline__ void interp_limit3(const EosC& e, const Tol& t, const double A[7],
                                              double hA, double B[7]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double qA = test_fn3(e, k, A);
    double eps = tol_of(t, k);
    double qB = test_fn3(e, k, B);
    if (qA < eps) {
#pragma unroll
      for (int v = 0; v < 7; ++v) B[v] = A[v];
    } else if (qB < eps) {
      double th = ddiv(qA - eps, qA - qB);
#pragma unroll
      for (int v = 0; v < 7; ++v) B[v] = (1.0 - th) * A[v] + th * B[v];
    }
  }
  double hB = rhoc2_tilde3(e, B);
  if (hA < t.eps_rhoc2) {
#pragma unroll
    for (int v = 0; v < 7; ++v) B[v] = A[v];
    hB = hA;
  } else if (hB < t.eps_rhoc2) {
    double th = ddiv(hA - t.eps_rhoc2, hA - hB);
#pragma unroll
    for (int v = 0; v < 7; ++v) B[v] = (1.0 - th) * A[v] + th * B[v];
    hB = rhoc2_tilde3(e, B);
  }
  bool fail = B[0] < t.hs_arho || B[1] < t.hs_arho || B[6] < t.hs_alpha ||
              1.0 - B[6] < t.hs_alpha || hB < t.hs_rhoc2;
  if (fail) {
#pragma unroll
    for (int v = 0; v < 7; ++v) B[v] = A[v];
  }
}

// Flux limiter, Algorithms 4-6 and the hard switch [Sec. 5.2]
__device__ __forceinline__ double flux_limit3(const EosC& e, const Tol& t, const double Wl[7],
                                              const double Wr[7], const double Fl[7],
                                              const double Fr[7], double lam,
                                              const double Hm[7], const double Hp[7],
                                              double Gm[7], double Gp[7]) {
  double thmin = 1.0;
  double hPG = 0.0, hMG = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double eps = tol_of(t, k);
    double qPH, qPG, qMH, qMG;
    if (k < 4) {
      const int v = k == 0 ? 0 : (k == 1 ? 1 : 6);
      qPH = half_state(0, Wl[v], lam, Hm[v], Fl[v]);
      qPG = half_state(0, Wl[v], lam, Gm[v], Fl[v]);
      qMH = half_state(1, Wr[v], lam, Hp[v], Fr[v]);
      qMG = half_state(1, Wr[v], lam, Gp[v], Fr[v]);
      if (k == 3) { qPH = 1.0 - qPH; qPG = 1.0 - qPG; qMH = 1.0 - qMH; qMG = 1.0 - qMG; }
    } else {
      double X[7];
#pragma unroll
      for (int v = 0; v < 7; ++v) X[v] = half_state(0, Wl[v], lam, Hm[v], Fl[v]);
      qPH = rhoc2_tilde3(e, X);
#pragma unroll
      for (int v = 0; v < 7; ++v) X[v] = half_state(0, Wl[v], lam, Gm[v], Fl[v]);
      qPG = rhoc2_tilde3(e, X);
#pragma unroll
      for (int v = 0; v < 7; ++v) X[v] = half_state(1, Wr[v], lam, Hp[v], Fr[v]);
      qMH = rhoc2_tilde3(e, X);
#pragma unroll
      for (int v = 0; v < 7; ++v) X[v] = half_state(1, Wr[v], lam, Gp[v], Fr[v]);
      qMG = rhoc2_tilde3(e, X);
      hPG = qPG;
      hMG = qMG;
    }
    double thp = limiter_theta(qPH, qPG, eps);
    double thm = limiter_theta(qMH, qMG, eps);
    double th = (thm < thp) ? thm : thp;
    if (th != 1.0) {
#pragma unroll
      for (int v = 0; v < 7; ++v) {
        Gp[v] = (1.0 - th) * Hp[v] + th * Gp[v];
        Gm[v] = (1.0 - th) * Hm[v] + th * Gm[v];
      }
      thmin = (th < thmin) ? th : thmin;
      if (k == 4) {
        double X[7];
#pragma unroll
        for (int v = 0; v < 7; ++v) X[v] = half_state(0, Wl[v], lam, Gm[v], Fl[v]);
        hPG = rhoc2_tilde3(e, X);
#pragma unroll
        for (int v = 0; v < 7; ++v) X[v] = half_state(1, Wr[v], lam, Gp[v], Fr[v]);
        hMG = rhoc2_tilde3(e, X);
      }
    }
  }
  bool fail = false;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const double* Wx = side == 0 ? Wl : Wr;
    const double* Fx = side == 0 ? Fl : Fr;
    const double* Gx = side == 0 ? Gm : Gp;
    double x0 = half_state(side, Wx[0], lam, Gx[0], Fx[0]);
    double x1 = half_state(side, Wx[1], lam, Gx[1], Fx[1]);
    double x6 = half_state(side, Wx[6], lam, Gx[6], Fx[6]);
    double hx = side == 0 ? hPG : hMG;
    fail = fail || x0 < t.hs_arho || x1 < t.hs_arho || x6 < t.hs_alpha || 1.0 - x6 < t.hs_alpha ||
           hx < t.hs_rhoc2;
  }
  if (fail) {
#pragma unroll
    for (int v = 0; v < 7; ++v) { Gm[v] = Hm[v]; Gp[v] = Hp[v]; }
    thmin = 0.0;
  }
  return thmin;
}

// ------------------------------------------------------------------ stencils
// Byte offsets of the 6 nodes of a face (after ghost mapping) along a line
// whose cell pos sits at base + pos*stride, and the reflective-ghost mask.
struct Sten3 {
  uint32_t off[6];
  uint32_t flip;
};

__device__ __forceinline__ Sten3 make_sten3(int g0, int n, int bc_lo, int bc_hi, long base,
                                            long stride) {
  Sten3 st;
  st.flip = 0;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    bool flip;
    int s = ghost_src(g0 + m, n, bc_lo, bc_hi, flip);
    if (flip) st.flip |= 1u << m;
    st.off[m] = (uint32_t)(base + (long)s * stride) * 8u;
  }
  return st;
}

// node m of a stencil in the frame of direction DIR
template <int DIR>
__device__ __forceinline__ void load_node3(const K3Args& a, const Sten3& st, int m, NodeQ3& q) {
  const uint32_t o = st.off[m];
  double Y[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) Y[k] = ldc(a.Wc[k], o);
  const double u = ldc(a.Pc[0], o), v = ldc(a.Pc[1], o), w = ldc(a.Pc[2], o);
  q.p = ldc(a.Pc[3], o);
  q.c = ldc(a.Pc[4], o);
  q.h = ldc(a.Pc[5], o);
  q.w[0] = Y[0]; q.w[1] = Y[1]; q.w[5] = Y[5]; q.w[6] = Y[6];
  if (DIR == 0) { q.w[2] = Y[2]; q.w[3] = Y[3]; q.w[4] = Y[4]; q.un = u; q.ut = v; q.us = w; }
  else if (DIR == 1) { q.w[2] = Y[3]; q.w[3] = Y[2]; q.w[4] = Y[4]; q.un = v; q.ut = u; q.us = w; }
  else { q.w[2] = Y[4]; q.w[3] = Y[2]; q.w[4] = Y[3]; q.un = w; q.ut = u; q.us = v; }
  const double sg = ((st.flip >> m) & 1u) ? -1.0 : 1.0;
  q.w[2] *= sg;
  q.un *= sg;
}

// characteristic field f of node q [App. A, one more passive field]
__device__ __forceinline__ double char_field3(int f, const NodeQ3& q, double fa1, double fa2,
                                              double k1, double k2) {
  switch (f) {
    case 0: return q.un - q.p * k1;
    case 1: return q.w[0] - fa1 * q.p * k2;
    case 2: return q.w[1] - fa2 * q.p * k2;
    case 3: return q.ut;
    case 4: return q.us;
    case 5: return q.w[6];
    default: return q.un + q.p * k1;
  }
}

// rotated component v of direction DIR -> state index
__device__ __forceinline__ int state_index3(int dir, int v) {
  if (v < 2 || v > 4 || dir == 0) return v;
  if (dir == 1) return v == 2 ? 3 : (v == 3 ? 2 : 4);
  return v == 2 ? 4 : (v == 3 ? 2 : 3);
}

// Stencil node m from global memory (offsets and wall flips of a Sten3)
template <int DIR>
struct GlobalLoad3 {
  const K3Args* a;
  Sten3 st;
  __device__ __forceinline__ void operator()(int m, NodeQ3& q) const { load_node3<DIR>(*a, st, m, q); }
};

// Stencil node m from LDS: value c of node m at p[m * sm + c * sc], values in
// the order w[0..6], un, ut, us, p, c, h of the sweep's frame
struct LdsLoad3 {
  const double* p;
  int sm, sc;
  __device__ __forceinline__ void operator()(int m, NodeQ3& q) const {
    const double* t = p + m * sm;
#pragma unroll
    for (int k = 0; k < 7; ++k) q.w[k] = t[k * sc];
    q.un = t[7 * sc];
    q.ut = t[8 * sc];
    q.us = t[9 * sc];
    q.p = t[10 * sc];
    q.c = t[11 * sc];
    q.h = t[12 * sc];
  }
};

// Stencil node m from LDS holding 11 values per node (w[0..6], un, ut, us,
// p); the sound speed and rho ctilde^2, which the face pipeline reads only at
// the two nodes next to the face (m = 2, 3), come from registers.
struct LdsLoad3C {
  const double* p;
  int sm, sc;
  double c2, h2, c3, h3;
  __device__ __forceinline__ void operator()(int m, NodeQ3& q) const {
    const double* t = p + m * sm;
#pragma unroll
    for (int k = 0; k < 7; ++k) q.w[k] = t[k * sc];
    q.un = t[7 * sc];
    q.ut = t[8 * sc];
    q.us = t[9 * sc];
    q.p = t[10 * sc];
    q.c = m == 2 ? c2 : (m == 3 ? c3 : 0.0);
    q.h = m == 2 ? h2 : (m == 3 ? h3 : 0.0);
  }
};

// The 13 staged values of the cell at byte offset o in the frame of DIR,
// normal momentum and velocity negated for a reflective ghost (the same
// values load_node3 returns)
template <int DIR>
__device__ __forceinline__ void node_values3(const K3Args& a, uint32_t o, bool flip, double v[13]) {
  double Y[7], P[6];
#pragma unroll
  for (int k = 0; k < 7; ++k) Y[k] = ldc(a.Wc[k], o);
#pragma unroll
  for (int k = 0; k < 6; ++k) P[k] = ldc(a.Pc[k], o);
  v[0] = Y[0]; v[1] = Y[1]; v[5] = Y[5]; v[6] = Y[6];
  if (DIR == 0) { v[2] = Y[2]; v[3] = Y[3]; v[4] = Y[4]; v[7] = P[0]; v[8] = P[1]; v[9] = P[2]; }
  else if (DIR == 1) { v[2] = Y[3]; v[3] = Y[2]; v[4] = Y[4]; v[7] = P[1]; v[8] = P[0]; v[9] = P[2]; }
  else { v[2] = Y[4]; v[3] = Y[2]; v[4] = Y[3]; v[7] = P[2]; v[8] = P[0]; v[9] = P[1]; }
  v[10] = P[3];
  v[11] = P[4];
  v[12] = P[5];
  if (flip) { v[2] = -v[2]; v[7] = -v[7]; }
}

// One face of a 3D sweep: WCNS steps 1-9 [Sec. 4.2] with both limiters, the
// stencil nodes (in the frame of DIR) from the loader `ld`.
template <int DIR, class LD>
__device__ __forceinline__ double face_flux3_core(const K3Args& a, const LD& ld, double lam,
                                                  double Gm[7], double Gp[7]) {
  const EosC& e = a.eos;
  double Hm[7], Hp[7];
  double fa1, fa2, frho, fc, k1, k2;
  {
    NodeQ3 nl, nr;
    ld(2, nl);
    ld(3, nr);
    HllcOut3 h1;
    hllc3(nl, nr, h1);
#pragma unroll
    for (int v = 0; v < 6; ++v) { Hm[v] = h1.F[v]; Hp[v] = h1.F[v]; }
    Hm[6] = h1.fa - nl.w[6] * h1.ss;
    Hp[6] = h1.fa - nr.w[6] * h1.ss;
    if (a.scheme == 1) {
#pragma unroll
      for (int v = 0; v < 7; ++v) { Gm[v] = Hm[v]; Gp[v] = Hp[v]; }
      return 0.0;
    }
    fa1 = 0.5 * (nl.w[0] + nr.w[0]);
    fa2 = 0.5 * (nl.w[1] + nr.w[1]);
    frho = 0.5 * ((nl.w[0] + nl.w[1]) + (nr.w[0] + nr.w[1]));
    fc = 0.5 * (nl.c + nr.c);
    k1 = ddiv(1.0, frho * fc);
    k2 = ddiv(1.0, frho * fc * fc);
  }
  // projection and IS-WENO, one field at a time
  double UL[7], UR[7];
#pragma unroll
  for (int f = 0; f < 7; ++f) {
    phase_barrier();
    double u[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      NodeQ3 q;
      ld(m, q);
      u[m] = char_field3(f, q, fa1, fa2, k1, k2);
    }
    UL[f] = weno_is(u[0], u[1], u[2], u[3], u[4], a.tol.weno_eps);
    UR[f] = weno_is(u[5], u[4], u[3], u[2], u[1], a.tol.weno_eps);
  }
  phase_barrier();
  // back-projection V = R U, then V -> W [App. A; Sec. 2]
  double WL[7], WR[7];
  {
    const double twoc = 2.0 * fc;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double* U = side == 0 ? UL : UR;
      double* X = side == 0 ? WL : WR;
      double d = U[6] - U[0];
      double a1r1 = U[1] + ddiv(fa1 * d, twoc);
      double a2r2 = U[2] + ddiv(fa2 * d, twoc);
      double un = 0.5 * (U[0] + U[6]);
      double ut = U[3];
      double us = U[4];
      double p = 0.5 * frho * fc * d;
      double a1 = U[5];
      double rho = a1r1 + a2r2;
      X[0] = a1r1;
      X[1] = a2r2;
      X[2] = rho * un;
      X[3] = rho * ut;
      X[4] = rho * us;
      double ke = un * un + ut * ut;
      ke = ke + us * us;
      X[5] = mix_gamma(e, a1) * p + mix_pi(e, a1) + 0.5 * rho * ke;
      X[6] = a1;
    }
  }
  if (a.interp_limiter) {
    NodeQ3 q;
    ld(2, q);
    interp_limit3(e, a.tol, q.w, q.h, WL);
    phase_barrier();
    ld(3, q);
    interp_limit3(e, a.tol, q.w, q.h, WR);
    phase_barrier();
  }
  // midpoint HLLC on the limited states [WCNS step 6]
  double acc[8];
  {
    NodeQ3 tl, tr;
#pragma unroll
    for (int v = 0; v < 7; ++v) { tl.w[v] = WL[v]; tr.w[v] = WR[v]; }
    recover3(e, tl.w, tl.un, tl.ut, tl.us, tl.p, tl.c, tl.h);
    recover3(e, tr.w, tr.un, tr.ut, tr.us, tr.p, tr.c, tr.h);
    HllcOut3 h2;
    hllc3(tl, tr, h2);
#pragma unroll
    for (int v = 0; v < 6; ++v) acc[v] = h2.F[v];
    acc[6] = h2.fa;
    acc[7] = h2.ss;
  }
  // HCS reconstruction of flux and velocity [Sec. 4.1; WCNS steps 7-8]
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    phase_barrier();
    NodeQ3 qa, qb;
    ld(2 - pr, qa);
    ld(3 + pr, qb);
    double ga[7], gb[7];
    node_flux3(qa, ga);
    node_flux3(qb, gb);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      double sum = v < 7 ? ga[v] + gb[v] : qa.un + qb.un;
      if (pr == 0) acc[v] = 3072.0 * acc[v] - 505.0 * sum;
      else if (pr == 1) acc[v] = acc[v] + 20.0 * sum;
      else acc[v] = cdiv(acc[v] - sum, 2100.0, R2100);
    }
  }
  const double uh = acc[7];
  // split fluxes G^{-+} [Sec. 3.2, WCNS step 9] and the flux limiter
  phase_barrier();
  NodeQ3 nl, nr;
  ld(2, nl);
  ld(3, nr);
#pragma unroll
  for (int v = 0; v < 6; ++v) { Gm[v] = acc[v]; Gp[v] = acc[v]; }
  Gm[6] = acc[6] - nl.w[6] * uh;
  Gp[6] = acc[6] - nr.w[6] * uh;
  if (a.flux_limiter) {
    double gl[7], gr[7];
    node_flux3(nl, gl);
    node_flux3(nr, gr);
    gl[6] = 0.0;
    gr[6] = 0.0;
    return flux_limit3(e, a.tol, nl.w, nr.w, gl, gr, lam, Hm, Hp, Gm, Gp);
  }
  return 1.0;
}

template <int DIR>
__device__ __forceinline__ double face_flux3(const K3Args& a, const Sten3& st, double lam,
                                             double Gm[7], double Gp[7]) {
  const GlobalLoad3<DIR> ld{&a, st};
  return face_flux3_core<DIR>(a, ld, lam, Gm, Gp);
}

// final write of one cell: L or the SSP-RK3 stage combination
__device__ __forceinline__ void write_cell3(const K3Args& a, long idx, long N, int k, double L) {
  if (a.out_mode == OUT_STORE) {
    a.out[k * N + idx] = L;
  } else {
    const double dt = a.step[0];
    a.out[k * N + idx] = a.ca * a.Un[k * N + idx] + a.cb * (a.W[k * N + idx] + dt * L);
  }
}

// The inputs of one cell's final write, loaded ahead of the stores (a store
// to a.out may alias a later load, so a load left between the stores waits
// for the one before): the earlier passes' L and, in the last pass of an RK
// stage, U^n, W and dt
struct CellIn3 {
  double lin[7], un[7], w[7], dt;
};
__device__ __forceinline__ void load_cell_in3(const K3Args& a, long idx, long N, CellIn3& c) {
#pragma unroll
  for (int k = 0; k < 7; ++k) c.lin[k] = a.Lin[k * N + idx];
  if (a.last && a.out_mode != OUT_STORE) {
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      c.un[k] = a.Un[k * N + idx];
      c.w[k] = a.W[k * N + idx];
    }
    c.dt = a.step[0];
  }
}
// write_cell3 (or L alone before the last pass) on preloaded inputs;
// returns the value written
__device__ __forceinline__ double write_cell3_in(const K3Args& a, long idx, long N, int k, double L,
                                                 const CellIn3& c) {
  const double v = (a.last && a.out_mode != OUT_STORE) ? a.ca * c.un[k] + a.cb * (c.w[k] + c.dt * L) : L;
  a.out[k * N + idx] = v;
  return v;
}

// Stage-result check of a cell the last pass of an RK stage finished (X in
// state order): counted when outside G (the lanes that get here vote).
__device__ __forceinline__ void stage_check3(const K3Args& a, const double X[7]) {
  if (!(a.viol && a.last && a.out_mode != OUT_STORE)) return;
  report_bad(a.viol, a.vflag, !admissible(X[0], X[1], X[6], rhoc2_tilde3(a.eos, X)));
}

// ------------------------------------------------------------------ kernels
__global__ __launch_bounds__(256) void k3_node(K3Args a, double* P, double* partial) {
  if (a.node_skip && a.step[STEP_SKIP] != 0.0) return;
  const long N = (long)a.nx * a.ny * a.nz;
  const bool check = a.viol && a.check_in;
  double m[3] = {0.0, 0.0, 0.0};
  for (long o = (long)blockIdx.x * blockDim.x + threadIdx.x; o < N;
       o += (long)gridDim.x * blockDim.x) {
    double X[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) X[k] = a.W[k * N + o];
    double u, v, w, p, c, h;
    recover3(a.eos, X, u, v, w, p, c, h);
    P[o] = u; P[N + o] = v; P[2 * N + o] = w;
    P[3 * N + o] = p; P[4 * N + o] = c; P[5 * N + o] = h;
    m[0] = fmax(m[0], fabs(u) + c);
    m[1] = fmax(m[1], fabs(v) + c);
    m[2] = fmax(m[2], fabs(w) + c);
    if (check) report_bad(a.viol, a.vflag, !admissible(X[0], X[1], X[6], h));
  }
  __shared__ double red[3][4];
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    m[d] = wave_max(m[d]);
    if (l == 0) red[d][wv] = m[d];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int d = threadIdx.x;
    double x = red[d][0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) x = fmax(x, red[d][k]);
    partial[3 * blockIdx.x + d] = x;
  }
}

// Time step and three-way split [Sec. 3.3]: tau_d = max(|u_d|+c)/h_d,
// dt = CFL/(tau_x + tau_y + tau_z), sigma_d = tau_d/(tau_x + tau_y + tau_z),
// lambda_d = dt/(h_d sigma_d).
// clock, nsteps, t_end: the time loop to t_end as in k_finalize (clock null:
// none)
__global__ __launch_bounds__(256) void k3_finalize(const double* partial, int nblk, int dt_mode,
                                                   double dt_in, double cfl, double dx, double dy,
                                                   double dz, double* step, double* dt_used,
                                                   double* clock, int64_t* nsteps, double t_end) {
  double m[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int d = 0; d < 3; ++d) m[d] = fmax(m[d], partial[3 * b + d]);
  __shared__ double red[3][4];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    m[d] = wave_max(m[d]);
    if (l == 0) red[d][w] = m[d];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int d = 0; d < 3; ++d)
    for (int k = 1; k < 4; ++k) m[d] = fmax(m[d], red[d][k]);
  if (dt_mode == DT_KEEP && step[STEP_SKIP] != 0.0) return;   // inside a skipped step
  double dt;
  if (dt_mode == DT_GIVEN) dt = dt_in;
  else if (dt_mode == DT_KEEP) dt = step[0];
  else dt = cfl / (m[0] / dx + m[1] / dy + m[2] / dz);
  if (dt_mode != DT_KEEP) {
    const bool run = !clock || clock_step(clock, nsteps, t_end, dt);
    step[STEP_SKIP] = run ? 0.0 : 1.0;
    if (!run) {
      if (dt_used) *dt_used = 0.0;
      return;
    }
  }
  const double h[3] = {dx, dy, dz};
  const double t[3] = {m[0] / dx, m[1] / dy, m[2] / dz};
  const double tot = t[0] + t[1] + t[2];
  step[0] = dt;
  for (int d = 0; d < 3; ++d) {
    step[1 + d] = dt / (h[d] * (t[d] / tot));
    step[4 + d] = m[d];
  }
  if (dt_used) *dt_used = dt;
}

// x pass: one wave per tile of tile_x flattened cells (rows of nx); lanes
// past the tile own the right faces of its row segments (as in 2D)
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k3_sweep_x(K3Args a) {
  if (a.step[STEP_SKIP] != 0.0) return;
  const int lane = threadIdx.x;
  const int nx = a.nx;
  const long N = (long)nx * a.ny * a.nz;
  const int T = a.tile_x;
  const long c0 = (long)blockIdx.x * T;
  const long c1 = (c0 + T < N ? c0 + T : N) - 1;
  const long j0 = c0 / nx, j1 = c1 / nx;
  long fj = 0;
  int fk = 0;
  bool active = false;
  if (lane < T) {
    long c = c0 + lane;
    if (c <= c1) { fj = c / nx; fk = (int)(c % nx); active = true; }
  } else {
    long r = lane - T;
    if (j0 + r <= j1) {
      fj = j0 + r;
      long last = (fj == j1) ? c1 : fj * nx + nx - 1;
      fk = (int)(last % nx) + 1;
      active = true;
    }
  }
  double Gm[7] = {0, 0, 0, 0, 0, 0, 0}, Gp[7] = {0, 0, 0, 0, 0, 0, 0};
  if (active) {
    const Sten3 st = make_sten3(fk - 3, nx, a.bc[0], a.bc[1], fj * nx, 1);
    face_flux3<0>(a, st, a.step[1], Gm, Gp);
  }
  int src = lane;
  const long c = c0 + lane;
  const bool owns_cell = lane < T && c <= c1;
  if (owns_cell) src = (c == c1 || (c % nx) == nx - 1) ? T + (int)(c / nx - j0) : lane + 1;
  double Gr[7];
#pragma unroll
  for (int v = 0; v < 7; ++v) Gr[v] = __shfl(Gm[v], src, 64);
  if (!owns_cell) return;
#pragma unroll
  for (int v = 0; v < 7; ++v) a.Lout[v * N + c] = hdiv(-(Gr[v] - Gp[v]), a.dx, a.rdx);
}

// x pass with each wave's stencil window staged in LDS (rows of at least
// XLDS_MIN_NX cells): flattened tiles of XT cells over the ny*nz rows with
// the window geometry of the 2D sweep, 13 values per slot in the x frame.
__global__ __launch_bounds__(64 * XW) void k3_sweep_xl(K3Args a) {
  if (a.step[STEP_SKIP] != 0.0) return;
  __shared__ double tile[XW][13 * XWIN];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nx = a.nx;
  const long N = (long)nx * a.ny * a.nz;
  const long tl = (long)blockIdx.x * XW + w;
  double* win = tile[w];
  XWin t{};
  if (tl * XT < N) {
    t = x_window(nx, N, tl);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int sl = lane + 64 * q;
      if (sl < t.slots) {
        int j, g;
        t.slot_cell(sl, j, g);
        bool flip;
        const int src = ghost_src(g, nx, a.bc[0], a.bc[1], flip);
        double v[13];
        node_values3<0>(a, ((uint32_t)j * (uint32_t)nx + (uint32_t)src) * 8u, flip, v);
#pragma unroll
        for (int c = 0; c < 13; ++c) win[c * XWIN + sl] = v[c];
      }
    }
  }
  wave_lds_sync();   // the window is this wave's own
  double Gm[7] = {0, 0, 0, 0, 0, 0, 0}, Gp[7] = {0, 0, 0, 0, 0, 0, 0};
  if (lane < t.nA + t.nB) {
    const LdsLoad3 ld{win + t.base(lane), 1, XWIN};
    face_flux3_core<0>(a, ld, a.step[1], Gm, Gp);
  }
  double Gr[7];   // (lane 63 owns no cell)
#pragma unroll
  for (int v = 0; v < 7; ++v) Gr[v] = from_next_lane(Gm[v]);
  if (!t.owner(lane)) return;
  const long c = t.cell(lane);
#pragma unroll
  for (int v = 0; v < 7; ++v) a.Lout[v * N + c] = hdiv(-(Gr[v] - Gp[v]), a.dx, a.rdx);
}

// Strided pass of direction DIR (1: y-lines in z slab blockIdx.z; 2: z-lines
// over the nx*ny columns) on tiles of 32 columns: a block of YW3/2 waves covers 32
// consecutive columns x YW3 face rows; lane (r = lane / 32, col = lane % 32)
// of wave w computes face row kb + 2w + r.  Stencil rows kb-3 .. kb+YW3+1
// are staged first (11 values per node in the frame of DIR; c and
// rho ctilde^2 of the two centre nodes from global memory into registers).
// Cell row kb + 2w takes G^- of face row kb + 2w + 1 from lane + 32 of its
// own wave; cell row kb + 2w + 1 takes it from wave w + 1 through LDS; the
// tile's first G^- and last G^+ go to the edge buffer for k3_fixup.  At 16
// face rows the tile is 59 KB: two 8-wave blocks per CU.
template <int DIR>
__device__ __forceinline__ void sweep3_tile32(const K3Args& a, double* tile) {
  constexpr int FR = YW3, W = YW3 / 2, ROWS = YW3 + 5;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane >> 5, cl = lane & 31;
  const long plane = (long)a.nx * a.ny;
  const long N = plane * a.nz;
  const long ncol = DIR == 1 ? a.nx : plane;
  const int nline = DIR == 1 ? a.ny : a.nz;
  const long stride = DIR == 1 ? a.nx : plane;
  const long slab = DIR == 1 ? (long)blockIdx.z * plane : 0;
  const double h = DIR == 1 ? a.dy : a.dz;
  const double rh = DIR == 1 ? a.rdy : a.rdz;
  const long col = (long)blockIdx.x * 32 + cl;
  const int by = blockIdx.y;
  const int kb = by * FR;
  const int fr = 2 * w + r;
  const int k = kb + fr;
  const bool active = col < ncol && k <= nline;
  // stage: slot t = thread + 64W q holds tile row t / 32, column t % 32
#pragma unroll
  for (int q = 0; q < (ROWS * 32 + 64 * W - 1) / (64 * W); ++q) {
    const int t = (int)threadIdx.x + 64 * W * q;
    const int tr = t >> 5;
    const long cc = (long)blockIdx.x * 32 + (t & 31);
    const int g = kb - 3 + tr;
    if (tr < ROWS && g <= nline + 2 && cc < ncol) {
      bool flip;
      const int s = ghost_src(g, nline, a.bc[2 * DIR], a.bc[2 * DIR + 1], flip);
      double v[13];
      node_values3<DIR>(a, (uint32_t)(slab + (long)s * stride + cc) * 8u, flip, v);
#pragma unroll
      for (int c = 0; c < 11; ++c) tile[(c * ROWS + tr) * 32 + (t & 31)] = v[c];
    }
  }
  __syncthreads();
  double Gm[7] = {0, 0, 0, 0, 0, 0, 0}, Gp[7] = {0, 0, 0, 0, 0, 0, 0};
  if (active) {
    bool flip;
    const int s2 = ghost_src(k - 1, nline, a.bc[2 * DIR], a.bc[2 * DIR + 1], flip);
    const int s3 = ghost_src(k, nline, a.bc[2 * DIR], a.bc[2 * DIR + 1], flip);
    const uint32_t o2 = (uint32_t)(slab + (long)s2 * stride + col) * 8u;
    const uint32_t o3 = (uint32_t)(slab + (long)s3 * stride + col) * 8u;
    const LdsLoad3C ld{tile + fr * 32 + cl, 32, ROWS * 32,
                       ldc(a.Pc[4], o2), ldc(a.Pc[5], o2), ldc(a.Pc[4], o3), ldc(a.Pc[5], o3)};
    face_flux3_core<DIR>(a, ld, a.step[1 + DIR], Gm, Gp);
  }
  // the owned cell's inputs, loaded while the block exchanges G^-
  const bool own = active && fr != FR - 1 && k < nline;
  const long idx = slab + (long)k * stride + col;
  CellIn3 cin;
  if (own) load_cell_in3(a, idx, N, cin);
  double Gn[7];   // G^- of face row k + 1 when r == 0 (same wave, upper half)
#pragma unroll
  for (int v = 0; v < 7; ++v) Gn[v] = __shfl(Gm[v], (lane + 32) & 63, 64);
  __syncthreads();   // every face has read the tile: reuse it for G^-
  double* sG = tile;   // [W][7][32]: G^- of each wave's lower face row
  if (r == 0) {
#pragma unroll
    for (int v = 0; v < 7; ++v) sG[(w * 7 + v) * 32 + cl] = Gm[v];
  }
  if (active) {
    double* e = a.edge + (((long)(DIR == 1 ? blockIdx.z : 0) * a.nbr + by) * 14) * ncol;
    if (fr == 0) {
#pragma unroll
      for (int v = 0; v < 7; ++v) e[v * ncol + col] = Gm[v];
    }
    if (fr == FR - 1 || k == nline) {
#pragma unroll
      for (int v = 0; v < 7; ++v) e[(7 + v) * ncol + col] = Gp[v];
    }
  }
  __syncthreads();
  if (!own) return;
  double X[7];
#pragma unroll
  for (int v = 0; v < 7; ++v) {
    const int s = state_index3(DIR, v);
    const double up = r == 0 ? Gn[v] : sG[((w + 1) * 7 + v) * 32 + cl];
    const double L = cin.lin[s] + hdiv(-(up - Gp[v]), h, rh);
    X[s] = write_cell3_in(a, idx, N, s, L, cin);
  }
  stage_check3(a, X);
}

// (measured at 256^3, ms per y / z pass: nodes loaded from global memory
// at their use, 64-column tiles 2.62 / 2.99; all 13 values staged 2.12 /
// 2.45; 11 values staged, c and rho ctilde^2 of the two centre nodes in
// registers, 1.81 / 1.93; the same on 32 columns x 8 rows 1.78 / 1.81)
template <int DIR>
__global__ __launch_bounds__(L3_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k3_sweep_l(K3Args a) {
  if (a.step[STEP_SKIP] != 0.0) return;
  __shared__ double tile32[11 * (YW3 + 5) * 32];
  sweep3_tile32<DIR>(a, tile32);
}

// the cell rows j = (b+1)*YW3 - 1 between tiles b and b+1 of a strided pass
template <int DIR>
__global__ __launch_bounds__(256) void k3_fixup(K3Args a) {
  if (a.step[STEP_SKIP] != 0.0) return;
  const long plane = (long)a.nx * a.ny;
  const long N = plane * a.nz;
  const long ncol = DIR == 1 ? a.nx : plane;
  const int nline = DIR == 1 ? a.ny : a.nz;
  const long stride = DIR == 1 ? a.nx : plane;
  const long nslab = DIR == 1 ? a.nz : 1;
  const long per_slab = (long)(a.nbr - 1) * ncol;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per_slab * nslab) return;
  const long sl = t / per_slab, r = t % per_slab;
  const int b = (int)(r / ncol);
  const long col = r % ncol;
  const int j = (b + 1) * YW3 - 1;
  if (j >= nline) return;
  const double h = DIR == 1 ? a.dy : a.dz;
  const double rh = DIR == 1 ? a.rdy : a.rdz;
  const double* lo = a.edge + ((sl * a.nbr + b) * 14 + 7) * ncol;   // G^+ of face row j
  const double* hi = a.edge + ((sl * a.nbr + b + 1) * 14) * ncol;   // G^- of face row j+1
  const long idx = sl * plane + (long)j * stride + col;
  double gl[7], gh[7];
#pragma unroll
  for (int v = 0; v < 7; ++v) {
    gl[v] = lo[v * ncol + col];
    gh[v] = hi[v * ncol + col];
  }
  CellIn3 cin;
  load_cell_in3(a, idx, N, cin);
  double X[7];
#pragma unroll
  for (int v = 0; v < 7; ++v) {
    const int s = state_index3(DIR, v);
    const double L = cin.lin[s] + hdiv(-(gh[v] - gl[v]), h, rh);
    X[s] = write_cell3_in(a, idx, N, s, L, cin);
  }
  stage_check3(a, X);
}

// V (a1r1, a2r2, u, v, w, p, a1) -> W [Sec. 2 mixture EOS]
__global__ __launch_bounds__(256) void k3_prim_to_cons(K3Args a, const double* V, double* W) {
  const long N = (long)a.nx * a.ny * a.nz;
  const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  double a1r1 = V[o], a2r2 = V[N + o], u = V[2 * N + o], v = V[3 * N + o], w = V[4 * N + o];
  double p = V[5 * N + o], a1 = V[6 * N + o];
  double rho = a1r1 + a2r2;
  W[o] = a1r1;
  W[N + o] = a2r2;
  W[2 * N + o] = rho * u;
  W[3 * N + o] = rho * v;
  W[4 * N + o] = rho * w;
  double ke = u * u + v * v;
  ke = ke + w * w;
  W[5 * N + o] = mix_gamma(a.eos, a1) * p + mix_pi(a.eos, a1) + 0.5 * rho * ke;
  W[6 * N + o] = a1;
}

// Admissible set G [Sec. 2]; NaN fails every comparison and counts as bad.
__global__ __launch_bounds__(256) void k3_admissible(K3Args a, unsigned long long* count) {
  const long N = (long)a.nx * a.ny * a.nz;
  const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (o < N) {
    double X[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) X[k] = a.W[k * N + o];
    double h = rhoc2_tilde3(a.eos, X);
    bad = !(X[6] >= 0.0 && X[6] <= 1.0 && X[0] >= 0.0 && X[1] >= 0.0 && h > 0.0);
  }
  unsigned long long n = __ballot(bad);
  if ((threadIdx.x & 63) == 0 && n) atomicAdd(count, (unsigned long long)__popcll(n));
}

// maxima of the step record for wcns_max_wavespeed (3 values)
__global__ void k3_copy_amax(const double* step, double* out) {
  if (threadIdx.x < 3) out[threadIdx.x] = step[4 + threadIdx.x];
}

}  // namespace wcns
