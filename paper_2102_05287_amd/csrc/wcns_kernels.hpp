// gfx950 kernels of the PP-WCNS-IS right-hand side and the SSP-RK3 step.
//
// Per RHS evaluation (2D):
//   k_node      one thread per cell: primitive recovery (u, v, p, c, rho
//               ctilde^2) written to scratch, plus per-block maxima of |u|+c
//               and |v|+c (Sec. 3.3 wave speeds).
//   k_finalize  one block: global maxima -> dt (CFL), sigma, lambda (Sec. 3.3)
//               kept on the device so a whole step can be graph-captured.
//   k_sweep_xl  one wave per flattened (row-major) tile of 62 cells with its
//               stencil window staged in LDS; each lane computes one x-face
//               with the full per-face pipeline and the flux difference uses
//               a cross-lane shuffle (k_sweep_x: the same tiling with global
//               loads, for rows narrower than 61 cells).
//   k_sweep_y   one block over 32 columns x 16 y-face rows (8 waves, two
//               face rows each), stencil rows staged in LDS; every face is
//               computed once; neighbours exchanged by shuffle and LDS; the
//               epilogue sums L_x + L_y and (for a step) applies the SSP-RK3
//               stage combination.
//   k_fixup_y   finishes the cell rows that straddle two y-tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcns_device.hpp"

// The FP64 path rounds every operation as written, in the same order as the
// serial reference (no FMA contraction, IEEE divides and square roots): the
// positivity limiters divide by differences of order 1e-8 near material
// interfaces, so any change of rounding upstream would move their blends by
// ~1e-8 relative.
#pragma clang fp contract(off)

namespace wcns {

enum { BC_PERIODIC = 0, BC_EXTRAP = 1, BC_REFLECT = 2, BC_DIRICHLET = 3 };
enum { OUT_STORE = 0, OUT_RK = 1 };
// Step record (device, one per solve): [0] dt, [1] lambda_x, [2] lambda_y,
// [3] max(|u|+c), [4] max(|v|+c) (3D: [1..3] lambda, [4..6] maxima), and at
// STEP_SKIP a flag set when a step of a time loop bounded by t_end would
// start at or after t_end: every kernel of that step then returns at once.
enum { STEP_SKIP = 7 };
// y-sweep tiles (single grid): 32 columns x 16 y-face rows, 8 waves and
// 48.6 KB of LDS per block, two blocks per CU.  Against 8-row tiles (four
// 4-wave blocks per CU) the y-sweep itself runs 0.5-2% slower, but the
// fixup has half the straddling cell rows: 1024^2 step 1.2%, 2048^2 FP64
// 1.1% and FP32 bulk 1.7% faster.
constexpr int Y_ROWS = 16;
constexpr int Y_COLS = 32;
constexpr int Y_THREADS = Y_COLS * Y_ROWS;   // 8 waves: each covers two face rows

struct KArgs {
  int32_t nx, ny, nv, tile_x;     // tile_x: cells per x-sweep wave
  double dx, dy;
  double rdx, rdy;                // checked reciprocals of dx, dy (0: divide)
  int32_t bc[4];
  int32_t dir_off[4];    // first Dirichlet ghost row of each side in dirW/dirP
  int32_t interp_limiter, flux_limiter, scheme, pad;
  EosC eos;
  Tol tol;
  const double* W;       // state differentiated
  const double* P;       // node primitives of W: [5][ny][nx] (u, v, p, c, h)
  const double* Wc[6];   // per-component bases of W in rotated-frame-free state
                         // order (1D: a1r1, a2r2, m, -, E, a1 with slot 3 unused)
  const double* Pc[5];   // per-component bases of P
  const double* dirW;    // Dirichlet ghost state of each boundary row/column
                         // [rows][6] (unrotated 6-comp; 1D: slot 3 is 0)
  const double* dirP;    // their node primitives [rows][5] (u, v, p, c, h)
  const double* step;    // [0] dt, [1] lam_x, [2] lam_y, [3] amax_x, [4] amax_y
  const double* Lx;      // x-part of L (read by the y-sweep)
  double* Lout;          // x-sweep output (L_x in 2D, full L in 1D)
  double* out;           // final output (L or next stage state)
  const double* Un;      // state at the start of the step (RK epilogue)
  double* edge;          // y-tile boundary fluxes [nbr][2][6][nx]
  double ca, cb;         // RK: out = ca*Un + cb*(W + dt*L)
  int32_t out_mode, nbr; // nbr: y-tile rows (edge buffer rows)
  double* partial;       // per-block wave-speed maxima of this instance
  double* Pw;            // node-primitive output of k_node (= P)
  int32_t nblk, ndim;    // node blocks of this instance; 1 or 2
  int32_t dt_mode, pad3; // stage's time-step mode (DT_GIVEN/DT_CFL/DT_KEEP)
  double cfl, dt_in;
  double* dt_used;       // optional copy of dt
  const int32_t* live;   // batched form: steps left for this instance (skip at 0)
  // Next stage's node primitives computed where the stage state is
  // finished (y-sweep epilogue and fixup) instead of by k_node: Pn [5][N]
  // (null: off) and per-block wave-speed maxima at partn[2b], partn[2b+1]
  // (y-sweep blocks first, the fixup's from fuse_off on)
  double* Pn;
  double* partn;
  int32_t fuse_off;
  int32_t check_out;     // one-pass first-order stage: also check its result
  // Lazy admissibility report [Sec. 2]: stage results outside G (and, with
  // check_in, k_node's input cells) are counted into *viol (null: not
  // counted) and raise the host-mapped flag *vflag (null: none).
  // node_skip: a k_node launch inside a step (not its first stage), which
  // returns at once when the step is skipped.
  unsigned long long* viol;
  int32_t* vflag;
  int32_t check_in, node_skip;
  double* sink;          // one-pass first-order stage: where lanes that finish no cell write
};

// ------------------------------------------------------------------ nodes
// Ghost mapping along a line of n cells [3 ghost layers; periodic, constant
// extrapolation, reflective, Dirichlet].  Returns the source cell or -1 for
// Dirichlet; flip = the wall-normal momentum changes sign.
__device__ __forceinline__ int ghost_src(int g, int n, int bc_lo, int bc_hi, bool& flip) {
  flip = false;
  if (g >= 0 && g < n) return g;
  int bc = g < 0 ? bc_lo : bc_hi;
  if (bc == BC_PERIODIC) { int r = g % n; return r < 0 ? r + n : r; }
  if (bc == BC_EXTRAP) return g < 0 ? 0 : n - 1;
  if (bc == BC_REFLECT) { flip = true; return g < 0 ? -1 - g : 2 * n - 1 - g; }
  return -1;
}

// Stencil of one face: byte offsets (within one component array) of the 6
// nodes i-2 .. i+3 after ghost mapping, a bit mask of reflective ghosts
// (normal momentum and velocity change sign) and, with Dirichlet sides, a
// mask of Dirichlet ghosts.  Computed once per face; every node load after
// that is a branch-free 32-bit-offset load from a per-component base.
struct Sten {
  uint32_t off[6];
  uint32_t flip, diri;
  int32_t drow[2];   // Dirichlet ghost rows of the face's line (lo, hi side)
};

template <int DIR>
__device__ __forceinline__ Sten make_sten(const KArgs& a, int line, int g0) {
  const int n = DIR == 0 ? a.nx : a.ny;
  Sten st;
  st.flip = 0;
  st.diri = 0;
  st.drow[0] = a.dir_off[2 * DIR] + line;
  st.drow[1] = a.dir_off[2 * DIR + 1] + line;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int g = g0 + m;
    bool flip;
    int s = ghost_src(g, n, a.bc[2 * DIR], a.bc[2 * DIR + 1], flip);
    if (s < 0) { st.diri |= 1u << m; s = 0; }
    if (flip) st.flip |= 1u << m;
    const uint32_t o = DIR == 0 ? (uint32_t)line * (uint32_t)a.nx + (uint32_t)s
                                : (uint32_t)s * (uint32_t)a.nx + (uint32_t)line;
    st.off[m] = o * 8u;
  }
  return st;
}

__device__ __forceinline__ double ldc(const double* base, uint32_t byte_off) {
  return *(const double*)((const char*)base + byte_off);
}

// Node m of a stencil in the frame rotated into direction DIR.
template <int DIR, bool HAS_T, bool DIRI>
__device__ __forceinline__ void load_node(const KArgs& a, const Sten& st, int m, int g0, NodeQ& q) {
  const uint32_t o = st.off[m];
  double Y[6], u, v;
  Y[0] = ldc(a.Wc[0], o);
  Y[1] = ldc(a.Wc[1], o);
  Y[2] = ldc(a.Wc[2], o);
  Y[3] = HAS_T ? ldc(a.Wc[3], o) : 0.0;
  Y[4] = ldc(a.Wc[4], o);
  Y[5] = ldc(a.Wc[5], o);
  u = ldc(a.Pc[0], o);
  v = HAS_T ? ldc(a.Pc[1], o) : 0.0;
  q.p = ldc(a.Pc[2], o);
  q.c = ldc(a.Pc[3], o);
  q.h = ldc(a.Pc[4], o);
  if (DIRI && ((st.diri >> m) & 1u)) {
    const int r = (g0 + m < 0) ? st.drow[0] : st.drow[1];
#pragma unroll
    for (int k = 0; k < 6; ++k) Y[k] = a.dirW[r * 6 + k];
    u = a.dirP[r * 5 + 0];
    v = a.dirP[r * 5 + 1];
    q.p = a.dirP[r * 5 + 2];
    q.c = a.dirP[r * 5 + 3];
    q.h = a.dirP[r * 5 + 4];
  }
  q.w[0] = Y[0]; q.w[1] = Y[1]; q.w[4] = Y[4]; q.w[5] = Y[5];
  if (DIR == 0) { q.w[2] = Y[2]; q.w[3] = Y[3]; q.un = u; q.ut = v; }
  else { q.w[2] = Y[3]; q.w[3] = Y[2]; q.un = v; q.ut = u; }
  const double sg = ((st.flip >> m) & 1u) ? -1.0 : 1.0;   // exact sign flip
  q.w[2] *= sg;
  q.un *= sg;
}

// ------------------------------------------------------------------ face
// Node loaders of the face pipeline: ld(m, q) fills node m (0..5 = i-2 ..
// i+3) of the face in the sweep's rotated frame.
// From global memory through the face's stencil offsets:
template <int DIR, bool HAS_T, bool DIRI>
struct GlobalLoad {
  const KArgs* a;
  Sten st;
  int g0;
  __device__ __forceinline__ void operator()(int m, NodeQ& q) const {
    load_node<DIR, HAS_T, DIRI>(*a, st, m, g0, q);
  }
};

// From a y-tile staged in LDS: value c (0..5 state, 6..8 u, v, p) of tile
// row r, column `col` at tile[(c * rows + r) * Y_COLS + col]; node m of the
// face of row w is tile row w + m.  Ghost rows are staged already mapped
// (reflective ones with the wall-normal momentum and velocity negated), so
// the node comes out as load_node would give it.  The sound speed and
// rho ctilde^2, which the face pipeline reads only at the two nodes next to
// the face (m = 2, 3), come from registers.
struct LdsLoadY {
  const double* tile;
  int rows, w, lane;
  double c2 = 0.0, h2 = 0.0, c3 = 0.0, h3 = 0.0;
  __device__ __forceinline__ void operator()(int m, NodeQ& q) const {
    const double* t = tile + (w + m) * Y_COLS + lane;
    const int cs = rows * Y_COLS;
    q.w[0] = t[0];
    q.w[1] = t[cs];
    q.w[2] = t[3 * cs];        // rho v: normal momentum of the y frame
    q.w[3] = t[2 * cs];
    q.w[4] = t[4 * cs];
    q.w[5] = t[5 * cs];
    q.ut = t[6 * cs];
    q.un = t[7 * cs];
    q.p = t[8 * cs];
    q.c = m == 2 ? c2 : (m == 3 ? c3 : 0.0);
    q.h = m == 2 ? h2 : (m == 3 ? h3 : 0.0);
  }
};

// One face i+1/2 of a sweep: WCNS steps 1-9 [Sec. 4.2] with the
// interpolation limiter [Sec. 5.1] and the flux limiter [Sec. 5.2].
// Node data are re-read (from the cache or the LDS tile) in each phase
// (phase_barrier) to keep the live register set small.  FO: compiled for
// the first-order scheme only (the rest of the pipeline is dead code, so
// the kernel keeps few registers).
template <int DIR, bool HAS_T, bool B32, bool FO = false, class LD>
__device__ __forceinline__ double face_flux_core(const KArgs& a, const LD& ld, double lam,
                                                 double Gm[6], double Gp[6]) {
  const EosC& e = a.eos;
  // first-order HLLC flux from W_i, W_{i+1} and its split [Sec. 3.2];
  // face averages for the projection [Sec. 4.2; App. A]
  double Hm[6], Hp[6];
  double fa1, fa2, frho, fc, k1, k2;
  {
    NodeQ nl, nr;
    ld(2, nl);
    ld(3, nr);
    HllcOut h1;
    hllc<HAS_T>(nl, nr, h1);
#pragma unroll
    for (int v = 0; v < 5; ++v) { Hm[v] = h1.F[v]; Hp[v] = h1.F[v]; }
    Hm[5] = h1.fa - nl.w[5] * h1.ss;
    Hp[5] = h1.fa - nr.w[5] * h1.ss;
    if (FO || a.scheme == 1) {
#pragma unroll
      for (int v = 0; v < 6; ++v) { Gm[v] = Hm[v]; Gp[v] = Hp[v]; }
      return 0.0;
    }
    fa1 = 0.5 * (nl.w[0] + nr.w[0]);
    fa2 = 0.5 * (nl.w[1] + nr.w[1]);
    frho = 0.5 * ((nl.w[0] + nl.w[1]) + (nr.w[0] + nr.w[1]));
    fc = 0.5 * (nl.c + nr.c);
    k1 = ddiv(1.0, frho * fc);
    k2 = ddiv(1.0, frho * fc * fc);
  }
  // characteristic projection U = R^{-1} V and IS-WENO, one field at a time
  // (FP32 interpolation in the precision form)
  double UL[6], UR[6];
  float ULf[6], URf[6];
  const float eps32 = fmaxf((float)a.tol.weno_eps, 1e-30f);
  // Fields in three groups that share their node data: (u_n, p) -> fields 0
  // and 5, (a1r1, a2r2, p) -> fields 1 and 2, (u_t, a1) -> fields 3 and 4.
  // The next group's node values are loaded before the current group's
  // interpolations run, so the cache latency overlaps the arithmetic.
  auto weno_pair = [&](int f, const double u[6]) {
    if constexpr (B32) {
      float v[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) v[m] = (float)u[m];
      ULf[f] = weno_is_f(v[0], v[1], v[2], v[3], v[4], eps32);
      URf[f] = weno_is_f(v[5], v[4], v[3], v[2], v[1], eps32);
    } else {
      UL[f] = weno_is(u[0], u[1], u[2], u[3], u[4], a.tol.weno_eps);
      UR[f] = weno_is(u[5], u[4], u[3], u[2], u[1], a.tol.weno_eps);
    }
  };
  double ra[6], rb[6], rc[6];   // raw node values of the group being formed
  phase_barrier();
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    NodeQ q;
    ld(m, q);
    ra[m] = q.un;
    rb[m] = q.p;
  }
  {
    // group (a1r1, a2r2, p) loaded ahead
    double na[6], nb[6], np[6];
    phase_barrier();
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      NodeQ q;
      ld(m, q);
      na[m] = q.w[0];
      nb[m] = q.w[1];
      np[m] = q.p;
    }
    double u0[6], u5[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      u0[m] = ra[m] - rb[m] * k1;
      u5[m] = ra[m] + rb[m] * k1;
    }
    weno_pair(0, u0);
    weno_pair(5, u5);
#pragma unroll
    for (int m = 0; m < 6; ++m) { ra[m] = na[m]; rb[m] = nb[m]; rc[m] = np[m]; }
  }
  {
    // group (u_t, a1) loaded ahead
    double nt[6], nw[6];
    phase_barrier();
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      NodeQ q;
      ld(m, q);
      nt[m] = q.ut;
      nw[m] = q.w[5];
    }
    double u1[6], u2[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      u1[m] = ra[m] - fa1 * rc[m] * k2;
      u2[m] = rb[m] - fa2 * rc[m] * k2;
    }
    weno_pair(1, u1);
    weno_pair(2, u2);
    if (HAS_T) {
      weno_pair(3, nt);
    } else {
      UL[3] = 0.0; UR[3] = 0.0; ULf[3] = 0.0f; URf[3] = 0.0f;
    }
    weno_pair(4, nw);
  }
  phase_barrier();
  if constexpr (B32) {
    // back-projection V = R U in FP32 [App. A]
    const float c2f = 2.0f * (float)fc, fa1f = (float)fa1, fa2f = (float)fa2;
    const float half_rc = 0.5f * (float)frho * (float)fc;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const float* U = side == 0 ? ULf : URf;
      double* V = side == 0 ? UL : UR;   // reused as primitive storage
      float d = U[5] - U[0];
      V[0] = (double)(U[1] + fdivf(fa1f * d, c2f));
      V[1] = (double)(U[2] + fdivf(fa2f * d, c2f));
      V[2] = (double)(0.5f * (U[0] + U[5]));
      V[3] = (double)U[3];
      V[4] = (double)(half_rc * d);
      V[5] = (double)U[4];
    }
  }
  // back-projection V = R U, then V -> W [App. A; Sec. 2]
  double WL[6], WR[6];
  if constexpr (B32) {
    // FP64 conservative state (the energy needs FP64: Pi ~ 4e8 vs Gamma p)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double* V = side == 0 ? UL : UR;
      double* X = side == 0 ? WL : WR;
      double rho = V[0] + V[1];
      X[0] = V[0];
      X[1] = V[1];
      X[2] = rho * V[2];
      X[3] = HAS_T ? rho * V[3] : 0.0;
      double ke = HAS_T ? (V[2] * V[2] + V[3] * V[3]) : V[2] * V[2];
      X[4] = mix_gamma(e, V[5]) * V[4] + mix_pi(e, V[5]) + 0.5 * rho * ke;
      X[5] = V[5];
    }
  } else {
    double twoc = 2.0 * fc;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double* U = side == 0 ? UL : UR;
      double* X = side == 0 ? WL : WR;
      double d = U[5] - U[0];
      double a1r1 = U[1] + ddiv(fa1 * d, twoc);
      double a2r2 = U[2] + ddiv(fa2 * d, twoc);
      double un = 0.5 * (U[0] + U[5]);
      double ut = U[3];
      double p = 0.5 * frho * fc * d;
      double a1 = U[4];
      double rho = a1r1 + a2r2;
      X[0] = a1r1;
      X[1] = a2r2;
      X[2] = rho * un;
      X[3] = HAS_T ? rho * ut : 0.0;
      double ke = HAS_T ? (un * un + ut * ut) : un * un;
      X[4] = mix_gamma(e, a1) * p + mix_pi(e, a1) + 0.5 * rho * ke;
      X[5] = a1;
    }
  }
  // interpolation limiter toward W_i (left value) and W_{i+1} (right value)
  if (a.interp_limiter) {
    NodeQ q;
    ld(2, q);
    interp_limit<HAS_T>(e, a.tol, q.w, q.h, WL);
    phase_barrier();
    ld(3, q);
    interp_limit<HAS_T>(e, a.tol, q.w, q.h, WR);
    phase_barrier();
  }
  // high-order midpoint flux from the limited states [WCNS step 6]
  // (p and c recovered in FP64; the flux itself in FP32 in the precision form)
  double acc[7];
  {
    NodeQ tl, tr;
#pragma unroll
    for (int v = 0; v < 6; ++v) { tl.w[v] = WL[v]; tr.w[v] = WR[v]; }
    recover<HAS_T>(e, tl.w, tl.un, tl.ut, tl.p, tl.c, tl.h);
    recover<HAS_T>(e, tr.w, tr.un, tr.ut, tr.p, tr.c, tr.h);
    if constexpr (B32) {
      NodeQf fl, fr;
#pragma unroll
      for (int v = 0; v < 6; ++v) { fl.w[v] = (float)tl.w[v]; fr.w[v] = (float)tr.w[v]; }
      fl.un = (float)tl.un; fl.ut = (float)tl.ut; fl.p = (float)tl.p; fl.c = (float)tl.c;
      fr.un = (float)tr.un; fr.ut = (float)tr.ut; fr.p = (float)tr.p; fr.c = (float)tr.c;
      HllcOutF h2;
      hllc_f<HAS_T>(fl, fr, h2);
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] = h2.F[v];
      acc[5] = h2.fa;
      acc[6] = h2.ss;
    } else {
      HllcOut h2;
      hllc<HAS_T>(tl, tr, h2);
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] = h2.F[v];
      acc[5] = h2.fa;
      acc[6] = h2.ss;
    }
  }
  // HCS reconstruction of flux and velocity [Sec. 4.1; WCNS steps 7-8]:
  // ((3072 gt - 505 s01) + 20 s12 - s03)/2100, node pairs s01 = (i, i+1),
  // s12 = (i-1, i+2), s03 = (i-2, i+3)
  float accf[7];
#pragma unroll
  for (int v = 0; v < 7; ++v) accf[v] = (float)acc[v];
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    phase_barrier();
    const int ma = 2 - pr, mb = 3 + pr;
    NodeQ qa, qb;
    ld(ma, qa);
    ld(mb, qb);
    double ga[6], gb[6];
    node_flux<HAS_T>(qa, ga);
    node_flux<HAS_T>(qb, gb);
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      if constexpr (B32) {
        float sum = v < 6 ? (float)ga[v] + (float)gb[v] : (float)qa.un + (float)qb.un;
        if (pr == 0) accf[v] = 3072.0f * accf[v] - 505.0f * sum;
        else if (pr == 1) accf[v] = accf[v] + 20.0f * sum;
        else accf[v] = (accf[v] - sum) * (1.0f / 2100.0f);
      } else {
        double sum = v < 6 ? ga[v] + gb[v] : qa.un + qb.un;
        if (pr == 0) acc[v] = 3072.0 * acc[v] - 505.0 * sum;
        else if (pr == 1) acc[v] = acc[v] + 20.0 * sum;
        else acc[v] = cdiv(acc[v] - sum, 2100.0, R2100);
      }
    }
  }
  if constexpr (B32) {
#pragma unroll
    for (int v = 0; v < 7; ++v) acc[v] = (double)accf[v];
  }
  const double uh = acc[6];
  // split fluxes G^{-+} [Sec. 3.2, WCNS step 9] and the flux limiter
  phase_barrier();
  NodeQ nl, nr;
  ld(2, nl);
  ld(3, nr);
#pragma unroll
  for (int v = 0; v < 5; ++v) { Gm[v] = acc[v]; Gp[v] = acc[v]; }
  Gm[5] = acc[5] - nl.w[5] * uh;
  Gp[5] = acc[5] - nr.w[5] * uh;
  if (a.flux_limiter) {
    double gl[6], gr[6];
    node_flux<HAS_T>(nl, gl);
    node_flux<HAS_T>(nr, gr);
    gl[5] = 0.0;
    gr[5] = 0.0;
    return flux_limit<HAS_T>(e, a.tol, nl.w, nr.w, gl, gr, lam, Hm, Hp, Gm, Gp);
  }
  return 1.0;
}

// Stencil nodes i-2 .. i+3 are g0 .. g0+5 along the line, read from global
// memory.
template <int DIR, bool HAS_T, bool DIRI, bool B32 = false>
__device__ __forceinline__ double face_flux(const KArgs& a, int line, int g0, double lam,
                                            double Gm[6], double Gp[6]) {
  const Sten st = make_sten<DIR>(a, line, g0);
  const GlobalLoad<DIR, HAS_T, DIRI> ld{&a, st, g0};
  return face_flux_core<DIR, HAS_T, B32>(a, ld, lam, Gm, Gp);
}

// map rotated flux component v of direction dir to the state index
__device__ __forceinline__ int state_index(int dir, int v, bool has_t) {
  if (!has_t) return v < 3 ? v : v - 1;      // 1D: (0,1,2,-,3,4)
  if (dir == 1 && (v == 2 || v == 3)) return 5 - v;
  return v;
}

// Neighbour lanes by DPP whole-wave shifts (a VALU move, no LDS round
// trip): from_next_lane gives lane L the value of lane L + 1 (lane 63 keeps
// its own), from_prev_lane the value of lane L - 1 (lane 0 keeps its own).
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  int lo = (int)(unsigned)u, hi = (int)(unsigned)(u >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double from_next_lane(double x) { return dpp_shift<0x130>(x); }   // wave_shl:1
__device__ __forceinline__ double from_prev_lane(double x) { return dpp_shift<0x138>(x); }   // wave_shr:1

// maximum over the 64 lanes of a wave
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// A state in the admissible set G [Sec. 2]: 0 <= a1 <= 1, a_k r_k >= 0 and
// h = rho e - pbar_inf > 0 (NaN fails every test).
__device__ __forceinline__ bool admissible(double a1r1, double a2r2, double a1, double h) {
  return a1 >= 0.0 && a1 <= 1.0 && a1r1 >= 0.0 && a2r2 >= 0.0 && h > 0.0;
}

// Lazy admissibility report: the cells of this wave with `bad` set are added
// to *viol and the host-visible flag is raised, by one lane and only when
// the wave has such a cell.
__device__ __forceinline__ void report_bad(unsigned long long* viol, int32_t* vflag, bool bad) {
  const unsigned long long m = __ballot(bad);
  if (m == 0ull) return;
  if ((int)(threadIdx.x & 63) == __ffsll((long long)m) - 1) {
    atomicAdd(viol, (unsigned long long)__popcll(m));
    if (vflag) __hip_atomic_store(vflag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// final write of one cell: L (store) or the SSP-RK3 combination [Sec. 4.1]
__device__ __forceinline__ double write_cell(const KArgs& a, double* dst, long idx, long N, int k,
                                             double L) {
  double v;
  if (a.out_mode == OUT_STORE) {
    v = L;
  } else {
    double dt = a.step[0];
    v = a.ca * a.Un[k * N + idx] + a.cb * (a.W[k * N + idx] + dt * L);
  }
  dst[k * N + idx] = v;
  return v;
}

// The inputs of one finished cell's write_cell, loaded ahead of use: L_x
// (2D) and (RK stage) U^n and W of the NC state components, and dt
struct CellIn {
  double lx[6], un[6], w[6], dt;
};
template <int NC = 6, bool LX = true>
__device__ __forceinline__ void load_cell_in(const KArgs& a, long idx, long N, CellIn& c) {
  if (LX) {
#pragma unroll
    for (int k = 0; k < NC; ++k) c.lx[k] = a.Lx[k * N + idx];
  }
  if (a.out_mode != OUT_STORE) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      c.un[k] = a.Un[k * N + idx];
      c.w[k] = a.W[k * N + idx];
    }
    c.dt = a.step[0];
  }
}
// write_cell on preloaded inputs (the same arithmetic)
__device__ __forceinline__ double write_cell_in(const KArgs& a, double* dst, long idx, long N, int k,
                                                double L, const CellIn& c) {
  const double v = a.out_mode == OUT_STORE ? L : a.ca * c.un[k] + a.cb * (c.w[k] + c.dt * L);
  dst[k * N + idx] = v;
  return v;
}

// Node primitives of a finished cell of the next stage's state X (state
// order) into a.Pn, and its wave speeds |u|+c, |v|+c into the running
// maxima: k_node's arithmetic [Sec. 2, 3.3] on the values just written.
// Returns whether X is admissible.
__device__ __forceinline__ bool next_prims(const KArgs& a, long idx, long N, const double X[6],
                                           double& mx, double& my) {
  double un, ut, p, c, h;
  recover<true>(a.eos, X, un, ut, p, c, h);
  double* P = a.Pn;
  P[idx] = un; P[N + idx] = ut; P[2 * N + idx] = p; P[3 * N + idx] = c; P[4 * N + idx] = h;
  mx = fmax(mx, fabs(un) + c);
  my = fmax(my, fabs(ut) + c);
  return admissible(X[0], X[1], X[5], h);
}

// Stage-result check of one finished 2D cell X (state order) when it is
// not made by next_prims: false if X lies outside G.
__device__ __forceinline__ bool stage_ok(const KArgs& a, const double X[6]) {
  return admissible(X[0], X[1], X[5], rhoc2_tilde<true>(a.eos, X));
}

// Block maxima of (mx, my) to out2[0], out2[1]; every thread of the block
// calls it (at most 16 waves).
__device__ __forceinline__ void block_max_out(double mx, double my, double* out2) {
  __shared__ double red[2][16];
  mx = wave_max(mx);
  my = wave_max(my);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { red[0][w] = mx; red[1][w] = my; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) { mx = fmax(mx, red[0][k]); my = fmax(my, red[1][k]); }
    out2[0] = mx;
    out2[1] = my;
  }
}

// ------------------------------------------------------------------ kernels
enum { DT_GIVEN = 0, DT_CFL = 1, DT_KEEP = 2 };

// Time step and directional split from the global maxima [Sec. 3.3]:
//   dt = CFL/(tau_x + tau_y), tau = max(|u|+c)/dx (1D: CFL dx/max(|u|+c)),
//   sigma_x = tau_x/(tau_x + tau_y), lambda_x = dt/(dx sigma_x) (1D: dt/dx).
struct FinArgs {
  int32_t ndim, dt_mode;
  double dx, dy, cfl, dt_in;
  double* step;       // step record (STEP_SKIP and the layout above)
  double* dt_used;    // optional copy of dt (0 for a skipped step)
  const double* damax;  // Dirichlet ghost maxima [2] or null
  // time loop to t_end (clock null: none): *clock is the time at the start
  // of the step, *nsteps (may be null) counts the steps taken
  double* clock;
  int64_t* nsteps;
  double t_end;
};

// The time loop's last step [Sec. 3.3 CFL step, shortened to land on
// t_end]: a step that would start at or after t_end is skipped; otherwise
// dt is clipped to t_end - t and the clock advanced.  Returns false for a
// skipped step.  (The order of the operations is that of the serial time
// loop.)  A step that would not advance the clock (dt not positive from an
// infinite wave speed, a NaN, or too small to change t) is skipped too, so
// the loop stops short of t_end instead of running on in place.
__device__ __forceinline__ bool clock_step(double* clock, int64_t* nsteps, double t_end, double& dt) {
  const double t = *clock;
  if (!(t < t_end)) return false;
  if (t + dt > t_end) dt = t_end - t;
  if (!(t + dt > t)) return false;
  *clock = t + dt;
  if (nsteps) *nsteps += 1;
  return true;
}

// Maxima over the per-block pairs (partial[2b], partial[2b+1]), b < nblk, of
// this thread's share: eight pairs per round with all loads issued together
// (fmax is exact, so the grouping does not change the result).
__device__ __forceinline__ void partial_max(const double* partial, int nblk, double& mx, double& my) {
  const double2* p2 = reinterpret_cast<const double2*>(partial);
  for (int b0 = threadIdx.x; b0 < nblk; b0 += 8 * (int)blockDim.x) {
    double2 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int b = b0 + k * (int)blockDim.x;
      v[k] = b < nblk ? p2[b] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      mx = fmax(mx, v[k].x);
      my = fmax(my, v[k].y);
    }
  }
}

// Node primitives (u, v, p, c, rho*ctilde^2) of every cell [Sec. 2] and the
// per-block wave-speed maxima.  (A last-block reduction here instead of
// k_finalize was measured 4x slower: its device-scope fence has to make the
// block's writes visible across the XCDs' separate L2s.)
template <bool HAS_T>
__global__ __launch_bounds__(256) void k_node(KArgs a, double* P, double* partial) {
  if (a.node_skip && a.step[STEP_SKIP] != 0.0) return;
  const long N = (long)a.nx * a.ny;
  const bool check = a.viol && a.check_in;
  double mx = 0.0, my = 0.0;
  for (long o = (long)blockIdx.x * blockDim.x + threadIdx.x; o < N;
       o += (long)gridDim.x * blockDim.x) {
    double X[6];
    if (HAS_T) {
#pragma unroll
      for (int k = 0; k < 6; ++k) X[k] = a.W[k * N + o];
    } else {
      X[0] = a.W[o]; X[1] = a.W[N + o]; X[2] = a.W[2 * N + o]; X[3] = 0.0;
      X[4] = a.W[3 * N + o]; X[5] = a.W[4 * N + o];
    }
    double un, ut, p, c, h;
    recover<HAS_T>(a.eos, X, un, ut, p, c, h);
    P[o] = un; P[N + o] = ut; P[2 * N + o] = p; P[3 * N + o] = c; P[4 * N + o] = h;
    mx = fmax(mx, fabs(un) + c);
    my = fmax(my, fabs(ut) + c);
    if (check) report_bad(a.viol, a.vflag, !admissible(X[0], X[1], X[5], h));
  }
  mx = wave_max(mx);
  my = wave_max(my);
  __shared__ double red[2][4];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { red[0][w] = mx; red[1][w] = my; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = red[0][0], a1v = red[1][0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) { a0 = fmax(a0, red[0][k]); a1v = fmax(a1v, red[1][k]); }
    partial[2 * blockIdx.x] = a0;
    partial[2 * blockIdx.x + 1] = a1v;
  }
}

// Global maxima -> dt, sigma and lambda in the device step record (one
// block), so a whole step needs no host round trip.
// (1024 threads: up to 8192 block maxima arrive in one round of loads)
__global__ __launch_bounds__(1024) void k_finalize(const double* partial, int nblk, FinArgs f) {
  double mx = 0.0, my = 0.0;
  partial_max(partial, nblk, mx, my);
  mx = wave_max(mx);
  my = wave_max(my);
  __shared__ double red[2][16];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { red[0][w] = mx; red[1][w] = my; }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { mx = fmax(mx, red[0][k]); my = fmax(my, red[1][k]); }
  if (f.damax) { mx = fmax(mx, f.damax[0]); my = fmax(my, f.damax[1]); }
  double* step = f.step;
  if (f.dt_mode == DT_KEEP && step[STEP_SKIP] != 0.0) return;   // inside a skipped step
  double dt;
  if (f.dt_mode == DT_GIVEN) dt = f.dt_in;
  else if (f.dt_mode == DT_KEEP) dt = step[0];
  else dt = f.ndim == 1 ? f.cfl * f.dx / mx : f.cfl / (mx / f.dx + my / f.dy);
  if (f.dt_mode != DT_KEEP) {
    const bool run = !f.clock || clock_step(f.clock, f.nsteps, f.t_end, dt);
    step[STEP_SKIP] = run ? 0.0 : 1.0;
    if (!run) {
      if (f.dt_used) *f.dt_used = 0.0;
      return;
    }
  }
  step[0] = dt;
  if (f.ndim == 1) {
    step[1] = dt / f.dx;
    step[2] = 0.0;
  } else {
    double tx = mx / f.dx, ty = my / f.dy;
    double sx = tx / (tx + ty), sy = ty / (tx + ty);
    step[1] = dt / (f.dx * sx);
    step[2] = dt / (f.dy * sy);
  }
  step[3] = mx;
  step[4] = my;
  if (f.dt_used) *f.dt_used = dt;
}

// Dirichlet ghost rows (one block): conservative states Wg (SoA [nvar][R],
// from k_prim_to_cons) -> unrotated 6-component rows dirW [R][6] and their
// node primitives dirP [R][5]; damax[d] = max(|u_d| + c) over the rows of
// the Dirichlet sides of direction d (0 when there are none), which the time
// step and lambda include [Sec. 3.3].
template <bool HAS_T>
__global__ __launch_bounds__(256) void k_dirichlet_rows(KArgs a, const double* Wg, int R,
                                                        double* dirW, double* dirP, double* damax) {
  double m[2] = {0.0, 0.0};
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    double X[6];
    X[0] = Wg[r];
    X[1] = Wg[R + r];
    X[2] = Wg[2 * R + r];
    X[3] = HAS_T ? Wg[3 * R + r] : 0.0;
    X[4] = Wg[(HAS_T ? 4 : 3) * R + r];
    X[5] = Wg[(HAS_T ? 5 : 4) * R + r];
#pragma unroll
    for (int k = 0; k < 6; ++k) dirW[r * 6 + k] = X[k];
    double un, ut, p, c, h;
    recover<HAS_T>(a.eos, X, un, ut, p, c, h);
    dirP[r * 5 + 0] = un; dirP[r * 5 + 1] = ut; dirP[r * 5 + 2] = p;
    dirP[r * 5 + 3] = c; dirP[r * 5 + 4] = h;
    int side = 3;
    while (side > 0 && r < a.dir_off[side]) --side;
    if (a.bc[side] == BC_DIRICHLET) {
      const int d = side >> 1;
      m[d] = fmax(m[d], fabs(d == 0 ? un : ut) + c);
    }
  }
  m[0] = wave_max(m[0]);
  m[1] = wave_max(m[1]);
  __shared__ double red[2][4];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { red[0][w] = m[0]; red[1][w] = m[1]; }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
    red[0][0] = fmax(red[0][0], red[0][k]);
    red[1][0] = fmax(red[1][0], red[1][k]);
  }
  damax[0] = red[0][0];
  damax[1] = red[1][0];
}

// One block of the node pass of one instance (batched form): cells
// [blk*256, blk*256 + 256), primitives to a.Pw, block maxima to partial[blk].
template <bool HAS_T>
__device__ __forceinline__ void node_block(const KArgs& a, int blk) {
  const long N = (long)a.nx * a.ny;
  const long o = (long)blk * blockDim.x + threadIdx.x;
  double mx = 0.0, my = 0.0;
  bool bad = false;
  if (o < N) {
    double X[6];
    if (HAS_T) {
#pragma unroll
      for (int k = 0; k < 6; ++k) X[k] = a.W[k * N + o];
    } else {
      X[0] = a.W[o]; X[1] = a.W[N + o]; X[2] = a.W[2 * N + o]; X[3] = 0.0;
      X[4] = a.W[3 * N + o]; X[5] = a.W[4 * N + o];
    }
    double un, ut, p, c, h;
    recover<HAS_T>(a.eos, X, un, ut, p, c, h);
    double* P = a.Pw;
    P[o] = un; P[N + o] = ut; P[2 * N + o] = p; P[3 * N + o] = c; P[4 * N + o] = h;
    mx = fabs(un) + c;
    my = fabs(ut) + c;
    bad = !admissible(X[0], X[1], X[5], h);
  }
  if (a.viol && a.check_in) report_bad(a.viol, a.vflag, bad);
  mx = wave_max(mx);
  my = wave_max(my);
  __shared__ double red[2][4];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { red[0][w] = mx; red[1][w] = my; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = red[0][0], a1v = red[1][0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) { a0 = fmax(a0, red[0][k]); a1v = fmax(a1v, red[1][k]); }
    a.partial[2 * blk] = a0;
    a.partial[2 * blk + 1] = a1v;
  }
}

// dt, sigma, lambda of one instance from its block maxima (one block)
__device__ __forceinline__ void finalize_inst(const KArgs& a) {
  double mx = 0.0, my = 0.0;
  partial_max(a.partial, a.nblk, mx, my);
  mx = wave_max(mx);
  my = wave_max(my);
  __shared__ double red[2][4];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { red[0][w] = mx; red[1][w] = my; }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < 4; ++k) { mx = fmax(mx, red[0][k]); my = fmax(my, red[1][k]); }
  double* step = (double*)a.step;
  double dt;
  if (a.dt_mode == DT_GIVEN) dt = a.dt_in;
  else if (a.dt_mode == DT_KEEP) dt = step[0];
  else dt = a.ndim == 1 ? a.cfl * a.dx / mx : a.cfl / (mx / a.dx + my / a.dy);
  step[0] = dt;
  if (a.ndim == 1) {
    step[1] = dt / a.dx;
    step[2] = 0.0;
  } else {
    double tx = mx / a.dx, ty = my / a.dy;
    double sx = tx / (tx + ty), sy = ty / (tx + ty);
    step[1] = dt / (a.dx * sx);
    step[2] = dt / (a.dy * sy);
  }
  step[3] = mx;
  step[4] = my;
  if (a.dt_used) *a.dt_used = dt;
}

// x-sweep: one wave per tile of tile_x flattened cells.  Lane t < T owns the
// left face of cell c0+t; lanes T.. own the right face of each row segment's
// last cell.  Cell c0+t then takes G^+ of its own face and G^- of the lane
// that owns its right face.
template <bool HAS_T, bool DIRI, bool B32>
__device__ __forceinline__ void sweep_x_tile(const KArgs& a, long tile) {
  const int lane = threadIdx.x;
  const int nx = a.nx;
  const long N = (long)nx * a.ny;
  const int T = a.tile_x;
  const long c0 = tile * T;
  const long c1 = (c0 + T < N ? c0 + T : N) - 1;
  const int j0 = (int)(c0 / nx), j1 = (int)(c1 / nx);
  int fj = 0, fk = 0;
  bool active = false;
  if (lane < T) {
    long c = c0 + lane;
    if (c <= c1) { fj = (int)(c / nx); fk = (int)(c % nx); active = true; }
  } else {
    int r = lane - T;
    if (j0 + r <= j1) {
      fj = j0 + r;
      long last = (fj == j1) ? c1 : (long)fj * nx + nx - 1;
      fk = (int)(last % nx) + 1;
      active = true;
    }
  }
  double Gm[6] = {0, 0, 0, 0, 0, 0}, Gp[6] = {0, 0, 0, 0, 0, 0};
  if (active) face_flux<0, HAS_T, DIRI, B32>(a, fj, fk - 3, a.step[1], Gm, Gp);
  // lane holding the right face of my cell
  int src = lane;
  const long c = c0 + lane;
  const bool owns_cell = lane < T && c <= c1;
  if (owns_cell) {
    const int cj = (int)(c / nx);
    src = (c == c1 || (c % nx) == nx - 1) ? T + (cj - j0) : lane + 1;
  }
  double Gr[6];
#pragma unroll
  for (int v = 0; v < 6; ++v) Gr[v] = __shfl(Gm[v], src, 64);
  if (!owns_cell) return;
  double* dst = (!HAS_T || a.Lout == nullptr) ? a.out : a.Lout;
  double X[6] = {0, 0, 0, 0, 0, 0};   // 1D: the stage result, in the rotated order
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    if (!HAS_T && v == 3) continue;
    const double L = hdiv(-(Gr[v] - Gp[v]), a.dx, a.rdx);
    const int k = state_index(0, v, HAS_T);
    if (HAS_T) {
      dst[k * N + c] = L;   // L_x; the y-sweep finishes the cell
    } else {
      X[v] = write_cell(a, a.out, c, N, k, L);
    }
  }
  if (!HAS_T && a.viol && a.out_mode == OUT_RK)
    report_bad(a.viol, a.vflag, !admissible(X[0], X[1], X[5], rhoc2_tilde<false>(a.eos, X)));
}

template <bool HAS_T, bool DIRI, bool B32>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_sweep_x(KArgs a) {
  if (a.step[STEP_SKIP] != 0.0) return;
  sweep_x_tile<HAS_T, DIRI, B32>(a, blockIdx.x);
}

// x-sweep with each wave's stencil window staged in LDS.  Waves take
// flattened (row-major) tiles of XT = 62 cells, which touch at most two rows
// when nx >= XLDS_MIN_NX.  The window holds 11 values (state and node
// primitives) per slot, ghost cells mapped while staging:
//   segment A, first row j0: faces k0 .. eA (nA faces), cells k0-3 .. eA+2 in
//              slots 0 .. nA+4;
//   segment B, row j0+1 when the tile crosses a row end: faces 0 .. eB (nB
//              faces), cells -3 .. eB+2 in slots nA+5 .. nA+nB+9.
// Lane L < nA computes face k0+L from slots L .. L+5, lane nA <= L < nA+nB
// face L-nA of row j0+1 from slots L+5 .. L+10.  A lane that does not hold
// the last face of its row owns the cell to the right of its face, whose
// right face is on lane L+1.
constexpr int XW = 4, XT = 62, XWIN = XT + 12, XLDS_MIN_NX = 61;

template <bool HAS_T>
struct LdsLoadX {
  const double* win;   // this wave's window [11][XWIN]
  int base;            // slot of the face's first stencil node
  __device__ __forceinline__ void operator()(int m, NodeQ& q) const {
    const double* t = win + base + m;
    q.w[0] = t[0];
    q.w[1] = t[XWIN];
    q.w[2] = t[2 * XWIN];
    q.w[3] = HAS_T ? t[3 * XWIN] : 0.0;
    q.w[4] = t[4 * XWIN];
    q.w[5] = t[5 * XWIN];
    q.un = t[6 * XWIN];
    q.ut = HAS_T ? t[7 * XWIN] : 0.0;
    q.p = t[8 * XWIN];
    q.c = t[9 * XWIN];
    q.h = t[10 * XWIN];
  }
};

// LDS written by this wave is visible to all its lanes, without waiting
// for the other waves of the block (for LDS only this wave uses)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Geometry of window tile `tile` over N cells in rows of nx (nx >= XLDS_MIN_NX)
struct XWin {
  long c0;
  int j0, k0, nA, nB, slots;
  // row and in-row position (ghosts -3 .. nx+2) of window slot sl < slots
  __device__ __forceinline__ void slot_cell(int sl, int& j, int& g) const {
    const bool segA = sl < nA + 5;
    j = segA ? j0 : j0 + 1;
    g = segA ? k0 - 3 + sl : sl - nA - 8;
  }
  // first stencil slot of the face on lane L < nA + nB
  __device__ __forceinline__ int base(int L) const { return L < nA ? L : L + 5; }
  // lane L owns the cell right of its face (flat index cell(L)); its right face is on L + 1
  __device__ __forceinline__ bool owner(int L) const { return L < nA - 1 || (L >= nA && L < nA + nB - 1); }
  __device__ __forceinline__ long cell(int L) const { return c0 + (L < nA ? L : L - 1); }
};

__device__ __forceinline__ XWin x_window(int nx, long N, long tile) {
  XWin t;
  t.c0 = tile * XT;
  const long c1 = (t.c0 + XT < N ? t.c0 + XT : N) - 1;
  t.j0 = (int)(t.c0 / nx);
  t.k0 = (int)(t.c0 - (long)t.j0 * nx);
  const int j1 = (int)(c1 / nx);
  const int e1 = (int)(c1 - (long)j1 * nx) + 1;   // last face of the tile in row j1
  if (j1 == t.j0) {
    t.nA = e1 - t.k0 + 1;
    t.nB = 0;
  } else {
    t.nA = nx - t.k0 + 1;
    t.nB = e1 + 1;
  }
  t.slots = t.nA + 5 + (t.nB > 0 ? t.nB + 5 : 0);
  return t;
}

// One tile per wave (`on` false: the wave has no tile and writes nothing).
template <bool HAS_T, bool DIRI, bool B32, bool FO = false>
__device__ __forceinline__ void sweep_x_window(const KArgs& a, long tile, bool on, double* win) {
  const int lane = threadIdx.x & 63;
  const int nx = a.nx;
  const long N = (long)nx * a.ny;
  XWin t{};
  if (on) {
    t = x_window(nx, N, tile);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int sl = lane + 64 * q;
      if (sl < t.slots) {
        int j, g;
        t.slot_cell(sl, j, g);
        bool flip;
        const int src = ghost_src(g, nx, a.bc[0], a.bc[1], flip);
        double v[11];
        if (DIRI && src < 0) {
          const int r = a.dir_off[g < 0 ? 0 : 1] + j;
#pragma unroll
          for (int c = 0; c < 6; ++c) v[c] = a.dirW[r * 6 + c];
#pragma unroll
          for (int c = 0; c < 5; ++c) v[6 + c] = a.dirP[r * 5 + c];
        } else {
          const uint32_t o = ((uint32_t)j * (uint32_t)nx + (uint32_t)src) * 8u;
#pragma unroll
          for (int c = 0; c < 6; ++c) v[c] = (!HAS_T && c == 3) ? 0.0 : ldc(a.Wc[c], o);
#pragma unroll
          for (int c = 0; c < 5; ++c) v[6 + c] = (!HAS_T && c == 1) ? 0.0 : ldc(a.Pc[c], o);
        }
        if (flip) { v[2] = -v[2]; v[6] = -v[6]; }   // rho u and u change sign at the wall
#pragma unroll
        for (int c = 0; c < 11; ++c) win[c * XWIN + sl] = v[c];
      }
    }
  }
  wave_lds_sync();   // the window is this wave's own
  const bool active = lane < t.nA + t.nB;
  double Gm[6] = {0, 0, 0, 0, 0, 0}, Gp[6] = {0, 0, 0, 0, 0, 0};
  if (active) {
    const LdsLoadX<HAS_T> ld{win, t.base(lane)};
    face_flux_core<0, HAS_T, B32, FO>(a, ld, a.step[1], Gm, Gp);
  }
  double Gr[6];   // (lane 63 owns no cell)
#pragma unroll
  for (int v = 0; v < 6; ++v) Gr[v] = from_next_lane(Gm[v]);
  if (!t.owner(lane)) return;
  const long c = t.cell(lane);
  double* dst = (!HAS_T || a.Lout == nullptr) ? a.out : a.Lout;
  CellIn cin;   // 1D: the stage's inputs, loaded before the first store
  if (!HAS_T) load_cell_in<5, false>(a, c, N, cin);
  double X[6] = {0, 0, 0, 0, 0, 0};   // 1D: the stage result, in the rotated order
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    if (!HAS_T && v == 3) continue;
    const double L = hdiv(-(Gr[v] - Gp[v]), a.dx, a.rdx);
    const int k = state_index(0, v, HAS_T);
    if (HAS_T) dst[k * N + c] = L;
    else X[v] = write_cell_in(a, a.out, c, N, k, L, cin);
  }
  if (!HAS_T && a.viol && a.out_mode == OUT_RK)
    report_bad(a.viol, a.vflag, !admissible(X[0], X[1], X[5], rhoc2_tilde<false>(a.eos, X)));
}

// waves per SIMD the windowed x-sweep is compiled for (VGPR budget 512 / this):
// 4 (110 VGPRs, no spills; compiled for 5 it spills and runs 2% slower)
constexpr int XL_WPE = 4;
// (FO: the first-order scheme, memory-bound: six waves per SIMD, the most
// the LDS windows allow)
template <bool HAS_T, bool DIRI, bool B32, bool FO = false>
__global__ __launch_bounds__(64 * XW) __attribute__((amdgpu_waves_per_eu(FO ? 6 : XL_WPE))) void k_sweep_xl(
    KArgs a) {
  if (a.step[STEP_SKIP] != 0.0) return;
  __shared__ double tile[XW][11 * XWIN];
  const int w = threadIdx.x >> 6;
  const long t = (long)blockIdx.x * XW + w;
  const long N = (long)a.nx * a.ny;
  sweep_x_window<HAS_T, DIRI, B32, FO>(a, t, t * XT < N, tile[w]);
}

// The y-tile on 32 columns: a block of FR/2 waves covers 32 columns x FR
// face rows; lane (r = lane / 32, col = lane % 32) of wave w computes face
// row kb + 2w + r.  Stencil rows kb-3 .. kb+FR+1 are staged first (9 values
// per node; c and rho ctilde^2 of the two centre nodes are read from global
// memory into registers).  Cell row kb + 2w takes G^- of face row
// kb + 2w + 1 from lane + 32 of its own wave (shuffle); cell row kb + 2w + 1
// takes it from wave w + 1 through LDS; the tile's first G^- and last G^+
// go to the edge buffer for the fixup.  The single-grid sweep uses 16 face
// rows (two 8-wave blocks per CU, half the fixup rows of 8-row tiles); the
// batched form instantiates 2 to 16.
// (part: this block's slot for its block maxima when a.Pn is set)
template <int FR, bool DIRI, bool B32>
__device__ __forceinline__ void sweep_y_tile32(const KArgs& a, int bx, int by, double* tile, long part) {
  constexpr int W = FR / 2;
  constexpr int ROWS = FR + 5;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane >> 5, col = lane & 31;
  const int i = bx * 32 + col;
  const int kb = by * FR;
  const int fr = 2 * w + r;
  const int k = kb + fr;
  const int nx = a.nx, ny = a.ny;
  const long N = (long)nx * ny;
  // stage: slot t = thread + 64W q holds tile row t / 32, column t % 32
#pragma unroll
  for (int q = 0; q < (ROWS * 32 + 64 * W - 1) / (64 * W); ++q) {
    const int t = (int)threadIdx.x + 64 * W * q;
    const int tr = t >> 5, ii = bx * 32 + (t & 31);
    const int g = kb - 3 + tr;
    if (tr < ROWS && g <= ny + 2 && ii < nx) {
      bool flip;
      const int s = ghost_src(g, ny, a.bc[2], a.bc[3], flip);
      double v[9];
      if (DIRI && s < 0) {
        const int rr = a.dir_off[g < 0 ? 2 : 3] + ii;
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = a.dirW[rr * 6 + c];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[6 + c] = a.dirP[rr * 5 + c];
      } else {
        const uint32_t o = ((uint32_t)s * (uint32_t)nx + (uint32_t)ii) * 8u;
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = ldc(a.Wc[c], o);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[6 + c] = ldc(a.Pc[c], o);
      }
      if (flip) { v[3] = -v[3]; v[7] = -v[7]; }   // rho v and v change sign at the wall
#pragma unroll
      for (int c = 0; c < 9; ++c) tile[(c * ROWS + tr) * 32 + (t & 31)] = v[c];
    }
  }
  __syncthreads();
  const bool active = i < nx && k <= ny;
  double Gm[6] = {0, 0, 0, 0, 0, 0}, Gp[6] = {0, 0, 0, 0, 0, 0};
  if (active) {
    LdsLoadY ld{tile, ROWS, fr, col};
#pragma unroll
    for (int q = 0; q < 2; ++q) {   // c and rho ctilde^2 of cell rows k-1 and k
      const int g = k - 1 + q;
      bool flip;
      const int s = ghost_src(g, ny, a.bc[2], a.bc[3], flip);
      double c, h;
      if (DIRI && s < 0) {
        const int rr = a.dir_off[g < 0 ? 2 : 3] + i;
        c = a.dirP[rr * 5 + 3];
        h = a.dirP[rr * 5 + 4];
      } else {
        const uint32_t o = ((uint32_t)s * (uint32_t)nx + (uint32_t)i) * 8u;
        c = ldc(a.Pc[3], o);
        h = ldc(a.Pc[4], o);
      }
      if (q == 0) { ld.c2 = c; ld.h2 = h; } else { ld.c3 = c; ld.h3 = h; }
    }
    face_flux_core<1, true, B32>(a, ld, a.step[2], Gm, Gp);
  }
  // the owned cell's L_x, U^n and W, loaded while the block exchanges G^-
  const bool own = active && fr != FR - 1 && k < ny;
  const long idx = (long)k * nx + i;
  CellIn cin;
  if (own) load_cell_in(a, idx, N, cin);
  double Gn[6];   // G^- of face row k + 1 when r == 0 (same wave, upper half)
#pragma unroll
  for (int v = 0; v < 6; ++v) Gn[v] = __shfl(Gm[v], (lane + 32) & 63, 64);
  __syncthreads();   // every face has read the tile: reuse it for G^-
  double* sG = tile;   // [W][6][32]: G^- of each wave's lower face row
  if (r == 0) {
#pragma unroll
    for (int v = 0; v < 6; ++v) sG[(w * 6 + v) * 32 + col] = Gm[v];
  }
  if (active) {
    double* e = a.edge + (long)by * 12 * nx;
    if (fr == 0) {
#pragma unroll
      for (int v = 0; v < 6; ++v) e[v * nx + i] = Gm[v];
    }
    if (fr == FR - 1 || k == ny) {
#pragma unroll
      for (int v = 0; v < 6; ++v) e[(6 + v) * nx + i] = Gp[v];
    }
  }
  __syncthreads();
  double mx = 0.0, my = 0.0;
  bool bad = false;
  if (own) {
    double X[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) {
      const int s = state_index(1, v, true);
      double L;
      {
        const double up = r == 0 ? Gn[v] : sG[((w + 1) * 6 + v) * 32 + col];
        double Ly = hdiv(-(up - Gp[v]), a.dy, a.rdy);
        L = cin.lx[s] + Ly;
      }
      X[s] = write_cell_in(a, a.out, idx, N, s, L, cin);
    }
    if (a.Pn) bad = !next_prims(a, idx, N, X, mx, my);
    else if (a.viol && a.out_mode == OUT_RK) bad = !stage_ok(a, X);
  }
  if (a.viol && a.out_mode == OUT_RK) report_bad(a.viol, a.vflag, bad);
  if (a.Pn) block_max_out(mx, my, a.partn + 2 * part);
}

// (the first-order scheme in 2D runs k_fo_stage instead)
template <bool DIRI, bool B32>
__global__ __launch_bounds__(Y_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_y(
    KArgs a) {
  if (a.step[STEP_SKIP] != 0.0) return;
  __shared__ double tile32[9 * (Y_ROWS + 5) * Y_COLS];
  sweep_y_tile32<Y_ROWS, DIRI, B32>(a, blockIdx.x, blockIdx.y, tile32,
                                        (long)blockIdx.y * gridDim.x + blockIdx.x);
}

// cell rows j = (b+1)*YW - 1 between y-tile b and b+1 (t: flat index over
// the boundary rows of one instance)
// (returns false for t past the boundary rows; else the cell's flat index
// and the values written, in state order)
__device__ __forceinline__ bool fixup_cell(const KArgs& a, long t, int yw, long& idx, double X[6]) {
  const int nx = a.nx, ny = a.ny;
  const long N = (long)nx * ny;
  const int b = (int)(t / nx), i = (int)(t % nx);
  if (b >= a.nbr - 1) return false;
  const int j = (b + 1) * yw - 1;
  if (j >= ny) return false;
  const double* lo = a.edge + (long)b * 12 * nx + 6 * nx;       // G^+ of face row j
  const double* hi = a.edge + (long)(b + 1) * 12 * nx;          // G^- of face row j+1
  idx = (long)j * nx + i;
  // every input first: a store to a.out may alias a later load, so loads
  // left between the stores would each wait for the one before
  double gl[6], gh[6];
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    gl[v] = lo[v * nx + i];
    gh[v] = hi[v * nx + i];
  }
  CellIn cin;
  load_cell_in(a, idx, N, cin);
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    const int s = state_index(1, v, true);
    double L;
    {
      double Ly = hdiv(-(gh[v] - gl[v]), a.dy, a.rdy);
      L = cin.lx[s] + Ly;
    }
    X[s] = write_cell_in(a, a.out, idx, N, s, L, cin);
  }
  return true;
}

// the fixup's stage-result check and next-stage primitives (blk: this
// block's slot after fuse_off for its block maxima)
__device__ __forceinline__ void fixup_finish(const KArgs& a, bool own, long idx, const double X[6],
                                             long blk) {
  double mx = 0.0, my = 0.0;
  bool bad = false;
  if (own) {
    if (a.Pn) bad = !next_prims(a, idx, (long)a.nx * a.ny, X, mx, my);
    else if (a.viol && a.out_mode == OUT_RK) bad = !stage_ok(a, X);
  }
  if (a.viol && a.out_mode == OUT_RK) report_bad(a.viol, a.vflag, bad);
  if (a.Pn) block_max_out(mx, my, a.partn + 2 * ((long)a.fuse_off + blk));
}

__global__ __launch_bounds__(256) void k_fixup_y(KArgs a) {
  if (a.step[STEP_SKIP] != 0.0) return;
  long idx = 0;
  double X[6];
  const bool own = fixup_cell(a, (long)blockIdx.x * blockDim.x + threadIdx.x, Y_ROWS, idx, X);
  fixup_finish(a, own, idx, X, blockIdx.x);
}

// Stand-alone flux limiter over the faces of one direction.
template <bool HAS_T>
__global__ __launch_bounds__(256) void k_limit(KArgs a, int dir, const double* Gho,
                                               const double* Glo, double* Gout, double* theta) {
  const int nx = a.nx, ny = a.ny;
  const long nf = dir == 0 ? (long)(nx + 1) * ny : (long)nx * (ny + 1);
  const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int line, k;
  if (dir == 0) { line = (int)(f / (nx + 1)); k = (int)(f % (nx + 1)); }
  else { k = (int)(f / nx); line = (int)(f % nx); }
  NodeQ nl, nr;
  if (dir == 0) {
    const Sten st = make_sten<0>(a, line, k - 3);
    load_node<0, HAS_T, true>(a, st, 2, k - 3, nl);
    load_node<0, HAS_T, true>(a, st, 3, k - 3, nr);
  } else {
    const Sten st = make_sten<1>(a, line, k - 3);
    load_node<1, HAS_T, true>(a, st, 2, k - 3, nl);
    load_node<1, HAS_T, true>(a, st, 3, k - 3, nr);
  }
  const int nv = HAS_T ? 6 : 5;
  double Gh[6], Hh[6];
  double uh = Gho[(long)nv * nf + f], uhh = Glo[(long)nv * nf + f];
  for (int v = 0; v < 6; ++v) {
    if (!HAS_T && v == 3) { Gh[v] = 0.0; Hh[v] = 0.0; continue; }
    const int s = state_index(dir, v, HAS_T);
    Gh[v] = Gho[(long)s * nf + f];
    Hh[v] = Glo[(long)s * nf + f];
  }
  double Gm[6], Gp[6], Hm[6], Hp[6];
  for (int v = 0; v < 5; ++v) { Gm[v] = Gh[v]; Gp[v] = Gh[v]; Hm[v] = Hh[v]; Hp[v] = Hh[v]; }
  {
    Gm[5] = Gh[5] - nl.w[5] * uh;
    Gp[5] = Gh[5] - nr.w[5] * uh;
    Hm[5] = Hh[5] - nl.w[5] * uhh;
    Hp[5] = Hh[5] - nr.w[5] * uhh;
  }
  double gl[6], gr[6];
  node_flux<HAS_T>(nl, gl);
  node_flux<HAS_T>(nr, gr);
  gl[5] = 0.0;
  gr[5] = 0.0;
  double lam = a.step[1 + dir];
  double th = flux_limit<HAS_T>(a.eos, a.tol, nl.w, nr.w, gl, gr, lam, Hm, Hp, Gm, Gp);
  for (int v = 0; v < 6; ++v) {
    if (!HAS_T && v == 3) continue;
    const int s = state_index(dir, v, HAS_T);
    Gout[(long)s * nf + f] = Gm[v];
    Gout[(long)(nv + s) * nf + f] = Gp[v];
  }
  if (theta) theta[f] = th;
}

// V (a1r1, a2r2, u, [v], p, a1) -> W  [Sec. 2 mixture EOS]
template <bool HAS_T>
__global__ __launch_bounds__(256) void k_prim_to_cons(KArgs a, const double* V, double* W) {
  const long N = (long)a.nx * a.ny;
  const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  const int nv = HAS_T ? 6 : 5;
  double a1r1 = V[o], a2r2 = V[N + o], u = V[2 * N + o];
  double v = HAS_T ? V[3 * N + o] : 0.0;
  double p = V[(nv - 2) * N + o], a1 = V[(nv - 1) * N + o];
  double rho = a1r1 + a2r2;
  W[o] = a1r1;
  W[N + o] = a2r2;
  W[2 * N + o] = rho * u;
  if (HAS_T) W[3 * N + o] = rho * v;
  double ke = HAS_T ? (u * u + v * v) : u * u;
  W[(nv - 2) * N + o] = mix_gamma(a.eos, a1) * p + mix_pi(a.eos, a1) + 0.5 * rho * ke;
  W[(nv - 1) * N + o] = a1;
}

// Admissible set G [Sec. 2]; NaN fails every comparison and counts as bad.
template <bool HAS_T>
__global__ __launch_bounds__(256) void k_admissible(KArgs a, unsigned long long* count) {
  const long N = (long)a.nx * a.ny;
  unsigned long long bad = 0;
  for (long o = (long)blockIdx.x * blockDim.x + threadIdx.x; o < N;
       o += (long)gridDim.x * blockDim.x) {
    double X[6];
    if (HAS_T) {
      for (int k = 0; k < 6; ++k) X[k] = a.W[k * N + o];
    } else {
      X[0] = a.W[o]; X[1] = a.W[N + o]; X[2] = a.W[2 * N + o]; X[3] = 0.0;
      X[4] = a.W[3 * N + o]; X[5] = a.W[4 * N + o];
    }
    double h = rhoc2_tilde<HAS_T>(a.eos, X);
    bool ok = X[5] >= 0.0 && X[5] <= 1.0 && X[0] >= 0.0 && X[1] >= 0.0 && h > 0.0;
    bad += ok ? 0ull : 1ull;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(count, bad);
}

// Division self-test: the IEEE quotient as compiled (`/`) next to ddiv.
__global__ __launch_bounds__(256) void k_selftest_div(const double* a, const double* b, double* q_ieee,
                                                       double* q_core, long n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  q_ieee[t] = a[t] / b[t];
  q_core[t] = ddiv(a[t], b[t]);
}

// The same for one divisor b and its checked reciprocal y (cdiv).
__global__ __launch_bounds__(256) void k_selftest_cdiv(const double* a, double b, double y,
                                                        double* q_ieee, double* q_core, long n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  q_ieee[t] = a[t] / b;
  q_core[t] = cdiv(a[t], b, y);
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0ull;
}

__global__ __launch_bounds__(256) void k_copy_amax(const double* step, double* out, int ndim) {
  if (threadIdx.x == 0) { out[0] = step[3]; if (ndim == 2) out[1] = step[4]; }
}

}  // namespace wcns
