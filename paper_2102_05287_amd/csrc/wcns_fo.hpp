// First-order HLLC scheme (the paper's comparison scheme, Sec. 3; theta = 0
// in both limiters) as one pass per SSP-RK3 stage in 2D.
//
// The mode needs only the face HLLC flux of the two cells next to a face,
// so a stage is memory-bound: it reads U^(s) (and U^n) and writes U^(s+1),
// 96 or 144 B per cell.  One wave owns a strip of 62 columns (lanes 1..62;
// lanes 0 and 63 hold the halo columns) and marches through a block of rows
// of it plus a halo row on either side, keeping two rows of node values in
// registers and the next row's state in flight.  Per row it recovers the
// primitives (Sec. 2), computes the x-face fluxes of the row (the right
// neighbour's node from the next lane by a DPP shift) and the y-face flux
// between the previous row and this one, which finishes the previous row's
// cells: L = L_x + L_y and the stage combination, the same arithmetic in
// the same order as the two-pass kernels (x-sweep L_x, y-sweep L_x + L_y),
// so the results are those of the oracle bit for bit.  Nothing but the
// stage result goes to memory: no node primitives, no L_x, no tile edges.
// At the last stage of a step that is followed by another, each wave also
// reduces the wave speeds |u|+c, |v|+c of its finished cells (Sec. 3.3) for
// the next step's time step.
//
// The rows of a strip are split into nrb near-equal blocks so that the grid
// has about as many waves as the GPU holds at once (three per SIMD): one
// round, no tail.  Wave tasks are dealt so that the row blocks of a strip
// run on one XCD (block b runs on XCD b % 8), and neighbouring blocks march
// in opposite directions: a block's halo rows are its neighbours' edge rows,
// read by both at about the same time and so found in that XCD's L2.
#pragma once
#include "wcns_kernels.hpp"

#pragma clang fp contract(off)

namespace wcns {

constexpr int FO_LANES = 62;     // owned columns per wave
constexpr int FO_WAVES = 4;      // waves per block
constexpr int FO_WPE = 3;        // waves per SIMD the kernel is compiled for
constexpr int FO_SINK_SLOTS = 1024;   // 8-double slots of the sink for lanes that write no cell
// (a four-wave budget of 128 VGPRs spills 108-224 B per lane)

// Column of a lane: its source column sx after the x ghost mapping (-1: an
// x-side Dirichlet ghost) and whether the wall-normal momentum flips.
struct FoCol {
  int c, sx;
  bool fx;
};

// State of node (column col.c in -1..nx, row g in -1..ny) as stored: ghosts
// mapped as in the sweeps, corner ghosts, which no face uses, clamped.
// (Only rows -1 and ny need the y mapping.)  One load per component for
// every lane, Dirichlet ghosts included, and no use of the values here
// (the wall flips are applied by fo_flip where the state is used): the
// loads of a row stay in flight while the previous row is computed.
template <bool DIRI>
__device__ __forceinline__ void fo_load(const KArgs& a, const FoCol& col, int g, double X[6]) {
  int sx = col.sx, sy = g;
  bool fy;
  if (g < 0 || g >= a.ny) sy = ghost_src(g, a.ny, a.bc[2], a.bc[3], fy);
  if (DIRI) {
    const bool gx = sx < 0 && sy >= 0;   // an x-side Dirichlet ghost
    const bool gy = sy < 0 && sx >= 0;   // a y-side one
    const long drow = gx ? (long)a.dir_off[col.c < 0 ? 0 : 1] + sy : (long)a.dir_off[g < 0 ? 2 : 3] + sx;
    if (sx < 0) sx = col.c < 0 ? 0 : a.nx - 1;
    if (sy < 0) sy = g < 0 ? 0 : a.ny - 1;
    const bool d = gx || gy;
    const double* src = d ? a.dirW + drow * 6 : a.W + ((long)sy * a.nx + sx);
    const long stride = d ? 1 : (long)a.nx * a.ny;
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = src[k * stride];
  } else {
    const uint32_t o = ((uint32_t)sy * (uint32_t)a.nx + (uint32_t)sx) * 8u;
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = ldc(a.Wc[k], o);
  }
}

// the wall flips of node (col, g): reflective ghosts negate the wall-normal
// momentum
__device__ __forceinline__ void fo_flip(const KArgs& a, const FoCol& col, int g, double X[6]) {
  bool fy = false;
  if (g < 0 || g >= a.ny) (void)ghost_src(g, a.ny, a.bc[2], a.bc[3], fy);
  if (col.fx) X[2] = -X[2];
  if (fy) X[3] = -X[3];
}

// the node of a loaded state: the state and its primitives [Sec. 2]
__device__ __forceinline__ void fo_node(const KArgs& a, const double X[6], NodeQ& q) {
#pragma unroll
  for (int k = 0; k < 6; ++k) q.w[k] = X[k];
  recover<true>(a.eos, X, q.un, q.ut, q.p, q.c, q.h);
}

// the node in the y frame (normal momentum rho v)
__device__ __forceinline__ NodeQ fo_yframe(const NodeQ& q) {
  NodeQ r = q;
  r.w[2] = q.w[3];
  r.w[3] = q.w[2];
  r.un = q.ut;
  r.ut = q.un;
  return r;
}

// split first-order HLLC fluxes H^- (alpha of the left cell), H^+ [Sec. 3.2]
__device__ __forceinline__ void fo_face(const NodeQ& l, const NodeQ& r, double Hm[6], double Hp[6]) {
  HllcOut h;
  hllc<true>(l, r, h);
#pragma unroll
  for (int v = 0; v < 5; ++v) { Hm[v] = h.F[v]; Hp[v] = h.F[v]; }
  Hm[5] = h.fa - l.w[5] * h.ss;
  Hp[5] = h.fa - r.w[5] * h.ss;
}

// the node of lane L + 1 (lane 63: its own, a face no cell uses)
__device__ __forceinline__ NodeQ next_lane_node(const NodeQ& q) {
  NodeQ r;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.w[k] = from_next_lane(q.w[k]);
  r.un = from_next_lane(q.un);
  r.ut = from_next_lane(q.ut);
  r.p = from_next_lane(q.p);
  r.c = from_next_lane(q.c);
  r.h = 0.0;
  return r;
}

// Cells of a wave outside G (nbad per lane) added to *viol, flag raised.
__device__ __forceinline__ void report_count(unsigned long long* viol, int32_t* vflag, int nbad) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) nbad += __shfl_xor(nbad, off, 64);
  if ((threadIdx.x & 63) == 0 && nbad > 0) {
    atomicAdd(viol, (unsigned long long)nbad);
    if (vflag) __hip_atomic_store(vflag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// One RK stage (or, out_mode OUT_STORE, the RHS) of the first-order scheme
// over waves of (strip, row block) tasks: strip = t % nstrip, row block
// rb = t / nstrip of nrb covering rows [rb ny / nrb, (rb + 1) ny / nrb).
// The grid is a multiple of 8 blocks.  USE_UN: an RK stage that combines
// with U^n (stages 2 and 3; stage 1 has ca = 0).  With a.partn set, the
// stage result's wave-speed maxima of wave t go to a.partn[2t], [2t+1].
//
// Every memory instruction of the row loop is issued by every lane with no
// branch around it: lanes that finish no cell of the row load a U^n value
// they do not use (a clamped cell, in cache) and write their stage values
// to the wave's slot of a.sink.  Vector memory operations complete in
// order, so a wait is counted back from the last operation issued; with no
// branch between them, the wait for this row's state does not also wait
// for the next row's loads or for this row's stores.
template <bool DIRI, bool USE_UN>
__global__ __launch_bounds__(64 * FO_WAVES) __attribute__((amdgpu_waves_per_eu(FO_WPE))) void k_fo_stage(
    KArgs a, int nstrip, int nrb, int ntask) {
  if (a.step[STEP_SKIP] != 0.0) return;
  const int lane = threadIdx.x & 63;
  // task of this wave: block b runs on XCD b % 8, so block rank
  // (b % 8) * per + b / 8 gives each XCD a contiguous range of tasks
  const int per = (int)gridDim.x / 8;
  const int b = blockIdx.x;
  const int bq = (b % 8) * per + b / 8;
  const int t = bq * FO_WAVES + (int)(threadIdx.x >> 6);
  const bool on = t < ntask;
  const int strip = on ? t % nstrip : 0;
  const int rb = on ? t / nstrip : 0;
  const int nx = a.nx, ny = a.ny;
  const long N = (long)nx * ny;
  const int c = strip * FO_LANES - 1 + lane;          // column of this lane (-1 .. )
  const int cc = c <= nx ? c : nx;                    // lanes past the halo repeat it
  const int cu = c < 0 ? 0 : (c < nx ? c : nx - 1);   // column of its U^n loads
  const int j0 = (int)((long)rb * ny / nrb);
  const int j1 = (int)((long)(rb + 1) * ny / nrb);    // first row of the next block
  const bool owner = on && lane >= 1 && lane <= FO_LANES && c < nx;
  const double dt = a.step[0];
  const bool rk = a.out_mode == OUT_RK;
  // admissibility: the stage's input cells (every stage result of a call
  // is the next stage's input) and, with check_out, its result
  const bool check_in = a.viol && a.check_in;
  const bool check_out = a.viol && a.check_out && rk;
  double* const sink = a.sink + (t & (FO_SINK_SLOTS - 1)) * 8;
  double mx = 0.0, my = 0.0;
  int nbad = 0;

  // Even row blocks march down (increasing rows), odd ones up, so that the
  // two blocks beside a block boundary read its rows at about the same time
  // (both first or both last) and the second read is served by the L2.
  // A march visits node rows first, first + dir, .., the halo row on one
  // side, the block's rows, the halo row on the other; at node row g the
  // y-face between rows g - dir and g finishes row g - dir.
  const int dir = (rb & 1) ? -1 : 1;
  const int first = dir > 0 ? j0 - 1 : j1;
  const int nit = on ? j1 - j0 + 1 : 0;

  // per lane, kept in LDS between rows (fewer live registers): L_x of the
  // previous row and the G^+ (marching down) or G^- (up) of its far y-face
  __shared__ double keep[FO_WAVES][2][6][64];
  double (*Lx_prev)[64] = keep[threadIdx.x >> 6][0];
  double (*G_prev)[64] = keep[threadIdx.x >> 6][1];
  FoCol col;
  col.c = cc;
  col.sx = ghost_src(cc, nx, a.bc[0], a.bc[1], col.fx);
  NodeQ prev;
  double X0[6], Xn[6];
  fo_load<DIRI>(a, col, first, X0);
  fo_load<DIRI>(a, col, first + dir, Xn);
  // six stores to the sink, as every row issues after its state's loads:
  // the first row's wait then counts the same as every other row's
  // (kept apart: six store instructions, not merged into wider ones)
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    sink[s] = 0.0;
    __asm__ volatile("" ::: "memory");
  }
  fo_flip(a, col, first, X0);
  fo_node(a, X0, prev);
  for (int k = 0; k < nit; ++k) {
    const int g = first + dir * (k + 1);
    NodeQ cur;
    fo_flip(a, col, g, Xn);
    fo_node(a, Xn, cur);
    const int r = g - dir;                 // the row this y-face finishes
    const bool fin = owner && k > 0;       // (r is a row of the block from k = 1 on)
    const long idx = (long)r * nx + c;
    // U^n of row r (k = 0: of row g, which the next row finishes), then the
    // next row's state (the last row: this one again), both in flight
    // while this row's y-face is computed
    double un[6];
    if (USE_UN) {
      int ur = k > 0 ? r : g;
      ur = ur < 0 ? 0 : (ur < ny ? ur : ny - 1);
      const long ui = (long)ur * nx + cu;
#pragma unroll
      for (int q = 0; q < 6; ++q) un[q] = a.Un[q * N + ui];
    }
    fo_load<DIRI>(a, col, k + 1 < nit ? g + dir : g, Xn);
    // y-face between the lower and the upper of rows r and g: row r takes
    // G^- of its upper face and G^+ of its lower face
    double Gm[6], Gp[6];
    if (dir > 0) fo_face(fo_yframe(prev), fo_yframe(cur), Gm, Gp);
    else fo_face(fo_yframe(cur), fo_yframe(prev), Gm, Gp);
    double X[6] = {0, 0, 0, 0, 0, 0};
    if (fin) {
#pragma unroll
      for (int v = 0; v < 6; ++v) {
        const int s = state_index(1, v, true);
        const double gu = dir > 0 ? Gm[v] : G_prev[v][lane];
        const double gd = dir > 0 ? G_prev[v][lane] : Gp[v];
        const double Ly = hdiv(-(gu - gd), a.dy, a.rdy);
        const double L = Lx_prev[s][lane] + Ly;
        X[s] = !rk ? L : (USE_UN ? a.ca * un[s] + a.cb * (prev.w[s] + dt * L)
                                 : a.cb * (prev.w[s] + dt * L));
      }
      if (a.partn) {
        double u, v, p, cs, h;
        recover<true>(a.eos, X, u, v, p, cs, h);
        mx = fmax(mx, fabs(u) + cs);
        my = fmax(my, fabs(v) + cs);
      }
      if (check_out) nbad += stage_ok(a, X) ? 0 : 1;
    }
    {
      double* const dst = fin ? a.out + idx : sink;
      const long st = fin ? N : 1;
#pragma unroll
      for (int s = 0; s < 6; ++s) dst[s * st] = X[s];
    }
#pragma unroll
    for (int v = 0; v < 6; ++v) G_prev[v][lane] = dir > 0 ? Gp[v] : Gm[v];
    // x-faces of row g (a row of this block): lane L holds face c + 1/2
    // (right neighbour by DPP lane shift); cell c takes G^+ of face c - 1/2
    // from lane L - 1
    if (g >= j0 && g < j1) {
      if (check_in && owner) nbad += admissible(cur.w[0], cur.w[1], cur.w[5], cur.h) ? 0 : 1;
      const NodeQ right = next_lane_node(cur);
      double Hm[6], Hp[6];
      fo_face(cur, right, Hm, Hp);
#pragma unroll
      for (int v = 0; v < 6; ++v) {
        const double gl = from_prev_lane(Hp[v]);   // (lane 0 owns no cell)
        Lx_prev[v][lane] = hdiv(-(Hm[v] - gl), a.dx, a.rdx);   // x frame = state order
      }
    }
    prev = cur;
  }
  if (check_in || check_out) report_count(a.viol, a.vflag, nbad);
  if (a.partn) {
    mx = wave_max(mx);
    my = wave_max(my);
    if (on && lane == 0) {
      a.partn[2 * t] = mx;
      a.partn[2 * t + 1] = my;
    }
  }
}

}  // namespace wcns
