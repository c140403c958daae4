// Whole runs of small 1D problems inside one workgroup.
//
// The paper's 1D experiments (Sec. 6.2-6.4: 200-401 cells, thousands of
// steps) are bound by launch latency when every SSP-RK3 stage is five
// launches.  Here one block of RUN1D_THREADS threads keeps the whole time
// loop on the device: per stage the node primitives and the wave-speed
// maximum (block reduction), the time step (CFL or fixed, the last one
// shortened to land on t_end) and lambda = dt/dx, every face of the line,
// then the flux difference and the stage combination, with block barriers
// between the phases.  The arithmetic of every phase is that of the
// multi-kernel path (the same device routines), so a run gives the same bits
// as stepping with wcns_ssprk3_step, and it counts the same cells outside the
// admissible set (the run's input and every stage result, Sec. 2).  A step
// that would not advance the time (an infinite wave speed) ends the run
// early.  A launch takes at most `chunk` steps and continues from the time
// and step count in its record, so a long run is a sequence of bounded
// launches.  Several instances run side by side, one per block, each with
// its own arguments and its own number of steps.
#pragma once
#include "wcns_kernels.hpp"

namespace wcns {

constexpr int RUN1D_THREADS = 512;   // 8 waves, 2 per SIMD (up to 256 VGPRs each)
constexpr int RUN1D_MAX_CELLS = 4096;
constexpr int64_t RUN1D_CHUNK = 1024;   // steps per launch (~0.05 s at 400 cells)

struct Run1D {
  KArgs a;             // the instance: W (state, updated in place), Wc/Pc, bc, eos, ...
  double* U1;          // stage states [5][n]
  double* U2;
  double* P;           // node primitives [5][n]
  double* G;           // face fluxes: G^- [6][n+1], then G^+ [6][n+1]
  const double* damax; // Dirichlet ghost maximum of |u|+c, or null
  double* dts;         // optional: dt of step k at dts[k] for k < dts_cap
  int64_t dts_cap;
  double t, t_end, dt_fixed, cfl;   // t: the time (in and out)
  int64_t max_steps, steps;         // steps: taken so far (in and out)
  int64_t last;                     // steps the last launch took (out)
  int32_t stopped, pad;             // 1: a step would not advance the time (out)
};

__device__ __forceinline__ double block_max_run1d(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double m = red[0];
  for (int k = 1; k < RUN1D_THREADS / 64; ++k) m = fmax(m, red[k]);
  return m;
}

template <bool DIRI, bool B32>
__global__ __launch_bounds__(RUN1D_THREADS) void k_run1d(Run1D* runs, int64_t chunk) {
  __shared__ double red[RUN1D_THREADS / 64];
  Run1D& r = runs[blockIdx.x];
  const KArgs a0 = r.a;
  const int n = a0.nx;
  const long N = n;
  const int tid = threadIdx.x;
  double* const W = const_cast<double*>(a0.W);
  double* const stage_in[3] = {W, r.U1, r.U2};
  double* const stage_out[3] = {r.U1, r.U2, W};
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0};
  const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
  double* const Gm = r.G;
  double* const Gp = r.G + 6 * (N + 1);
  double t = r.t;
  int64_t steps = r.steps, taken = 0;
  double dt = 0.0;
  bool stop = false;
  while (t < r.t_end && steps < r.max_steps && taken < chunk) {
    for (int s = 0; s < 3; ++s) {
      const double* in = stage_in[s];
      double* out = stage_out[s];
      // node primitives and the wave-speed maximum [Sec. 2, 3.3]; the
      // stage's input cells outside G are counted (the run's input, then
      // every stage result but the last, which is checked after the loop)
      double mx = 0.0;
      for (int i = tid; i < n; i += RUN1D_THREADS) {
        double X[6] = {in[i], in[N + i], in[2 * N + i], 0.0, in[3 * N + i], in[4 * N + i]};
        double un, ut, p, c, h;
        recover<false>(a0.eos, X, un, ut, p, c, h);
        r.P[i] = un; r.P[N + i] = ut; r.P[2 * N + i] = p; r.P[3 * N + i] = c; r.P[4 * N + i] = h;
        mx = fmax(mx, fabs(un) + c);
        if (a0.viol) report_bad(a0.viol, a0.vflag, !admissible(X[0], X[1], X[5], h));
      }
      mx = block_max_run1d(mx, red);
      if (r.damax) mx = fmax(mx, r.damax[0]);
      if (s == 0) {
        dt = r.dt_fixed > 0.0 ? r.dt_fixed : r.cfl * a0.dx / mx;
        if (t + dt > r.t_end) dt = r.t_end - t;
        // (dt is the same on every thread: the block maximum)
        if (!(t + dt > t)) {
          stop = true;
          break;
        }
      }
      const double lam = dt / a0.dx;
      // faces of the line [Sec. 4.2 steps, Sec. 5 limiters]
      KArgs a = a0;
      a.W = in;
      a.Wc[0] = in; a.Wc[1] = in + N; a.Wc[2] = in + 2 * N; a.Wc[3] = in;
      a.Wc[4] = in + 3 * N; a.Wc[5] = in + 4 * N;
      for (int k = 0; k < 5; ++k) a.Pc[k] = r.P + k * N;
      __syncthreads();
      for (int f = tid; f <= n; f += RUN1D_THREADS) {
        double gm[6], gp[6];
        face_flux<0, false, DIRI, B32>(a, 0, f - 3, lam, gm, gp);
#pragma unroll
        for (int v = 0; v < 6; ++v) {
          Gm[v * (N + 1) + f] = gm[v];
          Gp[v * (N + 1) + f] = gp[v];
        }
      }
      __syncthreads();
      // flux difference and the SSP-RK3 stage combination [Sec. 4.1, 5.3]
      for (int i = tid; i < n; i += RUN1D_THREADS) {
        // every input first: a store to `out` may alias a later load, so
        // loads left between the stores would each wait for the one before
        double gr[6], gl[6], wn[6], wi[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) {
          if (v == 3) continue;
          const int k = state_index(0, v, false);
          gr[v] = Gm[v * (N + 1) + i + 1];
          gl[v] = Gp[v * (N + 1) + i];
          wn[v] = W[k * N + i];
          wi[v] = in[k * N + i];
        }
#pragma unroll
        for (int v = 0; v < 6; ++v) {
          if (v == 3) continue;
          const double L = hdiv(-(gr[v] - gl[v]), a0.dx, a0.rdx);
          const int k = state_index(0, v, false);
          out[k * N + i] = ca[s] * wn[v] + cb[s] * (wi[v] + dt * L);
        }
      }
      __syncthreads();
    }
    if (stop) break;
    if (tid == 0 && r.dts && steps < r.dts_cap) r.dts[steps] = dt;
    t += dt;
    ++steps;
    ++taken;
  }
  // the last stage result, where the run ends (on t_end or max_steps: an
  // early stop has just checked it as the next step's input, and a launch
  // that ends on its chunk leaves it to the next launch's first stage)
  const bool more = !stop && taken == chunk && t < r.t_end && steps < r.max_steps;
  if (a0.viol && taken > 0 && !stop && !more) {
    for (int i = tid; i < n; i += RUN1D_THREADS) {
      const double X[6] = {W[i], W[N + i], W[2 * N + i], 0.0, W[3 * N + i], W[4 * N + i]};
      report_bad(a0.viol, a0.vflag, !admissible(X[0], X[1], X[5], rhoc2_tilde<false>(a0.eos, X)));
    }
  }
  if (tid == 0) {
    r.t = t;
    r.steps = steps;
    r.last = taken;
    r.stopped = stop ? 1 : 0;
  }
}

}  // namespace wcns
