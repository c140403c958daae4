// Host side of the C ABI declared in include/wcns.h: context creation and
// validation, scratch allocation (once), and kernel launch sequences for the
// RHS, the stand-alone flux limiter, the wave-speed reduction and the SSP-RK3
// step.  No allocation happens after wcns_create.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <utility>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/wcns.h"
#include "wcns_batch.hpp"
#include "wcns_3d.hpp"
#include "wcns_run1d.hpp"
#include "wcns_probe.hpp"
#include "wcns_fo.hpp"

#include <algorithm>
#include <vector>

using namespace wcns;

// k_node blocks at most (grid-stride beyond): its block maxima fit one
// round of k_finalize's loads
static constexpr long NODE_GRID_CAP = 2048;

struct wcns_ctx {
  wcns_grid grid;
  wcns_eos eos;
  wcns_params params;
  int32_t precision;
  hipStream_t stream;
  int nv;
  long N;
  double dx, dy;
  KArgs base;
  double *P, *L, *U1, *U2, *partial, *step, *dirW, *dirP, *edge;
  double* sink;   // first-order pass: stores of lanes that finish no cell (FO_SINK_SLOTS x 8)
  // 2D steps: the y-sweep and fixup of every stage but the last of a call
  // write the next stage's node primitives into the other buffer (P and P2
  // alternate) and their block maxima into `partial` (nfused pairs), so
  // only the first stage of a call runs k_node
  double* P2;
  int fuse, nfused;
  // count[0]: wcns_check_admissible's; count[1]: the cells the kernels found
  // outside G since creation or the last wcns_violations clear (viol)
  unsigned long long *count, *viol;
  int32_t* hflag;   // host-mapped pinned flag raised with viol (lazy error)
  int32_t* dflag;   // its device address
  double* damax;  // Dirichlet ghost wave-speed maxima [2] (inside dirP), or null
  // 3D: arguments shared by its kernels, strided-pass edge buffer, tile rows
  K3Args base3;
  double* edge3;
  int nbr_y3, nbr_z3;
  // 1D runs inside one workgroup (nx <= RUN1D_MAX_CELLS): face buffer, run record
  double* run_G;
  Run1D* run_dev;
  int node_grid, tile_x, x_grid, nbr;
  // first-order scheme in 2D: one pass per stage over (strip, row block) wave tasks
  int fo, fo_nstrip, fo_nrb, fo_ntask, fo_grid;
  int x_lds, xl_grid;   // x-sweep with LDS windows (rows of >= XLDS_MIN_NX cells), its grid
  // measurement aid: event pairs around launches (wcns_profile)
  int prof_on, prof_n, prof_cap;
  int prof_pend;   // 1 + slot of the open ProfScope whose event pair the next launch takes (0: none)
  hipEvent_t* ev;
  int* ev_cls;
  double prof_ms[WCNS_NPROF];
  int64_t prof_cnt[WCNS_NPROF];
};

// Fold recorded event pairs into the per-class sums (synchronises).  The
// pool is emptied either way: on a HIP error the pairs not yet folded are
// dropped rather than folded twice later.
static wcns_status prof_fold(wcns_ctx* c) {
  if (!c->prof_on || c->prof_n == 0) return WCNS_OK;
  const int n = c->prof_n;
  c->prof_n = 0;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return WCNS_ERR_HIP;
  for (int k = 0; k < n; ++k) {
    if (c->ev_cls[k] < 0) continue;   // a scope that launched nothing
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]) != hipSuccess) return WCNS_ERR_HIP;
    c->prof_ms[c->ev_cls[k]] += ms;
    c->prof_cnt[c->ev_cls[k]] += 1;
  }
  return WCNS_OK;
}

// One launch timed when profiling is on: the scope opens an event pair that
// the launch inside it (KLAUNCH) hands to hipExtLaunchKernelGGL, which
// stamps the pair with the kernel's own start and end, so the time excludes
// the dispatch that events recorded around the launch would include.
struct ProfScope {
  wcns_ctx* c;
  int slot;
  ProfScope(wcns_ctx* c_, int cls) : c(c_), slot(-1) {
    if (!c->prof_on) return;
    if (c->prof_n == c->prof_cap) (void)prof_fold(c);
    if (c->prof_n >= c->prof_cap) return;   // (no pool: the launch goes untimed)
    slot = c->prof_n++;
    c->ev_cls[slot] = cls;
    c->prof_pend = slot + 1;
  }
  ~ProfScope() {
    if (slot < 0 || c->prof_pend != slot + 1) return;
    // nothing was launched: keep the pair valid, count no launch
    (void)hipEventRecord(c->ev[2 * slot], c->stream);
    (void)hipEventRecord(c->ev[2 * slot + 1], c->stream);
    c->ev_cls[slot] = -1;
    c->prof_pend = 0;
  }
};

// hipLaunchKernelGGL, or, inside an open ProfScope of context C, the same
// launch stamping that scope's event pair
#define KLAUNCH(C, K, G, B, SHM, ST, ...)                                                      \
  do {                                                                                         \
    if ((C)->prof_pend > 0) {                                                                  \
      const int slot_ = (C)->prof_pend - 1;                                                    \
      (C)->prof_pend = 0;                                                                      \
      hipExtLaunchKernelGGL(K, G, B, SHM, ST, (C)->ev[2 * slot_], (C)->ev[2 * slot_ + 1], 0,  \
                            __VA_ARGS__);                                                      \
    } else {                                                                                   \
      hipLaunchKernelGGL(K, G, B, SHM, ST, __VA_ARGS__);                                       \
    }                                                                                          \
  } while (0)
enum { PROF_NODE = 0, PROF_FIN = 1, PROF_X = 2, PROF_Y = 3, PROF_FIX = 4, PROF_OTHER = 5, PROF_Z = 6,
       PROF_FO = 7, PROF_FO_UN = 8 };

#define HIP_TRY(x)                                   \
  do {                                               \
    hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) return WCNS_ERR_HIP;       \
  } while (0)
#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

extern "C" {

const char* wcns_status_str(wcns_status s) {
  switch (s) {
    case WCNS_OK: return "ok";
    case WCNS_ERR_ARG: return "invalid argument";
    case WCNS_ERR_EOS: return "fluids violate Lemma 1 (need one ideal gas and gamma_liquid >= gamma_gas)";
    case WCNS_ERR_NOMEM: return "device allocation failed";
    case WCNS_ERR_HIP: return "HIP runtime error";
    case WCNS_ERR_INADMISSIBLE: return "state outside the admissible set";
    case WCNS_ERR_CFL: return "invalid time step";
    case WCNS_ERR_TOO_LARGE: return "grid too large for the allocation-free scratch";
  }
  return "unknown status";
}

wcns_status wcns_params_default(wcns_params* p) {
  if (!p) return WCNS_ERR_ARG;
  memset(p, 0, sizeof(*p));
  p->eps_arho = 1e-10;
  p->eps_alpha = 1e-10;
  p->eps_rhoc2 = 1e-8;
  p->hs_arho = 1e-11;
  p->hs_alpha = 1e-11;
  p->hs_rhoc2 = 1e-9;
  p->weno_eps = 1e-40;
  p->cfl = 0.5;
  p->interp_limiter = 1;
  p->flux_limiter = 1;
  p->scheme = WCNS_SCHEME_PPWCNSIS;
  return WCNS_OK;
}

// Lemma 1 / Theorem 1: the admissible set is convex when one phase is an
// ideal gas (pinf = 0) and the other has a ratio of specific heats at least
// as large; gamma > 1 and pinf >= 0 for both.
static bool eos_ok(const wcns_eos* e) {
  if (!(e->gamma[0] > 1.0) || !(e->gamma[1] > 1.0)) return false;
  if (!(e->pinf[0] >= 0.0) || !(e->pinf[1] >= 0.0)) return false;
  if (e->pinf[1] == 0.0) return e->gamma[0] >= e->gamma[1];
  if (e->pinf[0] == 0.0) return e->gamma[1] >= e->gamma[0];
  return false;
}

// 1/h rounded once, if it is accurate to 2^-55 relative (the condition under
// which the kernels' reciprocal-and-correction divide by h is correctly
// rounded); 0 otherwise (the kernels then use the division core)
static double checked_recip(double h) {
  if (!(h > 0.0) || !isfinite(h)) return 0.0;
  const double y = 1.0 / h;
  const double e = fma(-h, y, 1.0);   // 1 - h*y: the relative error of y
  return fabs(e) <= ldexp(1.0, -55) ? y : 0.0;
}

static int pick_tile_x(int nx) {
  // largest T with T + (rows a run of T cells can touch) <= 64
  for (int T = 62; T >= 1; --T) {
    int rows = (T - 1 + nx - 1) / nx + 1;
    if (T + rows <= 64) return T;
  }
  return 1;
}

// (the pool is zero-filled at allocation, so events never created are null)
static void prof_release(wcns_ctx* c) {
  if (c->ev) {
    for (int k = 0; k < 2 * c->prof_cap; ++k)
      if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    free(c->ev);
    free(c->ev_cls);
  }
  c->ev = nullptr;
  c->ev_cls = nullptr;
  c->prof_cap = 0;
  c->prof_n = 0;
  c->prof_on = 0;
}

wcns_status wcns_destroy(wcns_ctx* c) {
  if (!c) return WCNS_ERR_ARG;
  prof_release(c);
  (void)hipStreamSynchronize(c->stream);
  double* bufs[] = {c->P, c->P2, c->L, c->U1, c->U2, c->partial, c->step, c->dirW, c->dirP, c->edge,
                    c->sink};
  for (double* b : bufs)
    if (b) (void)hipFree(b);
  if (c->count) (void)hipFree(c->count);
  if (c->hflag) (void)hipHostFree(c->hflag);
  if (c->edge3) (void)hipFree(c->edge3);
  if (c->run_G) (void)hipFree(c->run_G);
  if (c->run_dev) (void)hipFree(c->run_dev);
  free(c);
  return WCNS_OK;
}

static wcns_status create3(const wcns_grid* g, const wcns_eos* eos, const wcns_params* prm,
                           int32_t precision, void* stream, wcns_ctx** out);

// The admissible-count pair (zeroed) and the host-mapped violation flag.
static wcns_status alloc_report(wcns_ctx* c) {
  if (hipMalloc((void**)&c->count, 2 * sizeof(unsigned long long)) != hipSuccess) return WCNS_ERR_NOMEM;
  c->viol = c->count + 1;
  const unsigned long long z[2] = {0ull, 0ull};
  if (hipMemcpy(c->count, z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) return WCNS_ERR_HIP;
  if (hipHostMalloc((void**)&c->hflag, sizeof(int32_t), hipHostMallocMapped) != hipSuccess) {
    c->hflag = nullptr;
    return WCNS_ERR_NOMEM;
  }
  *c->hflag = 0;
  if (hipHostGetDevicePointer((void**)&c->dflag, c->hflag, 0) != hipSuccess) return WCNS_ERR_HIP;
  return WCNS_OK;
}

// weno_eps range: every IS-weight quotient tau_5/(beta + eps) then has a
// normal divisor at least eps and, for |tau_5| < 1e100, a normal quotient,
// the operand range on which the kernels' division core is the IEEE divide
static bool weno_eps_ok(double e) { return e >= 1e-200 && e <= 1e200; }

// Scheme options shared by every form: CFL number in (0, 0.5] (Sec. 3.3,
// 5.3), the IS-weight epsilon above, a known scheme, and the limiter and
// hard-switch tolerances of Sec. 5.1 finite and positive (the volume
// fraction ones below 1/2, so that [eps, 1 - eps] is not empty).
static bool params_ok(const wcns_params* p) {
  if (!(p->cfl > 0.0 && p->cfl <= 0.5) || !weno_eps_ok(p->weno_eps)) return false;
  if (p->scheme != WCNS_SCHEME_PPWCNSIS && p->scheme != WCNS_SCHEME_HLLC1) return false;
  for (double t : {p->eps_arho, p->eps_alpha, p->eps_rhoc2, p->hs_arho, p->hs_alpha, p->hs_rhoc2})
    if (!(t > 0.0) || !isfinite(t)) return false;
  return p->eps_alpha < 0.5 && p->hs_alpha < 0.5;
}

// A violation seen by earlier work on this context (lazy report): the
// entry points that enqueue work refuse to run until wcns_violations clears it.
static bool flagged(const wcns_ctx* c) {
  return c->hflag && __atomic_load_n(c->hflag, __ATOMIC_ACQUIRE) != 0;
}

// Validation of a 1D/2D grid, the fluids (Lemma 1) and the options.
static wcns_status check_setup(const wcns_grid* g, const wcns_eos* eos, const wcns_params* prm,
                               int32_t precision) {
  if (g->ndim != 1 && g->ndim != 2) return WCNS_ERR_ARG;
  if (g->nx < 1 || g->ny < 1 || (g->ndim == 1 && g->ny != 1)) return WCNS_ERR_ARG;
  // node loads use 32-bit byte offsets within one component array
  if ((long)g->nx * g->ny >= (1L << 29)) return WCNS_ERR_ARG;
  if (!(g->x1 > g->x0) || (g->ndim == 2 && !(g->y1 > g->y0))) return WCNS_ERR_ARG;
  for (int d = 0; d < g->ndim; ++d) {
    int lo = g->bc[2 * d], hi = g->bc[2 * d + 1];
    int n = d == 0 ? g->nx : g->ny;
    for (int b : {lo, hi})
      if (b < WCNS_BC_PERIODIC || b > WCNS_BC_DIRICHLET) return WCNS_ERR_ARG;
    if ((lo == WCNS_BC_PERIODIC) != (hi == WCNS_BC_PERIODIC)) return WCNS_ERR_ARG;
    if ((lo == WCNS_BC_REFLECT || hi == WCNS_BC_REFLECT) && n < 3) return WCNS_ERR_ARG;
  }
  if (!eos_ok(eos)) return WCNS_ERR_EOS;
  if (!params_ok(prm)) return WCNS_ERR_ARG;
  if (precision != WCNS_FP64 && precision != WCNS_FP32_BULK) return WCNS_ERR_ARG;
  return WCNS_OK;
}

// Dirichlet ghost states of a 1D/2D grid (primitive, per side or per
// boundary row): finite and inside the admissible set G of Sec. 2, i.e.
// partial densities >= 0 with a positive sum, 0 <= a1 <= 1, and
// rho e - pbar_inf = Gamma (p + pbar_inf) > 0 with Gamma > 0, so
// p + pbar_inf > 0 (Gamma, Pi and pbar_inf = Pi / (1 + Gamma) of the mixture).
static bool dirichlet_ok(const wcns_grid* g, const wcns_eos* e) {
  const int nv = g->ndim == 1 ? 5 : 6;
  for (int s = 0; s < 2 * g->ndim; ++s) {
    if (g->bc[s] != WCNS_BC_DIRICHLET) continue;
    const int n_side = g->dirichlet_rows[s] ? (s < 2 ? g->ny : g->nx) : 1;
    for (int l = 0; l < n_side; ++l) {
      const double* V = g->dirichlet_rows[s] ? g->dirichlet_rows[s] + (size_t)l * nv : g->dirichlet[s];
      for (int k = 0; k < nv; ++k)
        if (!isfinite(V[k])) return false;
      const double a1r1 = V[0], a2r2 = V[1], p = V[nv - 2], a1 = V[nv - 1];
      if (!(a1r1 >= 0.0 && a2r2 >= 0.0 && a1r1 + a2r2 > 0.0 && a1 >= 0.0 && a1 <= 1.0)) return false;
      const double Gam = a1 / (e->gamma[0] - 1.0) + (1.0 - a1) / (e->gamma[1] - 1.0);
      const double Pi = a1 * e->gamma[0] * e->pinf[0] / (e->gamma[0] - 1.0) +
                        (1.0 - a1) * e->gamma[1] * e->pinf[1] / (e->gamma[1] - 1.0);
      if (!(p + Pi / (1.0 + Gam) > 0.0)) return false;
    }
  }
  return true;
}

// Everything of a 1D/2D context but its device buffers: sizes, launch
// geometry and the kernel arguments (c zero-filled by the caller).
static void ctx_setup(wcns_ctx* c, const wcns_grid* g, const wcns_eos* eos, const wcns_params* prm,
                      int32_t precision, void* stream) {
  c->grid = *g;
  c->eos = *eos;
  c->params = *prm;
  c->precision = precision;
  c->stream = (hipStream_t)stream;
  c->nv = g->ndim == 1 ? 5 : 6;
  c->N = (long)g->nx * g->ny;
  c->dx = (g->x1 - g->x0) / g->nx;
  c->dy = g->ndim == 2 ? (g->y1 - g->y0) / g->ny : 1.0;

  KArgs& a = c->base;
  memset(&a, 0, sizeof(a));
  a.nx = g->nx;
  a.ny = g->ny;
  a.nv = c->nv;
  a.dx = c->dx;
  a.dy = c->dy;
  a.rdx = checked_recip(a.dx);
  a.rdy = checked_recip(a.dy);
  for (int k = 0; k < 4; ++k) a.bc[k] = g->bc[k];
  if (g->ndim == 1) { a.bc[2] = WCNS_BC_PERIODIC; a.bc[3] = WCNS_BC_PERIODIC; }
  a.interp_limiter = prm->interp_limiter ? 1 : 0;
  a.flux_limiter = prm->flux_limiter ? 1 : 0;
  a.scheme = prm->scheme;
  a.eos.g1 = 1.0 / (eos->gamma[0] - 1.0);
  a.eos.g2 = 1.0 / (eos->gamma[1] - 1.0);
  a.eos.q1 = eos->gamma[0] * eos->pinf[0] / (eos->gamma[0] - 1.0);
  a.eos.q2 = eos->gamma[1] * eos->pinf[1] / (eos->gamma[1] - 1.0);
  a.tol.eps_arho = prm->eps_arho;
  a.tol.eps_alpha = prm->eps_alpha;
  a.tol.eps_rhoc2 = prm->eps_rhoc2;
  a.tol.hs_arho = prm->hs_arho;
  a.tol.hs_alpha = prm->hs_alpha;
  a.tol.hs_rhoc2 = prm->hs_rhoc2;
  a.tol.weno_eps = prm->weno_eps;

  c->tile_x = pick_tile_x(g->nx);
  a.tile_x = c->tile_x;
  c->x_grid = (int)((c->N + c->tile_x - 1) / c->tile_x);
  c->x_lds = g->nx >= XLDS_MIN_NX;
  c->xl_grid = (int)(((c->N + XT - 1) / XT + XW - 1) / XW);
  long ng = (c->N + 255) / 256;
  c->node_grid = (int)(ng < NODE_GRID_CAP ? ng : NODE_GRID_CAP);
  c->nbr = (g->ny + 1 + Y_ROWS - 1) / Y_ROWS;
  a.nbr = c->nbr;
  c->fo = g->ndim == 2 && prm->scheme == WCNS_SCHEME_HLLC1;
  if (c->fo) {
    // as many (strip, row block) waves as the GPU holds at once
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
      ncu = 256;
    const long slots = 4L * FO_WPE * ncu;
    c->fo_nstrip = (g->nx + FO_LANES - 1) / FO_LANES;
    const long nrb = slots / c->fo_nstrip;   // never past the slots: a partial second round
                                             // of waves would double the pass
    c->fo_nrb = (int)std::max(1L, std::min(nrb, (long)g->ny));
    c->fo_ntask = c->fo_nstrip * c->fo_nrb;
    const int blocks = (c->fo_ntask + FO_WAVES - 1) / FO_WAVES;
    c->fo_grid = (blocks + 7) / 8 * 8;   // the task deal needs a multiple of 8 blocks
  }
}

wcns_status wcns_create(const wcns_grid* g, const wcns_eos* eos, const wcns_params* prm,
                        int32_t precision, void* stream, wcns_ctx** out) {
  if (!g || !eos || !prm || !out) return WCNS_ERR_ARG;
  *out = nullptr;
  if (g->ndim == 3) return create3(g, eos, prm, precision, stream, out);
  wcns_status chk = check_setup(g, eos, prm, precision);
  if (chk != WCNS_OK) return chk;
  if (!dirichlet_ok(g, eos)) return WCNS_ERR_INADMISSIBLE;

  wcns_ctx* c = (wcns_ctx*)calloc(1, sizeof(wcns_ctx));
  if (!c) return WCNS_ERR_NOMEM;
  ctx_setup(c, g, eos, prm, precision, stream);
  KArgs& a = c->base;

  wcns_status st = WCNS_OK;
  auto alloc = [&](double** p, size_t n) {
    if (st != WCNS_OK) return;
    if (hipMalloc((void**)p, n * sizeof(double)) != hipSuccess) { *p = nullptr; st = WCNS_ERR_NOMEM; }
  };
  alloc(&c->P, 5 * (size_t)c->N);
  alloc(&c->U1, (size_t)c->nv * c->N);
  alloc(&c->U2, (size_t)c->nv * c->N);
  if (g->ndim == 2) {
    alloc(&c->L, (size_t)c->nv * c->N);
    alloc(&c->edge, (size_t)c->nbr * 12 * g->nx);
  }
  // fused node primitives (2D): the y-tile epilogue and the fixup write
  // the next stage's
  c->fuse = g->ndim == 2;
  if (c->fuse) {
    const long nyb = (long)((g->nx + Y_COLS - 1) / Y_COLS) * c->nbr;
    const long nfb = c->nbr > 1 ? ((long)(c->nbr - 1) * g->nx + 255) / 256 : 0;
    c->nfused = (int)(nyb + nfb);
    alloc(&c->P2, 5 * (size_t)c->N);
  }
  const int npart = std::max(std::max(c->nfused, c->node_grid), c->fo_ntask);
  alloc(&c->partial, 2 * (size_t)npart);
  if (c->fo) alloc(&c->sink, 8 * (size_t)FO_SINK_SLOTS);
  alloc(&c->step, 8);
  if (g->ndim == 1 && g->nx <= RUN1D_MAX_CELLS) {
    alloc(&c->run_G, 12 * ((size_t)g->nx + 1));
    if (st == WCNS_OK && hipMalloc((void**)&c->run_dev, sizeof(Run1D)) != hipSuccess)
      st = WCNS_ERR_NOMEM;
  }
  // Dirichlet ghost rows: x-lo, x-hi (ny each), y-lo, y-hi (nx each)
  const int R = 2 * g->ny + 2 * g->nx;
  alloc(&c->dirW, 6 * (size_t)R);
  alloc(&c->dirP, 5 * (size_t)R + 2);
  if (st == WCNS_OK) st = alloc_report(c);
  if (st != WCNS_OK) { wcns_destroy(c); return st; }
  a.viol = c->viol;
  a.vflag = c->dflag;

  // Dirichlet ghost rows: primitive states from the grid (per row, or one
  // state for the whole side), converted on the device like any state
  a.dir_off[0] = 0;
  a.dir_off[1] = g->ny;
  a.dir_off[2] = 2 * g->ny;
  a.dir_off[3] = 2 * g->ny + g->nx;
  const int nv = c->nv;
  bool any_diri = false;
  double* V = (double*)malloc(sizeof(double) * nv * (size_t)R);
  if (!V) { wcns_destroy(c); return WCNS_ERR_NOMEM; }
  for (int s = 0; s < 4; ++s) {
    const int n_side = s < 2 ? g->ny : g->nx;
    const bool used = g->bc[s] == WCNS_BC_DIRICHLET && (g->ndim == 2 || s < 2);
    any_diri = any_diri || used;
    for (int l = 0; l < n_side; ++l) {
      const int r = a.dir_off[s] + l;
      for (int k = 0; k < nv; ++k) {
        double x;
        if (!used)   // admissible placeholder, never read
          x = k < 2 ? 1.0 : (k == nv - 2 ? 1e6 : (k == nv - 1 ? 0.5 : 0.0));
        else
          x = g->dirichlet_rows[s] ? g->dirichlet_rows[s][(size_t)l * nv + k] : g->dirichlet[s][k];
        V[(size_t)k * R + r] = x;
      }
    }
  }
  double *dV = nullptr, *dWg = nullptr;
  bool fail = hipMalloc((void**)&dV, sizeof(double) * nv * (size_t)R) != hipSuccess ||
              hipMalloc((void**)&dWg, sizeof(double) * nv * (size_t)R) != hipSuccess;
  fail = fail || hipMemcpy(dV, V, sizeof(double) * nv * (size_t)R, hipMemcpyHostToDevice) != hipSuccess;
  free(V);
  double zero8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  fail = fail || hipMemcpy(c->step, zero8, sizeof(zero8), hipMemcpyHostToDevice) != hipSuccess;
  a.dirW = c->dirW;
  a.dirP = c->dirP;
  a.step = c->step;
  a.edge = c->edge;
  c->damax = any_diri ? c->dirP + 5 * (size_t)R : nullptr;
  if (!fail) {
    KArgs ar = a;   // the rows as a 1-row grid of R cells
    ar.nx = R;
    ar.ny = 1;
    unsigned gr = (unsigned)((R + 255) / 256);
    if (g->ndim == 2) {
      hipLaunchKernelGGL(k_prim_to_cons<true>, dim3(gr), dim3(256), 0, c->stream, ar,
                         (const double*)dV, dWg);
      hipLaunchKernelGGL(k_dirichlet_rows<true>, dim3(1), dim3(256), 0, c->stream, a,
                         (const double*)dWg, R, c->dirW, c->dirP, c->dirP + 5 * (size_t)R);
    } else {
      hipLaunchKernelGGL(k_prim_to_cons<false>, dim3(gr), dim3(256), 0, c->stream, ar,
                         (const double*)dV, dWg);
      hipLaunchKernelGGL(k_dirichlet_rows<false>, dim3(1), dim3(256), 0, c->stream, a,
                         (const double*)dWg, R, c->dirW, c->dirP, c->dirP + 5 * (size_t)R);
    }
    fail = hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess;
  }
  if (dV) (void)hipFree(dV);
  if (dWg) (void)hipFree(dWg);
  if (fail) {
    wcns_destroy(c);
    return WCNS_ERR_HIP;
  }
  *out = c;
  return WCNS_OK;
}

// ---------------------------------------------------------------- 3D
// The direct 3D extension (Sec. 2): state [7][nz][ny][nx], FP64 only, sides
// periodic, extrapolated or reflective.
static wcns_status create3(const wcns_grid* g, const wcns_eos* eos, const wcns_params* prm,
                           int32_t precision, void* stream, wcns_ctx** out) {
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nz > 65535) return WCNS_ERR_ARG;
  const long N = (long)g->nx * g->ny * g->nz;
  if (N >= (1L << 29)) return WCNS_ERR_ARG;   // 32-bit byte offsets of node loads
  if (!(g->x1 > g->x0) || !(g->y1 > g->y0) || !(g->z1 > g->z0)) return WCNS_ERR_ARG;
  const int bc6[6] = {g->bc[0], g->bc[1], g->bc[2], g->bc[3], g->bc_z[0], g->bc_z[1]};
  const int len[3] = {g->nx, g->ny, g->nz};
  for (int d = 0; d < 3; ++d) {
    const int lo = bc6[2 * d], hi = bc6[2 * d + 1];
    for (int b : {lo, hi})
      if (b < WCNS_BC_PERIODIC || b > WCNS_BC_REFLECT) return WCNS_ERR_ARG;
    if ((lo == WCNS_BC_PERIODIC) != (hi == WCNS_BC_PERIODIC)) return WCNS_ERR_ARG;
    if ((lo == WCNS_BC_REFLECT || hi == WCNS_BC_REFLECT) && len[d] < 3) return WCNS_ERR_ARG;
  }
  if (!eos_ok(eos)) return WCNS_ERR_EOS;
  if (!params_ok(prm)) return WCNS_ERR_ARG;
  if (precision != WCNS_FP64) return WCNS_ERR_ARG;

  wcns_ctx* c = (wcns_ctx*)calloc(1, sizeof(wcns_ctx));
  if (!c) return WCNS_ERR_NOMEM;
  c->grid = *g;
  c->eos = *eos;
  c->params = *prm;
  c->precision = precision;
  c->stream = (hipStream_t)stream;
  c->nv = 7;
  c->N = N;
  c->dx = (g->x1 - g->x0) / g->nx;
  c->dy = (g->y1 - g->y0) / g->ny;
  K3Args& a = c->base3;
  memset(&a, 0, sizeof(a));
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.dx = c->dx;
  a.dy = c->dy;
  a.dz = (g->z1 - g->z0) / g->nz;
  a.rdx = checked_recip(a.dx);
  a.rdy = checked_recip(a.dy);
  a.rdz = checked_recip(a.dz);
  for (int k = 0; k < 6; ++k) a.bc[k] = bc6[k];
  a.interp_limiter = prm->interp_limiter ? 1 : 0;
  a.flux_limiter = prm->flux_limiter ? 1 : 0;
  a.scheme = prm->scheme;
  a.eos.g1 = 1.0 / (eos->gamma[0] - 1.0);
  a.eos.g2 = 1.0 / (eos->gamma[1] - 1.0);
  a.eos.q1 = eos->gamma[0] * eos->pinf[0] / (eos->gamma[0] - 1.0);
  a.eos.q2 = eos->gamma[1] * eos->pinf[1] / (eos->gamma[1] - 1.0);
  a.tol.eps_arho = prm->eps_arho;
  a.tol.eps_alpha = prm->eps_alpha;
  a.tol.eps_rhoc2 = prm->eps_rhoc2;
  a.tol.hs_arho = prm->hs_arho;
  a.tol.hs_alpha = prm->hs_alpha;
  a.tol.hs_rhoc2 = prm->hs_rhoc2;
  a.tol.weno_eps = prm->weno_eps;
  c->tile_x = pick_tile_x(g->nx);
  a.tile_x = c->tile_x;
  c->x_grid = (int)((N + c->tile_x - 1) / c->tile_x);
  c->x_lds = g->nx >= XLDS_MIN_NX;
  c->xl_grid = (int)(((N + XT - 1) / XT + XW - 1) / XW);
  const long ng = (N + 255) / 256;
  c->node_grid = (int)(ng < NODE_GRID_CAP ? ng : NODE_GRID_CAP);
  c->nbr_y3 = (g->ny + 1 + YW3 - 1) / YW3;
  c->nbr_z3 = (g->nz + 1 + YW3 - 1) / YW3;
  const size_t plane = (size_t)g->nx * g->ny;
  const size_t ey = (size_t)g->nz * c->nbr_y3 * 14 * g->nx, ez = (size_t)c->nbr_z3 * 14 * plane;

  wcns_status st = WCNS_OK;
  auto alloc = [&](double** p, size_t n) {
    if (st != WCNS_OK) return;
    if (hipMalloc((void**)p, n * sizeof(double)) != hipSuccess) { *p = nullptr; st = WCNS_ERR_NOMEM; }
  };
  alloc(&c->P, 6 * (size_t)N);
  alloc(&c->U1, 7 * (size_t)N);
  alloc(&c->U2, 7 * (size_t)N);
  alloc(&c->L, 7 * (size_t)N);
  alloc(&c->edge3, ey > ez ? ey : ez);
  alloc(&c->partial, 3 * (size_t)c->node_grid);
  alloc(&c->step, 8);
  if (st == WCNS_OK) st = alloc_report(c);
  if (st != WCNS_OK) { wcns_destroy(c); return st; }
  a.viol = c->viol;
  a.vflag = c->dflag;
  double zero8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (hipMemcpy(c->step, zero8, sizeof(zero8), hipMemcpyHostToDevice) != hipSuccess) {
    wcns_destroy(c);
    return WCNS_ERR_HIP;
  }
  a.step = c->step;
  for (int k = 0; k < 6; ++k) a.Pc[k] = c->P + (size_t)k * N;
  *out = c;
  return WCNS_OK;
}

// Time loop to t_end kept on the device (wcns_ssprk3_advance): the clock
// and step counter the first stage's finalize advances.
struct Clock {
  double* t;
  int64_t* n;
  double t_end;
};

static void set_bases3(const wcns_ctx* c, K3Args& a, const double* W) {
  a.W = W;
  for (int k = 0; k < 7; ++k) a.Wc[k] = W + (size_t)k * c->N;
}

// node primitives and maxima of W, then dt/lambda.  in_step: a stage after
// the first of a step (its k3_node returns when the step is skipped);
// check_in: k3_node also counts inadmissible input cells (the first stage
// of a call: later inputs are stage results, checked where they are made)
static wcns_status launch_node_finalize3(wcns_ctx* c, const double* W, int dt_mode, double dt,
                                         double* dt_used, bool in_step = false,
                                         bool check_in = true, const Clock* clk = nullptr) {
  K3Args a = c->base3;
  set_bases3(c, a, W);
  a.node_skip = in_step ? 1 : 0;
  a.check_in = check_in ? 1 : 0;
  {
    ProfScope ps(c, PROF_NODE);
    KLAUNCH(c, k3_node, dim3(c->node_grid), dim3(256), 0, c->stream, a, c->P, c->partial);
  }
  LAUNCH_CHECK();
  {
    ProfScope ps(c, PROF_FIN);
    KLAUNCH(c, k3_finalize, dim3(1), dim3(256), 0, c->stream, (const double*)c->partial,
                       c->node_grid, dt_mode, dt, c->params.cfl, a.dx, a.dy, a.dz, c->step,
                       dt_used, clk ? clk->t : nullptr, clk ? clk->n : nullptr,
                       clk ? clk->t_end : 0.0);
  }
  LAUNCH_CHECK();
  return WCNS_OK;
}

// x, y and z passes of state W into `out` (mode STORE: L; RK: next stage)
static wcns_status launch_sweeps3(wcns_ctx* c, const double* W, double* out, int mode,
                                  const double* Un, double ca, double cb) {
  K3Args a = c->base3;
  set_bases3(c, a, W);
  a.Un = Un;
  a.ca = ca;
  a.cb = cb;
  a.out_mode = mode;
  a.Lout = c->L;
  a.edge = c->edge3;
  const long nx = c->grid.nx, ny = c->grid.ny, nz = c->grid.nz;
  {
    ProfScope ps(c, PROF_X);
    if (c->x_lds)
      KLAUNCH(c, k3_sweep_xl, dim3(c->xl_grid), dim3(64 * XW), 0, c->stream, a);
    else
      KLAUNCH(c, k3_sweep_x, dim3(c->x_grid), dim3(64), 0, c->stream, a);
  }
  LAUNCH_CHECK();
  K3Args ay = a;   // y pass: L = L_x + L_y in place
  ay.Lin = c->L;
  ay.out = c->L;
  ay.last = 0;
  ay.nbr = c->nbr_y3;
  {
    ProfScope ps(c, PROF_Y);
    KLAUNCH(c, (k3_sweep_l<1>), dim3((unsigned)((nx + 31) / 32), c->nbr_y3, (unsigned)nz),
                       dim3(L3_THREADS), 0, c->stream, ay);
  }
  LAUNCH_CHECK();
  if (c->nbr_y3 > 1) {
    const long nt = (long)(c->nbr_y3 - 1) * nx * nz;
    ProfScope ps(c, PROF_FIX);
    KLAUNCH(c, (k3_fixup<1>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream,
                       ay);
    LAUNCH_CHECK();
  }
  K3Args az = a;   // z pass: L = (L_x + L_y) + L_z, then the output
  az.Lin = c->L;
  az.out = out;
  az.last = 1;
  az.nbr = c->nbr_z3;
  {
    ProfScope ps(c, PROF_Z);
    KLAUNCH(c, (k3_sweep_l<2>), dim3((unsigned)((nx * ny + 31) / 32), c->nbr_z3, 1),
                       dim3(L3_THREADS), 0, c->stream, az);
  }
  LAUNCH_CHECK();
  if (c->nbr_z3 > 1) {
    const long nt = (long)(c->nbr_z3 - 1) * nx * ny;
    ProfScope ps(c, PROF_FIX);
    KLAUNCH(c, (k3_fixup<2>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream,
                       az);
    LAUNCH_CHECK();
  }
  return WCNS_OK;
}

wcns_status wcns_set_stream(wcns_ctx* c, void* stream) {
  if (!c) return WCNS_ERR_ARG;
  // event pairs recorded on the old stream are folded while it is current
  const wcns_status st = prof_fold(c);
  c->stream = (hipStream_t)stream;
  return st;
}

// dt/lambda from the nblk block-maxima pairs in c->partial
static wcns_status launch_finalize(wcns_ctx* c, int nblk, int dt_mode, double dt, double* dt_used,
                                   const Clock* clk = nullptr) {
  FinArgs f;
  f.ndim = c->grid.ndim;
  f.dt_mode = dt_mode;
  f.dx = c->dx;
  f.dy = c->dy;
  f.cfl = c->params.cfl;
  f.dt_in = dt;
  f.step = c->step;
  f.dt_used = dt_used;
  f.damax = c->damax;
  f.clock = clk ? clk->t : nullptr;
  f.nsteps = clk ? clk->n : nullptr;
  f.t_end = clk ? clk->t_end : 0.0;
  ProfScope ps(c, PROF_FIN);
  KLAUNCH(c, k_finalize, dim3(1), dim3(1024), 0, c->stream, (const double*)c->partial,
                     nblk, f);
  LAUNCH_CHECK();
  return WCNS_OK;
}

// node primitives of state W into P + wave-speed maxima, then dt/lambda
// (in_step, check_in: as for launch_node_finalize3)
static wcns_status launch_node_finalize(wcns_ctx* c, const double* W, int dt_mode, double dt,
                                        double* dt_used, double* P = nullptr, bool in_step = false,
                                        bool check_in = true, const Clock* clk = nullptr) {
  if (!P) P = c->P;
  KArgs a = c->base;
  a.W = W;
  a.node_skip = in_step ? 1 : 0;
  a.check_in = check_in ? 1 : 0;
  {
    ProfScope ps(c, PROF_NODE);
    if (c->grid.ndim == 2)
      KLAUNCH(c, k_node<true>, dim3(c->node_grid), dim3(256), 0, c->stream, a, P, c->partial);
    else
      KLAUNCH(c, k_node<false>, dim3(c->node_grid), dim3(256), 0, c->stream, a, P, c->partial);
  }
  LAUNCH_CHECK();
  return launch_finalize(c, c->node_grid, dt_mode, dt, dt_used, clk);
}

// per-component base pointers of a state and of the node primitives
static void set_bases(wcns_ctx* c, KArgs& a, const double* W, const double* P) {
  const long N = c->N;
  if (c->grid.ndim == 2) {
    for (int k = 0; k < 6; ++k) a.Wc[k] = W + k * N;
  } else {
    a.Wc[0] = W; a.Wc[1] = W + N; a.Wc[2] = W + 2 * N; a.Wc[3] = W;
    a.Wc[4] = W + 3 * N; a.Wc[5] = W + 4 * N;
  }
  for (int k = 0; k < 5; ++k) a.Pc[k] = P + k * N;
}

static bool diri(const wcns_ctx* c, int dir) {
  return c->grid.bc[2 * dir] == WCNS_BC_DIRICHLET || c->grid.bc[2 * dir + 1] == WCNS_BC_DIRICHLET;
}

// the x-sweep of arguments `a`: LDS windows for rows of >= XLDS_MIN_NX cells
// (XG blocks; the first-order scheme takes its own instantiation, which runs
// no FP32 code in either precision), the flattened tiling otherwise
#define XSWEEP(HT, DI, BF, XG)                                                                 \
  do {                                                                                         \
    if (c->x_lds && c->params.scheme == WCNS_SCHEME_HLLC1)                                     \
      KLAUNCH(c, (k_sweep_xl<HT, DI, false, true>), dim3(XG), dim3(64 * XW), 0,         \
                         c->stream, a);                                                        \
    else if (c->x_lds)                                                                         \
      KLAUNCH(c, (k_sweep_xl<HT, DI, BF>), dim3(XG), dim3(64 * XW), 0, c->stream, a);   \
    else                                                                                       \
      KLAUNCH(c, (k_sweep_x<HT, DI, BF>), dim3(c->x_grid), dim3(64), 0, c->stream, a);  \
  } while (0)

#define XSWEEP_ALL(XG)                                \
  do {                                                \
    const bool d = diri(c, 0);                        \
    if (b32) {                                        \
      if (d) XSWEEP(true, true, true, XG);            \
      else XSWEEP(true, false, true, XG);             \
    } else {                                          \
      if (d) XSWEEP(true, true, false, XG);           \
      else XSWEEP(true, false, false, XG);            \
    }                                                 \
  } while (0)

// y-sweep of the first `rows` tile rows on stream s
static void ysweep(wcns_ctx* c, const KArgs& a, bool b32, int rows, hipStream_t s) {
  dim3 gy((c->grid.nx + Y_COLS - 1) / Y_COLS, rows);
  const bool d = diri(c, 1);
  if (b32) {
    if (d) KLAUNCH(c, (k_sweep_y<true, true>), gy, dim3(Y_THREADS), 0, s, a);
    else KLAUNCH(c, (k_sweep_y<false, true>), gy, dim3(Y_THREADS), 0, s, a);
  } else {
    if (d) KLAUNCH(c, (k_sweep_y<true, false>), gy, dim3(Y_THREADS), 0, s, a);
    else KLAUNCH(c, (k_sweep_y<false, false>), gy, dim3(Y_THREADS), 0, s, a);
  }
}

// x-sweep and (2D) y-sweep of state W into `out`; mode STORE (L) or RK.
// (P: node primitives of W; Pn: when not null, the finished cells' next
// stage primitives go there and their block maxima to c->partial)
static wcns_status launch_sweeps(wcns_ctx* c, const double* W, double* out, int mode,
                                 const double* Un, double ca, double cb,
                                 const double* P = nullptr, double* Pn = nullptr) {
  if (!P) P = c->P;
  KArgs a = c->base;
  a.W = W;
  a.P = P;
  a.out = out;
  a.Un = Un;
  a.ca = ca;
  a.cb = cb;
  a.out_mode = mode;
  set_bases(c, a, W, P);
  const bool b32 = c->precision == WCNS_FP32_BULK;
  if (c->grid.ndim == 1) {
    a.Lout = nullptr;
    ProfScope ps(c, PROF_X);
    const bool d = diri(c, 0);
    if (b32) {
      if (d) XSWEEP(false, true, true, c->xl_grid);
      else XSWEEP(false, false, true, c->xl_grid);
    } else {
      if (d) XSWEEP(false, true, false, c->xl_grid);
      else XSWEEP(false, false, false, c->xl_grid);
    }
    LAUNCH_CHECK();
    return WCNS_OK;
  }
  // 2D: L_x goes to `out` when storing L (summed in place by the y-sweep),
  // to the context's L buffer for a Runge-Kutta stage
  double* lx = mode == OUT_STORE ? out : c->L;
  a.Lout = lx;
  a.Lx = lx;
  if (Pn) {
    a.Pn = Pn;
    a.partn = c->partial;
    a.fuse_off = (int)((long)((c->grid.nx + Y_COLS - 1) / Y_COLS) * c->nbr);
  }
  {
    ProfScope ps(c, PROF_X);
    XSWEEP_ALL(c->xl_grid);
  }
  LAUNCH_CHECK();
  {
    ProfScope ps(c, PROF_Y);
    ysweep(c, a, b32, c->nbr, c->stream);
  }
  LAUNCH_CHECK();
  if (c->nbr > 1) {
    long nt = (long)(c->nbr - 1) * c->grid.nx;
    ProfScope ps(c, PROF_FIX);
    KLAUNCH(c, k_fixup_y, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream, a);
    LAUNCH_CHECK();
  }
  return WCNS_OK;
}

wcns_status wcns_prim_to_cons(wcns_ctx* c, const double* V, double* W) {
  if (!c || !V || !W) return WCNS_ERR_ARG;
  if (c->grid.ndim == 3) {
    unsigned g = (unsigned)((c->N + 255) / 256);
    hipLaunchKernelGGL(k3_prim_to_cons, dim3(g), dim3(256), 0, c->stream, c->base3, V, W);
    LAUNCH_CHECK();
    return WCNS_OK;
  }
  KArgs a = c->base;
  unsigned g = (unsigned)((c->N + 255) / 256);
  if (c->grid.ndim == 2)
    hipLaunchKernelGGL(k_prim_to_cons<true>, dim3(g), dim3(256), 0, c->stream, a, V, W);
  else
    hipLaunchKernelGGL(k_prim_to_cons<false>, dim3(g), dim3(256), 0, c->stream, a, V, W);
  LAUNCH_CHECK();
  return WCNS_OK;
}

static wcns_status launch_fo(wcns_ctx* c, const double* W, double* out, int mode, const double* Un,
                             double ca, double cb, bool maxima, bool check_out);

wcns_status wcns_rhs(wcns_ctx* c, const double* W, double* dWdt, double dt) {
  if (!c || !W || !dWdt || W == dWdt) return WCNS_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return WCNS_ERR_CFL;
  if (flagged(c)) return WCNS_ERR_INADMISSIBLE;
  if (c->grid.ndim == 3) {
    wcns_status s = launch_node_finalize3(c, W, DT_GIVEN, dt, nullptr);
    if (s != WCNS_OK) return s;
    return launch_sweeps3(c, W, dWdt, OUT_STORE, nullptr, 0.0, 0.0);
  }
  // (the first-order pass checks its input itself)
  wcns_status s = launch_node_finalize(c, W, DT_GIVEN, dt, nullptr, nullptr, false, !c->fo);
  if (s != WCNS_OK) return s;
  if (c->fo) return launch_fo(c, W, dWdt, OUT_STORE, nullptr, 0.0, 0.0, false, false);
  return launch_sweeps(c, W, dWdt, OUT_STORE, nullptr, 0.0, 0.0);
}

// one pass of the first-order scheme over state W into `out` (mode STORE:
// L; RK: next stage); maxima: the stage result's wave-speed maxima to
// c->partial (fo_ntask pairs) for the next step's finalize; the pass checks
// its input cells and, with check_out (the last stage of a call), its result
static wcns_status launch_fo(wcns_ctx* c, const double* W, double* out, int mode, const double* Un,
                             double ca, double cb, bool maxima, bool check_out) {
  KArgs a = c->base;
  a.check_in = 1;
  a.check_out = check_out ? 1 : 0;
  a.W = W;
  a.out = out;
  a.Un = Un;
  a.ca = ca;
  a.cb = cb;
  a.out_mode = mode;
  set_bases(c, a, W, c->P);
  a.partn = maxima ? c->partial : nullptr;
  a.sink = c->sink;
  const bool d = diri(c, 0) || diri(c, 1), un = mode == OUT_RK && ca != 0.0;
  ProfScope ps(c, un ? PROF_FO_UN : PROF_FO);
  const dim3 grid(c->fo_grid), block(64 * FO_WAVES);
  if (d && un) KLAUNCH(c, (k_fo_stage<true, true>), grid, block, 0, c->stream, a, c->fo_nstrip, c->fo_nrb, c->fo_ntask);
  else if (d) KLAUNCH(c, (k_fo_stage<true, false>), grid, block, 0, c->stream, a, c->fo_nstrip, c->fo_nrb, c->fo_ntask);
  else if (un) KLAUNCH(c, (k_fo_stage<false, true>), grid, block, 0, c->stream, a, c->fo_nstrip, c->fo_nrb, c->fo_ntask);
  else KLAUNCH(c, (k_fo_stage<false, false>), grid, block, 0, c->stream, a, c->fo_nstrip, c->fo_nrb, c->fo_ntask);
  LAUNCH_CHECK();
  return WCNS_OK;
}

// n steps of the first-order scheme in 2D: per step one finalize (dt from
// the maxima of U^n: k_node's for the first step of a call, then those the
// previous step's last stage reduced; the scheme uses no lambda, so stages
// 2 and 3 keep the step record) and one pass per stage.
static wcns_status steps_fo(wcns_ctx* c, double* W, int n, double dt, double* dts, const Clock* clk) {
  const double* in[3] = {W, c->U1, c->U2};
  double* outs[3] = {c->U1, c->U2, W};
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0};
  const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
  const int mode = dt > 0.0 ? DT_GIVEN : DT_CFL;
  for (int k = 0; k < n; ++k) {
    double* dt_used = dts ? dts + k : nullptr;
    wcns_status st = k == 0 ? launch_node_finalize(c, W, mode, dt, dt_used, c->P, false, false, clk)
                            : launch_finalize(c, c->fo_ntask, mode, dt, dt_used, clk);
    if (st != WCNS_OK) return st;
    for (int s = 0; s < 3; ++s) {
      const bool last = k == n - 1 && s == 2;
      st = launch_fo(c, in[s], outs[s], OUT_RK, W, ca[s], cb[s], s == 2 && !last, last);
      if (st != WCNS_OK) return st;
    }
  }
  return WCNS_OK;
}

// n SSP-RK3 steps of W in place (Shu-Osher form).  In 2D the node
// primitives and block maxima of every stage but the first of the call come
// from the previous stage's y-sweep and fixup (c->fuse): within one call no
// one else writes W between steps.  Step k's dt goes to dts[k] (device).
// clk: the time loop to t_end on the device (each step's first finalize
// clips dt or marks the step skipped; a skipped step's kernels return at
// once, and so do all later ones of the call, since the clock stays put).
static wcns_status steps_impl(wcns_ctx* c, double* W, int n, double dt, double* dts,
                              const Clock* clk = nullptr) {
  if (c->fo) return steps_fo(c, W, n, dt, dts, clk);
  const double* in[3] = {W, c->U1, c->U2};
  double* outs[3] = {c->U1, c->U2, W};
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0};
  const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
  double* Pcur = c->P;
  double* Pnext = c->P2;
  for (int k = 0; k < n; ++k) {
    double* dt_used = dts ? dts + k : nullptr;
    for (int s = 0; s < 3; ++s) {
      const int mode = s == 0 ? (dt > 0.0 ? DT_GIVEN : DT_CFL) : DT_KEEP;
      const bool first = k == 0 && s == 0, last = k == n - 1 && s == 2;
      const Clock* ck = s == 0 ? clk : nullptr;
      if (c->grid.ndim == 3) {
        wcns_status st = launch_node_finalize3(c, in[s], mode, dt, s == 0 ? dt_used : nullptr,
                                               s > 0, first, ck);
        if (st != WCNS_OK) return st;
        st = launch_sweeps3(c, in[s], outs[s], OUT_RK, W, ca[s], cb[s]);
        if (st != WCNS_OK) return st;
        continue;
      }
      wcns_status st = !first && c->fuse
                           ? launch_finalize(c, c->nfused, mode, dt, s == 0 ? dt_used : nullptr, ck)
                           : launch_node_finalize(c, in[s], mode, dt, s == 0 ? dt_used : nullptr,
                                                  Pcur, s > 0, first, ck);
      if (st != WCNS_OK) return st;
      double* Pn = c->fuse && !last ? Pnext : nullptr;
      st = launch_sweeps(c, in[s], outs[s], OUT_RK, W, ca[s], cb[s], Pcur, Pn);
      if (st != WCNS_OK) return st;
      if (Pn) std::swap(Pcur, Pnext);
    }
  }
  return WCNS_OK;
}

wcns_status wcns_ssprk3_step(wcns_ctx* c, double* W, double dt, double* dt_used) {
  if (!c || !W) return WCNS_ERR_ARG;
  if (!isfinite(dt)) return WCNS_ERR_CFL;
  if (flagged(c)) return WCNS_ERR_INADMISSIBLE;
  return steps_impl(c, W, 1, dt, dt_used);
}

wcns_status wcns_ssprk3_steps(wcns_ctx* c, double* W, int32_t nsteps, double dt, double* dts) {
  if (!c || !W || nsteps < 0) return WCNS_ERR_ARG;
  if (!isfinite(dt)) return WCNS_ERR_CFL;
  if (flagged(c)) return WCNS_ERR_INADMISSIBLE;
  return steps_impl(c, W, nsteps, dt, dts);
}

wcns_status wcns_ssprk3_advance(wcns_ctx* c, double* W, double dt, double t_end, int32_t nsteps,
                                double* t, int64_t* steps_taken, double* dts) {
  if (!c || !W || !t || nsteps < 0) return WCNS_ERR_ARG;
  if (!isfinite(t_end) || !isfinite(dt)) return WCNS_ERR_CFL;
  if (flagged(c)) return WCNS_ERR_INADMISSIBLE;
  const Clock clk{t, steps_taken, t_end};
  return steps_impl(c, W, nsteps, dt, dts, &clk);
}

wcns_status wcns_violations(wcns_ctx* c, int64_t* n_bad, int32_t clear) {
  if (!c || !n_bad) return WCNS_ERR_ARG;
  unsigned long long h = 0;
  HIP_TRY(hipMemcpyAsync(&h, c->viol, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *n_bad = (int64_t)h;
  if (clear) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, c->stream, c->viol, 1);
    LAUNCH_CHECK();
    HIP_TRY(hipStreamSynchronize(c->stream));
    __atomic_store_n(c->hflag, 0, __ATOMIC_RELEASE);
  }
  return h ? WCNS_ERR_INADMISSIBLE : WCNS_OK;
}

wcns_status wcns_run(wcns_ctx* c, double* W, double t0, double t_end, double dt_fixed,
                     int64_t max_steps, double* dts, int64_t dts_cap, int64_t* steps_out,
                     double* t_out) {
  if (!c || !W || !steps_out || !t_out || max_steps < 0 || dts_cap < 0) return WCNS_ERR_ARG;
  if (dts_cap > 0 && !dts) return WCNS_ERR_ARG;
  if (!c->run_dev) return WCNS_ERR_ARG;   // 1D grids of at most RUN1D_MAX_CELLS cells only
  if (!isfinite(t0) || !isfinite(t_end) || !(dt_fixed >= 0.0) || !isfinite(dt_fixed))
    return WCNS_ERR_CFL;
  if (flagged(c)) return WCNS_ERR_INADMISSIBLE;
  Run1D r;
  memset(&r, 0, sizeof(r));
  r.a = c->base;
  r.a.W = W;
  r.a.P = c->P;
  r.U1 = c->U1;
  r.U2 = c->U2;
  r.P = c->P;
  r.G = c->run_G;
  r.damax = c->damax;
  r.dts = dts;
  r.dts_cap = dts_cap;
  r.t = t0;
  r.t_end = t_end;
  r.dt_fixed = dt_fixed;
  r.cfl = c->params.cfl;
  r.max_steps = max_steps;
  HIP_TRY(hipMemcpyAsync(c->run_dev, &r, sizeof(r), hipMemcpyHostToDevice, c->stream));
  const bool d = diri(c, 0), b32 = c->precision == WCNS_FP32_BULK;
  // launches of at most RUN1D_CHUNK steps, each continuing from the record
  // the last one left, until one takes fewer (t_end, max_steps or a stop)
  for (;;) {
    {
      ProfScope ps(c, PROF_OTHER);
      const int64_t ch = RUN1D_CHUNK;
      if (b32) {
        if (d) KLAUNCH(c, (k_run1d<true, true>), dim3(1), dim3(RUN1D_THREADS), 0, c->stream, c->run_dev, ch);
        else KLAUNCH(c, (k_run1d<false, true>), dim3(1), dim3(RUN1D_THREADS), 0, c->stream, c->run_dev, ch);
      } else {
        if (d) KLAUNCH(c, (k_run1d<true, false>), dim3(1), dim3(RUN1D_THREADS), 0, c->stream, c->run_dev, ch);
        else KLAUNCH(c, (k_run1d<false, false>), dim3(1), dim3(RUN1D_THREADS), 0, c->stream, c->run_dev, ch);
      }
    }
    LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(&r, c->run_dev, sizeof(r), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (r.last < RUN1D_CHUNK || r.stopped || !(r.t < t_end) || r.steps >= max_steps) break;
  }
  *steps_out = r.steps;
  *t_out = r.t;
  // stopped short of t_end and of max_steps: a step that would not advance t
  return r.stopped ? WCNS_ERR_CFL : WCNS_OK;
}

wcns_status wcns_max_wavespeed(wcns_ctx* c, const double* W, double* d_amax) {
  if (!c || !W || !d_amax) return WCNS_ERR_ARG;
  if (flagged(c)) return WCNS_ERR_INADMISSIBLE;
  if (c->grid.ndim == 3) {
    wcns_status s = launch_node_finalize3(c, W, DT_GIVEN, 0.0, nullptr);
    if (s != WCNS_OK) return s;
    hipLaunchKernelGGL(k3_copy_amax, dim3(1), dim3(64), 0, c->stream, (const double*)c->step,
                       d_amax);
    LAUNCH_CHECK();
    return WCNS_OK;
  }
  wcns_status s = launch_node_finalize(c, W, DT_GIVEN, 0.0, nullptr);
  if (s != WCNS_OK) return s;
  hipLaunchKernelGGL(k_copy_amax, dim3(1), dim3(64), 0, c->stream, (const double*)c->step, d_amax,
                     c->grid.ndim);
  LAUNCH_CHECK();
  return WCNS_OK;
}

wcns_status wcns_limit(wcns_ctx* c, int32_t dir, const double* W, const double* G_ho,
                       const double* G_lo, double* G_out, double* theta, double dt) {
  if (!c || !W || !G_ho || !G_lo || !G_out) return WCNS_ERR_ARG;
  if (c->grid.ndim == 3) return WCNS_ERR_ARG;
  if (dir != 0 && !(dir == 1 && c->grid.ndim == 2)) return WCNS_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return WCNS_ERR_CFL;
  if (flagged(c)) return WCNS_ERR_INADMISSIBLE;
  wcns_status s = launch_node_finalize(c, W, DT_GIVEN, dt, nullptr);
  if (s != WCNS_OK) return s;
  KArgs a = c->base;
  a.W = W;
  a.P = c->P;
  set_bases(c, a, W, c->P);
  long nf = dir == 0 ? (long)(c->grid.nx + 1) * c->grid.ny : (long)c->grid.nx * (c->grid.ny + 1);
  unsigned g = (unsigned)((nf + 255) / 256);
  if (c->grid.ndim == 2)
    hipLaunchKernelGGL(k_limit<true>, dim3(g), dim3(256), 0, c->stream, a, (int)dir, G_ho, G_lo,
                       G_out, theta);
  else
    hipLaunchKernelGGL(k_limit<false>, dim3(g), dim3(256), 0, c->stream, a, (int)dir, G_ho, G_lo,
                       G_out, theta);
  LAUNCH_CHECK();
  return WCNS_OK;
}

wcns_status wcns_check_admissible(wcns_ctx* c, const double* W, long long* n_bad) {
  if (!c || !W || !n_bad) return WCNS_ERR_ARG;
  KArgs a = c->base;
  a.W = W;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, c->stream, c->count, 1);
  LAUNCH_CHECK();
  if (c->grid.ndim == 3) {
    K3Args a3 = c->base3;
    a3.W = W;
    hipLaunchKernelGGL(k3_admissible, dim3((unsigned)((c->N + 255) / 256)), dim3(256), 0,
                       c->stream, a3, c->count);
  } else if (c->grid.ndim == 2)
    hipLaunchKernelGGL(k_admissible<true>, dim3(c->node_grid), dim3(256), 0, c->stream, a, c->count);
  else
    hipLaunchKernelGGL(k_admissible<false>, dim3(c->node_grid), dim3(256), 0, c->stream, a, c->count);
  LAUNCH_CHECK();
  unsigned long long h = 0;
  HIP_TRY(hipMemcpyAsync(&h, c->count, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *n_bad = (long long)h;
  return WCNS_OK;
}

wcns_status wcns_selftest_division(const double* a, const double* b, double* q_ieee,
                                   double* q_core, int64_t n, void* stream) {
  if (!a || !b || !q_ieee || !q_core || n < 0) return WCNS_ERR_ARG;
  if (n == 0) return WCNS_OK;
  unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_selftest_div, dim3(g), dim3(256), 0, (hipStream_t)stream, a, b, q_ieee, q_core,
                     (long)n);
  LAUNCH_CHECK();
  return WCNS_OK;
}

wcns_status wcns_selftest_division_by(const double* a, double b, double* q_ieee, double* q_core,
                                      int64_t n, void* stream) {
  if (!a || !q_ieee || !q_core || n < 0) return WCNS_ERR_ARG;
  const double y = b == 2100.0 ? 1.0 / 2100.0 : checked_recip(b);
  if (y == 0.0) return WCNS_ERR_ARG;   // b does not take this path
  if (n == 0) return WCNS_OK;
  unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_selftest_cdiv, dim3(g), dim3(256), 0, (hipStream_t)stream, a, b, y, q_ieee,
                     q_core, (long)n);
  LAUNCH_CHECK();
  return WCNS_OK;
}

wcns_status wcns_issue_probe(int32_t op, int32_t iters, int32_t blocks, double* ms, void* stream) {
  if (op < PROBE_FMA || op > PROBE_SQRT_F32 || iters < 1 || !ms) return WCNS_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return WCNS_ERR_HIP;
  if (blocks <= 0) blocks = 32 * ncu;   // 8 waves on each of 4 SIMDs per CU
  double* out = nullptr;
  if (hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(double)) != hipSuccess) return WCNS_ERR_NOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  wcns_status st = WCNS_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = WCNS_ERR_HIP;
  const double c = 0.999999, d = 1e-6;
  if (st == WCNS_OK) {
    (void)hipEventRecord(e0, s);
    switch (op) {
      case PROBE_FMA: hipLaunchKernelGGL(k_issue_probe<PROBE_FMA>, dim3(blocks), dim3(256), 0, s, out, iters, c, d); break;
      case PROBE_ADD: hipLaunchKernelGGL(k_issue_probe<PROBE_ADD>, dim3(blocks), dim3(256), 0, s, out, iters, c, d); break;
      case PROBE_MUL: hipLaunchKernelGGL(k_issue_probe<PROBE_MUL>, dim3(blocks), dim3(256), 0, s, out, iters, c, d); break;
      case PROBE_DIV: hipLaunchKernelGGL(k_issue_probe<PROBE_DIV>, dim3(blocks), dim3(256), 0, s, out, iters, c, 1.5); break;
      case PROBE_SQRT: hipLaunchKernelGGL(k_issue_probe<PROBE_SQRT>, dim3(blocks), dim3(256), 0, s, out, iters, c, d); break;
      case PROBE_DIV_CORE: hipLaunchKernelGGL(k_issue_probe<PROBE_DIV_CORE>, dim3(blocks), dim3(256), 0, s, out, iters, c, 1.5); break;
      case PROBE_FMA_F32: hipLaunchKernelGGL(k_issue_probe_f32<PROBE_FMA_F32>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f); break;
      case PROBE_DIV_F32: hipLaunchKernelGGL(k_issue_probe_f32<PROBE_DIV_F32>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1.5f); break;
      default: hipLaunchKernelGGL(k_issue_probe_f32<PROBE_SQRT_F32>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f); break;
    }
    if (hipGetLastError() != hipSuccess) st = WCNS_ERR_HIP;
    (void)hipEventRecord(e1, s);
    float f = 0.0f;
    if (st == WCNS_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&f, e0, e1) != hipSuccess))
      st = WCNS_ERR_HIP;
    *ms = f;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  return st;
}

wcns_status wcns_profile(wcns_ctx* c, int32_t enable) {
  if (!c) return WCNS_ERR_ARG;
  if (enable && !c->prof_on) {
    const int cap = 4096;
    c->ev = (hipEvent_t*)calloc(2 * cap, sizeof(hipEvent_t));
    c->ev_cls = (int*)calloc(cap, sizeof(int));
    c->prof_cap = cap;
    if (!c->ev || !c->ev_cls) { prof_release(c); return WCNS_ERR_NOMEM; }
    for (int k = 0; k < 2 * cap; ++k) {
      if (hipEventCreate(&c->ev[k]) != hipSuccess) {
        c->ev[k] = nullptr;
        prof_release(c);
        return WCNS_ERR_HIP;
      }
    }
    c->prof_n = 0;
    c->prof_on = 1;
    for (int k = 0; k < WCNS_NPROF; ++k) { c->prof_ms[k] = 0.0; c->prof_cnt[k] = 0; }
  } else if (!enable && c->prof_on) {
    wcns_status s = prof_fold(c);
    prof_release(c);
    return s;
  }
  return WCNS_OK;
}

wcns_status wcns_profile_read(wcns_ctx* c, double* ms, int64_t* launches, int32_t reset) {
  if (!c || !ms || !launches) return WCNS_ERR_ARG;
  wcns_status s = prof_fold(c);
  if (s != WCNS_OK) return s;
  for (int k = 0; k < WCNS_NPROF; ++k) {
    ms[k] = c->prof_ms[k];
    launches[k] = c->prof_cnt[k];
    if (reset) { c->prof_ms[k] = 0.0; c->prof_cnt[k] = 0; }
  }
  return WCNS_OK;
}


}  // extern "C"

// ============================================================================
// Batched form
// ============================================================================
struct wcns_batch {
  int n = 0, ndim = 0, nv = 0, precision = 0;
  wcns_eos eos;
  wcns_params params;
  KArgs proto;
  hipStream_t stream = nullptr;
  double* arena = nullptr;
  size_t arena_cap = 0;        // doubles
  std::vector<wcns_grid> grids;
  std::vector<double*> W;
  std::vector<size_t> off;     // arena offset of each instance's scratch
  KArgs* d_ka = nullptr;       // [5][n]: stages 1-3, the RHS-only set, stage 1 of a continuing step
  size_t ka_cap = 0;
  Task* d_tasks = nullptr;
  size_t tasks_cap = 0;
  int n_node = 0, n_x = 0, n_y = 0, n_fix = 0;
  size_t o_node = 0, o_x = 0, o_y = 0, o_fix = 0;
  double* d_dt = nullptr;      // per-instance dt of the last step
  int32_t* d_live = nullptr;   // per-instance steps left (frozen at 0)
  unsigned long long* d_viol = nullptr;   // per-instance cells found outside G
  int dt_cap = 0;
  int ytile = 16, order = 0;
  bool x_lds = false;   // x-sweep with LDS windows (every instance has nx >= XLDS_MIN_NX)
  hipGraph_t graph = nullptr;     // first step of a call (node primitives by kb_node)
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph2 = nullptr;    // later steps (2D: primitives from the previous step)
  hipGraphExec_t exec2 = nullptr;
  bool dirty = true;
};

static size_t round32(size_t x) { return (x + 31) & ~(size_t)31; }

// scratch doubles of one instance: P, U1, U2, (L), edge (for the smallest
// y-tile), block maxima, step record
// block-maxima pairs of the fused next-stage primitives of a 2D instance
// (32-column y-tiles of yw face rows, then the fixup's blocks)
static size_t fused_pairs(const wcns_grid& g, int yw) {
  const size_t nbr = (size_t)(g.ny + 1 + yw - 1) / yw;
  const size_t nyb = (size_t)((g.nx + 31) / 32) * nbr;
  const size_t nfb = nbr > 1 ? ((nbr - 1) * (size_t)g.nx + 255) / 256 : 0;
  return nyb + nfb;
}

// block-maxima pairs an instance's scratch holds: k_node's blocks, or (2D)
// the fused ones at the smallest tile height
static size_t inst_pairs(const wcns_grid& g) {
  const size_t nblk = ((size_t)g.nx * g.ny + 255) / 256;
  if (g.ndim != 2) return nblk;
  const size_t f = fused_pairs(g, 2);
  return f > nblk ? f : nblk;
}

// instance scratch: P, (2D) P2, P3, U1, U2, block maxima, step record, (2D)
// L, edges
static size_t inst_doubles(const wcns_grid& g, int nv) {
  const size_t N = (size_t)g.nx * g.ny;
  size_t nbr = (size_t)(g.ny + 1 + 1) / 2;
  size_t d = round32(5 * N) + 2 * round32(nv * N) + round32(2 * inst_pairs(g)) + 32;
  if (g.ndim == 2) d += 2 * round32(5 * N) + round32(nv * N) + round32(nbr * 12 * g.nx);
  return d;
}

static wcns_status batch_check_grids(int n, const wcns_grid* grids, int ndim) {
  for (int b = 0; b < n; ++b) {
    const wcns_grid& g = grids[b];
    if (g.ndim != ndim) return WCNS_ERR_ARG;
    if (g.nx < 1 || g.ny < 1 || (ndim == 1 && g.ny != 1)) return WCNS_ERR_ARG;
    if ((long)g.nx * g.ny >= (1L << 29)) return WCNS_ERR_ARG;
    if (!(g.x1 > g.x0) || (ndim == 2 && !(g.y1 > g.y0))) return WCNS_ERR_ARG;
    for (int d = 0; d < ndim; ++d) {
      int lo = g.bc[2 * d], hi = g.bc[2 * d + 1];
      int m = d == 0 ? g.nx : g.ny;
      for (int k : {lo, hi})
        if (k < WCNS_BC_PERIODIC || k > WCNS_BC_REFLECT) return WCNS_ERR_ARG;   // no Dirichlet
      if ((lo == WCNS_BC_PERIODIC) != (hi == WCNS_BC_PERIODIC)) return WCNS_ERR_ARG;
      if ((lo == WCNS_BC_REFLECT || hi == WCNS_BC_REFLECT) && m < 3) return WCNS_ERR_ARG;
    }
  }
  return WCNS_OK;
}

static void batch_drop_graph(wcns_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->exec2) (void)hipGraphExecDestroy(b->exec2);
  if (b->graph2) (void)hipGraphDestroy(b->graph2);
  b->exec = nullptr;
  b->graph = nullptr;
  b->exec2 = nullptr;
  b->graph2 = nullptr;
  b->dirty = true;
}

// deal a task list to the 8 XCDs in contiguous chunks: block i runs on XCD
// i % 8, so position 8k + x takes the k-th task of chunk x
static void xcd_chunk(std::vector<Task>& t) {
  const size_t M = t.size();
  if (M < 16) return;
  std::vector<Task> out;
  out.reserve(M);
  const size_t per = (M + 7) / 8;
  for (size_t k = 0; k < per; ++k)
    for (size_t x = 0; x < 8; ++x) {
      size_t src = x * per + k;
      if (src < M) out.push_back(t[src]);
    }
  t.swap(out);
}

// The batch without an instance set (after a failed rebuild): no graph, no
// tasks; step and rhs refuse until a reset succeeds.
static void batch_invalidate(wcns_batch* b) {
  batch_drop_graph(b);
  b->n = 0;
  b->grids.clear();
  b->W.clear();
  b->off.clear();
  b->n_node = b->n_x = b->n_y = b->n_fix = 0;
}

// (re)build the per-instance arguments and the task lists
static wcns_status batch_build_impl(wcns_batch* b) {
  const int n = b->n;
  std::vector<KArgs> ka(5 * (size_t)n);
  std::vector<int> inst_order(n);
  for (int k = 0; k < n; ++k) inst_order[k] = k;
  if (b->order >= 1)
    std::stable_sort(inst_order.begin(), inst_order.end(), [&](int p, int q) {
      return (long)b->grids[p].nx * b->grids[p].ny > (long)b->grids[q].nx * b->grids[q].ny;
    });
  std::vector<Task> tn, tx, ty, tf;
  const int yw = b->ytile;
  for (int k = 0; k < n; ++k) {
    const wcns_grid& g = b->grids[k];
    const long N = (long)g.nx * g.ny;
    double* base = b->arena + b->off[k];
    double* P = base;
    // fused next-stage primitives (2D): stage 1 reads P, 2 reads P2, 3 reads
    // P3, and stage 3 leaves the next step's in P
    double* P2 = g.ndim == 2 ? P + round32(5 * N) : nullptr;
    double* P3 = g.ndim == 2 ? P2 + round32(5 * N) : nullptr;
    double* U1 = (P3 ? P3 : P) + round32(5 * N);
    double* U2 = U1 + round32((size_t)b->nv * N);
    double* part = U2 + round32((size_t)b->nv * N);
    const int nblk = (int)((N + 255) / 256);
    double* step = part + round32(2 * inst_pairs(g));
    double* L = step + 32;
    double* edge = L + round32((size_t)b->nv * N);
    const int nbr = (g.ny + 1 + yw - 1) / yw;
    KArgs a = b->proto;
    a.nx = g.nx;
    a.ny = g.ny;
    a.dx = (g.x1 - g.x0) / g.nx;
    a.dy = g.ndim == 2 ? (g.y1 - g.y0) / g.ny : 1.0;
    a.rdx = checked_recip(a.dx);
    a.rdy = checked_recip(a.dy);
    for (int q = 0; q < 4; ++q) a.bc[q] = g.bc[q];
    if (g.ndim == 1) { a.bc[2] = WCNS_BC_PERIODIC; a.bc[3] = WCNS_BC_PERIODIC; }
    a.tile_x = pick_tile_x(g.nx);
    a.P = P;
    a.Pw = P;
    for (int q = 0; q < 5; ++q) a.Pc[q] = P + q * N;
    a.step = step;
    a.partial = part;
    a.nblk = nblk;
    a.edge = g.ndim == 2 ? edge : nullptr;
    a.nbr = nbr;
    a.ndim = g.ndim;
    a.cfl = b->params.cfl;
    a.dt_used = b->d_dt + k;
    a.live = b->d_live + k;
    a.viol = b->d_viol + k;
    const double* in[3] = {b->W[k], U1, U2};
    double* outs[3] = {U1, U2, b->W[k]};
    const double cA[3] = {0.0, 0.75, 1.0 / 3.0};
    const double cB[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int set = 0; set < 5; ++set) {
      // sets 0-2: stages 1-3; 3: RHS only; 4: stage 1 of a step that follows
      // another in the same call
      const int s = set == 4 ? 0 : set;
      KArgs x = a;
      // the node pass checks its input only where no stage made it (the
      // first stage of a call, the RHS); stage results are checked where
      // they are written
      x.check_in = (set == 0 || set == 3) ? 1 : 0;
      const double* Ws = s < 3 ? in[s] : b->W[k];
      x.W = Ws;
      if (g.ndim == 2) {
        for (int q = 0; q < 6; ++q) x.Wc[q] = Ws + q * N;
      } else {
        x.Wc[0] = Ws; x.Wc[1] = Ws + N; x.Wc[2] = Ws + 2 * N; x.Wc[3] = Ws;
        x.Wc[4] = Ws + 3 * N; x.Wc[5] = Ws + 4 * N;
      }
      if (s < 3 && P2) {
        // the first step of a call runs kb_node into P; the y-sweep and
        // fixup of every stage leave the next stage's primitives (P2, P3,
        // then P for the next step) and the block maxima kb_finalize reduces
        const double* Pc = s == 0 ? P : (s == 1 ? P2 : P3);
        x.P = Pc;
        for (int q = 0; q < 5; ++q) x.Pc[q] = Pc + q * N;
        x.Pn = s == 0 ? P2 : (s == 1 ? P3 : P);
        x.partn = part;
        x.fuse_off = (int)((long)((g.nx + 31) / 32) * nbr);
        if (set != 0) x.nblk = (int)fused_pairs(g, yw);
      }
      if (s < 3) {
        x.out = outs[s];
        x.Un = b->W[k];
        x.ca = cA[s];
        x.cb = cB[s];
        x.out_mode = OUT_RK;
        x.dt_mode = s == 0 ? DT_CFL : DT_KEEP;
        x.Lout = g.ndim == 2 ? L : nullptr;
        x.Lx = L;
      } else {
        // RHS only: L into scratch U2 (summed in place in 2D), state untouched
        x.out = U2;
        x.Un = nullptr;
        x.out_mode = OUT_STORE;
        x.dt_mode = DT_CFL;
        x.Lout = g.ndim == 2 ? U2 : nullptr;
        x.Lx = U2;
        x.dt_used = nullptr;
        x.live = nullptr;
      }
      ka[(size_t)set * n + k] = x;
    }
  }
  b->x_lds = true;
  for (int k = 0; k < n; ++k) b->x_lds = b->x_lds && b->grids[k].nx >= XLDS_MIN_NX;
  for (int k : inst_order) {
    const wcns_grid& g = b->grids[k];
    const long N = (long)g.nx * g.ny;
    const int nblk = (int)((N + 255) / 256);
    for (int q = 0; q < nblk; ++q) tn.push_back({k, q, 0, 0});
    // x tasks: one tile of tile_x cells, or XW window tiles of XT cells
    const long nt = b->x_lds ? ((N + XT - 1) / XT + XW - 1) / XW : (N + ka[k].tile_x - 1) / ka[k].tile_x;
    for (long q = 0; q < nt; ++q) tx.push_back({k, (int)q, 0, 0});
    if (g.ndim == 2) {
      const int nbr = ka[k].nbr;
      const int nbx = (g.nx + 31) / 32;
      for (int by = 0; by < nbr; ++by)
        for (int bx = 0; bx < nbx; ++bx) ty.push_back({k, bx, by, 0});
      const long nfc = (long)(nbr - 1) * g.nx;
      for (long q = 0; q < (nfc + 255) / 256; ++q) tf.push_back({k, (int)q, 0, 0});
    }
  }
  if (b->order == 2) {
    xcd_chunk(tx);
    xcd_chunk(ty);
  }
  b->n_node = (int)tn.size();
  b->n_x = (int)tx.size();
  b->n_y = (int)ty.size();
  b->n_fix = (int)tf.size();
  std::vector<Task> all;
  b->o_node = all.size(); all.insert(all.end(), tn.begin(), tn.end());
  b->o_x = all.size(); all.insert(all.end(), tx.begin(), tx.end());
  b->o_y = all.size(); all.insert(all.end(), ty.begin(), ty.end());
  b->o_fix = all.size(); all.insert(all.end(), tf.begin(), tf.end());
  if (all.size() > b->tasks_cap) {
    if (b->d_tasks) (void)hipFree(b->d_tasks);
    b->d_tasks = nullptr;
    b->tasks_cap = 0;
    if (hipMalloc((void**)&b->d_tasks, all.size() * sizeof(Task)) != hipSuccess) return WCNS_ERR_NOMEM;
    b->tasks_cap = all.size();
  }
  if (ka.size() > b->ka_cap) {
    if (b->d_ka) (void)hipFree(b->d_ka);
    b->d_ka = nullptr;
    b->ka_cap = 0;
    if (hipMalloc((void**)&b->d_ka, ka.size() * sizeof(KArgs)) != hipSuccess) return WCNS_ERR_NOMEM;
    b->ka_cap = ka.size();
  }
  HIP_TRY(hipMemcpyAsync(b->d_tasks, all.data(), all.size() * sizeof(Task), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_ka, ka.data(), ka.size() * sizeof(KArgs), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  batch_drop_graph(b);
  return WCNS_OK;
}

// the rebuild, leaving no instance set bound if it fails part way (the
// device task list and arguments would no longer match the host's)
static wcns_status batch_build(wcns_batch* b) {
  const wcns_status st = batch_build_impl(b);
  if (st != WCNS_OK) batch_invalidate(b);
  return st;
}

// launches of stage s (3: RHS only); cont: stage 1 of a step that follows
// another in the same call
template <int YW>
static void batch_stage_launches(wcns_batch* b, int s, bool cont) {
  const KArgs* ka = b->d_ka + (size_t)(s == 0 && cont ? 4 : s) * b->n;
  const bool b32 = b->precision == WCNS_FP32_BULK;
  // 2D: only the first stage of a call (and the RHS) runs kb_node; the
  // others take their node primitives from the previous stage
  if (b->ndim == 2 && ((s == 0 && !cont) || s == 3))
    hipLaunchKernelGGL(kb_node<true>, dim3(b->n_node), dim3(256), 0, b->stream, ka, b->d_tasks + b->o_node);
  else if (b->ndim != 2)
    hipLaunchKernelGGL(kb_node<false>, dim3(b->n_node), dim3(256), 0, b->stream, ka, b->d_tasks + b->o_node);
  hipLaunchKernelGGL(kb_finalize, dim3(b->n), dim3(256), 0, b->stream, ka);
  const Task* tx = b->d_tasks + b->o_x;
  if (b->ndim == 2) {
    if (b->x_lds) {
      if (b32) hipLaunchKernelGGL((kb_sweep_xl<true, true>), dim3(b->n_x), dim3(64 * XW), 0, b->stream, ka, tx);
      else hipLaunchKernelGGL((kb_sweep_xl<true, false>), dim3(b->n_x), dim3(64 * XW), 0, b->stream, ka, tx);
    } else {
      if (b32) hipLaunchKernelGGL((kb_sweep_x<true, true>), dim3(b->n_x), dim3(64), 0, b->stream, ka, tx);
      else hipLaunchKernelGGL((kb_sweep_x<true, false>), dim3(b->n_x), dim3(64), 0, b->stream, ka, tx);
    }
    if (b32) hipLaunchKernelGGL((kb_sweep_y<YW, true>), dim3(b->n_y), dim3(32 * YW), 0, b->stream, ka, b->d_tasks + b->o_y);
    else hipLaunchKernelGGL((kb_sweep_y<YW, false>), dim3(b->n_y), dim3(32 * YW), 0, b->stream, ka, b->d_tasks + b->o_y);
    if (b->n_fix > 0)
      hipLaunchKernelGGL(kb_fixup<YW>, dim3(b->n_fix), dim3(256), 0, b->stream, ka, b->d_tasks + b->o_fix);
  } else if (b->x_lds) {
    if (b32) hipLaunchKernelGGL((kb_sweep_xl<false, true>), dim3(b->n_x), dim3(64 * XW), 0, b->stream, ka, tx);
    else hipLaunchKernelGGL((kb_sweep_xl<false, false>), dim3(b->n_x), dim3(64 * XW), 0, b->stream, ka, tx);
  } else {
    if (b32) hipLaunchKernelGGL((kb_sweep_x<false, true>), dim3(b->n_x), dim3(64), 0, b->stream, ka, tx);
    else hipLaunchKernelGGL((kb_sweep_x<false, false>), dim3(b->n_x), dim3(64), 0, b->stream, ka, tx);
  }
}

static void batch_stage(wcns_batch* b, int s, bool cont = false) {
  if (b->ytile == 2) batch_stage_launches<2>(b, s, cont);
  else if (b->ytile == 8) batch_stage_launches<8>(b, s, cont);
  else if (b->ytile == 16) batch_stage_launches<16>(b, s, cont);
  else batch_stage_launches<4>(b, s, cont);
  if (s == 2)
    hipLaunchKernelGGL(kb_tick, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->d_live, b->n);
}

static wcns_status batch_layout(wcns_batch* b, int n, const wcns_grid* grids, double* const* W) {
  size_t need = 0;
  std::vector<size_t> off(n);
  for (int k = 0; k < n; ++k) {
    off[k] = need;
    need += inst_doubles(grids[k], b->nv);
  }
  // (a set that does not fit, or per-instance arrays that cannot be
  // allocated, leave the bound set as it was; the caller has synchronised
  // the batch stream)
  if (need > b->arena_cap) return WCNS_ERR_NOMEM;
  if (n > b->dt_cap) {
    double* dt = nullptr;
    int32_t* live = nullptr;
    unsigned long long* viol = nullptr;
    if (hipMalloc((void**)&dt, sizeof(double) * n) != hipSuccess ||
        hipMalloc((void**)&live, sizeof(int32_t) * n) != hipSuccess ||
        hipMalloc((void**)&viol, sizeof(unsigned long long) * n) != hipSuccess) {
      if (dt) (void)hipFree(dt);
      if (live) (void)hipFree(live);
      if (viol) (void)hipFree(viol);
      return WCNS_ERR_NOMEM;
    }
    if (b->d_dt) (void)hipFree(b->d_dt);
    if (b->d_live) (void)hipFree(b->d_live);
    if (b->d_viol) (void)hipFree(b->d_viol);
    b->d_dt = dt;
    b->d_live = live;
    b->d_viol = viol;
    b->dt_cap = n;
  }
  b->n = n;
  b->grids.assign(grids, grids + n);
  b->W.assign(W, W + n);
  b->off = off;
  // every instance live for ever until told otherwise, no violation yet
  std::vector<int32_t> live(n, 0x7fffffff);
  std::vector<unsigned long long> zero(n, 0ull);
  if (hipMemcpy(b->d_live, live.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_viol, zero.data(), sizeof(unsigned long long) * n, hipMemcpyHostToDevice) !=
          hipSuccess) {
    batch_invalidate(b);
    return WCNS_ERR_HIP;
  }
  return batch_build(b);
}

extern "C" {

wcns_status wcns_batch_destroy(wcns_batch* b) {
  if (!b) return WCNS_ERR_ARG;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  batch_drop_graph(b);
  if (b->arena) (void)hipFree(b->arena);
  if (b->d_ka) (void)hipFree(b->d_ka);
  if (b->d_tasks) (void)hipFree(b->d_tasks);
  if (b->d_dt) (void)hipFree(b->d_dt);
  if (b->d_live) (void)hipFree(b->d_live);
  if (b->d_viol) (void)hipFree(b->d_viol);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return WCNS_OK;
}

wcns_status wcns_batch_create(int32_t n, const wcns_grid* grids, const wcns_eos* eos,
                              const wcns_params* prm, int32_t precision, double* const* W,
                              int64_t capacity_cells, wcns_batch** out) {
  if (!out) return WCNS_ERR_ARG;
  *out = nullptr;
  if (n < 1 || !grids || !eos || !prm || !W) return WCNS_ERR_ARG;
  for (int k = 0; k < n; ++k)
    if (!W[k]) return WCNS_ERR_ARG;
  const int ndim = grids[0].ndim;
  if (ndim != 1 && ndim != 2) return WCNS_ERR_ARG;
  wcns_status st = batch_check_grids(n, grids, ndim);
  if (st != WCNS_OK) return st;
  if (!eos_ok(eos)) return WCNS_ERR_EOS;
  if (!params_ok(prm)) return WCNS_ERR_ARG;
  if (precision != WCNS_FP64 && precision != WCNS_FP32_BULK) return WCNS_ERR_ARG;
  if (capacity_cells < 0) return WCNS_ERR_ARG;
  wcns_batch* b = new wcns_batch();
  b->ndim = ndim;
  b->nv = ndim == 1 ? 5 : 6;
  b->precision = precision;
  b->eos = *eos;
  b->params = *prm;
  KArgs& a = b->proto;
  memset(&a, 0, sizeof(a));
  a.nv = b->nv;
  a.interp_limiter = prm->interp_limiter ? 1 : 0;
  a.flux_limiter = prm->flux_limiter ? 1 : 0;
  a.scheme = prm->scheme;
  a.eos.g1 = 1.0 / (eos->gamma[0] - 1.0);
  a.eos.g2 = 1.0 / (eos->gamma[1] - 1.0);
  a.eos.q1 = eos->gamma[0] * eos->pinf[0] / (eos->gamma[0] - 1.0);
  a.eos.q2 = eos->gamma[1] * eos->pinf[1] / (eos->gamma[1] - 1.0);
  a.tol.eps_arho = prm->eps_arho;
  a.tol.eps_alpha = prm->eps_alpha;
  a.tol.eps_rhoc2 = prm->eps_rhoc2;
  a.tol.hs_arho = prm->hs_arho;
  a.tol.hs_alpha = prm->hs_alpha;
  a.tol.hs_rhoc2 = prm->hs_rhoc2;
  a.tol.weno_eps = prm->weno_eps;
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return WCNS_ERR_HIP;
  }
  // the Dirichlet slots of the arguments must point at readable memory
  size_t need = 32;
  for (int k = 0; k < n; ++k) need += inst_doubles(grids[k], b->nv);
  if (capacity_cells > 0) {
    wcns_grid big = grids[0];
    big.nx = (int32_t)std::min<int64_t>(capacity_cells, (1L << 29) - 1);
    big.ny = 1;
    size_t cap = inst_doubles(big, b->nv) + (size_t)n * 4096;
    need = std::max(need, cap);
  }
  if (hipMalloc((void**)&b->arena, need * sizeof(double)) != hipSuccess) {
    wcns_batch_destroy(b);
    return WCNS_ERR_NOMEM;
  }
  b->arena_cap = need - 32;
  double* dummy = b->arena + b->arena_cap;
  a.dirW = dummy;
  a.dirP = dummy;
  st = batch_layout(b, n, grids, W);
  if (st != WCNS_OK) {
    wcns_batch_destroy(b);
    return st;
  }
  *out = b;
  return WCNS_OK;
}

wcns_status wcns_batch_reset(wcns_batch* b, int32_t n, const wcns_grid* grids, double* const* W) {
  if (!b || n < 1 || !grids || !W) return WCNS_ERR_ARG;
  for (int k = 0; k < n; ++k)
    if (!W[k]) return WCNS_ERR_ARG;
  wcns_status st = batch_check_grids(n, grids, b->ndim);
  if (st != WCNS_OK) return st;
  HIP_TRY(hipStreamSynchronize(b->stream));
  return batch_layout(b, n, grids, W);
}

wcns_status wcns_batch_configure(wcns_batch* b, int32_t ytile, int32_t order) {
  if (!b || (ytile != 2 && ytile != 4 && ytile != 8 && ytile != 16) || order < 0 || order > 2)
    return WCNS_ERR_ARG;
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->ytile = ytile;
  b->order = order;
  return b->n > 0 ? batch_build(b) : WCNS_OK;   // (no set bound: the next reset builds)
}

wcns_status wcns_batch_step(wcns_batch* b, int32_t nsteps) {
  if (!b || nsteps < 0 || b->n < 1) return WCNS_ERR_ARG;
  if (b->dirty) {
    batch_drop_graph(b);
    for (int cont = 0; cont < 2; ++cont) {
      HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      for (int s = 0; s < 3; ++s) batch_stage(b, s, cont == 1);
      hipError_t e1 = hipGetLastError();
      hipError_t e2 = hipStreamEndCapture(b->stream, cont ? &b->graph2 : &b->graph);
      if (e1 != hipSuccess || e2 != hipSuccess) { batch_drop_graph(b); return WCNS_ERR_HIP; }
      HIP_TRY(hipGraphInstantiate(cont ? &b->exec2 : &b->exec, cont ? b->graph2 : b->graph,
                                  nullptr, nullptr, 0));
    }
    b->dirty = false;
  }
  // the first step of the call recovers the node primitives of the states
  // as given; the later ones take them from the step before
  for (int k = 0; k < nsteps; ++k) HIP_TRY(hipGraphLaunch(k == 0 ? b->exec : b->exec2, b->stream));
  return WCNS_OK;
}

wcns_status wcns_batch_rhs(wcns_batch* b) {
  if (!b || b->n < 1) return WCNS_ERR_ARG;
  batch_stage(b, 3);
  LAUNCH_CHECK();
  return WCNS_OK;
}

wcns_status wcns_batch_sync(wcns_batch* b) {
  if (!b) return WCNS_ERR_ARG;
  HIP_TRY(hipStreamSynchronize(b->stream));
  return WCNS_OK;
}

wcns_status wcns_batch_stream(wcns_batch* b, void** stream) {
  if (!b || !stream) return WCNS_ERR_ARG;
  *stream = (void*)b->stream;
  return WCNS_OK;
}

wcns_status wcns_batch_set_steps(wcns_batch* b, const int32_t* steps) {
  if (!b || !steps) return WCNS_ERR_ARG;
  if (b->n < 1) return WCNS_OK;
  for (int k = 0; k < b->n; ++k)
    if (steps[k] < 0) return WCNS_ERR_ARG;
  HIP_TRY(hipMemcpyAsync(b->d_live, steps, sizeof(int32_t) * b->n, hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return WCNS_OK;
}

wcns_status wcns_batch_steps_left(wcns_batch* b, int32_t* steps) {
  if (!b || !steps) return WCNS_ERR_ARG;
  if (b->n < 1) return WCNS_OK;
  HIP_TRY(hipMemcpyAsync(steps, b->d_live, sizeof(int32_t) * b->n, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return WCNS_OK;
}

wcns_status wcns_prim_to_cons_n(const wcns_eos* eos, int32_t ndim, int64_t ncell, const double* V,
                                double* W, void* stream) {
  if (!eos || !V || !W || (ndim != 1 && ndim != 2) || ncell < 1) return WCNS_ERR_ARG;
  if (!eos_ok(eos)) return WCNS_ERR_EOS;
  KArgs a;
  memset(&a, 0, sizeof(a));
  a.nx = (int32_t)std::min<int64_t>(ncell, 0x7fffffff);
  a.ny = 1;
  if (ncell > 0x7fffffff) return WCNS_ERR_ARG;
  a.eos.g1 = 1.0 / (eos->gamma[0] - 1.0);
  a.eos.g2 = 1.0 / (eos->gamma[1] - 1.0);
  a.eos.q1 = eos->gamma[0] * eos->pinf[0] / (eos->gamma[0] - 1.0);
  a.eos.q2 = eos->gamma[1] * eos->pinf[1] / (eos->gamma[1] - 1.0);
  unsigned g = (unsigned)((ncell + 255) / 256);
  if (ndim == 2)
    hipLaunchKernelGGL(k_prim_to_cons<true>, dim3(g), dim3(256), 0, (hipStream_t)stream, a, V, W);
  else
    hipLaunchKernelGGL(k_prim_to_cons<false>, dim3(g), dim3(256), 0, (hipStream_t)stream, a, V, W);
  LAUNCH_CHECK();
  return WCNS_OK;
}

wcns_status wcns_batch_violations(wcns_batch* b, int64_t* counts, int32_t clear) {
  if (!b || !counts) return WCNS_ERR_ARG;
  if (b->n < 1) return WCNS_OK;   // no instance set bound
  std::vector<unsigned long long> h(b->n);
  HIP_TRY(hipMemcpyAsync(h.data(), b->d_viol, sizeof(unsigned long long) * b->n,
                         hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int k = 0; k < b->n; ++k) counts[k] = (int64_t)h[k];
  if (clear) {
    hipLaunchKernelGGL(k_zero_u64, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->d_viol, b->n);
    LAUNCH_CHECK();
    HIP_TRY(hipStreamSynchronize(b->stream));
  }
  return WCNS_OK;
}

wcns_status wcns_batch_dt(wcns_batch* b, double* dt) {
  if (!b || !dt) return WCNS_ERR_ARG;
  if (b->n < 1) return WCNS_OK;
  HIP_TRY(hipMemcpyAsync(dt, b->d_dt, sizeof(double) * b->n, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return WCNS_OK;
}

}  // extern "C"

// the allocation-free right-hand side (uses the set-up and launch sequences above)
#include "wcns_noalloc.hpp"
