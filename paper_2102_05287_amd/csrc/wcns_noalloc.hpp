// Allocation-free right-hand side (included at the end of wcns_api.hip:
// it uses that file's validation, context set-up and launch sequences).
#pragma once
#include <mutex>

// ---------------------------------------------------------------- no allocation
// The allocation-free right-hand side keeps its scratch (node primitives,
// y-tile edge fluxes, block maxima, step record, the first-order pass's
// sink) in this file-scope device
// array: every GPU the library runs on holds its own copy until the process
// ends, and every call on that GPU shares it.  Its device address is taken
// once per device with hipGetSymbolAddress; the host-side name is only a
// stand-in and is never handed to a kernel or a copy.
static __device__ __align__(256) double scratch[WCNS_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[NOALLOC_MAX_DEVICES];

// device address of the current device's scratch (looked up on its first use)
static wcns_status noalloc_scratch(double** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return WCNS_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return WCNS_ERR_HIP;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return WCNS_OK;
}

static size_t round32d(size_t x) { return (x + 31) & ~(size_t)31; }

extern "C" wcns_status wcns_rhs_noalloc(const wcns_grid* g, const wcns_eos* eos, const wcns_params* prm,
                             int32_t precision, void* stream, const double* W, double* dWdt,
                             double dt) {
  if (!g || !eos || !prm || !W || !dWdt || W == dWdt) return WCNS_ERR_ARG;
  wcns_status chk = check_setup(g, eos, prm, precision);
  if (chk != WCNS_OK) return chk;
  for (int k = 0; k < 2 * g->ndim; ++k)
    if (g->bc[k] == WCNS_BC_DIRICHLET) return WCNS_ERR_ARG;
  if (!(dt >= 0.0) || !isfinite(dt)) return WCNS_ERR_CFL;
  wcns_ctx c;
  memset(&c, 0, sizeof(c));
  ctx_setup(&c, g, eos, prm, precision, stream);
  // scratch: P [5][N], (2D) edges [nbr][12][nx], block maxima, step record,
  // (first-order scheme) the sink of the one-pass stage
  const size_t nP = round32d(5 * (size_t)c.N);
  const size_t nE = g->ndim == 2 ? round32d((size_t)c.nbr * 12 * g->nx) : 0;
  const size_t nB = round32d(2 * (size_t)c.node_grid);
  const size_t nS = c.fo ? 8 * (size_t)FO_SINK_SLOTS : 0;
  if ((nP + nE + nB + 32 + nS) * sizeof(double) > WCNS_NOALLOC_SCRATCH_BYTES) return WCNS_ERR_TOO_LARGE;
  double* base = nullptr;
  wcns_status st = noalloc_scratch(&base);
  if (st != WCNS_OK) return st;
  c.P = base;
  c.edge = g->ndim == 2 ? base + nP : nullptr;
  c.partial = base + nP + nE;
  c.step = base + nP + nE + nB;
  c.sink = c.fo ? base + nP + nE + nB + 32 : nullptr;
  c.base.edge = c.edge;
  c.base.step = c.step;
  st = launch_node_finalize(&c, W, DT_GIVEN, dt, nullptr);
  if (st != WCNS_OK) return st;
  if (c.fo) return launch_fo(&c, W, dWdt, OUT_STORE, nullptr, 0.0, 0.0, false, false);
  return launch_sweeps(&c, W, dWdt, OUT_STORE, nullptr, 0.0, 0.0);
}

