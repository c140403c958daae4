// Drives the oracle (oracle/wcns_oracle.cpp, compiled into this translation
// unit) through small 1D, 2D and 3D solves with every side kind, both
// limiters active, the first-order scheme and Dirichlet rows, so that a build
// with AddressSanitizer and UndefinedBehaviorSanitizer checks every access and
// operation of the reference on the way.  Exits 0 when every solve stayed in
// the admissible set and finite; a sanitizer report aborts the run.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "wcns_oracle.cpp"

namespace {

Problem base(int ndim, int nx, int ny, int nz) {
  Problem P;
  std::memset(&P, 0, sizeof P);
  P.ndim = ndim;
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  P.dx = 1.0 / nx;
  P.dy = 1.0 / ny;
  P.dz = 1.0 / nz;
  P.gamma[0] = 6.12;
  P.gamma[1] = 1.4;
  P.pinf[0] = 3.43e8;
  P.pinf[1] = 0.0;
  P.eps_arho = 1e-10;
  P.eps_alpha = 1e-10;
  P.eps_rhoc2 = 1e-8;
  P.hs_arho = 1e-11;
  P.hs_alpha = 1e-11;
  P.hs_rhoc2 = 1e-9;
  P.weno_eps = 1e-40;
  P.cfl = 0.5;
  P.interp_limiter = 1;
  P.flux_limiter = 1;
  return P;
}

long ncells(const Problem& P) { return (long)P.nx * P.ny * (P.ndim == 3 ? P.nz : 1); }
int nvar(const Problem& P) { return P.ndim + 4; }

// Primitive state of one cell: shocked water left of x = 0.4 (p = 1e9),
// water at rest (p = 1e5) elsewhere, with an air bubble of radius 0.2 at the
// centre; volume-fraction floors of 1e-6.
void cell_prim(const Problem& P, int i, int j, int k, double* v) {
  const double x = (i + 0.5) / P.nx, y = P.ndim >= 2 ? (j + 0.5) / P.ny : 0.5;
  const double z = P.ndim == 3 ? (k + 0.5) / P.nz : 0.5;
  const double r2 = (x - 0.6) * (x - 0.6) + (y - 0.5) * (y - 0.5) + (z - 0.5) * (z - 0.5);
  const bool air = r2 < 0.04;
  const double a1 = air ? 1e-6 : 1.0 - 1e-6;
  const double p = x < 0.4 ? 1e9 : 1e5;
  const int nv = nvar(P);
  v[0] = 1000.0 * a1;
  v[1] = 1.0 * (1.0 - a1);
  for (int d = 0; d < P.ndim; ++d) v[2 + d] = (d == 0 && x < 0.4) ? 400.0 : 0.0;
  v[nv - 2] = p;
  v[nv - 1] = a1;
}

std::vector<double> initial(const Problem& P) {
  const long n = ncells(P);
  const int nv = nvar(P);
  std::vector<double> V(nv * n), W(nv * n), v(nv);
  const int nz = P.ndim == 3 ? P.nz : 1;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < P.ny; ++j)
      for (int i = 0; i < P.nx; ++i) {
        cell_prim(P, i, j, k, v.data());
        const long q = ((long)k * P.ny + j) * P.nx + i;
        for (int c = 0; c < nv; ++c) V[c * n + q] = v[c];
      }
  oracle_prim_to_cons(&P, V.data(), W.data(), n);
  return W;
}

bool finite(const std::vector<double>& a) {
  for (double x : a)
    if (!std::isfinite(x)) return false;
  return true;
}

int solve(const char* name, const Problem& P, int steps) {
  std::vector<double> W = initial(P), L(W.size());
  long bad = 0;
  double dt = 0.0;
  for (int s = 0; s < steps; ++s) bad += oracle_ssprk3_step(&P, W.data(), 0.0, &dt);
  if (oracle_rhs(&P, W.data(), L.data(), dt) != 0) bad += 1;
  double amax[3] = {0, 0, 0};
  oracle_max_wavespeed(&P, W.data(), amax);
  bad += oracle_count_inadmissible(&P, W.data());
  // every face of every direction, before and after limiting
  const int nd = P.ndim;
  long limited = 0;
  for (int dir = 0; dir < nd; ++dir) {
    const long n = dir == 0 ? P.nx : (dir == 1 ? P.ny : P.nz);
    const long nline = ncells(P) / n;
    const int nc = P.ndim == 3 ? 7 : 6;
    std::vector<double> Gm(nline * (n + 1) * nc), Gp(Gm.size()), th(nline * (n + 1));
    if (oracle_faces(&P, W.data(), dir, dt, Gm.data(), Gp.data(), th.data()) != 0) bad += 1;
    if (!finite(Gm) || !finite(Gp)) bad += 1;
    for (double x : th) limited += x < 1.0 ? 1 : 0;
  }
  const bool ok = bad == 0 && finite(W) && finite(L) && amax[0] > 0.0;
  std::printf("%-34s %s (dt %.3e, amax %.4e, %ld faces limited)\n", name, ok ? "ok" : "FAILED", dt,
              amax[0], limited);
  return ok ? 0 : 1;
}

}  // namespace

int main() {
  int fails = 0;
  {
    Problem P = base(1, 64, 1, 1);
    P.bc[0] = P.bc[1] = BC_EXTRAP;
    fails += solve("1D extrapolated", P, 4);
    double t = 0.0;
    std::vector<double> W = initial(P);
    const long steps = oracle_run(&P, W.data(), 3e-5, 0.0, 50, &t);
    std::printf("%-34s %s (%ld steps)\n", "1D run to t_end", steps > 0 ? "ok" : "FAILED", steps);
    fails += steps > 0 ? 0 : 1;
  }
  {
    Problem P = base(2, 24, 20, 1);
    P.bc[0] = P.bc[1] = BC_PERIODIC;
    P.bc[2] = P.bc[3] = BC_REFLECT;
    fails += solve("2D periodic x, reflective y", P, 3);
  }
  {
    Problem P = base(2, 16, 12, 1);
    P.bc[0] = BC_DIRICHLET;
    P.bc[1] = P.bc[2] = P.bc[3] = BC_EXTRAP;
    // conservative ghost state of each x-lo boundary row: the shocked water
    std::vector<double> rows(12 * 6), v(6), w(6);
    cell_prim(P, 0, 0, 0, v.data());
    oracle_prim_to_cons(&P, v.data(), w.data(), 1);
    for (int r = 0; r < 12; ++r)
      for (int c = 0; c < 6; ++c) rows[r * 6 + c] = w[c];
    P.dirichlet_rows[0] = rows.data();
    fails += solve("2D Dirichlet rows on x-lo", P, 3);
  }
  {
    Problem P = base(2, 16, 12, 1);
    P.bc[0] = P.bc[1] = P.bc[2] = P.bc[3] = BC_REFLECT;
    P.scheme = 1;
    fails += solve("2D first-order HLLC, all walls", P, 3);
  }
  {
    Problem P = base(3, 10, 8, 6);
    P.bc[0] = P.bc[1] = BC_PERIODIC;
    P.bc[2] = P.bc[3] = BC_EXTRAP;
    P.bcz[0] = P.bcz[1] = BC_REFLECT;
    fails += solve("3D periodic / extrapolated / walls", P, 2);
  }
  std::printf("fails=%d\n", fails);
  return fails;
}
