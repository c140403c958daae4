"""ctypes binding of the serial FP64 reference implementation (the oracle).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; the GPU library never calls it.

The C++ source is ``wcns_oracle.cpp`` next to this file; ``build()`` compiles
it with ``g++ -O2 -ffp-contract=off`` into ``liboracle.so``.

All arrays are numpy float64, SoA ``[nvar][ny][nx]`` with
nvar = 5 in 1D (a1r1, a2r2, rho u, E, a1) and 6 in 2D
(a1r1, a2r2, rho u, rho v, E, a1), and ``[7][nz][ny][nx]`` in 3D
(a1r1, a2r2, rho u, rho v, rho w, E, a1)  [paper Sec. 2/3, conservative W].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wcns_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_EXTRAP, BC_REFLECT, BC_DIRICHLET = 0, 1, 2, 3


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_FLAGS = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]


def build() -> str:
    """Compile the oracle (always; a few seconds): the serial library and
    the same source with OpenMP over grid rows and lines (the all-cores
    baseline)."""
    subprocess.check_call(_FLAGS + ["-Wno-unknown-pragmas", _SRC, "-o", _LIB + ".tmp"])
    os.replace(_LIB + ".tmp", _LIB)
    subprocess.check_call(_FLAGS + ["-fopenmp", _SRC, "-o", _LIB_OMP + ".tmp"])
    os.replace(_LIB_OMP + ".tmp", _LIB_OMP)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("pad0", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double),
        ("bc", C.c_int32 * 4),
        ("dirichlet_rows", C.c_void_p * 4),
        ("gamma", C.c_double * 2), ("pinf", C.c_double * 2),
        ("eps_arho", C.c_double), ("eps_alpha", C.c_double), ("eps_rhoc2", C.c_double),
        ("hs_arho", C.c_double), ("hs_alpha", C.c_double), ("hs_rhoc2", C.c_double),
        ("weno_eps", C.c_double), ("cfl", C.c_double),
        ("interp_limiter", C.c_int32), ("flux_limiter", C.c_int32), ("scheme", C.c_int32),
        ("pad1", C.c_int32),
        ("nz", C.c_int32), ("bcz", C.c_int32 * 2), ("pad2", C.c_int32),
        ("dz", C.c_double),
    ]


@dataclass
class Setup:
    """Grid, fluids and scheme options of one problem (oracle side)."""
    ndim: int
    nx: int
    ny: int = 1
    dx: float = 1.0
    dy: float = 1.0
    bc: tuple = (BC_PERIODIC,) * 4       # x-lo, x-hi, y-lo, y-hi [, z-lo, z-hi]
    nz: int = 1                          # 3D only
    dz: float = 1.0
    # Dirichlet sides: primitive ghost state (a1r1, a2r2, u, [v], p, a1), one
    # nvar-vector for the whole side or an array [n_side][nvar] per boundary
    # row (x sides: ny rows) or column (y sides: nx columns)
    dirichlet_prim: list = field(default_factory=lambda: [None] * 4)
    gamma: tuple = (6.12, 1.4)           # water, air   [Table 1]
    pinf: tuple = (3.43e8, 0.0)
    eps_arho: float = 1e-10              # [Sec. 5.1]
    eps_alpha: float = 1e-10
    eps_rhoc2: float = 1e-8
    hs_arho: float = 1e-11
    hs_alpha: float = 1e-11
    hs_rhoc2: float = 1e-9
    weno_eps: float = 1e-40
    cfl: float = 0.5                      # [Sec. 6]
    interp_limiter: bool = True
    flux_limiter: bool = True
    scheme: int = 0                       # 0 PP-WCNS-IS, 1 first-order HLLC

    @property
    def nvar(self) -> int:
        return {1: 5, 2: 6, 3: 7}[self.ndim]

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * (self.nz if self.ndim == 3 else 1)

    def c(self) -> _Problem:
        p = _Problem()
        p.ndim, p.nx, p.ny = self.ndim, self.nx, self.ny
        p.dx, p.dy = self.dx, self.dy
        p.nz = self.nz if self.ndim == 3 else 1
        p.dz = self.dz
        for k in range(4):
            p.bc[k] = int(self.bc[k])
        for k in range(2):
            p.bcz[k] = int(self.bc[4 + k]) if len(self.bc) > 4 else BC_PERIODIC
        p.gamma[0], p.gamma[1] = self.gamma
        p.pinf[0], p.pinf[1] = self.pinf
        p.eps_arho, p.eps_alpha, p.eps_rhoc2 = self.eps_arho, self.eps_alpha, self.eps_rhoc2
        p.hs_arho, p.hs_alpha, p.hs_rhoc2 = self.hs_arho, self.hs_alpha, self.hs_rhoc2
        p.weno_eps, p.cfl = self.weno_eps, self.cfl
        p.interp_limiter = int(bool(self.interp_limiter))
        p.flux_limiter = int(bool(self.flux_limiter))
        p.scheme = int(self.scheme)
        # conservative ghost rows of the Dirichlet sides, made once per
        # distinct input with the oracle's own EOS [Sec. 2] and kept alive
        # on the Setup for the Problem's pointers
        key = tuple((k, np.asarray(self.dirichlet_prim[k], dtype=np.float64).tobytes())
                    for k in range(4) if self.bc[k] == BC_DIRICHLET)
        key += (self.gamma, self.pinf, self.nx, self.ny, self.ndim)
        if getattr(self, "_rows_key", None) != key:
            rows = {}
            for k in range(4):
                if self.bc[k] != BC_DIRICHLET:
                    continue
                n_side = self.ny if k < 2 else self.nx
                V = np.asarray(self.dirichlet_prim[k], dtype=np.float64).reshape(-1, self.nvar)
                if V.shape[0] not in (1, n_side):
                    raise ValueError(f"Dirichlet side {k}: need 1 or {n_side} rows")
                Vt = np.ascontiguousarray(np.broadcast_to(V, (n_side, self.nvar)).T)
                Wt = np.empty_like(Vt)
                lib().oracle_prim_to_cons(C.byref(p), _dp(Vt), _dp(Wt), C.c_long(n_side))
                rows[k] = np.ascontiguousarray(Wt.T)
            self._rows, self._rows_key = rows, key
        for k, Wr in self._rows.items():
            p.dirichlet_rows[k] = Wr.ctypes.data
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if any(not os.path.exists(f) or os.path.getmtime(f) < os.path.getmtime(_SRC)
               for f in (_LIB, _LIB_OMP)):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER(_Problem)
        dp = C.POINTER(C.c_double)
        L.oracle_eos_valid.argtypes = [P]
        L.oracle_prim_to_cons.argtypes = [P, dp, dp, C.c_long]
        L.oracle_cons_to_prim.argtypes = [P, dp, dp, dp, C.c_long]
        L.oracle_rhs.argtypes = [P, dp, dp, C.c_double]
        L.oracle_rhs_cells.argtypes = [P, dp, C.c_double, C.POINTER(C.c_int64), C.c_long, dp]
        L.oracle_faces.argtypes = [P, dp, C.c_int, C.c_double, dp, dp, dp]
        L.oracle_flux_limit_face.argtypes = [P, dp, dp, C.c_double, dp, dp, dp, dp]
        L.oracle_flux_limit_face.restype = C.c_double
        L.oracle_interp_limit.argtypes = [P, dp, dp]
        L.oracle_weno_is.argtypes = [C.c_double] * 6
        L.oracle_weno_is.restype = C.c_double
        L.oracle_hcs.argtypes = [C.c_double] * 7
        L.oracle_hcs.restype = C.c_double
        L.oracle_hllc.argtypes = [P, dp, dp, dp, dp, dp]
        L.oracle_node.argtypes = [P, dp, dp]
        L.oracle_rhoc2_tilde.argtypes = [P, dp]
        L.oracle_rhoc2_tilde.restype = C.c_double
        L.oracle_project.argtypes = [P, dp, dp, dp, dp]
        L.oracle_back_project.argtypes = [P, dp, dp, dp, dp]
        L.oracle_max_wavespeed.argtypes = [P, dp, dp]
        L.oracle_stage_lambda.argtypes = [P, dp, C.c_double, dp]
        L.oracle_count_inadmissible.argtypes = [P, dp]
        L.oracle_count_inadmissible.restype = C.c_long
        L.oracle_cfl_dt.argtypes = [P, dp]
        L.oracle_cfl_dt.restype = C.c_double
        L.oracle_ssprk3_step.argtypes = [P, dp, C.c_double, dp]
        L.oracle_ssprk3_step.restype = C.c_long
        L.oracle_run.argtypes = [P, dp, C.c_double, C.c_double, C.c_long, dp]
        L.oracle_run.restype = C.c_long
        L.oracle_opcount_face.argtypes = [P, dp, C.c_double, C.POINTER(C.c_longlong)]
        L.oracle_opcount_face3.argtypes = [P, dp, C.c_double, C.POINTER(C.c_longlong)]
        L.oracle_opcount_phases.argtypes = [C.POINTER(C.c_longlong)]
        L.oracle_opcount_phases.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _arr(x, n=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


# ---------------------------------------------------------------- grid level
def eos_valid(s: Setup) -> bool:
    return bool(lib().oracle_eos_valid(C.byref(s.c())))


def prim_to_cons(s: Setup, V: np.ndarray) -> np.ndarray:
    V = _arr(V)
    n = V.size // s.nvar
    W = np.empty_like(V)
    lib().oracle_prim_to_cons(C.byref(s.c()), _dp(V), _dp(W), n)
    return W


def cons_to_prim(s: Setup, W: np.ndarray):
    W = _arr(W)
    n = W.size // s.nvar
    V = np.empty_like(W)
    c = np.empty(n)
    lib().oracle_cons_to_prim(C.byref(s.c()), _dp(W), _dp(V), _dp(c), n)
    return V, c.reshape(W.shape[1:])


def rhs(s: Setup, W: np.ndarray, dt: float) -> np.ndarray:
    W = _arr(W)
    L = np.empty_like(W)
    rc = lib().oracle_rhs(C.byref(s.c()), _dp(W), _dp(L), float(dt))
    if rc != 0:
        raise ValueError(f"oracle_rhs failed: {rc}")
    return L


_lib_omp = None


def _omp():
    global _lib_omp
    lib()   # builds both libraries when the source is newer
    if _lib_omp is None:
        L = C.CDLL(_LIB_OMP)
        L.oracle_rhs.argtypes = [C.POINTER(_Problem), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.c_double]
        L.oracle_run.restype = C.c_long
        L.oracle_run.argtypes = [C.POINTER(_Problem), C.POINTER(C.c_double), C.c_double,
                                 C.c_double, C.c_long, C.POINTER(C.c_double)]
        _lib_omp = L
    return _lib_omp


def rhs_parallel(s: Setup, W: np.ndarray, dt: float) -> np.ndarray:
    """rhs() from the OpenMP build of the same source (rows, in 3D lines,
    over the threads of OMP_NUM_THREADS): the same bits, on all cores."""
    _omp()
    W = _arr(W)
    out = np.empty_like(W)
    rc = _lib_omp.oracle_rhs(C.byref(s.c()), _dp(W), _dp(out), float(dt))
    if rc != 0:
        raise ValueError(f"oracle_rhs failed: {rc}")
    return out


def rhs_cells(s: Setup, W: np.ndarray, dt: float, cells: np.ndarray) -> np.ndarray:
    """RHS at flat cell indices j*nx+i only; returns [ncells][nvar]."""
    W = _arr(W)
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
    out = np.empty((cells.size, s.nvar))
    rc = lib().oracle_rhs_cells(C.byref(s.c()), _dp(W), float(dt),
                                cells.ctypes.data_as(C.POINTER(C.c_int64)), cells.size, _dp(out))
    if rc != 0:
        raise ValueError(f"oracle_rhs_cells failed: {rc}")
    return out


def faces(s: Setup, W: np.ndarray, direction: int, dt: float):
    """Limited G^-, G^+ and theta of every face, rotated frame:
    arrays [nline][n+1][NR] and [nline][n+1] (NR = 6, or 7 in 3D, where the
    lines of x, y, z run over (k, j), (k, i), (j, i))."""
    W = _arr(W)
    if s.ndim == 3:
        dims = (s.nx, s.ny, s.nz)
        n = dims[direction]
        nline = s.ncell // n
        nr = 7
    else:
        nline = s.ny if direction == 0 else s.nx
        n = s.nx if direction == 0 else s.ny
        nr = 6
    Gm = np.empty((nline, n + 1, nr))
    Gp = np.empty((nline, n + 1, nr))
    th = np.empty((nline, n + 1))
    rc = lib().oracle_faces(C.byref(s.c()), _dp(W), direction, float(dt), _dp(Gm), _dp(Gp), _dp(th))
    if rc != 0:
        raise ValueError(f"oracle_faces failed: {rc}")
    return Gm, Gp, th


def max_wavespeed(s: Setup, W: np.ndarray) -> np.ndarray:
    a = np.zeros(3 if s.ndim == 3 else 2)
    lib().oracle_max_wavespeed(C.byref(s.c()), _dp(_arr(W)), _dp(a))
    return a


def stage_lambda(s: Setup, W: np.ndarray, dt: float) -> np.ndarray:
    lam = np.zeros(3 if s.ndim == 3 else 2)
    lib().oracle_stage_lambda(C.byref(s.c()), _dp(_arr(W)), float(dt), _dp(lam))
    return lam


def count_inadmissible(s: Setup, W: np.ndarray) -> int:
    return int(lib().oracle_count_inadmissible(C.byref(s.c()), _dp(_arr(W))))


def cfl_dt(s: Setup, W: np.ndarray) -> float:
    return float(lib().oracle_cfl_dt(C.byref(s.c()), _dp(_arr(W))))


def ssprk3_step(s: Setup, W: np.ndarray, dt: float = 0.0):
    """One SSP-RK3 step on a copy; returns (W_new, dt_used, n_bad)."""
    W = _arr(W).copy()
    dtu = C.c_double(0.0)
    bad = lib().oracle_ssprk3_step(C.byref(s.c()), _dp(W), float(dt), C.byref(dtu))
    if bad < 0:
        raise ValueError(f"oracle_ssprk3_step failed: {bad}")
    return W, dtu.value, int(bad)


def run(s: Setup, W: np.ndarray, t_end: float, dt_fixed: float = 0.0, max_steps: int = 10**9):
    """Integrate to t_end on a copy; returns (W, steps, t). Raises if a stage
    produced an inadmissible state."""
    W = _arr(W).copy()
    t = C.c_double(0.0)
    steps = lib().oracle_run(C.byref(s.c()), _dp(W), float(t_end), float(dt_fixed),
                             int(max_steps), C.byref(t))
    if steps == -5:
        raise FloatingPointError(f"inadmissible state at t={t.value}")
    if steps < 0:
        raise ValueError(f"oracle_run failed: {steps}")
    return W, int(steps), t.value


def run_parallel(s: Setup, W: np.ndarray, t_end: float, dt_fixed: float = 0.0,
                 max_steps: int = 10**9):
    """run() from the OpenMP build (its RHS rows or lines over the threads): the same
    bits, on all cores, for the long runs that pin whole solves."""
    W = _arr(W).copy()
    t = C.c_double(0.0)
    steps = _omp().oracle_run(C.byref(s.c()), _dp(W), float(t_end), float(dt_fixed),
                              int(max_steps), C.byref(t))
    if steps == -5:
        raise FloatingPointError(f"inadmissible state at t={t.value}")
    if steps < 0:
        raise ValueError(f"oracle_run failed: {steps}")
    return W, int(steps), t.value


# ---------------------------------------------------------------- point level
def weno_is(a, b, c, d, e, eps=1e-40) -> float:
    return float(lib().oracle_weno_is(a, b, c, d, e, eps))


def hcs(gt, gm2, gm1, g0, gp1, gp2, gp3) -> float:
    return float(lib().oracle_hcs(gt, gm2, gm1, g0, gp1, gp2, gp3))


def hllc(s: Setup, WL, WR):
    """HLLC on rotated 6-states; returns (F[5], f_alpha, s*)."""
    F = np.zeros(5)
    fa = C.c_double(0.0)
    ss = C.c_double(0.0)
    lib().oracle_hllc(C.byref(s.c()), _dp(_arr(WL, 6)), _dp(_arr(WR, 6)), _dp(F),
                      C.byref(fa), C.byref(ss))
    return F, fa.value, ss.value


def node(s: Setup, X):
    """(rho, u_n, u_t, p, c, rho*ctilde^2) of a rotated 6-state."""
    out = np.zeros(6)
    lib().oracle_node(C.byref(s.c()), _dp(_arr(X, 6)), _dp(out))
    return out


def rhoc2_tilde(s: Setup, X) -> float:
    return float(lib().oracle_rhoc2_tilde(C.byref(s.c()), _dp(_arr(X, 6))))


def project(s: Setup, XL, XR, X):
    U = np.zeros(6)
    lib().oracle_project(C.byref(s.c()), _dp(_arr(XL, 6)), _dp(_arr(XR, 6)), _dp(_arr(X, 6)), _dp(U))
    return U


def back_project(s: Setup, XL, XR, U):
    X = np.zeros(6)
    lib().oracle_back_project(C.byref(s.c()), _dp(_arr(XL, 6)), _dp(_arr(XR, 6)), _dp(_arr(U, 6)), _dp(X))
    return X


def interp_limit(s: Setup, A, B):
    B = _arr(B, 6).copy()
    lib().oracle_interp_limit(C.byref(s.c()), _dp(_arr(A, 6)), _dp(B))
    return B


def flux_limit_face(s: Setup, Wl, Wr, lam, Hm, Hp, Gm, Gp):
    Gm = _arr(Gm, 6).copy()
    Gp = _arr(Gp, 6).copy()
    th = lib().oracle_flux_limit_face(C.byref(s.c()), _dp(_arr(Wl, 6)), _dp(_arr(Wr, 6)), float(lam),
                                      _dp(_arr(Hm, 6)), _dp(_arr(Hp, 6)), _dp(Gm), _dp(Gp))
    return Gm, Gp, th


def opcount_face(s: Setup, stencil, lam: float) -> dict:
    """Operation counts: per node (primitive recovery) and per face; a
    [6][6] rotated stencil, or [6][7] for a 3D face."""
    st = _arr(stencil)
    out = (C.c_longlong * 10)()
    if st.size == 42:
        lib().oracle_opcount_face3(C.byref(s.c()), _dp(st), float(lam), out)
    else:
        assert st.size == 36
        lib().oracle_opcount_face(C.byref(s.c()), _dp(st), float(lam), out)
    keys = ["add", "mul", "div", "sqrt", "cmp"]
    res = {"node": dict(zip(keys, out[0:5])), "face": dict(zip(keys, out[5:10]))}
    if st.size == 36:
        ph = (C.c_longlong * (5 * len(PHASES)))()
        assert lib().oracle_opcount_phases(ph) == len(PHASES)
        res["face_phases"] = {name: dict(zip(keys, ph[5 * k:5 * k + 5]))
                              for k, name in enumerate(PHASES)}
    return res


# steps of the face pipeline the op count is filed under (the oracle's PH_ order)
PHASES = ["first_order", "project", "weno", "back_v", "to_w", "interp_limit", "mid_recover",
          "mid_hllc", "hcs", "split_limit"]
