"""Thin ctypes binding of libwcns.so (the C ABI in include/wcns.h).

Argument marshalling only: every step of the right-hand side, the limiter
and the Runge-Kutta step runs in the library's HIP kernels.  Device buffers
are torch tensors on the ROCm device (torch's "cuda" device); their
``data_ptr()`` is passed straight to the C ABI, and calls are enqueued on
the current torch stream unless a stream is given.

The library must have been built (``python -m paper_2102_05287_amd.build``
or ``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwcns.so")

WCNS_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "fluids violate Lemma 1", -3: "out of memory",
          -4: "HIP error", -5: "inadmissible state", -6: "invalid time step",
          -7: "grid too large for the allocation-free scratch"}
WCNS_ERR_INADMISSIBLE = -5
BC_PERIODIC, BC_EXTRAP, BC_REFLECT, BC_DIRICHLET = 0, 1, 2, 3
FP64, FP32_BULK = 0, 1
SCHEME_PPWCNSIS, SCHEME_HLLC1 = 0, 1


class WcnsError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({code})")
        self.code = code


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("pad", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("bc", C.c_int32 * 4),
                ("dirichlet", (C.c_double * 6) * 4),
                ("dirichlet_rows", C.c_void_p * 4),
                ("nz", C.c_int32), ("bc_z", C.c_int32 * 2), ("reserved_z", C.c_int32),
                ("z0", C.c_double), ("z1", C.c_double)]


def _state_ptrs(grids, states):
    """Device pointers of the batch states, each checked against its grid:
    contiguous device float64 of [nvar][ny][nx] (nvar 6 in 2D, 5 in 1D)."""
    if len(states) != len(grids):
        raise ValueError(f"{len(grids)} grids but {len(states)} states")
    for k, (g, t) in enumerate(zip(grids, states)):
        n = (6 if g.ndim == 2 else 5) * g.nx * max(g.ny, 1)
        _dev_f64(t, n, f"state {k}")
        if t.numel() != n:
            raise ValueError(f"state {k}: {n} elements expected, got {t.numel()}")
    return (C.c_void_p * len(states))(*[t.data_ptr() for t in states])


class _Eos(C.Structure):
    _fields_ = [("gamma", C.c_double * 2), ("pinf", C.c_double * 2)]


class _Params(C.Structure):
    _fields_ = [("eps_arho", C.c_double), ("eps_alpha", C.c_double), ("eps_rhoc2", C.c_double),
                ("hs_arho", C.c_double), ("hs_alpha", C.c_double), ("hs_rhoc2", C.c_double),
                ("weno_eps", C.c_double), ("cfl", C.c_double),
                ("interp_limiter", C.c_int32), ("flux_limiter", C.c_int32),
                ("scheme", C.c_int32), ("reserved", C.c_int32)]


_lib = None

EXPORTS = ["wcns_params_default", "wcns_create", "wcns_destroy", "wcns_set_stream",
           "wcns_prim_to_cons", "wcns_rhs", "wcns_limit", "wcns_max_wavespeed",
           "wcns_ssprk3_step", "wcns_ssprk3_steps", "wcns_ssprk3_advance", "wcns_violations",
           "wcns_check_admissible", "wcns_profile",
           "wcns_profile_read",
           "wcns_selftest_division", "wcns_selftest_division_by", "wcns_issue_probe", "wcns_run",
           "wcns_batch_create", "wcns_batch_reset",
           "wcns_batch_configure", "wcns_batch_step", "wcns_batch_rhs", "wcns_batch_sync",
           "wcns_batch_stream", "wcns_batch_dt", "wcns_batch_destroy", "wcns_batch_set_steps",
           "wcns_batch_steps_left", "wcns_batch_violations", "wcns_prim_to_cons_n",
           "wcns_rhs_noalloc", "wcns_status_str"]
PROF_CLASSES = ["node", "finalize", "sweep_x", "sweep_y", "fixup_y", "other", "sweep_z", "fo_stage",
                "fo_stage_un"]


def lib():
    """Load libwcns.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m "
                              "paper_2102_05287_amd.build` (no CPU fallback exists)")
        # load torch first so the library binds to the HIP runtime torch
        # already uses (same soname) instead of a second copy
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.c_void_p
        L.wcns_params_default.argtypes = [C.POINTER(_Params)]
        L.wcns_create.argtypes = [C.POINTER(_Grid), C.POINTER(_Eos), C.POINTER(_Params), C.c_int32,
                                  vp, C.POINTER(vp)]
        L.wcns_destroy.argtypes = [vp]
        L.wcns_set_stream.argtypes = [vp, vp]
        L.wcns_prim_to_cons.argtypes = [vp, dp, dp]
        L.wcns_rhs.argtypes = [vp, dp, dp, C.c_double]
        L.wcns_limit.argtypes = [vp, C.c_int32, dp, dp, dp, dp, dp, C.c_double]
        L.wcns_max_wavespeed.argtypes = [vp, dp, dp]
        L.wcns_ssprk3_step.argtypes = [vp, dp, C.c_double, dp]
        L.wcns_ssprk3_steps.argtypes = [vp, dp, C.c_int32, C.c_double, dp]
        L.wcns_ssprk3_advance.argtypes = [vp, dp, C.c_double, C.c_double, C.c_int32, dp, dp, dp]
        L.wcns_violations.argtypes = [vp, C.POINTER(C.c_int64), C.c_int32]
        L.wcns_check_admissible.argtypes = [vp, dp, C.POINTER(C.c_longlong)]
        L.wcns_profile.argtypes = [vp, C.c_int32]
        L.wcns_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
        L.wcns_selftest_division.argtypes = [dp, dp, dp, dp, C.c_int64, vp]
        L.wcns_selftest_division_by.argtypes = [dp, C.c_double, dp, dp, C.c_int64, vp]
        L.wcns_issue_probe.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double), vp]
        L.wcns_run.argtypes = [vp, dp, C.c_double, C.c_double, C.c_double, C.c_int64, dp, C.c_int64,
                               C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.wcns_batch_create.argtypes = [C.c_int32, C.POINTER(_Grid), C.POINTER(_Eos), C.POINTER(_Params),
                                        C.c_int32, C.POINTER(C.c_void_p), C.c_int64, C.POINTER(vp)]
        L.wcns_batch_reset.argtypes = [vp, C.c_int32, C.POINTER(_Grid), C.POINTER(C.c_void_p)]
        L.wcns_batch_configure.argtypes = [vp, C.c_int32, C.c_int32]
        L.wcns_batch_step.argtypes = [vp, C.c_int32]
        L.wcns_batch_rhs.argtypes = [vp]
        L.wcns_batch_sync.argtypes = [vp]
        L.wcns_batch_stream.argtypes = [vp, C.POINTER(vp)]
        L.wcns_batch_dt.argtypes = [vp, C.POINTER(C.c_double)]
        L.wcns_batch_destroy.argtypes = [vp]
        L.wcns_batch_set_steps.argtypes = [vp, C.POINTER(C.c_int32)]
        L.wcns_batch_steps_left.argtypes = [vp, C.POINTER(C.c_int32)]
        L.wcns_batch_violations.argtypes = [vp, C.POINTER(C.c_int64), C.c_int32]
        L.wcns_prim_to_cons_n.argtypes = [C.POINTER(_Eos), C.c_int32, C.c_int64, dp, dp, vp]
        L.wcns_rhs_noalloc.argtypes = [C.POINTER(_Grid), C.POINTER(_Eos), C.POINTER(_Params),
                                       C.c_int32, vp, dp, dp, C.c_double]
        L.wcns_status_str.argtypes = [C.c_int]
        L.wcns_status_str.restype = C.c_char_p
        for name in EXPORTS:
            if name != "wcns_status_str":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code, where):
    if code != WCNS_OK:
        raise WcnsError(code, where)


def default_params(**overrides) -> _Params:
    p = _Params()
    _check(lib().wcns_params_default(C.byref(p)), "wcns_params_default")
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _dev_f64(t, n, what):
    """Check that t is a contiguous device float64 tensor of at least n
    elements (the library writes or reads that many doubles through its
    pointer); None passes."""
    import torch
    if t is None:
        return
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and t.numel() >= n):
        raise ValueError(f"{what}: a contiguous device float64 tensor of >= {n} elements is needed")


class Solver:
    """One grid + fluids + options, bound to a device context.

    grid: ndim, nx, ny, x0, x1, y0, y1, bc (4 kinds; 6 in 3D), dirichlet (per
    side: None, or the primitive ghost state (a1r1, a2r2, u, [v], p, a1) of a
    Dirichlet side as one nvar-vector or as an array [n_side][nvar] of one
    state per boundary row/column); 3D: nz, z0, z1 (state [7][nz][ny][nx])."""

    def __init__(self, ndim, nx, ny, x0, x1, y0=0.0, y1=1.0, bc=(BC_EXTRAP,) * 4,
                 gamma=(6.12, 1.4), pinf=(3.43e8, 0.0), precision=FP64, stream=None,
                 dirichlet=None, nz=1, z0=0.0, z1=1.0, **params):
        import torch
        g = make_grid(ndim, nx, ny, x0, x1, y0, y1, bc, dirichlet, nz, z0, z1)
        e = _Eos()
        e.gamma[0], e.gamma[1] = gamma
        e.pinf[0], e.pinf[1] = pinf
        p = default_params(**params)
        self.ndim, self.nx, self.ny = ndim, nx, ny
        self.nz = nz if ndim == 3 else 1
        self.nvar = {1: 5, 2: 6, 3: 7}[ndim]
        self.dx = (x1 - x0) / nx
        self.dy = (y1 - y0) / ny if ndim >= 2 else 1.0
        self.dz = (z1 - z0) / nz if ndim == 3 else 1.0
        self.params = p
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        ctx = C.c_void_p()
        _check(lib().wcns_create(C.byref(g), C.byref(e), C.byref(p), int(precision),
                                 C.c_void_p(stream), C.byref(ctx)), "wcns_create")
        self._ctx = ctx

    @classmethod
    def from_spec(cls, spec, **kw):
        """Build from a seeded ProblemSpec (paper_2102_05287_amd.problems)."""
        return cls(spec.ndim, spec.nx, spec.ny, spec.x0, spec.x1, spec.y0, spec.y1,
                   bc=spec.bc, gamma=spec.gamma, pinf=spec.pinf, cfl=spec.cfl,
                   dirichlet=spec.dirichlet_prim, nz=spec.nz, z0=spec.z0, z1=spec.z1, **kw)

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().wcns_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._stream = stream
        _check(lib().wcns_set_stream(self._ctx, C.c_void_p(stream)), "wcns_set_stream")

    # ----------------------------------------------------------- buffers
    def empty_state(self, dtype=None):
        import torch
        shape = (self.nvar, self.nz, self.ny, self.nx) if self.ndim == 3 else \
            (self.nvar, self.ny, self.nx)
        return torch.empty(shape, dtype=torch.float64, device="cuda")

    def _chk(self, t):
        n = self.nvar * self.nx * self.ny * self.nz
        _dev_f64(t, n, "state")
        if t.numel() != n:
            raise ValueError(f"state: {n} elements ([nvar]([nz])[ny][nx]) expected, got {t.numel()}")

    # ----------------------------------------------------------- entry points
    def prim_to_cons(self, V, W=None):
        self._chk(V)
        W = self.empty_state() if W is None else W
        self._chk(W)
        _check(lib().wcns_prim_to_cons(self._ctx, _ptr(V), _ptr(W)), "wcns_prim_to_cons")
        return W

    def rhs(self, W, dWdt=None, dt=0.0):
        self._chk(W)
        dWdt = self.empty_state() if dWdt is None else dWdt
        self._chk(dWdt)
        _check(lib().wcns_rhs(self._ctx, _ptr(W), _ptr(dWdt), float(dt)), "wcns_rhs")
        return dWdt

    def steps(self, W, n, dt=0.0, dts=None):
        """n SSP-RK3 steps in place on W (wcns_ssprk3_steps): the same bits
        as n calls of step(); dts: optional device float64 tensor of >= n
        elements receiving each step's dt."""
        self._chk(W)
        _dev_f64(dts, max(int(n), 0), "dts")
        _check(lib().wcns_ssprk3_steps(self._ctx, _ptr(W), int(n), float(dt), _ptr(dts)),
               "wcns_ssprk3_steps")

    def step(self, W, dt=0.0, dt_used=None):
        """One SSP-RK3 step in place on W; dt <= 0 selects the CFL step.
        dt_used: optional device float64 tensor of >= 1 element."""
        self._chk(W)
        _dev_f64(dt_used, 1, "dt_used")
        _check(lib().wcns_ssprk3_step(self._ctx, _ptr(W), float(dt), _ptr(dt_used)),
               "wcns_ssprk3_step")
        return W

    def _capture(self, enqueue):
        """A HIP graph of the library work `enqueue()` puts on this solver's
        stream (kernel nodes only: the entry points used here only launch
        kernels); replay() runs it on the current torch stream."""
        import torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        old = self._stream
        g = torch.cuda.CUDAGraph()
        self.set_stream(s.cuda_stream)
        try:
            with torch.cuda.graph(g, stream=s):
                enqueue()
        finally:
            self.set_stream(old)
        return g

    def capture_steps(self, W, n, dt_used):
        """A HIP graph of n device-CFL SSP-RK3 steps of W in place, step k
        writing its dt to dt_used[k]."""
        return self._capture(lambda: self.steps(W, n, 0.0, dts=dt_used))

    def capture_advance(self, W, t_end, n, clock, steps_taken):
        """A HIP graph of n steps of the device time loop toward t_end
        (advance_steps); replays continue from the device clock."""
        return self._capture(lambda: self.advance_steps(W, t_end, n, clock, steps_taken))

    def advance_steps(self, W, t_end, n, clock, steps_taken=None, dts=None, dt=0.0):
        """Enqueue up to n SSP-RK3 steps of the device time loop toward t_end
        (wcns_ssprk3_advance), each of size dt > 0 or the CFL step (dt <= 0):
        clock is a device float64 tensor holding the time (updated on the
        device), steps_taken an optional device int64 tensor counting the
        steps taken, dts an optional device tensor of >= n elements
        receiving each step slot's dt (0 when skipped)."""
        import torch
        self._chk(W)
        _dev_f64(clock, 1, "clock")
        _dev_f64(dts, max(int(n), 0), "dts")
        if steps_taken is not None and not (isinstance(steps_taken, torch.Tensor) and steps_taken.is_cuda
                                            and steps_taken.dtype == torch.int64
                                            and steps_taken.numel() >= 1):
            raise ValueError("steps_taken: a device int64 tensor is needed")
        _check(lib().wcns_ssprk3_advance(self._ctx, _ptr(W), float(dt), float(t_end), int(n),
                                         _ptr(clock), _ptr(steps_taken), _ptr(dts)),
               "wcns_ssprk3_advance")

    def advance(self, W, t_end, t=0.0, chunk=64, max_steps=1 << 40, dt=0.0):
        """March W in place from time t to t_end (the time loop of the
        paper's runs): the library takes steps of size dt > 0 or, by default,
        picks every CFL step, and shortens the last one to land on t_end,
        keeping the time on the device; the host only
        enqueues chunks of `chunk` steps and reads the step count once per
        chunk, stopping when a chunk took fewer steps than it enqueued.
        Raises WcnsError (inadmissible state) if the kernels found a cell
        outside the admissible set on the way, and WcnsError (invalid time
        step) if the device loop stopped short of t_end because a step was
        not positive.  Returns (steps, t)."""
        import torch
        clock = torch.full((1,), float(t), dtype=torch.float64, device="cuda")
        taken = torch.zeros(1, dtype=torch.int64, device="cuda")
        done = 0
        while done < max_steps:
            n = int(min(chunk, max_steps - done))
            self.advance_steps(W, t_end, n, clock, taken, dt=dt)
            now = int(taken.item())
            if now - done < n:
                done = now
                break
            done = now
        self.check_violations()
        t_now = float(clock.item())
        if done < max_steps and not t_now >= t_end:
            raise WcnsError(-6, f"the device time loop stopped at t = {t_now!r} < t_end "
                                "(a step would not advance the time)")
        return done, t_now

    def violations(self, clear=False) -> int:
        """Cells the kernels found outside the admissible set since creation
        or the last clear (wcns_violations; synchronises)."""
        n = C.c_int64(0)
        rc = lib().wcns_violations(self._ctx, C.byref(n), int(bool(clear)))
        if rc not in (WCNS_OK, -5):
            _check(rc, "wcns_violations")
        return int(n.value)

    def check_violations(self):
        """Raise WcnsError(-5) if the kernels found an inadmissible cell."""
        n = self.violations()
        if n:
            raise WcnsError(-5, f"{n} cells outside the admissible set")

    def run(self, W, t_end, t=0.0, dt_fixed=0.0, max_steps=1 << 40, dts=None):
        """1D grids of at most 4096 cells: the whole time loop to t_end in
        one device launch (wcns_run); W in place.  dts: optional device f64
        tensor receiving the dt of each step.  Returns (steps, t)."""
        self._chk(W)
        _dev_f64(dts, 0, "dts")
        n = C.c_int64(0)
        tt = C.c_double(0.0)
        cap = 0 if dts is None else dts.numel()
        _check(lib().wcns_run(self._ctx, _ptr(W), float(t), float(t_end), float(dt_fixed),
                              int(max_steps), _ptr(dts), cap, C.byref(n), C.byref(tt)), "wcns_run")
        return int(n.value), tt.value

    def max_wavespeed(self, W, out=None):
        import torch
        self._chk(W)
        if out is None:
            out = torch.zeros(3 if self.ndim == 3 else 2, dtype=torch.float64, device="cuda")
        _dev_f64(out, 3 if self.ndim == 3 else 2, "out")
        _check(lib().wcns_max_wavespeed(self._ctx, _ptr(W), _ptr(out)), "wcns_max_wavespeed")
        return out

    def limit(self, direction, W, G_ho, G_lo, dt, G_out=None, theta=None):
        import torch
        self._chk(W)
        nf = (self.nx + 1) * self.ny if direction == 0 else self.nx * (self.ny + 1)
        if G_out is None:
            G_out = torch.empty((2, self.nvar, nf), dtype=torch.float64, device="cuda")
        _dev_f64(G_ho, (self.nvar + 1) * nf, "G_ho")
        _dev_f64(G_lo, (self.nvar + 1) * nf, "G_lo")
        _dev_f64(G_out, 2 * self.nvar * nf, "G_out")
        _dev_f64(theta, nf, "theta")
        _check(lib().wcns_limit(self._ctx, int(direction), _ptr(W), _ptr(G_ho), _ptr(G_lo),
                                _ptr(G_out), _ptr(theta), float(dt)), "wcns_limit")
        return G_out

    def count_inadmissible(self, W) -> int:
        self._chk(W)
        n = C.c_longlong(0)
        _check(lib().wcns_check_admissible(self._ctx, _ptr(W), C.byref(n)), "wcns_check_admissible")
        return int(n.value)

    # ----------------------------------------------------------- measurement
    def profile(self, enable: bool):
        _check(lib().wcns_profile(self._ctx, int(bool(enable))), "wcns_profile")

    def profile_read(self, reset: bool = True) -> dict:
        ms = (C.c_double * len(PROF_CLASSES))()
        n = (C.c_int64 * len(PROF_CLASSES))()
        _check(lib().wcns_profile_read(self._ctx, ms, n, int(bool(reset))), "wcns_profile_read")
        return {k: (ms[i], n[i]) for i, k in enumerate(PROF_CLASSES)}


def selftest_division(a, b):
    """(IEEE quotient, kernels' division core) of device f64 tensors a, b."""
    import torch
    _dev_f64(a, 0, "a")
    _dev_f64(b, a.numel(), "b")
    qi = torch.empty_like(a)
    qc = torch.empty_like(a)
    _check(lib().wcns_selftest_division(_ptr(a), _ptr(b), _ptr(qi), _ptr(qc), a.numel(),
                                        C.c_void_p(torch.cuda.current_stream().cuda_stream)),
           "wcns_selftest_division")
    return qi, qc


def selftest_division_by(a, b: float):
    """(IEEE quotient, kernels' constant-divisor path) of device tensor a and
    the scalar b; None when b does not take that path."""
    import torch
    _dev_f64(a, 0, "a")
    qi = torch.empty_like(a)
    qc = torch.empty_like(a)
    rc = lib().wcns_selftest_division_by(_ptr(a), float(b), _ptr(qi), _ptr(qc), a.numel(),
                                         C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc == -1:
        return None
    _check(rc, "wcns_selftest_division_by")
    return qi, qc


PROBE_OPS = {"fma": 0, "add": 1, "mul": 2, "div": 3, "sqrt": 4, "div_core": 5,
             "fma_f32": 6, "div_f32": 7, "sqrt_f32": 8}


def issue_probe(op: str, iters: int, blocks: int = 0) -> float:
    """Device time (ms) of `iters` rounds of 8 independent chains of one FP64
    or FP32 operation per lane over a grid that fills every SIMD
    (wcns_issue_probe)."""
    import torch
    ms = C.c_double(0.0)
    _check(lib().wcns_issue_probe(PROBE_OPS[op], int(iters), int(blocks), C.byref(ms),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream)),
           "wcns_issue_probe")
    return ms.value


def issue_weights(iters: int = 2048) -> dict:
    """Issue cost of each probed operation in FP64 FMA slots: its time over
    the time of an FP64 FMA probe of equal work run just before it (so clock
    changes between probes cancel), plus the measured FMA issue rate in
    slots/s."""
    for _ in range(4):                            # warm-up: code load, clocks up
        issue_probe("fma", iters)
    for op in PROBE_OPS:                          # and once per op: the first measured
        issue_probe(op, iters)                    # pass ran ~8% off the later ones
    t, w = {}, {}
    for op in PROBE_OPS:
        tf = issue_probe("fma", iters)
        t[op] = issue_probe(op, iters)
        w[op] = t[op] / tf
    import torch
    props = torch.cuda.get_device_properties(0)
    lanes = 32 * props.multi_processor_count * 256
    return {"weights": w, "fma_slots_per_s": lanes * 8.0 * iters / (t["fma"] / 1e3),
            "ms": t, "iters": iters}


def prim_to_cons(V, ndim, gamma=(6.12, 1.4), pinf=(3.43e8, 0.0), W=None):
    """Device primitive -> conservative conversion without a solver context
    (V: device f64 [nvar][...]); enqueued on the current torch stream."""
    import torch
    W = torch.empty_like(V) if W is None else W
    e = _Eos()
    e.gamma[0], e.gamma[1] = gamma
    e.pinf[0], e.pinf[1] = pinf
    ncell = V.numel() // (5 if ndim == 1 else 6)
    _check(lib().wcns_prim_to_cons_n(C.byref(e), int(ndim), int(ncell), _ptr(V), _ptr(W),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream)),
           "wcns_prim_to_cons_n")
    return W


def make_grid(ndim, nx, ny, x0, x1, y0=0.0, y1=1.0, bc=(BC_EXTRAP,) * 4, dirichlet=None,
              nz=1, z0=0.0, z1=1.0) -> _Grid:
    """wcns_grid; dirichlet[side]: None, a primitive nvar-vector, or an array
    [n_side][nvar] (the grid keeps the array alive until it is dropped);
    3D: nz, z0, z1 and bc[4:6] for z-lo, z-hi."""
    g = _Grid()
    g.ndim, g.nx, g.ny = ndim, nx, ny
    g.x0, g.x1, g.y0, g.y1 = x0, x1, y0, y1
    g.nz, g.z0, g.z1 = (nz, z0, z1) if ndim == 3 else (1, 0.0, 1.0)
    if ndim == 3:
        g.bc_z[0], g.bc_z[1] = int(bc[4]), int(bc[5])
    nvar = {1: 5, 2: 6, 3: 7}[ndim]
    g._keep = []
    for k in range(4):
        g.bc[k] = int(bc[k])
        if dirichlet is None or dirichlet[k] is None:
            continue
        d = np.ascontiguousarray(np.asarray(dirichlet[k], dtype=np.float64))
        if d.ndim == 1:
            if d.size != nvar:
                raise ValueError(f"Dirichlet side {k}: need {nvar} values")
            for v in range(nvar):
                g.dirichlet[k][v] = float(d[v])
        else:
            n_side = ny if k < 2 else nx
            if d.shape != (n_side, nvar):
                raise ValueError(f"Dirichlet side {k}: need shape ({n_side}, {nvar})")
            g._keep.append(d)
            g.dirichlet_rows[k] = d.ctypes.data
    return g


def grid_of(spec) -> _Grid:
    return make_grid(spec.ndim, spec.nx, spec.ny, spec.x0, spec.x1, spec.y0, spec.y1, spec.bc,
                     spec.dirichlet_prim, spec.nz, spec.z0, spec.z1)


class Batch:
    """Many independent solves (same ndim, fluids, options, precision)
    advanced together by the batched kernels.

    grids: list of _Grid (see grid_of); states: list of device f64 tensors
    [nvar][ny][nx], stepped in place.  Work runs on the batch's own stream;
    step()/rhs() order it after the current torch stream and make the current
    torch stream wait for it, so torch code sees the results in order."""

    def __init__(self, grids, states, gamma=(6.12, 1.4), pinf=(3.43e8, 0.0), precision=FP64,
                 capacity_cells=0, **params):
        import torch
        n = len(grids)
        G = (_Grid * n)(*grids)
        e = _Eos()
        e.gamma[0], e.gamma[1] = gamma
        e.pinf[0], e.pinf[1] = pinf
        p = default_params(**params)
        ptrs = _state_ptrs(grids, states)
        ctx = C.c_void_p()
        _check(lib().wcns_batch_create(n, G, C.byref(e), C.byref(p), int(precision), ptrs,
                                       int(capacity_cells), C.byref(ctx)), "wcns_batch_create")
        self._b = ctx
        self.n = n
        self.states = list(states)
        st = C.c_void_p()
        _check(lib().wcns_batch_stream(self._b, C.byref(st)), "wcns_batch_stream")
        self.stream = torch.cuda.ExternalStream(st.value)

    def _enter(self):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream())

    def _leave(self):
        import torch
        torch.cuda.current_stream().wait_stream(self.stream)

    def configure(self, ytile=16, order=0):
        _check(lib().wcns_batch_configure(self._b, int(ytile), int(order)), "wcns_batch_configure")

    def reset(self, grids, states):
        n = len(grids)
        G = (_Grid * n)(*grids)
        ptrs = _state_ptrs(grids, states)
        self._enter()
        _check(lib().wcns_batch_reset(self._b, n, G, ptrs), "wcns_batch_reset")
        self.n = n
        self.states = list(states)

    def step(self, nsteps=1):
        self._enter()
        _check(lib().wcns_batch_step(self._b, int(nsteps)), "wcns_batch_step")
        self._leave()

    def rhs(self):
        self._enter()
        _check(lib().wcns_batch_rhs(self._b), "wcns_batch_rhs")
        self._leave()

    def sync(self):
        _check(lib().wcns_batch_sync(self._b), "wcns_batch_sync")

    def set_steps(self, steps):
        arr = (C.c_int32 * self.n)(*[int(x) for x in steps])
        self._enter()
        _check(lib().wcns_batch_set_steps(self._b, arr), "wcns_batch_set_steps")

    def steps_left(self):
        arr = (C.c_int32 * self.n)()
        _check(lib().wcns_batch_steps_left(self._b, arr), "wcns_batch_steps_left")
        return np.array(arr[:], dtype=np.int64)

    def violations(self, clear=False):
        """Per-instance count of cells found outside the admissible set
        (wcns_batch_violations; synchronises the batch stream)."""
        arr = (C.c_int64 * self.n)()
        _check(lib().wcns_batch_violations(self._b, arr, int(bool(clear))), "wcns_batch_violations")
        return np.array(arr[:], dtype=np.int64)

    def dt(self):
        out = (C.c_double * self.n)()
        _check(lib().wcns_batch_dt(self._b, out), "wcns_batch_dt")
        return np.array(out[:])

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            lib().wcns_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(batch, trials=3, candidates=None, margin=0.01):
    """Pick the batch schedule (y-tile height, task order) by the measured
    RHS time on the batch's own instances: each candidate is timed over
    `trials` separate RHS evaluations after one warm-up and scored by their
    median; of the candidates within `margin` of the fastest, the first in
    the candidate order (by default the library's own schedule, 16-row
    tiles in the given instance order, then the others in a fixed order) is
    taken, so schedules within the run-to-run noise of each other do not
    flip the pick.  Returns (best, {candidate: seconds})."""
    import time
    if candidates is None:
        candidates = [(16, 0)] + [(y, o) for y in (2, 4, 8, 16) for o in (0, 1, 2) if (y, o) != (16, 0)]
    times = {}
    for cand in candidates:
        batch.configure(*cand)
        batch.rhs()
        batch.sync()
        ts = []
        for _ in range(max(1, int(trials))):
            t0 = time.perf_counter()
            batch.rhs()
            batch.sync()
            ts.append(time.perf_counter() - t0)
        times[cand] = sorted(ts)[len(ts) // 2]
    fastest = min(times.values())
    best = next(c for c in candidates if times[c] <= fastest * (1.0 + margin))
    batch.configure(*best)
    return best, times
