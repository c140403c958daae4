"""Continuous-batching request server for PP-WCNS-IS solves on one GPU.

Requests (a grid, an initial state, a number of SSP-RK3 steps, a precision)
arrive over time.  The server
  * admits queued requests in arrival order while their HBM footprint fits
    the budget and a slot is free (no reordering, so no starvation);
  * keeps every admitted solve's state resident on the device;
  * groups active solves by (ndim, precision) into batches (wcns.Batch), each
    on its own stream so the groups' kernels overlap on the GPU;
  * advances all active solves together in ticks of `chunk` graph-replayed
    steps; a per-instance step budget on the device freezes a solve the
    moment its own step count is reached, so solves of any length share the
    same ticks;
  * between ticks retires finished solves and admits newly arrived ones
    (membership changes rebind the batch inside its existing scratch, which
    grows by doubling only when needed);
  * retires, marked failed, a solve whose kernels found a cell outside the
    admissible set (the batch's per-instance report, read once per tick), so
    it neither runs on nor disturbs the others.

Every solve in a batch runs exactly the arithmetic it runs alone (the batched
kernels are the single-solve kernels per tile), so a result does not depend
on what it was batched with.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import wcns


def footprint_bytes(ndim: int, nx: int, ny: int) -> int:
    """Device bytes one solve holds: its state plus its batch scratch
    (primitives, two stage states, block maxima; in 2D two more primitive
    buffers for the next stages, L and the y-tile edges)."""
    nv = 5 if ndim == 1 else 6
    N = nx * ny
    pairs = (N + 255) // 256
    if ndim == 2:   # block maxima of the fused next-stage primitives, 2-row tiles
        nbr = (ny + 2) // 2
        pairs = max(pairs, ((nx + 31) // 32) * nbr + ((nbr - 1) * nx + 255) // 256)
    d = nv * N + 5 * N + 2 * nv * N + 2 * pairs + 64
    if ndim == 2:   # two more primitive buffers (next-stage primitives), L, edges
        d += 2 * 5 * N + nv * N + ((ny + 2) // 2) * 12 * nx
    return 8 * d


@dataclass
class Solve:
    rid: int
    arrival: float
    spec: object           # problems.ProblemSpec (prim on the host)
    steps: int
    fp32: bool
    state: object = None   # device tensor while active
    taken: int = 0         # steps completed
    admitted: float = -1.0
    done: float = -1.0
    result: object = None  # host copy of the final state (when kept)
    failed: bool = False   # retired after a cell left the admissible set
    bad_cells: int = 0


@dataclass
class _Group:
    ndim: int
    fp32: bool
    members: list = field(default_factory=list)
    batch: object = None
    cap_cells: int = 0
    dirty: bool = True


class Server:
    def __init__(self, hbm_budget: int = 32 << 30, max_slots: int = 512, chunk: int = 20,
                 gamma=(6.12, 1.4), pinf=(3.43e8, 0.0), keep_results: bool = False,
                 ytile: int = 16, order: int = 2):
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.chunk = chunk
        self.gamma, self.pinf = gamma, pinf
        self.keep = keep_results
        self.ytile, self.order = ytile, order
        self.groups: dict = {}
        self.used = 0
        self.active = 0

    # ------------------------------------------------------------ admission
    def _fits(self, s: Solve) -> bool:
        fp = footprint_bytes(s.spec.ndim, s.spec.nx, s.spec.ny)
        return self.active < self.max_slots and self.used + fp <= self.budget

    def _admit(self, s: Solve, now: float):
        import torch
        sp = s.spec
        V = torch.from_numpy(np.ascontiguousarray(sp.prim)).cuda()
        s.state = wcns.prim_to_cons(V, sp.ndim, self.gamma, self.pinf)
        s.admitted = now
        key = (sp.ndim, s.fp32)
        g = self.groups.get(key)
        if g is None:
            g = self.groups[key] = _Group(sp.ndim, s.fp32)
        g.members.append(s)
        g.dirty = True
        self.used += footprint_bytes(sp.ndim, sp.nx, sp.ny)
        self.active += 1

    def _retire(self, g: _Group, s: Solve, now: float):
        s.done = now
        if self.keep:
            s.result = s.state.cpu().numpy()
        s.state = None
        self.used -= footprint_bytes(s.spec.ndim, s.spec.nx, s.spec.ny)
        self.active -= 1

    # ------------------------------------------------------------ batches
    def _rebind(self, g: _Group):
        """Bind the group's batch to its current members (grow if needed)."""
        if not g.members:
            return
        cells = sum(m.spec.nx * m.spec.ny for m in g.members)
        grids = [wcns.grid_of(m.spec) for m in g.members]
        states = [m.state for m in g.members]
        prec = wcns.FP32_BULK if g.fp32 else wcns.FP64
        if g.batch is None or cells > g.cap_cells:
            if g.batch is not None:
                g.batch.close()
            g.cap_cells = max(2 * cells, 1 << 18)
            g.batch = wcns.Batch(grids, states, self.gamma, self.pinf, precision=prec,
                                 capacity_cells=g.cap_cells)
            g.batch.configure(self.ytile, self.order)
        else:
            g.batch.reset(grids, states)
        g.batch.set_steps([m.steps - m.taken for m in g.members])
        g.dirty = False

    # ------------------------------------------------------------ serving
    def run(self, solves, realtime: bool = True, log=None):
        """Serve `solves` (arrival-sorted).  realtime: arrivals follow the
        wall clock from the start of the call; otherwise every request is
        queued at once.  Returns the per-request records and a summary."""
        import torch
        pending = list(solves)
        for s in pending:
            s.taken = 0
        self.peak_used = 0
        queue = []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        finished = []
        ticks = 0
        work = 0.0
        spent = {"admit": 0.0, "rebind": 0.0, "step": 0.0, "check": 0.0, "idle": 0.0}
        while pending or queue or self.active:
            ta = time.perf_counter()
            tnow = now()
            while pending and (not realtime or pending[0].arrival <= tnow):
                queue.append(pending.pop(0))
            while queue and self._fits(queue[0]):
                self._admit(queue.pop(0), tnow)
            self.peak_used = max(self.peak_used, self.used)
            tb = time.perf_counter()
            spent["admit"] += tb - ta
            if queue and self.active == 0:
                raise RuntimeError(f"request {queue[0].rid} exceeds the HBM budget")
            if not self.active:
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - now(), 0.05)))
                spent["idle"] += time.perf_counter() - tb
                continue
            live = [g for g in self.groups.values() if g.members]
            for g in live:
                if g.dirty:
                    self._rebind(g)
            torch.cuda.synchronize()
            tc = time.perf_counter()
            spent["rebind"] += tc - tb
            for g in live:
                g.batch.step(self.chunk)
            for g in live:
                g.batch.sync()
            ticks += 1
            tdone = now()
            td = time.perf_counter()
            spent["step"] += td - tc
            for g in live:
                left = g.batch.steps_left()
                viol = g.batch.violations()
                keep = []
                for m, l, nb in zip(g.members, left, viol):
                    before = m.steps - m.taken
                    m.taken = m.steps - int(l)
                    work += 3.0 * m.spec.nx * m.spec.ny * (before - int(l))
                    if nb:
                        m.failed, m.bad_cells = True, int(nb)
                    if l == 0 or nb:
                        self._retire(g, m, tdone)
                        finished.append(m)
                    else:
                        keep.append(m)
                if len(keep) != len(g.members):
                    g.members = keep
                    g.dirty = True
            spent["check"] += time.perf_counter() - td
            if log:
                log(f"tick {ticks} t={tdone:.2f}s active={self.active} queued={len(queue)} "
                    f"pending={len(pending)} done={len(finished)}")
        makespan = now()
        lat = np.array([s.done - s.arrival for s in finished]) if realtime else \
            np.array([s.done for s in finished])
        summary = {
            "requests": len(finished),
            "failed": sum(1 for s in finished if s.failed),
            "makespan_s": makespan,
            "solves_per_s": len(finished) / makespan,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "mcell_updates_per_s": work / makespan / 1e6,
            "ticks": ticks,
            "chunk_steps": self.chunk,
            "host_seconds": spent,
        }
        for g in self.groups.values():
            if g.batch is not None:
                g.batch.close()
                g.batch = None
        return finished, summary
