"""Benchmark of the PP-WCNS-IS hot path on one MI355X.

Workload (default): 2D shock-bubble interaction on a 1024 x 1024 grid in
FP64 (planar water shock at 1e9 Pa hitting an air bubble in water), SSP-RK3
steps at CFL 0.5 with the time step computed on the device.  One timed "step"
is one full SSP-RK3 step = 3 right-hand-side evaluations with their wave-speed
reductions, limiters, flux differences and stage combinations.

value = cell-updates per second per RHS (3 x cells x steps / time), in
Mcell-updates/s, inputs resident in HBM before the timed region.

Also reported:
  roofline      the dominant kernel's algorithmic FP64 work per launch over
                its average duration (HIP events around each launch on the
                library's stream), against the FP64 VALU issue rate
  cpu_baseline  the serial FP64 oracle timed on a bounded sample of the same
                workload on this host (rank 0, N = 1 only)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s per RHS, FP64 vs FP32/batched; solves/s and p99 latency"
# FP64 VALU: 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 issue slots/s
# (78.6 TFLOP/s when every slot is an FMA counted as 2 flops)
VALU_F64_SLOTS = 256 * 64 * 2.4e9
# Issue cost of a correctly rounded FP64 divide and square root in FMA issue
# slots, measured at start-up with the library's issue probe
# (wcns_issue_probe: time per operation over an FMA probe of equal work,
# median of 3 runs).  A divide is weighted by the cheapest exact sequence
# available, the kernels' division core (8 instructions, one a quarter-rate
# reciprocal: 11 issue units); the compiler's IEEE divide (11 instructions,
# 14 issue units) is reported beside it.  Until measured: the issue units.
# FP32 (the precision form's bulk): a non-packed operation issues like an
# FP64 one; its quotient is a quarter-rate reciprocal and a product.
OP_WEIGHTS = {"div": 11.0, "sqrt": 19.0, "f32": 1.0, "div_f32": 5.0, "sqrt_f32": 5.0,
              "source": "issue units of the instruction sequences"}
# steps of the face pipeline the precision form runs in FP32 (the others,
# and the per-cell difference and RK combination, stay FP64)
FP32_PHASES = ("weno", "back_v", "mid_hllc", "hcs")


def measure_weights():
    import statistics
    from paper_2102_05287_amd import wcns
    runs = [wcns.issue_weights(4096) for _ in range(3)]
    med = {op: round(statistics.median(r["weights"][op] for r in runs), 2)
           for op in ("div_core", "div", "sqrt", "fma_f32", "div_f32", "sqrt_f32")}
    OP_WEIGHTS["div"] = med["div_core"]
    OP_WEIGHTS["sqrt"] = med["sqrt"]
    OP_WEIGHTS["div_ieee_sequence"] = med["div"]
    OP_WEIGHTS["f32"] = med["fma_f32"]
    OP_WEIGHTS["div_f32"] = med["div_f32"]
    OP_WEIGHTS["sqrt_f32"] = med["sqrt_f32"]
    OP_WEIGHTS["source"] = "issue probe (wcns_issue_probe), median of 3; div = division core"
    OP_WEIGHTS["fma_slots_per_s"] = statistics.median(r["fma_slots_per_s"] for r in runs)


def weighted(c, w_div=None, w_sqrt=None):
    w_div = OP_WEIGHTS["div"] if w_div is None else w_div
    w_sqrt = OP_WEIGHTS["sqrt"] if w_sqrt is None else w_sqrt
    return c["add"] + c["mul"] + c["cmp"] + w_div * c["div"] + w_sqrt * c["sqrt"]


def weighted_f32(c, unit=False):
    """FP32 operations in FP64 FMA issue slots (unit: every operation 1)."""
    if unit:
        return c["add"] + c["mul"] + c["cmp"] + c["div"] + c["sqrt"]
    return (OP_WEIGHTS["f32"] * (c["add"] + c["mul"] + c["cmp"]) + OP_WEIGHTS["div_f32"] * c["div"]
            + OP_WEIGHTS["sqrt_f32"] * c["sqrt"])


def face_weighted(oc, fp32_bulk=False, w_div=None, w_sqrt=None):
    """Weighted algorithmic operations of one face: FP64 throughout, or the
    precision form's split (FP32_PHASES priced as FP32, the rest as FP64)."""
    if not fp32_bulk:
        return weighted(oc["face"], w_div, w_sqrt)
    unit = w_div == 1 and w_sqrt == 1
    return sum(weighted_f32(c, unit) if k in FP32_PHASES else weighted(c, w_div, w_sqrt)
               for k, c in oc["face_phases"].items())


def kernel_ops(nx, ny, scheme="ppwcnsis", w_div=None, w_sqrt=None, fused=2.0 / 3.0,
               fp32_bulk=False):
    """Algorithmic (issue-weighted) ops per launch of each kernel, in FP64
    FMA issue slots; w_div = w_sqrt = 1 gives the plain operation count.
    `fused`: share of the y-sweep launches that also recover the next
    stage's node primitives in place of k_node (2/3 for single-step calls;
    1 - 1/(3K) for K steps in one call).  fp32_bulk: the precision form's
    split of the face work by precision."""
    w_div = OP_WEIGHTS["div"] if w_div is None else w_div
    w_sqrt = OP_WEIGHTS["sqrt"] if w_sqrt is None else w_sqrt
    with open(os.path.join(ROOT, "tests", "golden", "opcount.json")) as f:
        oc = json.load(f)["counts"][scheme]
    face = face_weighted(oc, fp32_bulk, w_div, w_sqrt)
    node = weighted(oc["node"], w_div, w_sqrt)
    cells = nx * ny
    diff = 6 * (1 + w_div)                 # -(G^- - G^+)/dx per component
    rk = 6 * 5                             # ca*Un + cb*(W + dt*L)
    return {
        "node": cells * (node + 4),        # + |u|+c, |v|+c, two max
        "sweep_x": (nx + 1) * ny * face + cells * diff,
        "sweep_y": nx * (ny + 1) * face + cells * (diff + 6 + rk) + fused * cells * (node + 4),
    }


def source_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2102_05287_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter runs, or
    None when the kernel sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != source_hash() or kernel not in t["kernels"]:
        return None
    k, c = t["kernels"][kernel], t["calibration"]
    return (k["fetch_kib"] * c["fetch_factor"] + k["write_kib"] * c["write_factor"]) * 1024.0


def time_steps(sol, W0, steps, warmup):
    """Seconds for `steps` device-CFL SSP-RK3 steps from W0 (after warmup),
    enqueued as one multi-step call (wcns_ssprk3_steps)."""
    import torch
    W = W0.clone()
    sol.steps(W, warmup, 0.0)
    W.copy_(W0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.steps(W, steps, 0.0)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, W


def precision_form(n=2048, prof_steps=20):
    """Underwater explosion at n^2 (2048^2: the precision form's workload)
    to its final time t = 2e-4 s, FP64 and FP32 bulk each through the
    library's time loop on the same device (each takes its own CFL steps):
    time to solution and Mcell-updates/s per RHS of each, the relative L1
    per variable of the FP32-bulk final state against the FP64 one, the
    relative L1 per variable of one FP32-bulk RHS of the initial state (its
    sharp material interfaces) against the FP64 RHS, and the ALU roofline of
    the FP32-bulk sweeps with each step of the face pipeline priced at its
    own precision (the FP64 path equals the oracle bit for bit, so the FP64
    runs stand for it at this size)."""
    import torch
    from paper_2102_05287_amd import problems as pb
    from paper_2102_05287_amd import wcns
    spec = pb.underwater_explosion(n)
    V = torch.from_numpy(spec.prim).cuda()
    spec.prim = None
    cells = spec.nx * spec.ny
    out = {"workload": f"2D underwater explosion near a wall, {n}x{n}, to t = {spec.t_end} s"}
    finals = {}
    W0 = None
    for name, prec in (("fp64", wcns.FP64), ("fp32_bulk", wcns.FP32_BULK)):
        sol = wcns.Solver.from_spec(spec, precision=prec)
        if W0 is None:
            W0 = sol.prim_to_cons(V)
        W = W0.clone()
        sol.steps(W, 3, 0.0)               # warm-up
        W.copy_(W0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, t = sol.advance(W, spec.t_end, chunk=128)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"{name}_steps"] = steps
        out[f"{name}_wall_s"] = el
        out[f"{name}_mcells_per_s"] = 3 * cells * steps / el / 1e6
        out[f"{name}_violations"] = sol.violations()
        out[f"{name}_inadmissible_at_end"] = sol.count_inadmissible(W)
        finals[name] = W
        # one RHS of the initial state (material interfaces), at the CFL step
        if prec == wcns.FP64:
            Wc = W0.clone()
            dtu = torch.zeros(1, dtype=torch.float64, device="cuda")
            sol.step(Wc, 0.0, dt_used=dtu)
            finals["dt0"] = float(dtu.item())
            finals["amax"] = float(sol.max_wavespeed(W0).max())
            del Wc
        finals[name + "_rhs"] = sol.rhs(W0, dt=finals["dt0"]).clone()
        if prec == wcns.FP32_BULK:
            Wp = W0.clone()
            sol.profile(True)
            sol.steps(Wp, prof_steps, 0.0)
            prof = sol.profile_read(reset=True)
            sol.profile(False)
            del Wp
        sol.close()
    A, B = finals["fp64"], finals["fp32_bulk"]
    out["rel_l1_fp32_vs_fp64_final_per_variable"] = [
        float((B[v] - A[v]).abs().sum() / A[v].abs().sum()) for v in range(6)]
    # one Euler step of the CFL size with each RHS of the initial state: the
    # FP32-bulk change per variable relative to the state (momenta, zero at
    # t = 0, against rho times the largest wave speed)
    La, Lb = finals["fp64_rhs"], finals["fp32_bulk_rhs"]
    rho = W0[0] + W0[1]
    scale = [float(W0[v].abs().sum()) for v in range(6)]
    scale[2] = scale[3] = float(rho.sum()) * finals["amax"]
    out["euler_step_fp32_vs_fp64_initial_per_variable"] = [
        float(finals["dt0"] * (Lb[v] - La[v]).abs().sum() / scale[v]) for v in range(6)]
    out["speedup_fp32_bulk"] = out["fp32_bulk_mcells_per_s"] / out["fp64_mcells_per_s"]
    ops = kernel_ops(spec.nx, spec.ny, fused=1.0 - 1.0 / (3 * prof_steps), fp32_bulk=True)
    ops1 = kernel_ops(spec.nx, spec.ny, w_div=1, w_sqrt=1, fused=1.0 - 1.0 / (3 * prof_steps),
                      fp32_bulk=True)
    roof32 = {}
    for k in ("sweep_x", "sweep_y"):
        avg = prof[k][0] / 1e3 / prof[k][1]
        roof32[k] = {"avg_launch_ms": avg * 1e3, "ops_per_launch": ops[k],
                     "achieved": ops[k] / avg / 1e12, "frac": ops[k] / avg / VALU_F64_SLOTS,
                     "frac_unweighted": ops1[k] / avg / VALU_F64_SLOTS}
    out["roofline_fp32_bulk"] = {
        "bound": "alu", "peak": VALU_F64_SLOTS / 1e12, "unit": "TFLOP/s", "kernels": roof32,
        "op_model": "oracle op count per face filed by pipeline step (tests/golden/opcount.json "
                    "face_phases); " + ", ".join(FP32_PHASES) + " priced as FP32 (f32, div_f32, "
                    "sqrt_f32 of op_weights), the rest and the per-cell work as FP64; peak = "
                    "the FP64 / non-packed FP32 VALU issue rate 256 CU x 64 lanes x 2.4 GHz",
        "op_weights": dict(OP_WEIGHTS)}
    del A, B, La, Lb, W0, V, finals
    torch.cuda.empty_cache()
    return out


def batched_form(n_inst, steps, seq_steps):
    """512 seeded random water/air instances (sides 64..512) advanced together
    by the batched kernels, FP64 and FP32-bulk, after autotuning the schedule;
    compared with the plain FP64 path solving the same instances one by one."""
    import numpy as np
    import torch
    from paper_2102_05287_amd import problems as pb
    from paper_2102_05287_amd import wcns
    specs = [pb.random_instance(i) for i in range(n_inst)]
    conv = {}
    W0 = []
    for sp in specs:
        if sp.nx not in conv:
            conv[sp.nx] = wcns.Solver.from_spec(sp)
        W0.append(conv[sp.nx].prim_to_cons(torch.from_numpy(sp.prim).cuda()))
    for sp in specs:
        sp.prim = None
    cells = sum(sp.nx * sp.ny for sp in specs)
    grids = [wcns.grid_of(sp) for sp in specs]
    out = {"workload": f"{n_inst} seeded 2D water/air instances, sides "
                       f"{sorted(set(sp.nx for sp in specs))}, {cells} cells in total",
           "steps": steps, "cells": cells}
    for name, prec in (("fp64", wcns.FP64), ("fp32_bulk", wcns.FP32_BULK)):
        states = [w.clone() for w in W0]
        b = wcns.Batch(grids, states, precision=prec)
        best, times = wcns.autotune(b, trials=3)
        for k in range(n_inst):
            states[k].copy_(W0[k])
        b.step(1)
        b.sync()
        for k in range(n_inst):
            states[k].copy_(W0[k])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        b.sync()
        el = time.perf_counter() - t0
        bad = sum(conv[specs[k].nx].count_inadmissible(states[k]) for k in range(n_inst))
        out[f"batched_{name}_mcells_per_s"] = 3 * cells * steps / el / 1e6
        orders = ["given", "largest_first", "xcd_chunked"]
        out[f"batched_{name}_schedule"] = {"ytile": best[0], "order": orders[best[1]]}
        out[f"batched_{name}_autotune_rhs_ms"] = {f"{y}/{orders[o]}": round(t * 1e3, 3)
                                                  for (y, o), t in times.items()}
        out[f"batched_{name}_inadmissible"] = bad
        b.close()
        del states
    # plain FP64 path, one instance after another (a shorter run, same rate unit)
    states = [w.clone() for w in W0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_inst):
        sol = conv[specs[k].nx]
        for _ in range(seq_steps):
            sol.step(states[k], 0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["sequential_fp64_mcells_per_s"] = 3 * cells * seq_steps / el / 1e6
    out["sequential_steps"] = seq_steps
    out["speedup_batched_fp64_vs_sequential"] = (out["batched_fp64_mcells_per_s"]
                                                 / out["sequential_fp64_mcells_per_s"])
    return out


def serving_form(n_req=2000, rate=200.0, budget_gib=64, chunk=20):
    """The Poisson request stream (seed 4) at `rate` req/s replayed in real
    time through the continuous-batching server: the whole 2000-request
    trace of mixed 1D (200-20000 cells) and 2D (64^2-1024^2) water/air
    solves of 100-2000 steps, FP64 or FP32 bulk.  Offered over capacity, so
    latency there is mostly queueing: the rate sweep gives the sustainable
    rate."""
    from paper_2102_05287_amd import problems as pb
    from paper_2102_05287_amd import serve
    reqs = pb.serving_trace(n_req, rate, seed=4)
    solves = [serve.Solve(r.rid, r.arrival, pb.request_problem(r), r.steps, r.fp32) for r in reqs]
    srv = serve.Server(hbm_budget=budget_gib << 30, chunk=chunk)
    done, summary = srv.run(solves, realtime=True)
    offered = sum(3.0 * s.spec.nx * s.spec.ny * s.steps for s in solves) / (reqs[-1].arrival or 1.0)
    summary.update({"workload": f"the seed-4 trace, {n_req} requests at {rate} req/s (Poisson), "
                                f"mixed 1D/2D, FP64/FP32-bulk",
                    "offered_mcell_updates_per_s": offered / 1e6,
                    "hbm_budget_gib": budget_gib, "peak_hbm_used_gib": srv.peak_used / 2**30})
    return summary


def serving_rate_sweep(n_req=300, rates=(8.0, 12.0, 16.0, 20.0, 28.0), budget_gib=64, chunk=20):
    """The first n_req requests of the seed-4 trace (the same solves at every
    rate) replayed at several Poisson arrival rates: completion rate and
    latency against offered rate.  A rate is sustained while latency stays
    bounded (p50 within 2x and p99 within 3x their values at the lowest
    rate); the sustainable rate is the highest such rate."""
    from paper_2102_05287_amd import problems as pb
    from paper_2102_05287_amd import serve
    rows = []
    for r in rates:
        reqs = pb.serving_trace(2000, r, seed=4)[:n_req]
        solves = [serve.Solve(q.rid, q.arrival, pb.request_problem(q), q.steps, q.fp32) for q in reqs]
        srv = serve.Server(hbm_budget=budget_gib << 30, chunk=chunk)
        _, sm = srv.run(solves, realtime=True)
        offered = n_req / reqs[-1].arrival
        rows.append({"rate_req_per_s": r, "offered_req_per_s": offered,
                     "solves_per_s": sm["solves_per_s"],
                     "latency_p50_s": sm["latency_p50_s"], "latency_p99_s": sm["latency_p99_s"],
                     "makespan_s": sm["makespan_s"],
                     "mcell_updates_per_s": sm["mcell_updates_per_s"]})
        print(f"#   rate {r}: {sm['solves_per_s']:.1f} solves/s, p50 {sm['latency_p50_s']:.2f} s, "
              f"p99 {sm['latency_p99_s']:.2f} s", flush=True)
    p50, p99 = rows[0]["latency_p50_s"], rows[0]["latency_p99_s"]
    for row in rows:
        row["sustained"] = bool(row["latency_p50_s"] <= 2.0 * p50 and row["latency_p99_s"] <= 3.0 * p99)
    ok = [row["rate_req_per_s"] for row in rows if row["sustained"]]
    return {"requests_per_rate": n_req, "rates": rows,
            "sustainable_rate_req_per_s": max(ok) if ok else None,
            "rule": "latency stays bounded: p50 <= 2x and p99 <= 3x those at the lowest rate "
                    "(beyond it a queue builds and latency grows with the offered rate)"}


HBM_PEAK = 8.0e12     # MI355X HBM3E, bytes/s


def first_order_form(n=1024, steps=200, warmup=10):
    """The first-order HLLC product mode on the default workload (n^2
    shock-bubble, FP64, device-CFL steps in one call): Mcell-updates/s per
    RHS and, since the mode has no interpolation, limiter or midpoint
    arithmetic, an HBM roofline against its algorithmic bytes: a stage reads
    U^(s) and (stages 2, 3) U^n and writes U^(s+1) (6 FP64 components),
    96 + 144 + 144 B per cell per step.  In 2D each stage is one launch of
    the one-pass kernel, so `achieved` is those bytes per launch (the
    three-stage mean, 128 B per cell) over its mean launch time (HIP events
    around each launch); `stages` splits it into stage 1 (96 B per cell) and
    stages 2 and 3 (144 B); `step` prices the whole step, finalize
    included."""
    import torch
    from paper_2102_05287_amd import problems as pb
    from paper_2102_05287_amd import wcns
    spec = pb.shock_bubble(n)
    sol = wcns.Solver.from_spec(spec, scheme=1)
    W0 = sol.prim_to_cons(torch.from_numpy(spec.prim).cuda())
    el, W = time_steps(sol, W0, steps, warmup)
    cells = spec.nx * spec.ny
    W.copy_(W0)
    sol.profile(True)
    sol.steps(W, steps, 0.0)
    prof = sol.profile_read(reset=True)
    sol.profile(False)
    bad = sol.count_inadmissible(W)
    step_bytes = (96.0 + 144.0 + 144.0) * cells
    launch_bytes = step_bytes / 3.0
    # stage 1 (class fo_stage: no U^n) and stages 2, 3 (fo_stage_un)
    (ms1, n1), (ms23, n23) = prof["fo_stage"], prof["fo_stage_un"]
    t_launch = (ms1 + ms23) / 1e3 / (n1 + n23)
    dev_step = sum(v[0] for v in prof.values()) / 1e3 / steps
    stages = {}
    for name, ms, nl, b in (("stage1", ms1, n1, 96.0), ("stages23", ms23, n23, 144.0)):
        t = ms / 1e3 / nl
        stages[name] = {"bytes_per_cell": b, "avg_launch_ms": t * 1e3, "achieved": b * cells / t / 1e9,
                        "frac": b * cells / t / HBM_PEAK}
    roof = {"bound": "hbm", "kernel": "fo_stage", "unit": "GB/s", "peak": HBM_PEAK / 1e9,
            "bytes_per_launch": launch_bytes, "avg_launch_ms": t_launch * 1e3,
            "achieved": launch_bytes / t_launch / 1e9, "frac": launch_bytes / t_launch / HBM_PEAK,
            "traffic": measured_traffic("fo_stage"), "stages": stages,
            "step": {"bytes": step_bytes, "device_ms": dev_step * 1e3,
                     "frac": step_bytes / dev_step / HBM_PEAK,
                     "frac_wall": step_bytes / (el / steps) / HBM_PEAK}}
    del W, W0
    sol.close()
    return {"workload": f"2D shock-bubble {n}x{n}, first-order HLLC (scheme 1), FP64",
            "steps": steps, "mcells_per_s": 3 * cells * steps / el / 1e6,
            "ms_per_step": el / steps * 1e3, "inadmissible_after": bad,
            "per_kernel_ms_per_launch": {k: v[0] / v[1] for k, v in prof.items() if v[1]},
            "launches_per_step": {k: v[1] / steps for k, v in prof.items() if v[1]},
            "roofline": roof}


def sizes_form(sizes=(1024, 1448, 2048), steps=(60, 30, 16)):
    """Per-launch times of the two 2D sweeps on the shock-bubble at three
    grid sizes (kernel-stamped events, one multi-step call each after a
    warm-up), and the least-squares fit time = a + b * cells of each sweep:
    a is the fixed cost of a launch (its first round of waves staging before
    any arithmetic, its last round draining), b the cost per cell."""
    import numpy as np
    import torch
    from paper_2102_05287_amd import problems as pb
    from paper_2102_05287_amd import wcns
    rows = []
    for n, k in zip(sizes, steps):
        spec = pb.shock_bubble(n)
        sol = wcns.Solver.from_spec(spec)
        W = sol.prim_to_cons(torch.from_numpy(spec.prim).cuda())
        spec.prim = None
        sol.steps(W, 3, 0.0)
        torch.cuda.synchronize()
        sol.profile(True)
        sol.steps(W, k, 0.0)
        prof = sol.profile_read(reset=True)
        sol.profile(False)
        sol.close()
        rows.append({"grid": [n, n], "cells": n * n, "steps": k,
                     "sweep_x_us": prof["sweep_x"][0] / prof["sweep_x"][1] * 1e3,
                     "sweep_y_us": prof["sweep_y"][0] / prof["sweep_y"][1] * 1e3})
        print(f"#   {n}^2: x {rows[-1]['sweep_x_us']:.1f} us, y {rows[-1]['sweep_y_us']:.1f} us per launch",
              flush=True)
    cells = np.array([r["cells"] for r in rows], dtype=float)
    fit = {}
    for key in ("sweep_x_us", "sweep_y_us"):
        t = np.array([r[key] for r in rows])
        b, a = np.polyfit(cells, t, 1)
        fit[key.replace("_us", "")] = {"fixed_us_per_launch": a, "ps_per_cell": b * 1e6,
                                       "fixed_share_at_smallest": a / t[0],
                                       "fixed_share_at_largest": a / t[-1]}
    return {"workload": "2D shock-bubble, FP64, sweep launch times at three grid sizes",
            "sizes": rows, "fit_a_plus_b_cells": fit}


def three_d_form(n=256, steps=10, warmup=2):
    """3D underwater explosion near a wall at n^3 (FP64, the direct 3D
    extension): Mcell-updates/s per RHS, per-kernel device time and the
    x-, y- and z-sweep roofline fractions (3D face op count)."""
    import torch
    from paper_2102_05287_amd import problems as pb
    from paper_2102_05287_amd import wcns
    spec = pb.underwater_explosion_3d(n)
    sol = wcns.Solver.from_spec(spec)
    W0 = sol.prim_to_cons(torch.from_numpy(spec.prim).cuda())
    spec.prim = None
    el, W = time_steps(sol, W0, steps, warmup)
    cells = n ** 3
    W.copy_(W0)
    sol.profile(True)
    sol.steps(W, steps, 0.0)
    prof = sol.profile_read(reset=True)
    sol.profile(False)
    bad = sol.count_inadmissible(W)
    with open(os.path.join(ROOT, "tests", "golden", "opcount.json")) as f:
        oc = json.load(f)["counts"]["ppwcnsis_3d"]
    face = weighted(oc["face"])
    diff = 7 * (1 + OP_WEIGHTS["div"])
    faces = (n + 1) * n * n
    ops_x = faces * face + cells * diff
    ops_y = faces * face + cells * (diff + 7)             # + L_x
    ops_z = faces * face + cells * (diff + 7 + 7 * 5)     # + (L_x + L_y), RK stage
    nrhs = 3 * steps
    roof = {}
    for k, ops in (("sweep_x", ops_x), ("sweep_y", ops_y), ("sweep_z", ops_z)):
        t = prof[k][0] / 1e3 / nrhs          # seconds per RHS in this class
        roof[k] = {"ms_per_rhs": t * 1e3, "achieved": ops / t / 1e12, "frac": ops / t / VALU_F64_SLOTS}
    del W, W0
    sol.close()
    return {"workload": f"3D underwater explosion near a wall, {n}^3 ({cells} cells), FP64",
            "steps": steps, "mcells_per_s": 3 * cells * steps / el / 1e6,
            "ms_per_step": el / steps * 1e3, "inadmissible_after": bad,
            "per_kernel_ms_per_rhs": {k: v[0] / nrhs for k, v in prof.items() if v[1]},
            "roofline": {"bound": "alu", "peak": VALU_F64_SLOTS / 1e12, "unit": "TFLOP/s",
                         "face_ops_weighted": face, "op_weights": dict(OP_WEIGHTS), "kernels": roof}}


def time_to_solution_form():
    """The paper's runs to their final times on the device time loop
    (Solver.advance), and the 1024^2 shock-bubble over its full 1000 steps
    (its final state checked against the oracle's whole solve): the 1D
    water-air tube (400 cells, t = 2.4e-4 s), the
    1D multi-material Sedov blast (401 cells, 4000 fixed steps), and the two
    2D robustness problems, Mach 10 shock-water cylinder (1152 x 768, 16 us)
    and Mach 100 water jet (1024 x 512, 4 us), with PP-WCNS-IS and with the
    first-order HLLC scheme; plus the cylinder with both limiters off, which
    has to fail."""
    import torch
    from paper_2102_05287_amd import problems as pb
    from paper_2102_05287_amd import wcns
    out = {}

    def run(name, spec, **kw):
        sol = wcns.Solver.from_spec(spec, **kw)
        W = sol.prim_to_cons(torch.from_numpy(spec.prim).cuda())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n, t = sol.advance(W, spec.t_end, chunk=64 if spec.ndim == 2 else 32, dt=spec.dt_fixed)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        a1 = W[-1]
        rec = {"grid": [spec.nx, spec.ny] if spec.ndim == 2 else [spec.nx], "t_end": spec.t_end,
               "steps": n, "wall_s": el, "ms_per_step": el / n * 1e3,
               "mcell_updates_per_s": 3.0 * spec.nx * spec.ny * n / el / 1e6,
               "inadmissible_at_end": sol.count_inadmissible(W),
               "alpha1_min": float(a1.min()), "alpha1_max": float(a1.max())}
        out[name] = rec
        print(f"#   {name}: {n} steps in {el:.2f} s", flush=True)
        sol.close()

    run("water_air_tube_1d", pb.water_air_shock_tube(400))
    run("sedov_1d", pb.sedov_multimaterial(401))
    # the same two 1D runs with the whole time loop in one workgroup (wcns_run)
    for name, spec in (("water_air_tube_1d_device_loop", pb.water_air_shock_tube(400)),
                       ("sedov_1d_device_loop", pb.sedov_multimaterial(401))):
        sol = wcns.Solver.from_spec(spec)
        W = sol.prim_to_cons(torch.from_numpy(spec.prim).cuda())
        sol.run(W.clone(), spec.t_end, dt_fixed=spec.dt_fixed, max_steps=3)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n, t = sol.run(W, spec.t_end, dt_fixed=spec.dt_fixed)
        el = time.perf_counter() - t0
        out[name] = {"grid": [spec.nx], "t_end": spec.t_end, "steps": n, "wall_s": el,
                     "ms_per_step": el / n * 1e3, "inadmissible_at_end": sol.count_inadmissible(W)}
        print(f"#   {name}: {n} steps in {el:.3f} s", flush=True)
        sol.close()
    run("mach10_cylinder", pb.mach10_cylinder())
    run("mach10_cylinder_hllc1", pb.mach10_cylinder(), scheme=1)
    run("mach100_jet", pb.mach100_jet())
    run("mach100_jet_hllc1", pb.mach100_jet(), scheme=1)
    # negative control: no limiters; the library's lazy report refuses the
    # next chunk once a stage result has left the admissible set
    spec = pb.mach10_cylinder()
    sol = wcns.Solver.from_spec(spec, interp_limiter=False, flux_limiter=False)
    W = sol.prim_to_cons(torch.from_numpy(spec.prim).cuda())
    refused_after, n = None, 0
    while n < 8000 and refused_after is None:
        try:
            sol.steps(W, 50, 0.0)
            n += 50
            torch.cuda.synchronize()
        except wcns.WcnsError as e:
            if e.code != wcns.WCNS_ERR_INADMISSIBLE:
                raise
            refused_after = n
    nviol = sol.violations(clear=True)
    out["mach10_cylinder_limiters_off"] = {"refused_after_steps": refused_after,
                                           "chunk_steps": 50, "max_steps": 8000,
                                           "stage_results_outside_G": nviol}
    sol.close()
    # the shock-bubble workload over its full 1000 CFL steps in one call; the
    # final state's SHA-256 against the digest of the oracle's own whole
    # solve (tests/golden/full_runs.json, written by a script that calls
    # only the oracle)
    import hashlib
    spec = pb.shock_bubble(1024)
    sol = wcns.Solver.from_spec(spec)
    W = sol.prim_to_cons(torch.from_numpy(spec.prim).cuda())
    spec.prim = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.steps(W, 1000, 0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    digest = hashlib.sha256(W.cpu().numpy().astype("<f8").tobytes()).hexdigest()
    with open(os.path.join(ROOT, "tests", "golden", "full_runs.json")) as f:
        golden = json.load(f)["runs"]["shock_bubble_1024_1000_steps"]["sha256"]
    out["shock_bubble_1024_1000_steps"] = {
        "grid": [spec.nx, spec.ny], "steps": 1000, "wall_s": el, "ms_per_step": el,
        "mcell_updates_per_s": 3.0 * spec.nx * spec.ny * 1000 / el / 1e6,
        "inadmissible_at_end": sol.count_inadmissible(W),
        "final_state_sha256_equals_oracle": digest == golden}
    print(f"#   shock_bubble_1024_1000_steps: {el:.2f} s, oracle digest "
          f"{'matched' if digest == golden else 'DIFFERS'}", flush=True)
    sol.close()
    return out


def cpu_baseline(spec, target_s=10.0):
    """The oracle on the same initial state, timed on this host: as many
    full-grid RHS evaluations as fit in about target_s seconds, serially (1
    thread) and with the OpenMP build of the same source over all host
    cores (bit-identical results); `value` is the all-cores rate."""
    from oracle import oracle as orc
    s = orc.Setup(ndim=spec.ndim, nx=spec.nx, ny=spec.ny, dx=spec.dx, dy=spec.dy, bc=spec.bc)
    W = orc.prim_to_cons(s, spec.prim)
    dt = orc.cfl_dt(s, W)

    def rate(fn):
        t0 = time.perf_counter()
        fn(s, W, dt)
        one = time.perf_counter() - t0
        calls = max(1, int(target_s / max(one, 1e-3)) - 1)
        t0 = time.perf_counter()
        for _ in range(calls):
            fn(s, W, dt)
        el = time.perf_counter() - t0
        return spec.nx * spec.ny * calls / el / 1e6, calls

    serial, n1 = rate(orc.rhs)
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    allc, nall = rate(orc.rhs_parallel)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": allc, "unit": "Mcell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{nall} full-grid RHS evaluations of the {spec.nx}x{spec.ny} shock-bubble "
                      f"initial state, FP64 C++ oracle built with OpenMP over grid rows "
                      f"({threads} threads; bit-identical to the serial build)",
            "serial": {"value": serial, "cores": 1,
                       "sample": f"{n1} RHS evaluations, the serial build, 1 thread"},
            "host": {"cpu": cpu, "logical_cpus": os.cpu_count(), "nproc": len(os.sched_getaffinity(0))}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision/batched/serving forms")
    ap.add_argument("--form", choices=("precision", "batched", "serving", "solutions", "rates",
                                       "3d", "first_order", "sizes"),
                    default=None,
                    help="run only this form and print its record")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 3}))
        return
    if args.form:
        import torch
        torch.cuda.set_device(0)
        measure_weights()
        run = {"precision": precision_form,
               "batched": lambda: batched_form(512, 200, 20),
               "serving": serving_form,
               "solutions": time_to_solution_form,
               "rates": serving_rate_sweep,
               "3d": three_d_form,
               "sizes": sizes_form,
               "first_order": first_order_form}[args.form]
        print(json.dumps({"form": args.form, **run()}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2102_05287_amd import problems as pb
    from paper_2102_05287_amd import wcns

    torch.cuda.set_device(0)
    spec = pb.shock_bubble(args.n)
    sol = wcns.Solver.from_spec(spec)
    V = torch.from_numpy(spec.prim).cuda()
    W0 = sol.prim_to_cons(V)
    W = W0.clone()
    # the issue probes (about half a second of sustained GPU work) run right
    # before the warm-up steps: after host-side set-up the GPU needs ~15 ms
    # of sustained load to reach its working clock, longer than a few
    # warm-up steps take (measured: the first 20-step call after an idle
    # gap ran 0.75-0.77 ms per step against 0.70-0.71 when kept busy)
    measure_weights()
    print(f"# workload {spec.name} {spec.nx}x{spec.ny} fp64; warmup {args.warmup}", flush=True)
    sol.steps(W, args.warmup, 0.0)
    torch.cuda.synchronize()
    W.copy_(W0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.steps(W, args.steps, 0.0)       # K device-CFL steps, one call
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    cells = spec.nx * spec.ny
    value = 3 * cells * args.steps / el / 1e6
    bad = sol.count_inadmissible(W)
    print(f"# timed {args.steps} steps in {el:.3f}s; inadmissible cells after: {bad}", flush=True)

    # per-kernel device time over the same number of steps (events on the
    # library's stream); the dominant kernel gives the roofline
    W.copy_(W0)
    sol.profile(True)
    sol.steps(W, args.steps, 0.0)
    prof = sol.profile_read(reset=True)
    sol.profile(False)
    fused = 1.0 - 1.0 / (3 * args.steps)   # y-sweeps that also recover the next primitives
    ops = kernel_ops(spec.nx, spec.ny, fused=fused)
    dom = max((k for k in ops), key=lambda k: prof[k][0])
    ms, n = prof[dom]
    avg_s = ms / 1e3 / n
    achieved = ops[dom] / avg_s / 1e12
    peak = VALU_F64_SLOTS / 1e12
    ops1 = kernel_ops(spec.nx, spec.ny, w_div=1, w_sqrt=1, fused=fused)
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": measured_traffic(dom),
                "frac_unweighted": ops1[dom] / avg_s / VALU_F64_SLOTS,
                "avg_launch_ms": avg_s * 1e3,
                "ops_per_launch": ops[dom],
                "op_model": "oracle op count per face (tests/golden/opcount.json), divide "
                            "and sqrt weighted by op_weights; peak = FP64 VALU issue rate "
                            "256 CU x 64 lanes x 2.4 GHz",
                "op_weights": dict(OP_WEIGHTS)}
    # both sweeps, each against the same peak (the dominant one is above)
    roofline["kernels"] = {
        k: {"avg_launch_ms": prof[k][0] / prof[k][1],
            "achieved": ops[k] / (prof[k][0] / 1e3 / prof[k][1]) / 1e12,
            "frac": ops[k] / (prof[k][0] / 1e3 / prof[k][1]) / VALU_F64_SLOTS}
        for k in ("sweep_x", "sweep_y") if prof[k][1]}
    per_kernel = {k: {"ms_total": v[0], "launches": v[1]} for k, v in prof.items() if v[1]}

    # pure RHS rate (no stage combination) for reference
    dWdt = torch.empty_like(W)
    dt = 1e-8
    for _ in range(3):
        sol.rhs(W0, dWdt, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nr = max(10, args.steps)
    for _ in range(nr):
        sol.rhs(W0, dWdt, dt)
    torch.cuda.synchronize()
    rhs_rate = cells * nr / (time.perf_counter() - t0) / 1e6

    forms = {}
    if not args.no_forms:
        print("# precision form (2048^2 underwater explosion) ...", flush=True)
        forms["precision_fp32_bulk"] = precision_form()
        print("# batched form (512 instances) ...", flush=True)
        forms["batched"] = batched_form(512, 200, 20)
        print("# serving form ...", flush=True)
        forms["serving"] = serving_form()
        print("# serving rate sweep ...", flush=True)
        forms["serving_rate_sweep"] = serving_rate_sweep()
        print("# 3D form ...", flush=True)
        forms["three_d"] = three_d_form()
        print("# first-order mode ...", flush=True)
        forms["first_order"] = first_order_form()
        print("# time to solution (paper runs) ...", flush=True)
        forms["time_to_solution"] = time_to_solution_form()

    cpu = None
    if not args.no_cpu:
        print("# cpu baseline (oracle) ...", flush=True)
        cpu = cpu_baseline(spec)

    out = {
        "metric": METRIC, "value": value, "unit": "Mcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D shock-bubble interaction, {spec.nx}x{spec.ny}, FP64 "
                               "PP-WCNS-IS, SSP-RK3 at CFL 0.5 (device dt)",
                   "cells": cells, "rhs_per_step": 3, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "rhs_only_mcells_per_s": rhs_rate,
        "per_kernel": per_kernel,
        "inadmissible_after": bad,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
