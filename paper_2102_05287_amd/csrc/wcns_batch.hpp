// Batched form: many independent solves of uneven grid sizes advanced
// together.  Each phase of an SSP-RK3 stage (node primitives, dt/lambda,
// x-sweep, y-sweep, y-tile fixup) is one launch over a device task list of
// (instance, tile) pairs, reading per-instance arguments from a device array
// prepared once per stage.  A whole step is therefore a fixed sequence of
// launches, captured once into a HIP graph and replayed (in 2D a second
// graph without the node launch serves the later steps of a call, whose
// node primitives the previous step's last stage left).
#pragma once
#include "wcns_kernels.hpp"

namespace wcns {

struct Task {
  int32_t inst, a, b, pad;   // instance and its tile coordinates
};

// An instance whose step counter reached 0 is frozen: every block of it
// returns at once (the counter is uniform over the block, so no barrier is
// skipped by part of a block).
__device__ __forceinline__ bool frozen(const KArgs& a) { return a.live && *a.live <= 0; }

template <bool HAS_T>
__global__ __launch_bounds__(256) void kb_node(const KArgs* ka, const Task* t) {
  const Task task = t[blockIdx.x];
  const KArgs& a = ka[task.inst];
  if (frozen(a)) return;
  node_block<HAS_T>(a, task.a);
}

__global__ __launch_bounds__(256) void kb_finalize(const KArgs* ka) {
  const KArgs& a = ka[blockIdx.x];
  if (frozen(a)) return;
  finalize_inst(a);
}

// The sweeps copy their instance's arguments into registers first: read
// through the pointer, every use would be a fresh scalar load (the stores of
// the sweep may alias them), which measured 14% (FP64) and 28% (FP32-bulk)
// slower than the copy.
template <bool HAS_T, bool B32>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void kb_sweep_x(
    const KArgs* ka, const Task* t) {
  const Task task = t[blockIdx.x];
  const KArgs a = ka[task.inst];
  if (frozen(a)) return;
  sweep_x_tile<HAS_T, false, B32>(a, task.a);
}

// x-sweep with LDS windows: task.a = group of XW tiles of XT cells
template <bool HAS_T, bool B32>
__global__ __launch_bounds__(64 * XW) void kb_sweep_xl(const KArgs* ka, const Task* t) {
  __shared__ double tile[XW][11 * XWIN];
  const Task task = t[blockIdx.x];
  const KArgs a = ka[task.inst];
  if (frozen(a)) return;
  const int w = threadIdx.x >> 6;
  const long tl = (long)task.a * XW + w;
  sweep_x_window<HAS_T, false, B32>(a, tl, tl * XT < (long)a.nx * a.ny, tile[w]);
}

// y-sweep over 32-column tiles of YW face rows (YW/2 waves): task.a = column
// block, task.b = tile row
template <int YW, bool B32>
__global__ __launch_bounds__(32 * YW) __attribute__((amdgpu_waves_per_eu(YW >= 4 ? 4 : 3))) void kb_sweep_y(
    const KArgs* ka, const Task* t) {
  __shared__ double tile[9 * (YW + 5) * 32];
  const Task task = t[blockIdx.x];
  const KArgs a = ka[task.inst];
  if (frozen(a)) return;
  sweep_y_tile32<YW, false, B32>(a, task.a, task.b, tile, (long)task.b * ((a.nx + 31) / 32) + task.a);
}

template <int YW>
__global__ __launch_bounds__(256) void kb_fixup(const KArgs* ka, const Task* t) {
  const Task task = t[blockIdx.x];
  const KArgs& a = ka[task.inst];
  if (frozen(a)) return;
  long idx = 0;
  double X[6];
  const bool own = fixup_cell(a, (long)task.a * 256 + threadIdx.x, YW, idx, X);
  fixup_finish(a, own, idx, X, task.a);
}

// end of a step: one step fewer for every live instance
__global__ __launch_bounds__(256) void kb_tick(int32_t* live, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && live[k] > 0) live[k] -= 1;
}

}  // namespace wcns
