// Batched form: many independent solves of uneven grid sizes advanced
// together.  Each phase of an SSP-RK3 stage (node primitives, dt/lambda,
// x-sweep, y-sweep, y-tile fixup) is one launch over a device task list of
// (instance, tile) pairs, reading per-instance arguments from a device array
// prepared once per stage.  A whole step is therefore a fixed sequence of 15
// launches that is captured once into a HIP graph and replayed.
#pragma once
#include "wcns_kernels.hpp"

namespace wcns {

struct Task {
  int32_t inst, a, b, pad;   // instance and its tile coordinates
};

template <bool HAS_T>
__global__ __launch_bounds__(256) void kb_node(const KArgs* ka, const Task* t) {
  const Task task = t[blockIdx.x];
  node_block<HAS_T>(ka[task.inst], task.a);
}

__global__ __launch_bounds__(256) void kb_finalize(const KArgs* ka) {
  finalize_inst(ka[blockIdx.x]);
}

template <bool HAS_T, bool B32>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void kb_sweep_x(
    const KArgs* ka, const Task* t) {
  const Task task = t[blockIdx.x];
  sweep_x_tile<HAS_T, false, B32>(ka[task.inst], task.a);
}

template <int YW, bool B32>
__global__ __launch_bounds__(64 * YW) void kb_sweep_y(const KArgs* ka, const Task* t) {
  __shared__ double sGm[YW][6][64];
  const Task task = t[blockIdx.x];
  sweep_y_tile<YW, false, B32>(ka[task.inst], task.a, task.b, sGm);
}

template <int YW>
__global__ __launch_bounds__(256) void kb_fixup(const KArgs* ka, const Task* t) {
  const Task task = t[blockIdx.x];
  fixup_cell(ka[task.inst], (long)task.a * 256 + threadIdx.x, YW);
}

}  // namespace wcns
