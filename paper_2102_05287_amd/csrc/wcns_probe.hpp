// Issue-cost probe of FP64 and FP32 operations (a measurement aid for the
// ALU roofline of the sweeps).
//
// Every lane runs `iters` rounds of 8 independent chains of one operation,
// with the grid sized to keep 8 waves on every SIMD, so the device time
// measures issue throughput, not latency.  The time per operation relative
// to the FMA's is the operation's cost in FMA issue slots: the weight of a
// divide or a square root in the algorithmic operation count of a face.
// Constants arrive as kernel arguments so no chain can be folded.
#pragma once
#include "wcns_device.hpp"

#pragma clang fp contract(off)

namespace wcns {

enum { PROBE_FMA = 0, PROBE_ADD = 1, PROBE_MUL = 2, PROBE_DIV = 3, PROBE_SQRT = 4, PROBE_DIV_CORE = 5,
       PROBE_FMA_F32 = 6, PROBE_DIV_F32 = 7, PROBE_SQRT_F32 = 8 };

template <int OP>
__global__ __launch_bounds__(256) void k_issue_probe(double* out, int iters, double c, double d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 1.0 + 1e-3 * (double)(t & 255) + 0.125 * k;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (OP == PROBE_FMA) x[k] = __builtin_fma(x[k], c, d);   // -> d / (1 - c)
      else if (OP == PROBE_ADD) x[k] = x[k] + d;
      else if (OP == PROBE_MUL) x[k] = x[k] * c;
      else if (OP == PROBE_DIV) x[k] = d / x[k];                // alternates
      else if (OP == PROBE_SQRT) x[k] = __builtin_sqrt(x[k]);   // -> 1
      else x[k] = ddiv(d, x[k]);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s = s + x[k];
  out[t] = s;
}

// The same for FP32 (the precision form's bulk): non-packed FMA, the
// kernels' FP32 quotient (fdivf: hardware reciprocal and a product) and the
// compiler's FP32 square root.
template <int OP>
__global__ __launch_bounds__(256) void k_issue_probe_f32(double* out, int iters, float c, float d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 1.0f + 1e-3f * (float)(t & 255) + 0.125f * k;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (OP == PROBE_FMA_F32) x[k] = __builtin_fmaf(x[k], c, d);
      else if (OP == PROBE_DIV_F32) x[k] = fdivf(d, x[k]);
      else x[k] = __builtin_sqrtf(x[k]);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s = s + x[k];
  out[t] = (double)s;
}

}  // namespace wcns
