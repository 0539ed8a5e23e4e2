// Device helpers shared by the gfx950 kernels of the U(1)-symmetric MPS
// engine: complex arithmetic on double2, wave64 reductions, and the FP64
// matrix-core product v_mfma_f64_16x16x4f64.
#pragma once

#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"

namespace u1mps {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// FP64 matrix-core product D[16x16] += A[16x4] B[4x16] on one wavefront.
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; register r of lane
// l holds D[4 r + l / 16][l % 16].
typedef double v4d __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace u1mps
