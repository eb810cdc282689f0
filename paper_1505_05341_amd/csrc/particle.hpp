// Per-particle arithmetic shared by the row sort and the assignment kernels, so that
// both derive a particle's base cell from the same FP32 operations.
//
// Mass assignment (Sec. 4 names cloud-in-cell; the triangular-shaped cloud is the
// next order): nodes at box_min + j H, u = (x - box_min) / H.
//   CIC: i = floor(u), f = u - i, weights (1 - f, f) on cells (i, i + 1);
//   TSC: i = floor(u + 1/2), d = u - i, weights (1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2)
//        on cells (i - 1, i, i + 1).
// Cell indices wrap modulo N (periodic box).
#pragma once
#include <hip/hip_runtime.h>

#include "pk.h"

namespace pk {

__device__ __forceinline__ float grid_coord(float x, float bmin, float invH) {
  return __fmul_rn(__fsub_rn(x, bmin), invH);
}

// Squared distance of a particle to the observer in FP32, with the rounding of every
// operation fixed (no contraction left to the compiler), so that the validity test of
// the sort and the line of sight of the assignment take the same value: a particle
// whose FP32 position equals the FP32 observer (a zero line of sight) is rejected by
// the one and never reaches the other.
__device__ __forceinline__ float los_norm2(float x, float y, float z, float ox, float oy, float oz) {
  const float dx = __fsub_rn(x, ox), dy = __fsub_rn(y, oy), dz = __fsub_rn(z, oz);
  return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}

// N is a power of two (the supported grid sizes), so the periodic wrap is a mask.
template <int ASSIGN>
__device__ __forceinline__ int base_index(float u, int N) {
  const float t = ASSIGN == PK_CIC ? u : __fadd_rn(u, 0.5f);
  return (int)floorf(t) & (N - 1);
}

// Offset of u from its base node (f for CIC, d for TSC).
template <int ASSIGN>
__device__ __forceinline__ float base_offset(float u) {
  const float t = ASSIGN == PK_CIC ? u : __fadd_rn(u, 0.5f);
  return __fsub_rn(u, floorf(t));
}

// Weight of the cell at base + o for offset o in [0, 1] (CIC) or [-1, 1] (TSC).
template <int ASSIGN>
__device__ __forceinline__ float stencil_weight(float f, int o) {
  if (ASSIGN == PK_CIC) return o == 0 ? 1.0f - f : f;
  if (o == 0) return 0.75f - f * f;
  const float h = o < 0 ? 0.5f - f : 0.5f + f;
  return 0.5f * h * h;
}

}  // namespace pk
