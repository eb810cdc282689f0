// Per-particle arithmetic shared by the row sort and the assignment kernels, so that
// both derive a particle's base cell from the same operations.
//
// Mass assignment (Sec. 4 names cloud-in-cell; the triangular-shaped cloud is the
// next order): nodes at box_min + j H, u = (x - box_min) / H, H = L / N.
//   CIC: i = floor(u), f = u - i, weights (1 - f, f) on cells (i, i + 1);
//   TSC: i = floor(u + 1/2), d = u - i, weights (1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2)
//        on cells (i - 1, i, i + 1).
// Cell indices wrap modulo N (periodic box).
#pragma once
#include <hip/hip_runtime.h>

#include "pk.h"

namespace pk {

// Squared distance of a particle to the observer in FP32, with the rounding of every
// operation fixed (no contraction left to the compiler), so that the validity test of
// the sort and the line of sight of the assignment take the same value: a particle
// whose FP32 position equals the FP32 observer (a zero line of sight) is rejected by
// the one and never reaches the other.
__device__ __forceinline__ float los_norm2(float x, float y, float z, float ox, float oy, float oz) {
  const float dx = __fsub_rn(x, ox), dy = __fsub_rn(y, oy), dz = __fsub_rn(z, oz);
  return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}

// Cell of a coordinate along one axis: u = (x - box_min) N / L formed in FP64 from the FP32
// position (as the FP64 oracle forms it, so both take the same cell decisions), the base
// node i (wrapped modulo N; N is a power of two, so the wrap is a mask) and the offset
// f = u - floor(t) in [0, 1) (CIC, t = u) or [-1/2, 1/2) (TSC, t = u + 1/2), rounded to FP32
// only once it is small, so that it keeps FP32's relative precision at any N (u formed in
// FP32 would put every offset off by up to |u| 2^-24, ~6e-5 of a cell at N = 1024). The cost
// is a few FP64 vector instructions (half the FP32 rate) per particle and axis.
struct AxisCell {
  int i;    // base node
  float f;  // offset from it
};

template <int ASSIGN>
__device__ __forceinline__ AxisCell axis_cell(float x, double bmin, double invH, int N) {
  // every operation rounded on its own (no fused multiply-add), so that each caller takes
  // the same cells as the others and as the oracle
#pragma clang fp contract(off)
  const double u = ((double)x - bmin) * invH;
  const double fl = floor(ASSIGN == PK_CIC ? u : u + 0.5);
  AxisCell c;
  c.i = (int)fl & (N - 1);
  c.f = (float)(u - fl);
  return c;
}

// Weight of the cell at base + o for offset o in [0, 1] (CIC) or [-1, 1] (TSC). Both TSC
// forms are evaluated and one is selected: o often differs between the lanes of a wave,
// and a branch on it would run both sides one after the other.
template <int ASSIGN>
__device__ __forceinline__ float stencil_weight(float f, int o) {
  if (ASSIGN == PK_CIC) return o == 0 ? 1.0f - f : f;
  const float h = 0.5f + (o < 0 ? -f : f);
  const float side = 0.5f * h * h;
  const float mid = 0.75f - f * f;
  return o == 0 ? mid : side;
}

}  // namespace pk
