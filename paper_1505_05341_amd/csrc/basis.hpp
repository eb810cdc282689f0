// Reduced basis of the LOS-weighted grids. Every particle's line of sight is a unit
// vector, rhat_x^2 + rhat_y^2 + rhat_z^2 = 1, so for the monomial grids G_(a,b,c) =
// F rhat_x^a rhat_y^b rhat_z^c of Sec. 3 (Eqs. 11, 13)
//   G_(a,b,c+2) = G_(a,b,c) - G_(a+2,b,c) - G_(a,b+2,c),
// and the same holds after any linear transform. Only the monomials with a power of
// rhat_z below 2 are gathered and transformed along x: 1, 6 and 15 of the 1, 7 and 22
// (ell_max 0, 2, 4); the other x-transformed rows are written as these combinations:
//   (0,0,2) = (0,0,0) - (2,0,0) - (0,2,0)
//   (2,0,2) = (2,0,0) - (4,0,0) - (2,2,0)      (1,1,2) = (1,1,0) - (3,1,0) - (1,3,0)
//   (1,0,3) = (1,0,1) - (3,0,1) - (1,2,1)      (0,2,2) = (0,2,0) - (2,2,0) - (0,4,0)
//   (0,1,3) = (0,1,1) - (2,1,1) - (0,3,1)
//   (0,0,4) = (0,0,2) - (2,0,2) - (0,2,2)
//           = (0,0,0) - 2 (2,0,0) - 2 (0,2,0) + (4,0,0) + 2 (2,2,0) + (0,4,0).
// Monomial indices follow plan.hpp (degree 0; degree 2: xx xy xz yy yz zz; degree 4:
// 400 310 301 220 211 202 130 121 112 103 040 031 022 013 004).
#pragma once

namespace pk {

// gathered ("kept") monomials for ell_max and their number
__host__ __device__ constexpr int kept_count(int ell) { return ell == 0 ? 1 : (ell == 2 ? 6 : 15); }
__host__ __device__ constexpr int dep_count(int ell) { return ell == 0 ? 0 : (ell == 2 ? 1 : 7); }

// monomial index of kept grid j (the 15 with c <= 1, in monomial order)
__host__ __device__ constexpr int kept_monomial(int j) {
  constexpr int m[15] = {0, 1, 2, 3, 4, 5, 7, 8, 9, 10, 11, 13, 14, 17, 18};
  return m[j];
}

// dependent grid d: its monomial index, number of terms, and term t as (kept j, coefficient)
__host__ __device__ constexpr int dep_monomial(int d) {
  constexpr int m[7] = {6, 12, 15, 16, 19, 20, 21};
  return m[d];
}
__host__ __device__ constexpr int dep_terms(int d) { return d == 6 ? 6 : 3; }
__host__ __device__ constexpr int dep_kept(int d, int t) {
  constexpr int j[7][6] = {{0, 1, 4, 0, 0, 0},  {1, 6, 9, 0, 0, 0},  {2, 7, 11, 0, 0, 0}, {3, 8, 12, 0, 0, 0},
                           {4, 9, 13, 0, 0, 0}, {5, 10, 14, 0, 0, 0}, {0, 1, 4, 6, 9, 13}};
  return j[d][t];
}
__host__ __device__ constexpr float dep_coef(int d, int t) {
  constexpr float c[7][6] = {{1, -1, -1, 0, 0, 0}, {1, -1, -1, 0, 0, 0}, {1, -1, -1, 0, 0, 0}, {1, -1, -1, 0, 0, 0},
                             {1, -1, -1, 0, 0, 0}, {1, -1, -1, 0, 0, 0}, {1, -2, -2, 1, 2, 1}};
  return c[d][t];
}

}  // namespace pk
