// Sums of the gathered monomials of one particle visit (the reduced basis of basis.hpp,
// in its gathered order): acc[j] += w rhat^m(j) for the NG = 1, 6, 15 or 28 monomials with a
// power of rhat_z below 2. Each product is one multiply-add from two factors already at
// hand, w rhat_x^2 or w rhat_y^2 times a monomial two degrees lower: 24 vector operations
// for the 15 sums of ell_max = 4, where forming every monomial and then w times it takes 29.
// Host and device (the host check of basis.hpp compares it with kept_monomials).
#pragma once

namespace pk {

template <int NG>
__host__ __device__ inline void add_monomial_sums(float (&acc)[NG], float w, float rx, float ry, float rz) {
  acc[0] += w;
  if constexpr (NG > 1) {
    const float wx = w * rx, wy = w * ry;
    const float wxx = wx * rx, wyy = wy * ry;
    acc[1] += wxx;      // 200
    acc[2] += wx * ry;  // 110
    acc[3] += wx * rz;  // 101
    acc[4] += wyy;      // 020
    acc[5] += wy * rz;  // 011
    if constexpr (NG > 6) {
      const float xx = rx * rx, xy = rx * ry, xz = rx * rz, yy = ry * ry, yz = ry * rz;
      acc[6] += wxx * xx;   // 400
      acc[7] += wxx * xy;   // 310
      acc[8] += wxx * xz;   // 301
      acc[9] += wxx * yy;   // 220
      acc[10] += wxx * yz;  // 211
      acc[11] += wyy * xy;  // 130
      acc[12] += wyy * xz;  // 121
      acc[13] += wyy * yy;  // 040
      acc[14] += wyy * yz;  // 031
      if constexpr (NG > 15) {
        const float m400 = xx * xx, m310 = xx * xy, m301 = xx * xz, m220 = xx * yy, m211 = xx * yz;
        const float m130 = yy * xy, m121 = yy * xz, m040 = yy * yy, m031 = yy * yz;
        acc[15] += wxx * m400;  // 600
        acc[16] += wxx * m310;  // 510
        acc[17] += wxx * m301;  // 501
        acc[18] += wxx * m220;  // 420
        acc[19] += wxx * m211;  // 411
        acc[20] += wxx * m130;  // 330
        acc[21] += wxx * m121;  // 321
        acc[22] += wxx * m040;  // 240
        acc[23] += wxx * m031;  // 231
        acc[24] += wyy * m130;  // 150
        acc[25] += wyy * m121;  // 141
        acc[26] += wyy * m040;  // 060
        acc[27] += wyy * m031;  // 051
      }
    }
  }
}

}  // namespace pk
