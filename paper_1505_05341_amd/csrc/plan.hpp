// Host/device plan of one estimator call: sizes, workspace carve-up, the monomial
// and z-power group tables, and the launchers of every kernel (one per stage).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "pk.h"

namespace pk {

constexpr int kMaxGrids = 50;       // 1 + 6 + 15 + 28 monomial grids (ell_max = 6)
constexpr int kMaxGroups = 16;      // z-power groups: 1 + 3 + 5 + 7
constexpr int kMaxMembers = 7;
constexpr int kMaxTiles = 256;      // kx tiles: 16 columns up to N = 512, 8 at 1024, 4 at 2048
constexpr int kStatsBlocks = 2048;  // blocks of the catalogue-scalar reduction
constexpr int kScanChunk = 4096;    // counters per scan block
constexpr int kScanTopMax = 4096;   // scan blocks of one scan (N^2 kRowHistParts / kScanChunk at N = 2048)
constexpr int kSortBlocks = 2048;   // level-A sort blocks (one contiguous particle range each)
constexpr int kRowHistParts = 4;    // level-B blocks per plane
constexpr int kNumSums = 7;         // per-bin sums: count, |n|, Q0, Q2, Q4, noise, Q6

// Device scalars written by the catalogue-scalar kernels.
enum ScalarSlot {
  kSumWg = 0, kSumWr, kSumWg2, kSumWr2, kSumWg2Nbar, kSumWr2Nbar,
  kAlpha, kNormI, kNoiseS, kNumScalars
};

// Error-flag bits (device).
enum FlagBits {
  kFlagNonFinitePos = 1, kFlagOutOfBox = 2, kFlagAtObserver = 4, kFlagNonFiniteWeight = 8,
  kFlagBadNorm = 16
};

// Exponents of monomial m in the fixed order used everywhere: degree 0, 2, 4, then 6,
// each with the power of x descending, then the power of y descending.
struct Monomial { int a, b, c; };
__host__ __device__ inline Monomial monomial(int m) {
  // degree 0: m = 0; degree 2: m = 1..6; degree 4: m = 7..21; degree 6: m = 22..49
  int n = m == 0 ? 0 : (m <= 6 ? 2 : (m <= 21 ? 4 : 6));
  int r = m == 0 ? 0 : (m <= 6 ? m - 1 : (m <= 21 ? m - 7 : m - 22));
  for (int a = n; a >= 0; --a) {
    for (int b = n - a; b >= 0; --b) {
      if (r == 0) return Monomial{a, b, n - a - b};
      --r;
    }
  }
  return Monomial{0, 0, 0};
}

// Group (n, c) of the monomials of degree n with power c of z: after the transforms
// along x and y they are summed with weights coef kx^a ky^b, so that one transform
// along z serves the whole group (the FFT along z is linear and kx, ky are constant
// along it).
struct GroupTable {
  int ngroups;
  int n[kMaxGroups];
  int c[kMaxGroups];
  int count[kMaxGroups];
  int grid[kMaxGroups][kMaxMembers];
  int a[kMaxGroups][kMaxMembers];
  int b[kMaxGroups][kMaxMembers];
  float coef[kMaxGroups][kMaxMembers];
  // the same members flattened in the order the y pass takes them (group by group,
  // largest power of y first); group g ends before member mend[g]
  int nmem;
  int mgrid[kMaxGrids];
  int ma[kMaxGrids];
  float mcoef[kMaxGrids];
  int mend[kMaxGroups];
};

// Tile table of the y and z passes: per kx tile the largest |ky| kept (M), the
// float2 offset of the tile's region inside one H group, and the first z item.
struct TileTable {
  int M[kMaxTiles];
  int64_t regoff[kMaxTiles];
  int64_t item0[kMaxTiles + 1];
};

struct Plan {
  // configuration
  int N, assign, ell_max, los, compensate, dn, nbins, norm_from;
  double box_min[3], L, observer[3];
  int64_t n_gal, n_ran;
  // derived
  int G;          // LOS-weighted grids: 1, 7, 22
  int K;          // nbins * dn: modes with |n| < K are binned
  int TK;         // kx columns per FFT tile
  int Kx;         // kx columns kept after the x transform (multiple of TK, <= N/2)
  int nkt;        // kx tiles
  int xs;         // z planes per slab of the x and y passes (divides N)
  int xr;         // slabs X holds: 1 (xs = N) or 2 (slab i uses slot i % 2)
  int z_blocks;   // persistent blocks of the z pass
  int col_e[2];   // values per thread of the column transforms of the y and z passes (8 or 16)
  int64_t z_items;
  GroupTable groups;
  TileTable tiles;
  // workspace offsets (bytes)
  size_t off_scalars, off_partials, off_flags, off_tw, off_invw2, off_alias, off_tables;
  size_t off_rowcnt, off_rowoff, off_rowhist, off_blocksum, off_tmp, off_rowkey, off_sorted, off_X, off_H, off_zpart, off_result;
  size_t total;
  size_t H_group_stride;   // float2 elements per group in H
  int64_t result_doubles;
};

int sort_blocks(int64_t ntot);
pk_status make_plan(const pk_config* cfg, int64_t n_gal, int64_t n_ran, Plan* plan, const char** why);

// Launchers (queued on `s`; they return the launch error, if any).
hipError_t launch_init(const Plan& p, char* ws, hipStream_t s);  // also copies the group and tile tables
hipError_t launch_stats(const Plan& p, const pk_catalog& gal, const pk_catalog& ran, char* ws, hipStream_t s);
hipError_t launch_sort(const Plan& p, const pk_catalog& gal, const pk_catalog& ran, char* ws, hipStream_t s);
// The x and y passes work on the slab of planes [z0, z0 + xs): the x pass writes the
// slab's x-transformed rows into planes [pbase, pbase + xs) of X (which holds xr xs
// planes), the y pass reads them there.
hipError_t launch_xpass(const Plan& p, char* ws, hipStream_t s, int z0, int pbase);
hipError_t launch_ypass(const Plan& p, char* ws, hipStream_t s, int z0, int pbase);
hipError_t launch_zpass(const Plan& p, char* ws, hipStream_t s);
hipError_t launch_finalize(const Plan& p, char* ws, double* d_result, hipStream_t s);

template <class T>
__host__ __device__ inline T* at(char* ws, size_t off) { return reinterpret_cast<T*>(ws + off); }

}  // namespace pk
