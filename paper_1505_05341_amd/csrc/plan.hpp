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
constexpr int kYSetGroups = 6;      // z-power groups one y-pass block sums at once (8-value schedule)
constexpr int kMaxYSets = 6;        // sets of groups per schedule (ell_max = 6 with sets of 3)
constexpr int kMaxYMembers = 64;    // gathered grids loaded by all sets of one schedule
constexpr int kMaxYTerms = 128;     // weight terms of all sets of one schedule
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

// kx columns per tile of X (tile-major, written by the x pass) and of H (y and z passes):
// 16 (128-byte rows) up to N = 512; 8 at N = 1024, where a 16-column tile would need
// 1024-thread y blocks and their 128-register cap; 4 at 2048, where the 8-value schedule
// needs 256 threads per column.
template <int N>
__host__ __device__ constexpr int tile_cols() { return N >= 2048 ? 4 : (N >= 1024 ? 8 : (N / 2 < 16 ? N / 2 : 16)); }

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
};

// The groups written from the gathered grids alone. X holds only the monomials with a
// power of rhat_z below 2; a member (a, b, c) of group (n, c) with c >= 2 is the integer
// combination of gathered monomials that rhat_z^2 = 1 - rhat_x^2 - rhat_y^2 gives, so
//   H_(n,c) = sum_j Q_(j,n,c)(tx, ty) Y_j,  Q = sum of terms coef tx^a ty^b,
// over gathered grids j (no rhat_z for even c, one power for odd c). A set is up to
// kYSetGroups (8-value column schedule) or 3 (16-value schedule, whose registers hold
// fewer sums) groups of one parity of c: one y-pass launch per set loads each of the set's
// grids once and adds it, with its terms, into every group of the set.
struct YSetTable {
  float tcoef[kMaxYTerms];                // weight of a term
  int32_t nsets;
  int16_t mem0[kMaxYSets + 1];            // members of set s: [mem0[s], mem0[s + 1])
  int16_t term0[kMaxYMembers + 1];        // terms of member i: [term0[i], term0[i + 1])
  int8_t ngroups[kMaxYSets];              // groups in set s
  int8_t group[kMaxYSets][kYSetGroups];   // H group of slot k of set s
  int8_t mgrid[kMaxYMembers];             // X grid (gathered index) of a member
  int8_t tslot[kMaxYTerms];               // slot (group of the set) of a term
  int8_t ta[kMaxYTerms], tb[kMaxYTerms];  // powers of tx and ty of a term
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
  int G;          // LOS-weighted grids: 1, 7, 22, 50
  int GK;         // of them gathered and stored in X (power of rhat_z below 2): 1, 6, 15, 28
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
  YSetTable ysets[2];  // y-pass sets of the 8- and 16-value schedules
  TileTable tiles;
  // workspace offsets (bytes)
  size_t off_scalars, off_partials, off_flags, off_tw, off_invw2, off_alias, off_tables;
  size_t off_rowcnt, off_rowoff, off_rowhist, off_blocksum, off_tmp, off_rowkey, off_sorted, off_X, off_H, off_zpart, off_result;
  size_t total;
  size_t H_group_stride;   // float2 elements per group in H
  int64_t result_doubles;
};

// Workspace offsets of the device tables (from off_tables).
constexpr size_t ysets_offset(int schedule) { return (size_t)schedule * sizeof(YSetTable); }
constexpr size_t tiles_offset() { return 2 * sizeof(YSetTable); }
constexpr size_t tables_bytes() { return 2 * sizeof(YSetTable) + sizeof(TileTable); }

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
