// Transforms along y and z, the k-hat contraction and the shell binning
// (Sec. 3, Eqs. 6-13).
//
// H is stored in tiles of TKH kx columns (tile_cols): for each group, tile and z, the
// rows |ky| <= M(tile) of TKH complex values.
// y pass: one block owns TK kx columns (a whole H tile, or half of one at N = 512 and
//   1024) at one z and one set of groups of one parity of c. X holds only the gathered
//   monomials (power of rhat_z below 2); a group's other members are combinations of them
//   (rhat_z^2 = 1 - rhat_x^2 - rhat_y^2), so H_{n,c} = sum_j Q_j(tx, ty) Y_j over gathered
//   grids j with polynomial weights Q_j. For each gathered grid of the set the block loads
//   the N x TK tile (TK complex values per row, coalesced), transforms along y and adds it
//   with its weights into every group of the set, whose sums stay in registers; each group
//   leaves a single grid H_{n,c}. Only the rows with kx0^2 + ky^2 < K^2 are stored
//   (kx0 = the H tile's smallest kx).
// z pass: a persistent block walks (kx tile, ky) columns (a whole H tile, or half of
//   one at N = 512). It transforms H_{0,0} along z to A_0, accumulates
//   A_n = |t|^-n sum_c tz^c FFT_z[H_{n,c}] for n = 2, 4 (and 6) (t = 2n/N), and adds
//   per mode mu Re[A_0 A_l^*] / W^2, the noise and the mode count to FP64 bin sums in
//   LDS (mu = 1 on the kx = 0 plane, 2 elsewhere: the other half of the lattice holds
//   the complex conjugates). Each block writes its bin sums once.
//
// By linearity, A_n = |t|^-n sum_{a+b+c=n} coef tx^a ty^b tz^c FFT_xyz[F rhat^(a,b,c)]
// equals the paper's Eqs. (10) and (12); regrouping by the power of z only moves the
// kx, ky factors in front of the z transform.
#include <hip/hip_runtime.h>

#include "fft_dev.hpp"
#include "plan.hpp"

namespace pk {

struct YArgs {
  int Kx;
  int z0;                 // first plane of the slab
  int pbase;              // plane of X that holds plane z0
  int64_t x_grid_stride;  // xr xs N Kx
  int64_t h_group_stride;
  const YSetTable* yt;    // device copies (dynamic indexing of by-value kernel
  const TileTable* tt;    // arguments would push them to scratch)
};

__device__ __forceinline__ float ipow(float x, int e) {
  float r = 1.0f;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

// LDS slot of row `idx` of column `c`: rows of TK complex values (128 bytes for
// TK = 16), so a wave touching 16 columns of 4 rows is conflict-free.
template <int TK>
struct ColSlot {
  int c;
  __device__ __forceinline__ int operator()(int idx) const { return idx * TK + c; }
};

// kx columns per y-pass block: half a tile of H at N = 512 and 1024, so that two blocks
// (8 and 16 values per thread respectively need 96 and ~230 registers) share a CU and
// one block's barriers overlap the other's work; two neighbouring blocks (on one XCD)
// fill the two halves of each H tile row. A whole tile elsewhere.
template <int N>
constexpr int ytile_cols() { return (N == 512 || N == 1024) ? tile_cols<N>() / 2 : tile_cols<N>(); }

// kx columns per z-pass block: half an H tile (8 columns, 512 threads) at N = 512, so that
// two blocks of ~128 registers share a CU instead of one (z pass 1.29 -> 1.16 ms at 512^3);
// at 1024 half tiles (4 columns) were slower (11.7 -> 12.1 ms): whole tiles there.
template <int N>
constexpr int ztile_cols() { return N == 512 ? tile_cols<N>() / 2 : tile_cols<N>(); }

// Linear block id -> logical id such that blocks with consecutive logical ids run on one
// XCD (workgroups go to the 8 XCDs round-robin): tiles narrower than a 128-byte line
// share lines with their neighbours, which then meet in that XCD's L2. Needs a multiple
// of 8 blocks; otherwise the identity.
__device__ __forceinline__ uint32_t xcd_group(uint32_t lin, uint32_t nblk) {
  return (nblk & 7u) ? lin : (lin & 7u) * (nblk >> 3) + (lin >> 3);
}

// Column transforms come in two schedules, picked per plan (the autotuner times both):
// EC = 16 values per thread (radices 16, 8, 4 at 512: fewer threads) or EC = 8 (radices
// 8, 8, 8: half the registers). With EC = 8 the thread's row index is hidden from the
// optimiser where it is used, so that the addresses derived from it are recomputed
// instead of being held in registers across the loops (that would cost the occupancy the
// smaller schedule is for); with EC = 16 the code is left to the optimiser.
template <int EC>
__device__ __forceinline__ int col_hide(int v) {
  if constexpr (EC == 8) asm volatile("" : "+v"(v));
  return v;
}

// Loads the column tile of member grid m (plane pbase + zs of X) in stage-0 order.
template <int N, int TK, int EC>
__device__ __forceinline__ void load_member(const float2* __restrict__ X, const YArgs& a, int m, int zs, int kt,
                                            int tid0, float2 (&d)[Fft<N, EC>::E]) {
  using F = Fft<N, EC>;
  const int tid = col_hide<EC>(tid0);
  const int c = tid % TK, t = tid / TK;
  // tile-major X: [plane][kx / TW][y][kx % TW], the block's TK columns inside one tile
  constexpr int TW = tile_cols<N>();
  static_assert(TW % TK == 0, "a y block reads a part of one X tile");
  const int kx = kt * TK + c;
  const float2* __restrict__ src =
      X + (size_t)m * a.x_grid_stride + (size_t)(a.pbase + zs) * N * a.Kx + (size_t)(kx / TW) * TW * N + (kx % TW);
#pragma unroll
  for (int e = 0; e < F::E; ++e) d[e] = src[(size_t)F::in_index(t, e) * TW];
}

// One set of z-power groups (YSetTable) for TK kx columns at one z: every member (a
// gathered grid of the set) is loaded once, transformed along y, and added into each group
// of the set it has terms in, with weight sum coef tx^a ty^b; the NGS group sums stay in
// registers until the end.
template <int N, int TK, int EC, int TKH, int NGS>
__global__ __launch_bounds__((TK * Fft<N, EC>::T)) void ypass_kernel(const float2* __restrict__ X, float2* __restrict__ H,
                                                                  const float2* __restrict__ tw, const YArgs a,
                                                                  const int set) {
  static_assert(TKH % TK == 0, "a y tile is a part of an H tile");
  using F = Fft<N, EC>;
  extern __shared__ float2 T[];
  // The set's members and terms and the twiddles, in LDS: loads of global memory retire
  // in order, so reading either from global memory inside a transform would also wait
  // for the next member's tile, which is in flight meanwhile.
  float2* twl = T + TK * N;
  __shared__ int s_grid[kMaxYMembers], s_t0[kMaxYMembers + 1], s_term[kMaxYTerms], s_group[kYSetGroups];
  __shared__ float s_coef[kMaxYTerms];
  const int tid0 = threadIdx.x;
  const uint32_t nblk = gridDim.x * gridDim.y;
  const uint32_t lb = xcd_group(blockIdx.x + blockIdx.y * gridDim.x, nblk);
  const int kt = (int)(lb % gridDim.x), zs = (int)(lb / gridDim.x), z = a.z0 + zs;
  const YSetTable& yt = *a.yt;
  const int m0 = yt.mem0[set], nmem = yt.mem0[set + 1] - m0, ngs = yt.ngroups[set];
  const int q0 = yt.term0[m0], nterm = yt.term0[m0 + nmem] - q0;
  for (int i = tid0; i < nmem; i += blockDim.x) s_grid[i] = yt.mgrid[m0 + i];
  for (int i = tid0; i <= nmem; i += blockDim.x) s_t0[i] = yt.term0[m0 + i] - q0;
  for (int i = tid0; i < nterm; i += blockDim.x) {
    s_term[i] = yt.tslot[q0 + i] | (yt.ta[q0 + i] << 8) | (yt.tb[q0 + i] << 16);  // slot, a, b
    s_coef[i] = yt.tcoef[q0 + i];
  }
  for (int i = tid0; i < ngs; i += blockDim.x) s_group[i] = yt.group[set][i];
  for (int i = tid0; i < N; i += blockDim.x) twl[i] = tw[i];
  // the H tile (TKH columns) this block's TK columns belong to, and their offset in it
  const int kth = kt * TK / TKH, ch = kt * TK - kth * TKH;
  const int M = a.tt->M[kth];
  const int64_t regoff = a.tt->regoff[kth];
  const int nslot = 2 * M + 1;
  // ty of each of the thread's output values, and tx of its column
  float tyv[F::E];
#pragma unroll
  for (int e = 0; e < F::E; ++e) tyv[e] = (float)signed_freq<N>(F::out_index(tid0 / TK, e)) * (2.0f / N);
  const float tx = (float)(kt * TK + tid0 % TK) * (2.0f / N);
  __syncthreads();
  float2 acc[NGS][F::E];
#pragma unroll
  for (int g = 0; g < NGS; ++g)
#pragma unroll
    for (int e = 0; e < F::E; ++e) acc[g][e] = make_float2(0.0f, 0.0f);
  {
    // member j + 1 is loaded while member j is transformed
    float2 nd[F::E];
    load_member<N, TK, EC>(X, a, s_grid[0], zs, kt, tid0, nd);
    for (int j = 0; j < nmem; ++j) {
      float2 d[F::E];
#pragma unroll
      for (int e = 0; e < F::E; ++e) d[e] = nd[e];
      if (j + 1 < nmem) load_member<N, TK, EC>(X, a, s_grid[j + 1], zs, kt, tid0, nd);
      const int tid = col_hide<EC>(tid0);
      F::run(d, tid / TK, twl, T, ColSlot<TK>{tid % TK});
      // the member's terms: coef tx^a ty^b into group slot s (block-uniform: scalar branches)
      const int qe = __builtin_amdgcn_readfirstlane(s_t0[j + 1]);
      for (int q = __builtin_amdgcn_readfirstlane(s_t0[j]); q < qe; ++q) {
        const int term = __builtin_amdgcn_readfirstlane(s_term[q]);
        const int s = term & 0xff, pa = (term >> 8) & 0xff, pb = term >> 16;
        float k = s_coef[q];
        for (int i = 0; i < pa; ++i) k *= tx;
        float w[F::E];
#pragma unroll
        for (int e = 0; e < F::E; ++e) w[e] = k;
        for (int i = 0; i < pb; ++i)
#pragma unroll
          for (int e = 0; e < F::E; ++e) w[e] *= tyv[e];
#pragma unroll
        for (int g = 0; g < NGS; ++g) {
          if (g == s) {
#pragma unroll
            for (int e = 0; e < F::E; ++e) {
              acc[g][e].x += w[e] * d[e].x;
              acc[g][e].y += w[e] * d[e].y;
            }
          }
        }
      }
    }
  }
  const int c = tid0 % TK, t = tid0 / TK;
#pragma unroll
  for (int g = 0; g < NGS; ++g) {
    if (g < ngs) {
      float2* __restrict__ dst =
          H + (size_t)s_group[g] * a.h_group_stride + regoff + (size_t)z * nslot * TKH + ch + c;
#pragma unroll
      for (int e = 0; e < F::E; ++e) {
        const int ky = signed_freq<N>(F::out_index(t, e));
        if (ky >= -M && ky <= M) dst[(size_t)(ky + M) * TKH] = acc[g][e];
      }
    }
  }
}

// Register sums per schedule: the 8-value schedule takes sets of up to 6 groups (built as
// 1, 3 or 6 slots) up to N = 512, the 16-value one sets of up to 3 (1 or 3 slots). From
// N = 1024 on the 8-value schedule also takes the sets of up to 3: at 1024 the 6-slot
// kernel (~167 registers) leaves one 512-thread block per CU, whose barriers in the
// four-stage transform then stall the CU (32.9 ms against 29.8 ms with sets of 3 and two
// blocks per CU, although sets of 3 load 19 grids instead of 15); at 2048, whose
// 1024-thread blocks cap a thread at 128 registers, 6 slots would spill. At 512 the sets of
// 6 take 3.10 ms against 3.50 ms for the G member grids of the full basis.
template <int N, int TK, int EC, int TKH, int NGS>
static void launch_yset(const Plan& p, char* ws, hipStream_t s, const YArgs& a, int set) {
  const size_t shmem = (size_t)(TK + 1) * N * sizeof(float2);  // column tile + twiddles
  const int ntiles = p.nkt * (TKH / TK);                      // y tiles: Kx / TK
  hipFuncSetAttribute(reinterpret_cast<const void*>(&ypass_kernel<N, TK, EC, TKH, NGS>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  hipLaunchKernelGGL((ypass_kernel<N, TK, EC, TKH, NGS>), dim3(ntiles, p.xs), dim3(TK * Fft<N, EC>::T), shmem, s,
                     at<const float2>(ws, p.off_X), at<float2>(ws, p.off_H), at<const float2>(ws, p.off_tw), a, set);
}

template <int N, int TK, int TKH>
static hipError_t launch_y2(const Plan& p, char* ws, hipStream_t s, int z0, int pbase) {
  const bool ec8 = N >= 2048 || p.col_e[0] == 8;
  const int sched = (ec8 && N < 1024) ? 0 : 1;  // set table: up to 6 groups, or up to 3
  YArgs a;
  a.Kx = p.Kx;
  a.z0 = z0;
  a.pbase = pbase;
  a.x_grid_stride = (int64_t)p.xr * p.xs * p.N * p.Kx;
  a.h_group_stride = (int64_t)p.H_group_stride;
  a.yt = at<const YSetTable>(ws, p.off_tables + ysets_offset(sched));
  a.tt = at<const TileTable>(ws, p.off_tables + tiles_offset());
  const YSetTable& yt = p.ysets[sched];
  for (int set = 0; set < yt.nsets; ++set) {
    const int ng = yt.ngroups[set];
    if (ec8) {
      if (ng <= 1) launch_yset<N, TK, 8, TKH, 1>(p, ws, s, a, set);
      else if (ng <= 3) launch_yset<N, TK, 8, TKH, 3>(p, ws, s, a, set);
      else if constexpr (N < 1024) launch_yset<N, TK, 8, TKH, 6>(p, ws, s, a, set);
    } else if constexpr (N < 2048) {
      if (ng <= 1) launch_yset<N, TK, 16, TKH, 1>(p, ws, s, a, set);
      else launch_yset<N, TK, 16, TKH, 3>(p, ws, s, a, set);
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// z pass with the contraction and the binning
// ---------------------------------------------------------------------------------
struct ZArgs {
  int Kx;
  int K2;          // K^2: modes with |n|^2 < K2 are binned
  int dn;
  int nbins;
  int compensate;
  int nkt;
  int64_t h_group_stride;
  int64_t n_items;
  const TileTable* tt;
};

// Lane i - S of the same 16-lane row (DPP row shift; a lane with no source reads 0).
template <int S>
__device__ __forceinline__ int dpp_shr(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x110 + S, 0xf, 0xf, true);
}
template <int S>
__device__ __forceinline__ double dpp_shr(double v) {
  const int lo = dpp_shr<S>(__double2loint(v)), hi = dpp_shr<S>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// The TK lanes c = 0 .. TK-1 of a column tile hold the same (ky, kz) at kx = kx0 + c, so
// their bins do not decrease with c and lanes of one bin are adjacent. A segmented
// inclusive sum over each run of equal keys (DPP row shifts: TK <= 16 divides the row)
// leaves the run's totals in its last lane, which alone adds them to LDS; this takes the
// same-address conflicts out of the atomics. Every lane of the wave must execute the
// shifts (a disabled source lane would be read as 0).
template <int TK>
struct Runs {
  static_assert(TK <= 16 && (TK & (TK - 1)) == 0, "tiles of up to 16 columns");
  bool take[4];  // step s (shift 2^s): the lane 2^s below is in this lane's run
  bool last;     // this lane ends its run: it alone adds the run's totals

  __device__ __forceinline__ Runs(int c, int key) {
    // every shift is taken by every lane (as the right operand of a short-circuit && a
    // shift would run only where the left one holds, and read the other lanes as disabled)
    take[0] = (c >= 1) & (dpp_shr<1>(key) == key);
    take[1] = (c >= 2) & (dpp_shr<2>(key) == key);
    take[2] = (c >= 4) & (dpp_shr<4>(key) == key);
    take[3] = (c >= 8) & (dpp_shr<8>(key) == key);
    const int next = __builtin_amdgcn_update_dpp(0, key, 0x101, 0xf, 0xf, true);  // lane i + 1 (row_shl:1)
    last = (c == TK - 1) | (next != key);
  }

  // Inclusive segmented sums of v over the runs (a few values at a time keeps the shifted
  // copies in few registers).
  template <int NV>
  __device__ __forceinline__ void sum(double (&v)[NV]) const {
    step<1>(v);
    if constexpr (TK > 2) step<2>(v);
    if constexpr (TK > 4) step<4>(v);
    if constexpr (TK > 8) step<8>(v);
  }
  template <int S, int NV>
  __device__ __forceinline__ void step(double (&v)[NV]) const {
    constexpr int k = S == 1 ? 0 : (S == 2 ? 1 : (S == 4 ? 2 : 3));
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const double u = dpp_shr<S>(v[j]);
      v[j] += take[k] ? u : 0.0;
    }
  }
};

__device__ __forceinline__ int isqrt_i(int n) {
  int s = (int)sqrtf((float)n);
  if (s * s > n) --s;
  if ((s + 1) * (s + 1) <= n) ++s;
  return s;
}

// Column (kx tile, ky) of the z pass: its H address (group 0), tile, part of the tile and
// row stride. A block takes TK columns: a whole H tile (HP = 1) or one of its HP parts;
// the HP parts of one (tile, ky) are consecutive items, which go to one XCD.
struct ZItem {
  const float2* base;
  int kt, part, M, s, zstride;
};

template <int TK, int HP>
__device__ __forceinline__ ZItem z_item(int64_t item, const float2* __restrict__ H, const int64_t* item0,
                                        const int64_t* regoff, const int* Mt, int nkt, int c) {
  const int64_t key = item / HP;  // the (tile, ky) column
  int kt = 0, hi = nkt;           // the tile: the last kt with item0[kt] <= key
  while (hi - kt > 1) {
    const int mid = (kt + hi) >> 1;
    if (item0[mid] <= key) kt = mid; else hi = mid;
  }
  ZItem z;
  z.kt = kt;
  z.part = (int)(item - key * HP);
  z.M = Mt[kt];
  z.s = (int)(key - item0[kt]);
  z.zstride = (2 * z.M + 1) * TK * HP;
  z.base = H + regoff[kt] + (size_t)z.s * TK * HP + z.part * TK + c;
  return z;
}

template <int N, int EC>
__device__ __forceinline__ void z_load(const float2* __restrict__ col, int zstride, int t0,
                                       float2 (&d)[Fft<N, EC>::E]) {
  using F = Fft<N, EC>;
  const int t = col_hide<EC>(t0);
#pragma unroll
  for (int e = 0; e < F::E; ++e) d[e] = col[(size_t)F::in_index(t, e) * zstride];
}

// z-power group taken at step k of a column: H_00 first, then each degree from the
// highest power of z down (Horner in tz): (2,2) (2,1) (2,0) (4,4) .. (4,0) (6,6) .. (6,0).
__host__ __device__ constexpr int zseq(int k) { return k == 0 ? 0 : (k <= 3 ? 4 - k : (k <= 8 ? 12 - k : 24 - k)); }

// Step k: takes the prefetched column of group zseq(k) into d, starts loading the next
// one (the next group of this column, or group 0 of the next column), then transforms d.
template <int N, int TK, int EC, int NG>
__device__ __forceinline__ void z_step(int k, float2 (&nd)[Fft<N, EC>::E], float2 (&d)[Fft<N, EC>::E],
                                       const ZItem& cur, const ZItem& nxt, bool more, int64_t gstride, int c, int t,
                                       const float2* twl, float2* T) {
  using F = Fft<N, EC>;
#pragma unroll
  for (int e = 0; e < F::E; ++e) d[e] = nd[e];
  if (k + 1 < NG)
    z_load<N, EC>(cur.base + (size_t)zseq(k + 1) * gstride, cur.zstride, t, nd);
  else if (more)
    z_load<N, EC>(nxt.base, nxt.zstride, t, nd);
  F::run(d, col_hide<EC>(t), twl, T, ColSlot<TK>{c});
}

// acc <- acc tz + FFT_z[H_(n, c)] over steps k0 .. k0 + CMAX (c = CMAX .. 0).
template <int N, int TK, int EC, int NG, int CMAX>
__device__ __forceinline__ void z_horner(int k0, float2 (&nd)[Fft<N, EC>::E], float2 (&acc)[Fft<N, EC>::E],
                                         const ZItem& cur, const ZItem& nxt, bool more, int64_t gstride, int c,
                                         int t, const float2* twl, float2* T) {
  using F = Fft<N, EC>;
#pragma unroll
  for (int e = 0; e < F::E; ++e) acc[e] = make_float2(0.0f, 0.0f);
  auto step = [&](int k) {
    float2 u[F::E];
    z_step<N, TK, EC, NG>(k, nd, u, cur, nxt, more, gstride, c, t, twl, T);
    const int tt = col_hide<EC>(t);
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
      const float tz = (float)signed_freq<N>(F::out_index(tt, e)) * (2.0f / N);
      acc[e].x = acc[e].x * tz + u[e].x;
      acc[e].y = acc[e].y * tz + u[e].y;
    }
  };
  if constexpr (EC == 8) {
    // one transform at a time: unrolled, the loads of several would be hoisted together
#pragma unroll 1
    for (int k = k0; k <= k0 + CMAX; ++k) step(k);
  } else {
    for (int k = k0; k <= k0 + CMAX; ++k) step(k);
  }
}

// Bytes of the z pass's LDS: the transform area, the twiddles, the FP64 bin sums, the
// tile table and the per-axis window tables.
__host__ __device__ constexpr size_t zpass_lds_bytes(int N, int TK, int nbins, int nkt) {
  return (size_t)TK * N * 8 + (size_t)N * 8 + (size_t)nbins * kNumSums * 8 + (size_t)(2 * nkt + 1) * 8 +
         (size_t)2 * N * 4 + (size_t)nkt * 4;
}

template <int N, int TK, int ELL, int EC, int HP>
__global__ __launch_bounds__((TK * Fft<N, EC>::T)) __attribute__((amdgpu_waves_per_eu(EC == 8 ? 4 : 1, 8))) void zpass_kernel(const float2* __restrict__ H,
                                                                  const float2* __restrict__ tw,
                                                                  const float* __restrict__ invw2,
                                                                  const float* __restrict__ alias,
                                                                  const double* __restrict__ scal,
                                                                  double* __restrict__ zpart, const ZArgs a) {
  using F = Fft<N, EC>;
  constexpr int NG = ELL == 0 ? 1 : (ELL == 2 ? 4 : (ELL == 4 ? 9 : 16));
  // LDS: every table the loop reads, so that no wait inside it drains the prefetch of the
  // next column (loads of global memory retire in order)
  extern __shared__ __align__(16) char smem[];
  float2* T = reinterpret_cast<float2*>(smem);
  float2* twl = T + TK * N;
  double* bins = reinterpret_cast<double*>(twl + N);
  int64_t* item0 = reinterpret_cast<int64_t*>(bins + a.nbins * kNumSums);
  int64_t* regoff = item0 + a.nkt + 1;
  float* ivw = reinterpret_cast<float*>(regoff + a.nkt);
  float* alw = ivw + N;
  int* Mt = reinterpret_cast<int*>(alw + N);
  const int tid = threadIdx.x;
  const int c = tid % TK, t = tid / TK;
  for (int i = tid; i < a.nbins * kNumSums; i += blockDim.x) bins[i] = 0.0;
  for (int i = tid; i < N; i += blockDim.x) {
    twl[i] = tw[i];
    ivw[i] = invw2[i];
    alw[i] = alias[i];
  }
  for (int i = tid; i <= a.nkt; i += blockDim.x) item0[i] = a.tt->item0[i];
  for (int i = tid; i < a.nkt; i += blockDim.x) {
    regoff[i] = a.tt->regoff[i];
    Mt[i] = a.tt->M[i];
  }
  const double S = scal[kNoiseS];
  const float twoN = 2.0f / N;
  __syncthreads();
  // consecutive items (neighbouring ky columns of one tile, which share lines when the
  // tile is narrower than 128 bytes) go to blocks of one XCD
  int64_t item = xcd_group(blockIdx.x, gridDim.x);
  ZItem cur = z_item<TK, HP>(item < a.n_items ? item : 0, H, item0, regoff, Mt, a.nkt, c);
  float2 nd[F::E];  // defined on every path (an undefined value can pin its register)
#pragma unroll
  for (int e = 0; e < F::E; ++e) nd[e] = make_float2(0.0f, 0.0f);
  if (item < a.n_items) z_load<N, EC>(cur.base, cur.zstride, t, nd);
  for (; item < a.n_items; item += gridDim.x) {
    const int64_t nitem = item + gridDim.x;
    const bool more = nitem < a.n_items;
    const ZItem nxt = more ? z_item<TK, HP>(nitem, H, item0, regoff, Mt, a.nkt, c) : cur;
    const int M = cur.M;
    const int ky = cur.s - M;
    const int kx = cur.kt * (TK * HP) + cur.part * TK + c;
    const float tx = (float)kx * twoN, ty = (float)ky * twoN;
    const float wxy = ivw[kx] * ivw[ky & (N - 1)];
    const float cxy = alw[kx] * alw[ky & (N - 1)];
    const int n2xy = kx * kx + ky * ky;
    // 1 or 2: its products with FP32 values are exact in FP32 (kept so: one register)
    const float mu = kx == 0 ? 1.0f : 2.0f;

    float2 a0[F::E];
    z_step<N, TK, EC, NG>(0, nd, a0, cur, nxt, more, a.h_group_stride, c, t, twl, T);

    float2 acc[F::E];
    if (ELL >= 2) z_horner<N, TK, EC, NG, 2>(1, nd, acc, cur, nxt, more, a.h_group_stride, c, t, twl, T);
    {
      // pass 1: counts, |n|, Q0, Q2 (ell_max >= 2) and the noise
      const int tt = col_hide<EC>(t);
#pragma unroll
      for (int e = 0; e < F::E; ++e) {
        const int kzi = F::out_index(tt, e);
        const int kz = signed_freq<N>(kzi);
        const int n2 = n2xy + kz * kz;
        const bool valid = n2 > 0 && n2 < a.K2;
        const int b = valid ? isqrt_i(n2) / a.dn : 0;
        float iw = 1.0f, noise_f = 1.0f;
        if (a.compensate >= 1) iw = wxy * ivw[kzi];
        if (a.compensate == 2) noise_f = cxy * alw[kzi] * iw;
        const float2 z0 = a0[e];
        const float q0 = (z0.x * z0.x + z0.y * z0.y) * iw;
        double w4[4];
        w4[0] = (double)mu;
        w4[1] = (double)(mu * sqrtf((float)n2));
        w4[2] = (double)(mu * q0);
        w4[3] = 0.0;
        if (ELL >= 2) {
          const float tz = (float)kz * twoN;
          const float inv_t2 = 1.0f / (tx * tx + ty * ty + tz * tz);
          const float2 A2 = acc[e];
          w4[3] = (double)(mu * ((z0.x * A2.x + z0.y * A2.y) * inv_t2 * iw));
        }
        // slots: 0 count, 1 |n|, 2 Q0, 3 Q2, 4 Q4, 5 noise, 6 Q6
        const Runs<TK> runs(c, valid ? b : -1 - c);  // invalid lanes: a key no neighbour holds
        const bool add = valid && runs.last;
        double wa[3] = {w4[0], w4[1], S * (double)(mu * noise_f)};
        runs.sum(wa);
        if (add) {
          atomicAdd(&bins[b * kNumSums + 0], wa[0]);
          atomicAdd(&bins[b * kNumSums + 1], wa[1]);
          atomicAdd(&bins[b * kNumSums + 5], wa[2]);
        }
        double wb[2] = {w4[2], w4[3]};
        runs.sum(wb);
        if (add) {
          atomicAdd(&bins[b * kNumSums + 2], wb[0]);
          atomicAdd(&bins[b * kNumSums + 3], wb[1]);
        }
      }
    }
    if (ELL >= 4) {
      z_horner<N, TK, EC, NG, 4>(4, nd, acc, cur, nxt, more, a.h_group_stride, c, t, twl, T);
      const int tt = col_hide<EC>(t);
#pragma unroll
      for (int e = 0; e < F::E; ++e) {
        const int kzi = F::out_index(tt, e);
        const int kz = signed_freq<N>(kzi);
        const int n2 = n2xy + kz * kz;
        const bool valid = n2 > 0 && n2 < a.K2;
        const int b = valid ? isqrt_i(n2) / a.dn : 0;
        const float iw = a.compensate >= 1 ? wxy * ivw[kzi] : 1.0f;
        const float tz = (float)kz * twoN;
        const float t2 = tx * tx + ty * ty + tz * tz;
        const float inv_t4 = 1.0f / (t2 * t2);
        const float2 z0 = a0[e];
        const float2 A4 = acc[e];
        double w[1] = {(double)(mu * ((z0.x * A4.x + z0.y * A4.y) * inv_t4 * iw))};
        const Runs<TK> runs(c, valid ? b : -1 - c);
        runs.sum(w);
        if (valid && runs.last) atomicAdd(&bins[b * kNumSums + 4], w[0]);
      }
    }
    if (ELL >= 6) {
      // A_6 = |t|^-6 sum_c tz^c FFT_z[H_(6,c)], groups 9 .. 15
      z_horner<N, TK, EC, NG, 6>(9, nd, acc, cur, nxt, more, a.h_group_stride, c, t, twl, T);
      const int tt = col_hide<EC>(t);
#pragma unroll
      for (int e = 0; e < F::E; ++e) {
        const int kzi = F::out_index(tt, e);
        const int kz = signed_freq<N>(kzi);
        const int n2 = n2xy + kz * kz;
        const bool valid = n2 > 0 && n2 < a.K2;
        const int b = valid ? isqrt_i(n2) / a.dn : 0;
        const float iw = a.compensate >= 1 ? wxy * ivw[kzi] : 1.0f;
        const float tz = (float)kz * twoN;
        const float t2 = tx * tx + ty * ty + tz * tz;
        const float inv_t6 = 1.0f / (t2 * t2 * t2);
        const float2 z0 = a0[e];
        const float2 A6 = acc[e];
        double w[1] = {(double)(mu * ((z0.x * A6.x + z0.y * A6.y) * inv_t6 * iw))};
        const Runs<TK> runs(c, valid ? b : -1 - c);
        runs.sum(w);
        if (valid && runs.last) atomicAdd(&bins[b * kNumSums + 6], w[0]);
      }
    }
    cur = nxt;
  }
  __syncthreads();
  double* out = zpart + (size_t)blockIdx.x * a.nbins * kNumSums;
  for (int i = tid; i < a.nbins * kNumSums; i += blockDim.x) out[i] = bins[i];
}

template <int N, int TK, int ELL, int EC, int HP>
static hipError_t launch_z4(const Plan& p, char* ws, const ZArgs& a, hipStream_t s) {
  const size_t shmem = zpass_lds_bytes(N, TK, p.nbins, p.nkt);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&zpass_kernel<N, TK, ELL, EC, HP>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  hipLaunchKernelGGL((zpass_kernel<N, TK, ELL, EC, HP>), dim3(p.z_blocks), dim3(TK * Fft<N, EC>::T), shmem, s,
                     at<const float2>(ws, p.off_H), at<const float2>(ws, p.off_tw), at<const float>(ws, p.off_invw2),
                     at<const float>(ws, p.off_alias), at<const double>(ws, p.off_scalars),
                     at<double>(ws, p.off_zpart), a);
  return hipGetLastError();
}

// At N = 2048 only the 8-value schedule is built: with 16 values per thread the column
// transforms need more than 256 registers.
template <int N, int TK, int ELL, int HP>
static hipError_t launch_z3(const Plan& p, char* ws, const ZArgs& a, hipStream_t s) {
  if constexpr (N >= 2048) {
    return launch_z4<N, TK, ELL, 8, HP>(p, ws, a, s);
  } else {
    return p.col_e[1] == 8 ? launch_z4<N, TK, ELL, 8, HP>(p, ws, a, s) : launch_z4<N, TK, ELL, 16, HP>(p, ws, a, s);
  }
}

// TKH: columns of an H tile; the z blocks take ztile_cols<N>() of them.
template <int N, int TKH>
static hipError_t launch_z2(const Plan& p, char* ws, hipStream_t s) {
  constexpr int TK = ztile_cols<N>(), HP = TKH / TK;
  static_assert(TKH % TK == 0, "a z block takes a part of an H tile");
  ZArgs a;
  a.Kx = p.Kx;
  a.K2 = p.K * p.K;
  a.dn = p.dn;
  a.nbins = p.nbins;
  a.compensate = p.compensate;
  a.nkt = p.nkt;
  a.h_group_stride = (int64_t)p.H_group_stride;
  a.n_items = p.z_items * HP;
  a.tt = at<const TileTable>(ws, p.off_tables + tiles_offset());
  switch (p.ell_max) {
    case 0: return launch_z3<N, TK, 0, HP>(p, ws, a, s);
    case 2: return launch_z3<N, TK, 2, HP>(p, ws, a, s);
    case 6:
      if constexpr (N <= 1024) return launch_z3<N, TK, 6, HP>(p, ws, a, s);
      else return hipErrorInvalidValue;
    default: return launch_z3<N, TK, 4, HP>(p, ws, a, s);
  }
}



hipError_t launch_ypass(const Plan& p, char* ws, hipStream_t s, int z0, int pbase) {
  switch (p.N) {
    case 8: return launch_y2<8, ytile_cols<8>(), tile_cols<8>()>(p, ws, s, z0, pbase);
    case 16: return launch_y2<16, ytile_cols<16>(), tile_cols<16>()>(p, ws, s, z0, pbase);
    case 32: return launch_y2<32, ytile_cols<32>(), tile_cols<32>()>(p, ws, s, z0, pbase);
    case 64: return launch_y2<64, ytile_cols<64>(), tile_cols<64>()>(p, ws, s, z0, pbase);
    case 128: return launch_y2<128, ytile_cols<128>(), tile_cols<128>()>(p, ws, s, z0, pbase);
    case 256: return launch_y2<256, ytile_cols<256>(), tile_cols<256>()>(p, ws, s, z0, pbase);
    case 512: return launch_y2<512, ytile_cols<512>(), tile_cols<512>()>(p, ws, s, z0, pbase);
    case 1024: return launch_y2<1024, ytile_cols<1024>(), tile_cols<1024>()>(p, ws, s, z0, pbase);
    case 2048: return launch_y2<2048, ytile_cols<2048>(), tile_cols<2048>()>(p, ws, s, z0, pbase);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zpass(const Plan& p, char* ws, hipStream_t s) {
  switch (p.N) {
    case 8: return launch_z2<8, tile_cols<8>()>(p, ws, s);
    case 16: return launch_z2<16, tile_cols<16>()>(p, ws, s);
    case 32: return launch_z2<32, tile_cols<32>()>(p, ws, s);
    case 64: return launch_z2<64, tile_cols<64>()>(p, ws, s);
    case 128: return launch_z2<128, tile_cols<128>()>(p, ws, s);
    case 256: return launch_z2<256, tile_cols<256>()>(p, ws, s);
    case 512: return launch_z2<512, tile_cols<512>()>(p, ws, s);
    case 1024: return launch_z2<1024, tile_cols<1024>()>(p, ws, s);
    case 2048: return launch_z2<2048, tile_cols<2048>()>(p, ws, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pk
