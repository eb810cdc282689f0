// Catalogue stages: workspace initialisation, the FP64 catalogue scalars (Sec. 2:
// alpha, I and the shot-noise amplitude of Eq. 3), input validation, the counting
// sort of particles by grid row, and the final FP64 reduction into P_0, P_2, P_4
// (Sec. 3, Eqs. 6-8).
#include <hip/hip_runtime.h>
#include <string.h>

#include "plan.hpp"
#include "particle.hpp"

namespace pk {

// --------------------------------------------------------------------------------
// Workspace initialisation: flags, row counters, the FFT twiddle table and the
// per-axis window tables, all computed here in FP64 and stored as FP32.
// --------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void init_kernel(int N, int assign, int* flags, float2* tw, float* invw2,
                                                   float* alias) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *flags = 0;
  if (t < N) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)N, &s, &c);   // exp(-2 pi i t / N)
    tw[t] = make_float2((float)c, (float)s);
    const int n = t < N / 2 ? t : t - N;
    const double x = (double)n / (double)N;           // in units of pi
    const double sn = sinpi(x);
    const double sinc = n == 0 ? 1.0 : sn / (M_PI * x);
    double w = sinc * sinc;                            // sinc^2 (CIC window)
    if (assign == PK_TSC) w *= sinc;                   // sinc^3 (TSC window)
    invw2[t] = (float)(1.0 / (w * w));
    const double s2 = sn * sn;
    const double C = assign == PK_CIC ? 1.0 - (2.0 / 3.0) * s2 : 1.0 - s2 + (2.0 / 15.0) * s2 * s2;
    alias[t] = (float)C;
  }
}

// Copies the group and tile tables into the workspace, passed by value as 32-bit words
// in pieces of at most 2 KB of kernel arguments (so that a captured graph holds them).
constexpr int kTableChunkWords = 512;
constexpr int kTableWords = (int)((tables_bytes() + 3) / 4);
struct TableChunk {
  uint32_t w[kTableChunkWords];
};

__global__ __launch_bounds__(256) void copy_tables_kernel(const TableChunk c, int n, uint32_t* out) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = c.w[i];
}

hipError_t launch_init(const Plan& p, char* ws, hipStream_t s) {
  uint32_t words[kTableWords];
  memset(words, 0, sizeof(words));
  memcpy(reinterpret_cast<char*>(words) + ysets_offset(0), &p.ysets[0], sizeof(YSetTable));
  memcpy(reinterpret_cast<char*>(words) + ysets_offset(1), &p.ysets[1], sizeof(YSetTable));
  memcpy(reinterpret_cast<char*>(words) + tiles_offset(), &p.tiles, sizeof(TileTable));
  for (int w0 = 0; w0 < kTableWords; w0 += kTableChunkWords) {
    const int n = kTableWords - w0 < kTableChunkWords ? kTableWords - w0 : kTableChunkWords;
    TableChunk c;
    memset(&c, 0, sizeof(c));
    memcpy(c.w, words + w0, sizeof(uint32_t) * n);
    hipLaunchKernelGGL(copy_tables_kernel, dim3(1), dim3(256), 0, s, c, n, at<uint32_t>(ws, p.off_tables) + w0);
  }
  const int blocks = (p.N + 255) / 256;
  hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, s, p.N, p.assign, at<int>(ws, p.off_flags),
                     at<float2>(ws, p.off_tw), at<float>(ws, p.off_invw2), at<float>(ws, p.off_alias));
  return hipGetLastError();
}

// --------------------------------------------------------------------------------
// Catalogue scalars (Sec. 2). Per-block FP64 partial sums in a fixed order, then a
// single block adds the partials in block order: the result does not depend on
// scheduling.
// --------------------------------------------------------------------------------
__device__ __forceinline__ bool finite_f(float v) { return isfinite(v); }

// Adds one particle's w, w^2 and (with_nb) w^2 nbar to s[0], s[1], s[2].
__device__ __forceinline__ void stats_add(float w, float nb, bool with_nb, double (&s)[3], bool& bad) {
  bad |= !finite_f(w);
  const double wd = w;
  s[0] += wd;
  s[1] += wd * wd;
  if (with_nb) {
    bad |= !finite_f(nb);
    s[2] += wd * wd * (double)nb;
  }
}

// Sums over one catalogue, grid-stride: 16-byte loads of four weights (and densities)
// where the arrays are 16-byte aligned, single elements for the rest.
__device__ __forceinline__ void stats_range(const float* w, const float* nb, int64_t n, bool with_nb, int64_t t0,
                                            int64_t stride, double (&s)[3], bool& bad) {
  const uintptr_t al = reinterpret_cast<uintptr_t>(w) | (with_nb ? reinterpret_cast<uintptr_t>(nb) : 0);
  int64_t done = 0;
  if ((al & 15) == 0) {
    const int64_t n4 = n / 4;
    for (int64_t i = t0; i < n4; i += stride) {
      const float4 wv = reinterpret_cast<const float4*>(w)[i];
      const float4 nv = with_nb ? reinterpret_cast<const float4*>(nb)[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      stats_add(wv.x, nv.x, with_nb, s, bad);
      stats_add(wv.y, nv.y, with_nb, s, bad);
      stats_add(wv.z, nv.z, with_nb, s, bad);
      stats_add(wv.w, nv.w, with_nb, s, bad);
    }
    done = 4 * n4;
  }
  for (int64_t i = done + t0; i < n; i += stride) stats_add(w[i], with_nb ? nb[i] : 0.0f, with_nb, s, bad);
}

__global__ __launch_bounds__(256) void stats_kernel(pk_catalog gal, pk_catalog ran, int norm_from,
                                                    double* partials, int* flags) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sg[3] = {0, 0, 0}, sr[3] = {0, 0, 0};
  stats_range(gal.w, gal.nbar, gal.n, norm_from == 1, t0, stride, sg, bad);
  stats_range(ran.w, ran.nbar, ran.n, norm_from == 0, t0, stride, sr, bad);
  // slots: 0 sum w_g, 1 sum w_r, 2 sum w_g^2, 3 sum w_r^2, 4 sum w_g^2 nbar_g, 5 sum w_r^2 nbar_r
  double acc[6] = {sg[0], sr[0], sg[1], sr[1], sg[2], sr[2]};
  if (bad) atomicOr(flags, (int)kFlagNonFiniteWeight);
  __shared__ double red[6][256];
#pragma unroll
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
#pragma unroll
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) partials[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Sum of the block partials in block order: thread k of a 256-thread block adds every
// 256th partial of slot j, then a fixed tree combines the 256 sums.
__global__ __launch_bounds__(256) void stats_final_kernel(const double* partials, int nblk, int norm_from, double* scal,
                                                          int* flags) {
  __shared__ double red[6][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double s = 0.0;
    for (int b = t; b < nblk; b += 256) s += partials[b * 6 + j];
    red[j][t] = s;
  }
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int j = 0; j < 6; ++j) red[j][t] += red[j][t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    double sums[6];
    for (int j = 0; j < 6; ++j) {
      sums[j] = red[j][0];
      scal[kSumWg + j] = sums[j];
    }
    const double alpha = sums[0] / sums[1];
    const double I = norm_from == 0 ? alpha * sums[5] : sums[4];
    const double S = sums[2] + alpha * alpha * sums[3];
    scal[kAlpha] = alpha;
    scal[kNormI] = I;
    scal[kNoiseS] = S;
    if (!(sums[1] != 0.0) || !isfinite(alpha) || !(I > 0.0) || !isfinite(I) || !isfinite(S))
      atomicOr(flags, (int)kFlagBadNorm);
  }
}

hipError_t launch_stats(const Plan& p, const pk_catalog& gal, const pk_catalog& ran, char* ws, hipStream_t s) {
  hipLaunchKernelGGL(stats_kernel, dim3(kStatsBlocks), dim3(256), 0, s, gal, ran, p.norm_from,
                     at<double>(ws, p.off_partials), at<int>(ws, p.off_flags));
  hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(256), 0, s, at<double>(ws, p.off_partials),
                     kStatsBlocks, p.norm_from, at<double>(ws, p.off_scalars), at<int>(ws, p.off_flags));
  return hipGetLastError();
}

// --------------------------------------------------------------------------------
// Counting sort of the particles by grid row (y, z), in two privatised levels so that
// no device-scope atomics are needed: level A sorts by z plane with per-block LDS
// histograms, level B sorts each plane by row y in one block. The payload is
// (x, y, z, w') with w' = w for galaxies and -alpha w for randoms (Eq. 1). Invalid
// particles are flagged and left out; the host turns a flag into an error.
// --------------------------------------------------------------------------------
struct SortGeom {
  double invH;     // N / L
  double bmin_d[3];
  double L;
  float obs[3];   // the observer rounded to FP32, as the assignment takes it
  int N;
  int los;
};

// The one validity test of both sort passes (they must agree particle by particle).
template <bool RAISE>
__device__ __forceinline__ bool valid_particle(const SortGeom& g, float x, float y, float z, int* flags) {
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    if (RAISE) atomicOr(flags, (int)kFlagNonFinitePos);
    return false;
  }
  const double dx = (double)x - g.bmin_d[0], dy = (double)y - g.bmin_d[1], dz = (double)z - g.bmin_d[2];
  if (!(dx >= 0.0 && dx < g.L && dy >= 0.0 && dy < g.L && dz >= 0.0 && dz < g.L)) {
    if (RAISE) atomicOr(flags, (int)kFlagOutOfBox);
    return false;
  }
  if (g.los == 0) {
    if (!(los_norm2(x, y, z, g.obs[0], g.obs[1], g.obs[2]) > 0.0f)) {
      if (RAISE) atomicOr(flags, (int)kFlagAtObserver);
      return false;
    }
  }
  return true;
}

// Level A, pass 1: per-block histogram over z planes in LDS, stored plane-major
// (ph[plane * B + block]) so that one exclusive scan gives every block's first slot in
// every plane. Each block owns the contiguous particle range [blk * per, (blk+1) * per).
template <int ASSIGN>
__global__ __launch_bounds__(256) void plane_hist_kernel(pk_catalog gal, pk_catalog ran, SortGeom g, int64_t per,
                                                         uint32_t* ph, int* flags) {
  extern __shared__ uint32_t h[];
  for (int i = threadIdx.x; i < g.N; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const int64_t ntot = gal.n + ran.n;
  const int64_t i0 = (int64_t)blockIdx.x * per;
  const int64_t i1 = i0 + per < ntot ? i0 + per : ntot;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const float* q = i < gal.n ? gal.xyz + 3 * i : ran.xyz + 3 * (i - gal.n);
    const float x = q[0], y = q[1], z = q[2];
    if (!valid_particle<true>(g, x, y, z, flags)) continue;
    atomicAdd(&h[axis_cell<ASSIGN>(z, g.bmin_d[2], g.invH, g.N).i], 1u);
  }
  __syncthreads();
  for (int pl = threadIdx.x; pl < g.N; pl += blockDim.x) ph[(int64_t)pl * gridDim.x + blockIdx.x] = h[pl];
}

// Exclusive scan of a[0, n) (n <= 4 NT) held in LDS, by a block of NT threads; writes
// the starts back into a and returns the total to every thread.
template <int NT>
__device__ __forceinline__ uint32_t block_scan_lds(uint32_t* a, int n) {
  constexpr int PER = 4;
  __shared__ uint32_t wsum[NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t v[PER];
  uint32_t loc = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid * PER + j;
    v[j] = idx < n ? a[idx] : 0u;
    loc += v[j];
  }
  uint32_t inc = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  uint32_t ex = inc - loc, tot = 0;
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wv) ex += wsum[w];
    tot += wsum[w];
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid * PER + j;
    if (idx < n) a[idx] = ex;
    ex += v[j];
  }
  __syncthreads();
  return tot;
}

// Both scatters write through an LDS tile: a tile of particles is counting-sorted by
// bucket in LDS and then copied out bucket run by bucket run, so that consecutive
// threads store consecutive slots of one bucket (runs of ~tile/buckets particles)
// instead of scattering 16-byte stores over all buckets, which costs a partial-line
// write per particle.
// Tiles of 6144 particles (6 per thread): the largest multiple of the block that leaves
// the staging within the 160 KB of LDS at N = 2048 (24 KB of bucket tables + 120 KB);
// measured 7-8% faster than 4096 at 512^3 and 1024^3 (longer runs, fewer tile rounds).
constexpr int kSortThreads = 1024;
constexpr int kSortTile = 6144;
constexpr int kSortPer = kSortTile / kSortThreads;

// LDS of one staged scatter: cur, tcnt, gb (uint32[nb] each), stage float4[tile],
// skey and sval (uint16[tile] each).
__host__ __device__ constexpr size_t staged_lds_bytes(int nb) {
  return (size_t)3 * nb * 4 + (size_t)kSortTile * (16 + 2 + 2);
}

// Level A, pass 2: the same particles, scattered plane by plane into tmp as
// (x, y, z, w') with w' = w for galaxies and -alpha w for randoms (Eq. 1); the row index
// of each particle goes to rowkey at the same slot, for level B.
template <int ASSIGN>
__global__ __launch_bounds__(kSortThreads) void plane_scatter_kernel(pk_catalog gal, pk_catalog ran, SortGeom g,
                                                                     int64_t per, const uint32_t* phoff,
                                                                     const double* scal, float4* tmp,
                                                                     uint16_t* rowkey) {
  extern __shared__ __align__(16) uint32_t sm[];
  const int nb = g.N;
  uint32_t* cur = sm;        // next global slot of each plane for this block
  uint32_t* tcnt = cur + nb;  // tile counts, then tile starts
  uint32_t* gb = tcnt + nb;   // global slot of the first particle of each plane's run in the tile
  float4* stage = reinterpret_cast<float4*>(sm + 3 * nb);
  uint16_t* skey = reinterpret_cast<uint16_t*>(stage + kSortTile);
  uint16_t* sval = skey + kSortTile;
  const int tid = threadIdx.x;
  for (int pl = tid; pl < nb; pl += kSortThreads) cur[pl] = phoff[(int64_t)pl * gridDim.x + blockIdx.x];
  const float alpha = (float)scal[kAlpha];
  const int64_t ntot = gal.n + ran.n;
  const int64_t i0 = (int64_t)blockIdx.x * per;
  const int64_t i1 = i0 + per < ntot ? i0 + per : ntot;
  // raw (x, y, z, w) of this thread's particles of the next tile, loaded one tile ahead
  float4 nraw[kSortPer];
  auto load_tile = [&](int64_t t0) {
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      const int64_t i = t0 + tid + j * kSortThreads;
      if (i < i1) {
        const bool isg = i < gal.n;
        const float* q = isg ? gal.xyz + 3 * i : ran.xyz + 3 * (i - gal.n);
        nraw[j] = make_float4(q[0], q[1], q[2], isg ? gal.w[i] : ran.w[i - gal.n]);
      }
    }
  };
  load_tile(i0);
  for (int64_t t0 = i0; t0 < i1; t0 += kSortTile) {
    float4 raw[kSortPer];
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) raw[j] = nraw[j];
    if (t0 + kSortTile < i1) load_tile(t0 + kSortTile);
    __syncthreads();  // the previous tile's copy-out is done (and cur is set)
    for (int k = tid; k < nb; k += kSortThreads) tcnt[k] = 0u;
    __syncthreads();
    float4 v[kSortPer];
    int key[kSortPer], row[kSortPer];
    uint32_t rank[kSortPer];
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      const int64_t i = t0 + tid + j * kSortThreads;
      key[j] = -1;
      row[j] = 0;
      rank[j] = 0u;
      v[j] = raw[j];
      // flags were raised by the histogram pass; here invalid particles are skipped
      if (i < i1 && valid_particle<false>(g, raw[j].x, raw[j].y, raw[j].z, nullptr)) {
        key[j] = axis_cell<ASSIGN>(raw[j].z, g.bmin_d[2], g.invH, g.N).i;
        row[j] = axis_cell<ASSIGN>(raw[j].y, g.bmin_d[1], g.invH, g.N).i;
        if (i >= gal.n) v[j].w = -alpha * raw[j].w;
        rank[j] = atomicAdd(&tcnt[key[j]], 1u);
      }
    }
    __syncthreads();
    for (int k = tid; k < nb; k += kSortThreads) {
      gb[k] = cur[k];
      cur[k] += tcnt[k];
    }
    const uint32_t ntile = block_scan_lds<kSortThreads>(tcnt, nb);  // barriers inside
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      if (key[j] >= 0) {
        const uint32_t lp = tcnt[key[j]] + rank[j];
        stage[lp] = v[j];
        skey[lp] = (uint16_t)key[j];
        sval[lp] = (uint16_t)row[j];
      }
    }
    __syncthreads();
    for (uint32_t lp = tid; lp < ntile; lp += kSortThreads) {
      const int k = skey[lp];
      const uint32_t dst = gb[k] + (lp - tcnt[k]);
      if (dst < (uint32_t)ntot) {
        tmp[dst] = stage[lp];
        rowkey[dst] = sval[lp];
      }
    }
  }
}

// Level B splits each plane into kRowParts contiguous parts, one block each, so that
// the whole chip works on it. Pass 1: each block counts its part's particles per row
// into rh[(plane N + row) kRowParts + part]; one exclusive scan of rh (row-major, parts
// innermost) then gives every block its first slot in every row, and rh at part 0 is
// the row offset.
constexpr int kRowParts = kRowHistParts;

__device__ __forceinline__ void plane_part(const uint32_t* phoff, int B, int pl, int q, uint32_t& lo, uint32_t& hi) {
  const uint32_t a = phoff[(int64_t)pl * B], b = phoff[(int64_t)(pl + 1) * B];
  const uint32_t len = (b - a + kRowParts - 1) / kRowParts;
  lo = a + (uint32_t)q * len < b ? a + (uint32_t)q * len : b;
  hi = lo + len < b ? lo + len : b;
}

__global__ __launch_bounds__(kSortThreads) void row_hist_kernel(const uint16_t* __restrict__ rowkey,
                                                                const uint32_t* __restrict__ phoff, int B, int N,
                                                                uint32_t* __restrict__ rh) {
  extern __shared__ uint32_t hc[];
  const int q = blockIdx.x, pl = blockIdx.y, tid = threadIdx.x;
  uint32_t lo, hi;
  plane_part(phoff, B, pl, q, lo, hi);
  for (int i = tid; i < N; i += kSortThreads) hc[i] = 0u;
  __syncthreads();
  // eight keys per 16-byte load over the aligned middle of the part, single keys at its ends
  // (rowkey starts on a 256-byte boundary of the workspace)
  const uint32_t a0 = (lo + 7u) & ~7u, a1 = hi & ~7u;
  if (a0 < a1) {
    for (uint32_t j = a0 / 8 + tid; j < a1 / 8; j += kSortThreads) {
      const uint4 v = reinterpret_cast<const uint4*>(rowkey)[j];
      const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        atomicAdd(&hc[u[k] & 0xffffu], 1u);
        atomicAdd(&hc[u[k] >> 16], 1u);
      }
    }
    if ((uint32_t)tid < a0 - lo) atomicAdd(&hc[rowkey[lo + tid]], 1u);
    if ((uint32_t)tid < hi - a1) atomicAdd(&hc[rowkey[a1 + tid]], 1u);
  } else {
    for (uint32_t i = lo + tid; i < hi; i += kSortThreads) atomicAdd(&hc[rowkey[i]], 1u);
  }
  __syncthreads();
  for (int y = tid; y < N; y += kSortThreads) rh[((int64_t)pl * N + y) * kRowParts + q] = hc[y];
}

__device__ __forceinline__ void load_row_tile(const float4* __restrict__ tmp, const uint16_t* __restrict__ rowkey,
                                              uint32_t t0, uint32_t hi, int tid, float4 (&nv)[kSortPer],
                                              int (&nk)[kSortPer]) {
#pragma unroll
  for (int j = 0; j < kSortPer; ++j) {
    const uint32_t i = t0 + tid + j * kSortThreads;
    nk[j] = -1;
    nv[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (i < hi) {
      nk[j] = rowkey[i];
      nv[j] = tmp[i];
    }
  }
}

// Pass 2: each block scatters its part by row through the LDS tile; part 0 also writes
// the row offsets rowoff[z N + y] (rowoff[N N] = total).
__global__ __launch_bounds__(kSortThreads) void row_sort_kernel(const float4* __restrict__ tmp,
                                                                const uint16_t* __restrict__ rowkey,
                                                                const uint32_t* __restrict__ phoff, int B, int N,
                                                                const uint32_t* __restrict__ rstart,
                                                                float4* __restrict__ sorted,
                                                                uint32_t* __restrict__ rowoff) {
  extern __shared__ __align__(16) uint32_t sm[];
  const int nb = N;
  uint32_t* cur = sm;
  uint32_t* tcnt = cur + nb;
  uint32_t* gb = tcnt + nb;
  float4* stage = reinterpret_cast<float4*>(sm + 3 * nb);
  uint16_t* skey = reinterpret_cast<uint16_t*>(stage + kSortTile);
  const int tid = threadIdx.x;
  const int q = blockIdx.x, pl = blockIdx.y;
  uint32_t lo, hi;
  plane_part(phoff, B, pl, q, lo, hi);
  for (int y = tid; y < nb; y += kSortThreads) {
    cur[y] = rstart[((int64_t)pl * nb + y) * kRowParts + q];
    if (q == 0) rowoff[(int64_t)pl * nb + y] = cur[y];
  }
  if (q == 0 && pl == nb - 1 && tid == 0) rowoff[(int64_t)nb * nb] = phoff[(int64_t)nb * B];
  // this thread's particles and keys of the next tile, loaded one tile ahead
  float4 nv[kSortPer];
  int nk[kSortPer];
  const uint32_t total = phoff[(int64_t)nb * B];
  load_row_tile(tmp, rowkey, lo, hi, tid, nv, nk);
  for (uint32_t t0 = lo; t0 < hi; t0 += kSortTile) {
    float4 v[kSortPer];
    int key[kSortPer];
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      v[j] = nv[j];
      key[j] = nk[j];
    }
    if (t0 + kSortTile < hi) load_row_tile(tmp, rowkey, t0 + kSortTile, hi, tid, nv, nk);
    __syncthreads();  // the previous tile's copy-out is done (and cur is set)
    for (int k = tid; k < nb; k += kSortThreads) tcnt[k] = 0u;
    __syncthreads();
    uint32_t rank[kSortPer];
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) rank[j] = key[j] >= 0 ? atomicAdd(&tcnt[key[j]], 1u) : 0u;
    __syncthreads();
    for (int k = tid; k < nb; k += kSortThreads) {
      gb[k] = cur[k];
      cur[k] += tcnt[k];
    }
    const uint32_t ntile = block_scan_lds<kSortThreads>(tcnt, nb);
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      if (key[j] >= 0) {
        const uint32_t lp = tcnt[key[j]] + rank[j];
        stage[lp] = v[j];
        skey[lp] = (uint16_t)key[j];
      }
    }
    __syncthreads();
    for (uint32_t lp = tid; lp < ntile; lp += kSortThreads) {
      const int k = skey[lp];
      const uint32_t dst = gb[k] + (lp - tcnt[k]);
      if (dst < total) sorted[dst] = stage[lp];
    }
  }
}

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t* cnt, int64_t n, uint32_t* blocksum) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t s = 0;
  for (int k = threadIdx.x; k < kScanChunk; k += 256) {
    const int64_t i = base + k;
    if (i < n) s += cnt[i];
  }
  __shared__ uint32_t red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) blocksum[blockIdx.x] = red[0];
}

// Exclusive scan of up to kScanTopMax block sums in one block of 1024 threads, four
// consecutive sums per thread.
__global__ __launch_bounds__(1024) void scan_top_kernel(uint32_t* blocksum, int nb) {
  constexpr int PER = kScanTopMax / 1024;
  __shared__ uint32_t a[1024];
  const int t = threadIdx.x;
  uint32_t v[PER];
  uint32_t loc = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = t * PER + j;
    v[j] = i < nb ? blocksum[i] : 0u;
    loc += v[j];
  }
  a[t] = loc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t add = t >= off ? a[t - off] : 0u;
    __syncthreads();
    a[t] += add;
    __syncthreads();
  }
  uint32_t run = a[t] - loc;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = t * PER + j;
    if (i < nb) blocksum[i] = run;
    run += v[j];
  }
}

// Exclusive scan, second level: out[i] = offset of element i (in place allowed), out[n] = total.
__global__ __launch_bounds__(256) void scan_down_kernel(const uint32_t* cnt, int64_t n, const uint32_t* blocksum,
                                                        uint32_t* out) {
  constexpr int PER = kScanChunk / 256;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * PER;
  uint32_t v[PER];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? cnt[i] : 0u;
    s += v[k];
  }
  __shared__ uint32_t a[256];
  a[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t add = (int)threadIdx.x >= off ? a[threadIdx.x - off] : 0u;
    __syncthreads();
    a[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = a[threadIdx.x] - s + blocksum[blockIdx.x];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) out[n] = run;
}

static SortGeom sort_geom(const Plan& p) {
  SortGeom g;
  for (int i = 0; i < 3; ++i) {
    g.bmin_d[i] = p.box_min[i];
    g.obs[i] = (float)p.observer[i];
  }
  g.invH = (double)p.N / p.L;
  g.L = p.L;
  g.N = p.N;
  g.los = p.los;
  return g;
}

int sort_blocks(int64_t ntot) {
  int64_t b = (ntot + 255) / 256;
  if (b > kSortBlocks) b = kSortBlocks;
  return b < 1 ? 1 : (int)b;
}

hipError_t launch_sort(const Plan& p, const pk_catalog& gal, const pk_catalog& ran, char* ws, hipStream_t s) {
  const SortGeom g = sort_geom(p);
  const int64_t ntot = p.n_gal + p.n_ran;
  const int B = sort_blocks(ntot);
  const int64_t per = (ntot + B - 1) / B;
  uint32_t* ph = at<uint32_t>(ws, p.off_rowcnt);
  const size_t shA = sizeof(uint32_t) * p.N;
  if (p.assign == PK_CIC)
    hipLaunchKernelGGL(plane_hist_kernel<PK_CIC>, dim3(B), dim3(256), shA, s, gal, ran, g, per, ph, at<int>(ws, p.off_flags));
  else
    hipLaunchKernelGGL(plane_hist_kernel<PK_TSC>, dim3(B), dim3(256), shA, s, gal, ran, g, per, ph, at<int>(ws, p.off_flags));
  const int64_t nph = (int64_t)p.N * B;
  const int nb = (int)((nph + kScanChunk - 1) / kScanChunk);
  const int64_t nrh = (int64_t)p.N * p.N * kRowParts;
  const int nbr = (int)((nrh + kScanChunk - 1) / kScanChunk);
  if (nb > kScanTopMax || nbr > kScanTopMax) return hipErrorInvalidValue;  // the block-sum buffer
  uint32_t* bsum = at<uint32_t>(ws, p.off_blocksum);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(256), 0, s, ph, nph, bsum);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, s, bsum, nb);
  hipLaunchKernelGGL(scan_down_kernel, dim3(nb), dim3(256), 0, s, ph, nph, bsum, ph);
  float4* tmp = at<float4>(ws, p.off_tmp);
  uint16_t* rowkey = at<uint16_t>(ws, p.off_rowkey);
  const size_t shS = staged_lds_bytes(p.N);  // above 64 KB at N = 2048
  hipFuncSetAttribute(reinterpret_cast<const void*>(&plane_scatter_kernel<PK_CIC>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shS);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&plane_scatter_kernel<PK_TSC>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shS);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&row_sort_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shS);
  if (p.assign == PK_CIC)
    hipLaunchKernelGGL(plane_scatter_kernel<PK_CIC>, dim3(B), dim3(kSortThreads), shS, s, gal, ran, g, per, ph,
                       at<const double>(ws, p.off_scalars), tmp, rowkey);
  else
    hipLaunchKernelGGL(plane_scatter_kernel<PK_TSC>, dim3(B), dim3(kSortThreads), shS, s, gal, ran, g, per, ph,
                       at<const double>(ws, p.off_scalars), tmp, rowkey);
  uint32_t* rh = at<uint32_t>(ws, p.off_rowhist);
  hipLaunchKernelGGL(row_hist_kernel, dim3(kRowParts, p.N), dim3(kSortThreads), sizeof(uint32_t) * p.N, s, rowkey, ph,
                     B, p.N, rh);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(nbr), dim3(256), 0, s, rh, nrh, bsum);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, s, bsum, nbr);
  hipLaunchKernelGGL(scan_down_kernel, dim3(nbr), dim3(256), 0, s, rh, nrh, bsum, rh);
  hipLaunchKernelGGL(row_sort_kernel, dim3(kRowParts, p.N), dim3(kSortThreads), shS, s, tmp, rowkey, ph, B, p.N, rh,
                     at<float4>(ws, p.off_sorted), at<uint32_t>(ws, p.off_rowoff));
  return hipGetLastError();
}

// --------------------------------------------------------------------------------
// Final reduction (Sec. 3, Eqs. 6-8): per-bin sums over the z-pass blocks in block
// order, then the Legendre combinations, the noise on ell = 0 only and 1/I.
// Result layout: k_eff[nb], P[(ell_max/2+1) nb], noise[nb], nmodes[nb], wedges[2 nb],
// alpha, I, S, flags.
// --------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void finalize_kernel(const double* zpart, int zblocks, int nbins, int ell_max,
                                                       double kf, const double* scal, const int* flags,
                                                       double* res) {
  // one block per bin: thread t adds the partials of blocks t, t + 256, ... in order, then
  // a fixed tree combines them
  __shared__ double red[kNumSums][256];
  const int b = blockIdx.x, t = threadIdx.x;
  double s[kNumSums] = {};
  for (int blk = t; blk < zblocks; blk += 256) {
    const double* q = zpart + ((size_t)blk * nbins + b) * kNumSums;
#pragma unroll
    for (int j = 0; j < kNumSums; ++j) s[j] += q[j];
  }
#pragma unroll
  for (int j = 0; j < kNumSums; ++j) red[j][t] = s[j];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int j = 0; j < kNumSums; ++j) red[j][t] += red[j][t + h];
    }
    __syncthreads();
  }
  if (t != 0) return;
  const double I = scal[kNormI];
  const int nl = ell_max / 2 + 1;
  double* k_eff = res;
  double* P = res + nbins;
  double* noise = P + (size_t)nl * nbins;
  double* nmodes = noise + nbins;
  double* wedge = nmodes + nbins;  // P_perp[nbins], then P_par[nbins]
  double* tail = wedge + 2 * nbins;
  const double cnt = red[0][0];
  if (cnt > 0.0) {
    const double den = I * cnt;
    k_eff[b] = kf * red[1][0] / cnt;
    P[b] = (red[2][0] - red[5][0]) / den;
    if (nl > 1) P[nbins + b] = 2.5 * (3.0 * red[3][0] - red[2][0]) / den;
    if (nl > 2) P[2 * nbins + b] = 1.125 * (35.0 * red[4][0] - 30.0 * red[3][0] + 3.0 * red[2][0]) / den;
    // ell = 6 by the same construction: 13/16 (231 Q6 - 315 Q4 + 105 Q2 - 5 Q0), from L_6
    if (nl > 3)
      P[3 * nbins + b] =
          0.8125 * (231.0 * red[6][0] - 315.0 * red[4][0] + 105.0 * red[3][0] - 5.0 * red[2][0]) / den;
    noise[b] = red[5][0] / den;
    // wedges mu in [0, 1/2] and [1/2, 1] from the multipoles (Sec. 5): the top-hat means
    // of L_2 and L_4 over those ranges are -+3/8 and +-15/128 (missing multipoles are 0)
    const double p2 = nl > 1 ? P[nbins + b] : 0.0, p4 = nl > 2 ? P[2 * nbins + b] : 0.0;
    wedge[b] = P[b] - 0.375 * p2 + (15.0 / 128.0) * p4;
    wedge[nbins + b] = P[b] + 0.375 * p2 - (15.0 / 128.0) * p4;
  } else {
    k_eff[b] = 0.0;
    for (int l = 0; l < nl; ++l) P[l * nbins + b] = 0.0;
    noise[b] = 0.0;
    wedge[b] = 0.0;
    wedge[nbins + b] = 0.0;
  }
  nmodes[b] = cnt;
  if (b == 0) {
    tail[0] = scal[kAlpha];
    tail[1] = scal[kNormI];
    tail[2] = scal[kNoiseS];
    tail[3] = (double)*flags;
  }
}

hipError_t launch_finalize(const Plan& p, char* ws, double* d_result, hipStream_t s) {
  const double kf = 2.0 * M_PI / p.L;
  hipLaunchKernelGGL(finalize_kernel, dim3(p.nbins), dim3(256), 0, s, at<double>(ws, p.off_zpart), p.z_blocks, p.nbins,
                     p.ell_max, kf, at<double>(ws, p.off_scalars), at<int>(ws, p.off_flags), d_result);
  return hipGetLastError();
}

}  // namespace pk
