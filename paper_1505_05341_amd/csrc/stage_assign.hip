// LOS-weighted mass assignment fused with the FFT along x (Sec. 3, Eqs. 11 and 13;
// Sec. 4 for the assignment).
//
// One block owns one target grid row (y, z) of the 1, 7, 22 or 50 monomial grids
// F rhat^m. Only the 1, 6, 15 or 28 monomials with a power of rhat_z below 2 are gathered,
// transformed and stored; the others follow exactly from rhat_x^2 + rhat_y^2 + rhat_z^2 = 1
// and enter the y pass as combinations of the stored rows (basis.hpp). The particles whose
// stencil reaches the row are those of a few source rows, which the counting sort made
// contiguous. They are processed in chunks:
//   1. each particle's own line of sight rhat = (x - observer)/|x - observer|, its
//      base cell along x, its x offset and its weight w' W_y W_z go to LDS;
//   2. the chunk is counting-sorted by base cell in LDS (integer atomics only): a
//      particle's rank in its cell is the count its atomic returns, and its record goes
//      straight from registers to its slot;
//   3. each thread owns target cells and gathers, from the particles of the 2 (CIC)
//      or 3 (TSC) source cells that reach it, w' W rhat^m for every gathered monomial,
//      summing in registers.
// No floating-point atomics are used: on gfx950 LDS float atomics run several times
// slower than integer ones, and a scatter would need one per particle, cell and grid.
// The finished rows never go to HBM in real space: two real rows are packed as one
// complex row, transformed along x in registers and LDS, separated into their two half
// spectra, and only kx < Kx is written (every mode with |kx| >= Kx lies outside the
// binned sphere).
#include <hip/hip_runtime.h>

#include "basis.hpp"
#include "fft_dev.hpp"
#include "monomial_sums.hpp"
#include "particle.hpp"
#include "plan.hpp"

namespace pk {

struct XArgs {
  double bmin[3];
  double invH;
  float obs[3];
  int los;
  int Kx;
  int z0;               // first plane of the slab
  int pbase;            // plane of X that receives plane z0
  int64_t grid_stride;  // float2 elements per grid of X: xr * xs * N * Kx
};

// Block geometry: 512 threads up to N = 512; from N = 1024 on, blocks of 1024 threads (one
// cell per thread at 1024, two at 2048). Particles per LDS chunk: 3 per thread for CIC at
// 512 and TSC at 1024, where the chunk area then still fits beside the transformed rows for
// 4 (512) or 2 (1024) blocks per CU and the records held through the counting sort fit the
// register budget (fewer chunk rounds per row, each with its barriers: 4.75 -> 4.46 ms at
// 512^3 CIC, 66.8 -> 61.7 ms at 1024^3 TSC; 4 per thread was slower at 512; TSC at 512 and
// CIC at 1024 would spill), 2 elsewhere.
template <int N, int ASSIGN>
struct XGeom {
  static constexpr int NT = N >= 1024 ? 1024 : 512;  // threads
  static constexpr int PER = ((N == 512 && ASSIGN == PK_CIC) || (N == 1024 && ASSIGN == PK_TSC)) ? 3 : 2;
  static constexpr int CHUNK = NT * PER;              // particles per LDS chunk
};

// Bytes of the gather-phase LDS area: the chunk's particles in base-cell order, pa
// float4[XCHUNK] (fx, w' W_y W_z, rx, ry) and pr float[XCHUNK] (rz); cnt uint32[N] (counts)
// and st uint32[N + 1] (first particle of each cell).
template <int N, int ASSIGN>
constexpr size_t gather_lds_bytes() {
  return (size_t)XGeom<N, ASSIGN>::CHUNK * (16 + 4) + (size_t)N * 4 + (size_t)(N + 1) * 4;
}

// Exclusive scan of cnt[0, N) into st[0, N] (st[N] = total); cnt[i] = st[i] on exit.
template <int N>
__device__ __forceinline__ void scan_counts(uint32_t* cnt, uint32_t* st) {
  constexpr int NT = XGeom<N, PK_CIC>::NT;
  constexpr int PER = (N + NT - 1) / NT;
  __shared__ uint32_t wsum[NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t v[PER];
  uint32_t loc = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid * PER + j;
    v[j] = idx < N ? cnt[idx] : 0u;
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
  uint32_t ex = inc - loc;
  for (int w = 0; w < wv; ++w) ex += wsum[w];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid * PER + j;
    if (idx < N) {
      st[idx] = ex;
      cnt[idx] = ex;
    }
    ex += v[j];
  }
  if (tid == NT - 1) st[N] = ex;
  __syncthreads();
}

// Adds a chunk particle (pa = (f, w W_y W_z, rx, ry), rz) with stencil offset o along x to
// the NG kept-monomial sums of a target cell: CIC weights (1 - f, f) for o = (0, 1); TSC
// 3/4 - d^2 for o = 0 and (1/2 + o d)^2 / 2 for o = +-1.
template <int NG, int ASSIGN>
__device__ __forceinline__ void add_particle(float (&acc)[NG], const float4 p, const float rz, const int o) {
  add_monomial_sums<NG>(acc, p.y * stencil_weight<ASSIGN>(p.x, o), p.z, p.w, rz);
}

// Gathers the NG kept monomial rows of the block's target row into LDS rows[g][x]
// (rows NG .. 2*NP-1 are zeroed). S*S source rows: particles beg[s] .. beg[s] + len.
template <int N, int ASSIGN, int NG, int NP, int S = (ASSIGN == PK_CIC ? 2 : 3)>
__device__ __forceinline__ void gather_rows(float* lds, const float4* __restrict__ sorted, const uint32_t (&beg)[S * S],
                                            const uint32_t (&pre)[S * S + 1], const XArgs& a) {
  constexpr int O0 = ASSIGN == PK_CIC ? 0 : -1;
  using XG = XGeom<N, ASSIGN>;
  constexpr int NT = XG::NT, XCHUNK = XG::CHUNK, XPER = XG::PER;
  constexpr int CPT = (N + NT - 1) / NT;  // target cells per thread
  char* base = reinterpret_cast<char*>(lds);
  float4* pa = reinterpret_cast<float4*>(base);
  float* pr = reinterpret_cast<float*>(base + XCHUNK * 16);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(base + XCHUNK * 20);
  uint32_t* st = cnt + N;
  const int tid = threadIdx.x;
  // FP32 register sums; the order in which a cell's particles arrive is set by atomics
  // in the sorts, so repeated runs differ at the FP32 rounding level of a cell. Each
  // thread owns target cells and gathers from the S base cells that reach them. (Adding
  // each particle once to the S cells of its stencil, with S sets of sums, was measured
  // slower at every size once the sums fit 64 registers: it costs the second block per CU.)
  float acc[CPT][NG];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[c][g] = 0.0f;
  // index shift from a particle's place in the concatenated source rows to its place in
  // the sorted array, per source row (modulo 2^32, like every particle index here)
  __shared__ uint32_t shift[S * S];
#pragma unroll
  for (int k = 0; k < S * S; ++k)  // constant indices: beg and pre stay in scalar registers
    if (tid == k) shift[k] = beg[k] - pre[k];
  for (int i = tid; i < N; i += NT) cnt[i] = 0u;
  __syncthreads();
  const uint32_t total = pre[S * S];
  for (uint32_t c0 = 0; c0 < total; c0 += XCHUNK) {
    const int n = (int)(total - c0 < (uint32_t)XCHUNK ? total - c0 : (uint32_t)XCHUNK);
    // 1. per-particle values: all of this thread's loads are issued first
    // defined on every path: a value left undefined for the threads past the chunk end
    // can be kept in its register across iterations, which costs registers
    float4 qv[XPER];
#pragma unroll
    for (int j = 0; j < XPER; ++j) qv[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    // source row of each particle: the number of row starts at or before its place f
    // (compares against scalars; selecting the row's start and offset alongside took three
    // selects per row), then its index in the sorted array through the row's shift: all
    // LDS reads first, then all global loads
    int sv[XPER];
    uint32_t gi[XPER];
#pragma unroll
    for (int j = 0; j < XPER; ++j) {
      const uint32_t f = c0 + tid + j * NT;
      int k0 = 0;
#pragma unroll
      for (int k = 1; k < S * S; ++k) k0 += f >= pre[k] ? 1 : 0;
      sv[j] = k0;
      gi[j] = f + shift[k0];
    }
#pragma unroll
    for (int j = 0; j < XPER; ++j)
      if (tid + j * NT < n) qv[j] = sorted[gi[j]];
    // each particle's record stays in registers until its slot in base-cell order is
    // known: its rank inside its cell is the count the atomic returns, its cell's first
    // slot comes from the scan (no unsorted copy, no index permutation)
    float4 rec[XPER];
    float rzv[XPER];
    uint32_t slot[XPER];  // base cell << 16 | rank in the cell
#pragma unroll
    for (int j = 0; j < XPER; ++j) {
      const int i = tid + j * NT;
      rec[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      rzv[j] = 0.0f;
      slot[j] = 0u;
      if (i >= n) continue;
      const float4 q = qv[j];
      const int oy = O0 + sv[j] % S, oz = O0 + sv[j] / S;
      // the source row fixes the base cells along y and z; their offsets set the weights
      const float wyz = q.w * stencil_weight<ASSIGN>(axis_cell<ASSIGN>(q.y, a.bmin[1], a.invH, N).f, oy) *
                        stencil_weight<ASSIGN>(axis_cell<ASSIGN>(q.z, a.bmin[2], a.invH, N).f, oz);
      const AxisCell cx = axis_cell<ASSIGN>(q.x, a.bmin[0], a.invH, N);
      const int ix = cx.i;
      float rx = 0.0f, ry = 0.0f, rz = 1.0f;
      if (a.los == 0) {
        // the sort left out every particle with a zero FP32 line of sight (los_norm2)
        const float dx = q.x - a.obs[0], dy = q.y - a.obs[1], dz = q.z - a.obs[2];
        const float inv = rsqrtf(los_norm2(q.x, q.y, q.z, a.obs[0], a.obs[1], a.obs[2]));
        rx = dx * inv;
        ry = dy * inv;
        rz = dz * inv;
      }
      rec[j] = make_float4(cx.f, wyz, rx, ry);
      rzv[j] = rz;
      slot[j] = ((uint32_t)ix << 16) | atomicAdd(&cnt[ix], 1u);
    }
    __syncthreads();
    // 2. counting sort of the chunk by base cell: starts, then every record to its slot
    scan_counts<N>(cnt, st);
#pragma unroll
    for (int j = 0; j < XPER; ++j) {
      if (tid + j * NT < n) {
        const uint32_t pos = st[slot[j] >> 16] + (slot[j] & 0xffffu);
        pa[pos] = rec[j];
        pr[pos] = rzv[j];
      }
    }
    __syncthreads();
    // 3. gather
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int x = tid + c * NT;
      if (x < N) {
        // Target cell x receives from the base cells x - 1 ... x - O0 (stencil offset
        // o = x - base, 1 down to O0). Their particles are adjacent in the chunk (sorted by
        // base cell), so one loop walks them all and takes o from the cell boundaries:
        // the lanes of a wave then wait for the largest sum of S counts rather than for
        // the largest count S times. The periodic neighbours of x = 0 (cell N - 1) and,
        // for TSC, of x = N - 1 (cell 0) follow in a loop of their own.
        const uint32_t sx = st[x];
        const uint32_t sx1 = st[x + 1];
        const uint32_t kb = st[x > 0 ? x - 1 : 0];
        const uint32_t ke = ASSIGN == PK_CIC ? sx1 : st[x + 2 < N ? x + 2 : N];
        for (uint32_t k = kb; k < ke; ++k) {
          const int o = ASSIGN == PK_CIC ? (int)(k < sx) : (int)(k < sx) - (int)(k >= sx1);
          add_particle<NG, ASSIGN>(acc[c], pa[k], pr[k], o);
        }
        const bool wrap_lo = x == 0, wrap_hi = ASSIGN != PK_CIC && x == N - 1;
        if (wrap_lo || wrap_hi) {
          const uint32_t k1 = wrap_lo ? st[N] : st[1];
          for (uint32_t k = wrap_lo ? st[N - 1] : st[0]; k < k1; ++k)
            add_particle<NG, ASSIGN>(acc[c], pa[k], pr[k], wrap_lo ? 1 : -1);
        }
        cnt[x] = 0u;  // ready for the next chunk (only this thread touches cell x here)
      }
    }
    __syncthreads();
  }
  // rows alias the gather area (all gathers are done: barrier above)
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int x = tid + c * NT;
    if (x < N) {
#pragma unroll
      for (int g = 0; g < NG; ++g) lds[g * N + x] = acc[c][g];
#pragma unroll
      for (int g = NG; g < 2 * NP; ++g) lds[g * N + x] = 0.0f;
    }
  }
  __syncthreads();
}

// LDS slot of index i of one transform: an XOR swizzle inside each block of 16
// that spreads the stride-R writes of the first exchange over the banks.
struct XSwizzle {
  __device__ __forceinline__ int operator()(int i) const { return i ^ ((i >> 4) & 15); }
};

// Planes per band of the x pass's row order (see xpass_kernel).
constexpr int kZBand = 8;

// Waves per SIMD the registers are budgeted for (<= 64 VGPRs at 8): 8 up to N = 1024, i.e.
// 4 blocks of 512 threads per CU (up to 512) or 2 of 1024 threads (at 1024), as the LDS
// of the 15 gathered rows allows (measured 11% faster than 6 at 512, 14-30% than 4 at
// 1024); 4 at 2048, where the rows take 128 KB of LDS (one block per CU), and for the 28
// gathered rows of ell_max = 6.
template <int N, int ELL>
constexpr int xpass_waves() { return (N >= 2048 || ELL >= 6) ? 4 : 8; }

// Bytes before the x pass's LDS twiddle table: the larger of the gather area and the
// 2 NP transformed rows (which alias each other).
template <int N, int ASSIGN, int NP>
constexpr size_t xpass_tw_offset() {
  const size_t rows = (size_t)2 * NP * N * sizeof(float);
  const size_t g = gather_lds_bytes<N, ASSIGN>();
  return ((rows > g ? rows : g) + 15) / 16 * 16;
}

template <int N, int ASSIGN, int ELL>
__global__ __launch_bounds__((XGeom<N, ASSIGN>::NT)) __attribute__((amdgpu_waves_per_eu(xpass_waves<N, ELL>(), 8))) void xpass_kernel(const float4* __restrict__ sorted, const uint32_t* __restrict__ rowoff,
                                                    const float2* __restrict__ tw, float2* __restrict__ X, XArgs a) {
  constexpr int GK = kept_count(ELL);   // gathered, transformed and stored rows
  constexpr int NP = (GK + 1) / 2;
  constexpr int S = ASSIGN == PK_CIC ? 2 : 3;
  constexpr int O0 = ASSIGN == PK_CIC ? 0 : -1;
  using F = Fft<N>;
  static_assert(NP * F::T <= XGeom<N, ASSIGN>::NT, "row pairs do not fit the block");
  // 16-byte aligned: the records are read and written as float4, and the static LDS
  // (scan sums, row shifts) in front of this area need not be a multiple of 16 bytes
  extern __shared__ __align__(16) float lds[];
  const int tid = threadIdx.x;
  // first thread index of this wave, a scalar: the output stage forms its kx from it and
  // the hardware lane count instead of holding tid through the gather and the transform
  // (at N = 1024 with TSC that long-lived register was spilled to scratch, ~8 GB a launch)
  const int wave0 = __builtin_amdgcn_readfirstlane(tid) & ~63;
  // Workgroups go to the 8 XCDs round-robin by linear id; remap so that XCD j takes the
  // rows of the slab's planes [j xs/8, (j+1) xs/8) (xs = gridDim.y) and the source rows
  // that neighbouring target rows share stay in that XCD's L2. Where the planes split into
  // bands of kZBand, the XCD walks each band with y outer and z inner, so the rows of
  // planes z - 1 and z + 1 are still in L2 when plane z needs them (a particle is fetched
  // about once per band rather than once per plane that it reaches); else in plane order.
  const uint32_t lin = blockIdx.x + blockIdx.y * (uint32_t)N;
  const uint32_t xcd_rows = (uint32_t)(N * gridDim.y / 8), l = lin >> 3;
  uint32_t logical = (lin & 7u) * xcd_rows + l;
  if (gridDim.y % (8 * kZBand) == 0) {
    const uint32_t band = l / (uint32_t)(N * kZBand), r = l % (uint32_t)(N * kZBand);
    logical = (lin & 7u) * xcd_rows + (band * kZBand + r % kZBand) * (uint32_t)N + r / kZBand;
  }
  const int y = (int)(logical % N), zs = (int)(logical / N), z = a.z0 + zs;

  // source rows: the particles whose base cell (iy, iz) = (y - oy, z - oz) reach this row
  uint32_t beg[S * S], pre[S * S + 1];
  pre[0] = 0;
#pragma unroll
  for (int s = 0; s < S * S; ++s) {
    const int oy = O0 + s % S, oz = O0 + s / S;
    const int sy = (y - oy) & (N - 1), sz = (z - oz) & (N - 1);
    const int64_t r = (int64_t)sz * N + sy;
    beg[s] = rowoff[r];
    const uint32_t end = rowoff[r + 1];
    // offsets are non-decreasing; the sums are block-uniform and kept in scalar registers
    // (the clamped difference is a vector instruction, which would hold S * S VGPRs)
    pre[s + 1] = __builtin_amdgcn_readfirstlane(pre[s] + (end > beg[s] ? end - beg[s] : 0u));
  }
  // the twiddles of the x transform in LDS (the barriers of the gather make them visible)
  float2* twl = reinterpret_cast<float2*>(reinterpret_cast<char*>(lds) + xpass_tw_offset<N, ASSIGN, NP>());
  for (int i = tid; i < N; i += XGeom<N, ASSIGN>::NT) twl[i] = tw[i];
  gather_rows<N, ASSIGN, GK, NP>(lds, sorted, beg, pre, a);

  // transform along x: rows (2q, 2q+1) as the real and imaginary parts of one row
  const int q = tid / F::T, t = tid % F::T;
  const bool active = q < NP;
  float2* T = reinterpret_cast<float2*>(lds);  // pair q uses T[q N, (q + 1) N), its two rows
  float2 d[F::E];  // zero for the inactive threads (defined on every path)
#pragma unroll
  for (int e = 0; e < F::E; ++e) d[e] = make_float2(0.0f, 0.0f);
  if (active) {
    const float* r0 = lds + 2 * q * N;
    const float* r1 = r0 + N;
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
      const int x = F::in_index(t, e);
      d[e] = make_float2(r0[x], r1[x]);
    }
  }
  float2* Tq = T + (active ? q * N : 0);
  F::run(d, t, twl, Tq, XSwizzle(), active);
  __syncthreads();
  if (active) {
#pragma unroll
    for (int e = 0; e < F::E; ++e) Tq[XSwizzle()(F::out_index(t, e))] = d[e];
  }
  __syncthreads();
  // Thread kx < Kx (Kx <= N / 2 <= block size) unpacks each gathered spectrum at kx and
  // stores it at its gathered index. Rows (2q, 2q+1) were transformed as one complex row
  // Z, so X_2q[k] = (Z[k] + conj Z[N-k]) / 2 and X_2q+1[k] = -i (Z[k] - conj Z[N-k]) / 2.
  const int Kx = a.Kx;
  const int kx = wave0 + (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  if (kx < Kx) {
    // tile-major X: [plane][kx / TW][y][kx % TW], so that a y-pass block reads its columns
    // of a plane as one contiguous run (with rows of Kx values it read 64-byte pieces
    // 2-4 KB apart: y pass 29.9 -> 27.0 ms at 1024^3 for +0.8 ms here, the same at 512^3)
    constexpr int TW = tile_cols<N>();
    const size_t o = (size_t)(a.pbase + zs) * N * (size_t)Kx + (size_t)(kx / TW) * (TW * N) + TW * y + (kx % TW);
    const int ik = XSwizzle()(kx), im = XSwizzle()((N - kx) & (N - 1));
    // the grid stride is opaque here: otherwise the compiler forms all GK products with
    // it up front and holds them in (spilled) scalar registers through the kernel
    int64_t gs = a.grid_stride;
    asm volatile("" : "+s"(gs));
#pragma unroll
    for (int qq = 0; qq < NP; ++qq) {
      const float2 zk = T[qq * N + ik], zm = T[qq * N + im];
      X[(size_t)(2 * qq) * gs + o] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      if (2 * qq + 1 < GK) X[(size_t)(2 * qq + 1) * gs + o] = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
    }
  }
}

template <int N, int ASSIGN, int ELL>
static hipError_t launch_x3(const Plan& p, char* ws, const XArgs& a, hipStream_t s) {
  constexpr int NP = (kept_count(ELL) + 1) / 2;
  const size_t rows = (size_t)2 * NP * N * sizeof(float);
  (void)rows;
  const size_t shmem = xpass_tw_offset<N, ASSIGN, NP>() + (size_t)N * sizeof(float2);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&xpass_kernel<N, ASSIGN, ELL>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  hipLaunchKernelGGL((xpass_kernel<N, ASSIGN, ELL>), dim3(N, p.xs), dim3(XGeom<N, ASSIGN>::NT), shmem, s,
                     at<const float4>(ws, p.off_sorted), at<const uint32_t>(ws, p.off_rowoff),
                     at<const float2>(ws, p.off_tw), at<float2>(ws, p.off_X), a);
  return hipGetLastError();
}

template <int N, int ASSIGN>
static hipError_t launch_x2(const Plan& p, char* ws, const XArgs& a, hipStream_t s) {
  switch (p.ell_max) {
    case 0: return launch_x3<N, ASSIGN, 0>(p, ws, a, s);
    case 2: return launch_x3<N, ASSIGN, 2>(p, ws, a, s);
    case 6:   // 14 row pairs of 2048 cells would need 1792 threads: built up to N = 1024
      if constexpr (N <= 1024) return launch_x3<N, ASSIGN, 6>(p, ws, a, s);
      else return hipErrorInvalidValue;
    default: return launch_x3<N, ASSIGN, 4>(p, ws, a, s);
  }
}

template <int N>
static hipError_t launch_x1(const Plan& p, char* ws, const XArgs& a, hipStream_t s) {
  return p.assign == PK_CIC ? launch_x2<N, PK_CIC>(p, ws, a, s) : launch_x2<N, PK_TSC>(p, ws, a, s);
}

hipError_t launch_xpass(const Plan& p, char* ws, hipStream_t s, int z0, int pbase) {
  XArgs a;
  for (int i = 0; i < 3; ++i) {
    a.bmin[i] = p.box_min[i];
    a.obs[i] = (float)p.observer[i];
  }
  a.invH = (double)p.N / p.L;
  a.los = p.los;
  a.Kx = p.Kx;
  a.z0 = z0;
  a.pbase = pbase;
  a.grid_stride = (int64_t)p.xr * p.xs * p.N * p.Kx;
  switch (p.N) {
    case 8: return launch_x1<8>(p, ws, a, s);
    case 16: return launch_x1<16>(p, ws, a, s);
    case 32: return launch_x1<32>(p, ws, a, s);
    case 64: return launch_x1<64>(p, ws, a, s);
    case 128: return launch_x1<128>(p, ws, a, s);
    case 256: return launch_x1<256>(p, ws, a, s);
    case 512: return launch_x1<512>(p, ws, a, s);
    case 1024: return launch_x1<1024>(p, ws, a, s);
    case 2048: return launch_x1<2048>(p, ws, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pk
