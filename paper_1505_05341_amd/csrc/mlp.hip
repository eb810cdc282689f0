// Coarse-grid correction network: a multilayer perceptron with 3 hidden layers of width
// 128 and SiLU activations, trained and evaluated with hand-written BF16 MFMA kernels
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), FP32 master weights and Adam.
//
// Layers: z_l = h_{l-1} W_l + b_l (W_l stored [in, out]), h_l = silu(z_l), y = h_3 W_4 + b_4.
// Padded widths: the input to KPAD and the output to 32 (multiples of the MFMA depth).
// Every GEMM is one of three shapes:
//   forward   Z[M, N]   = H[M, K] W[K, N]          (A = H rows, B = W^T rows)
//   backward  dH[M, K]  = dZ[M, N] W[K, N]^T        (A = dZ rows, B = W rows)
//   gradient  dW[K, N] = sum_m H[m, K]^T dZ[m, N]   (per-block partials, fixed-order sum)
//
// MFMA 16x16x32 operand layout (lane l): A[i][k] with i = l % 16, k = 8 (l / 16) + j;
// B[k][n] with n = l % 16, k = 8 (l / 16) + j (j = 0..7); D[i][n] with n = l % 16,
// i = 4 (l / 16) + r (r = 0..3).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "pk.h"

namespace pk {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kWidth = 128;
constexpr int kLayers = 4;       // 3 hidden + output
constexpr int kOutPad = 32;   // output width padded to the MFMA depth
constexpr int kRowsPerBlock = 64;  // 4 waves x 16 rows
constexpr int kGradRows = 256;     // rows per weight-gradient partial

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

// ---------------------------------------------------------------------------------
// Row GEMM: C[M, N] = A[M, K] * B'[N, K]^T, A and B' row-major BF16 (B' = the right
// operand stored by its columns). One wave: 16 rows x N columns.
// EPI 0: forward hidden  (z = c + bias -> Zout fp32, Hout = bf16(silu(z)))
// EPI 1: forward output  (y = c + bias -> Zout fp32)
// EPI 2: backward hidden (dh = c; dz = dh silu'(Zin) -> Zout fp32, Hout bf16(dz))
// ---------------------------------------------------------------------------------
template <int K, int N, int EPI>
__global__ __launch_bounds__(256) void mlp_rows_kernel(const uint16_t* __restrict__ A, const uint16_t* __restrict__ Bt,
                                                       const float* __restrict__ bias, const float* __restrict__ Zin,
                                                       float* __restrict__ Zout, uint16_t* __restrict__ Hout, int64_t M) {
  constexpr int NT = N / 16;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock + wv * 16;
  const int li = lane & 15, lg = lane >> 4;
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t arow = r0 + li < M ? r0 + li : M - 1;  // clamp reads of the ragged tail
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    const bf16x8 a = load8(A + arow * K + k0 + 8 * lg);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bf16x8 b = load8(Bt + (int64_t)(16 * t + li) * K + k0 + 8 * lg);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int n = 16 * t + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + 4 * lg + r;
      if (row >= M) continue;
      const float c = acc[t][r];
      const int64_t o = row * N + n;
      if (EPI == 0) {
        const float z = c + bias[n];
        Zout[o] = z;
        Hout[o] = f2bf(silu(z));
      } else if (EPI == 1) {
        Zout[o] = c + bias[n];
      } else {
        const float dz = c * silu_grad(Zin[o]);
        Zout[o] = dz;
        Hout[o] = f2bf(dz);
      }
    }
  }
}

// Weight gradient partial: P[blk][K][N] = sum over rows of the block's chunk of
// H[m][k] dZ[m][n]; both chunks go through LDS (64 rows at a time). Block: 4 waves;
// wave w owns output row tiles w, w+4, ... of the K x N result.
template <int K, int N>
__global__ __launch_bounds__(256) void mlp_wgrad_kernel(const uint16_t* __restrict__ H, const uint16_t* __restrict__ dZ,
                                                        float* __restrict__ part, int64_t M) {
  constexpr int KT = K / 16, NT = N / 16, TPW = (KT * NT + 3) / 4;
  constexpr int CH = 64;
  __shared__ uint16_t sh[CH][K + 8];
  __shared__ uint16_t sd[CH][N + 8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  f32x4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t m0 = (int64_t)blockIdx.x * kGradRows;
  for (int c0 = 0; c0 < kGradRows; c0 += CH) {
    __syncthreads();
    for (int e = threadIdx.x; e < CH * K; e += 256) {
      const int r = e / K, k = e % K;
      const int64_t m = m0 + c0 + r;
      sh[r][k] = m < M ? H[m * K + k] : (uint16_t)0;
    }
    for (int e = threadIdx.x; e < CH * N; e += 256) {
      const int r = e / N, n = e % N;
      const int64_t m = m0 + c0 + r;
      sd[r][n] = m < M ? dZ[m * N + n] : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < CH; s += 32) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tile = wv + 4 * t;
        if (tile >= KT * NT) continue;
        const int kt = tile / NT, nt = tile % NT;
        uint16_t av[8], bv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          av[j] = sh[s + 8 * lg + j][16 * kt + li];   // A[i = k index][depth = row]
          bv[j] = sd[s + 8 * lg + j][16 * nt + li];   // B[depth = row][n]
        }
        bf16x8 a, b;
        __builtin_memcpy(&a, av, 16);
        __builtin_memcpy(&b, bv, 16);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
      }
    }
  }
  float* out = part + (size_t)blockIdx.x * K * N;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wv + 4 * t;
    if (tile >= KT * NT) continue;
    const int kt = tile / NT, nt = tile % NT;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(16 * kt + 4 * lg + r) * N + 16 * nt + li] = acc[t][r];
  }
}

// Fixed-order sum of the gradient partials; bias gradients are column sums of the FP32
// dZ, also in a fixed order.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* part, int nblk, int KN, float* g) {
  // g may alias part (block 0): each thread reads all partials of index i before writing g[i]
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KN) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * KN + i];
  g[i] = s;
}

__global__ __launch_bounds__(256) void mlp_colsum_kernel(const float* __restrict__ dz, int64_t M, int N,
                                                         float* __restrict__ g) {
  // one block per column; fixed strided order, then a fixed tree
  __shared__ float red[256];
  const int n = blockIdx.x;
  float s = 0.0f;
  for (int64_t m = threadIdx.x; m < M; m += 256) s += dz[m * N + n];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[n] = red[0];
}

// Packs the FP32 input rows (din columns) into BF16 rows of KPAD columns.
__global__ __launch_bounds__(256) void mlp_pack_kernel(const float* __restrict__ x, int64_t M, int din, int kpad,
                                                       uint16_t* __restrict__ xb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * kpad) return;
  const int64_t m = i / kpad;
  const int k = (int)(i % kpad);
  xb[i] = k < din ? f2bf(x[m * din + k]) : (uint16_t)0;
}

// Output: y[m][j] = Y[m][j] for j < dout; loss partial and dY = 2 (y - t) / (M dout)
// as FP32 and BF16 (padded columns get 0).
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                       int64_t M, int dout, float* __restrict__ dY,
                                                       uint16_t* __restrict__ dYb, double* __restrict__ lpart) {
  __shared__ double red[256];
  double s = 0.0;
  const float scale = 2.0f / (float)((double)M * dout);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M * kOutPad;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i / kOutPad;
    const int j = (int)(i % kOutPad);
    float d = 0.0f;
    if (j < dout) {
      d = Y[i] - T[m * dout + j];
      s += (double)d * d;
    }
    dY[i] = d * scale;
    dYb[i] = f2bf(d * scale);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ void mlp_loss_final_kernel(const double* lpart, int nblk, int64_t count, float* loss) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += lpart[b];
  *loss = (float)(s / (double)count);
}

// Adam on every FP32 master parameter, then the BF16 copies W (row-major [in, out])
// and W^T ([out, in]) of each padded layer.
struct MlpDims {
  int din, dout, kpad;
  int in[kLayers], out[kLayers], pin[kLayers], pout[kLayers];
  int64_t woff[kLayers], boff[kLayers];      // offsets in the master arrays (floats)
  int64_t bfoff[kLayers];                     // offsets of the padded BF16 copies (elements)
  int64_t nparams;
  int64_t nbf;
};

__global__ __launch_bounds__(256) void mlp_zero_kernel(float* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ w, float* __restrict__ m,
                                                       float* __restrict__ v, const float* __restrict__ g, int64_t n,
                                                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void mlp_bf16_copies_kernel(const float* __restrict__ w, MlpDims d,
                                                              uint16_t* __restrict__ wb, uint16_t* __restrict__ wtb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.nbf) return;
  int l = 0;
  while (l + 1 < kLayers && i >= d.bfoff[l + 1]) ++l;
  const int64_t e = i - d.bfoff[l];
  const int r = (int)(e / d.pout[l]), c = (int)(e % d.pout[l]);   // padded [pin, pout]
  const float val = (r < d.in[l] && c < d.out[l]) ? w[d.woff[l] + (int64_t)r * d.out[l] + c] : 0.0f;
  wb[i] = f2bf(val);
  wtb[d.bfoff[l] + (int64_t)c * d.pin[l] + r] = f2bf(val);
}

// --------------------------------------------------------------------------- host side

struct MlpPlan {
  MlpDims d;
  // state (bytes): master w, m, v (nparams floats each), padded biases (4 x 128 floats), wb, wtb
  size_t st_w, st_m, st_v, st_bias, st_wb, st_wtb, st_total;
  // workspace (bytes) for M rows
  size_t ws_xb, ws_z[kLayers], ws_h[kLayers], ws_dz, ws_dzb, ws_dh, ws_dhb, ws_part, ws_grad, ws_lpart, ws_total;
  int64_t M;
  int grad_blocks;
};

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

static bool mlp_plan(const pk_mlp_shape* s, int64_t M, MlpPlan* P) {
  if (!s || s->din < 1 || s->din > 64 || s->dout < 1 || s->dout > 16 || s->width != kWidth || s->depth != 3 ||
      M < 0)
    return false;
  MlpDims& d = P->d;
  memset(&d, 0, sizeof(d));
  d.din = s->din;
  d.dout = s->dout;
  d.kpad = (s->din + 31) / 32 * 32;
  const int dims[5] = {s->din, kWidth, kWidth, kWidth, s->dout};
  const int pdims[5] = {d.kpad, kWidth, kWidth, kWidth, kOutPad};
  int64_t off = 0, bf = 0;
  for (int l = 0; l < kLayers; ++l) {
    d.in[l] = dims[l];
    d.out[l] = dims[l + 1];
    d.pin[l] = pdims[l];
    d.pout[l] = pdims[l + 1];
    d.woff[l] = off;
    off += (int64_t)dims[l] * dims[l + 1];
    d.boff[l] = off;
    off += dims[l + 1];
    d.bfoff[l] = bf;
    bf += (int64_t)pdims[l] * pdims[l + 1];
  }
  d.nparams = off;
  d.nbf = bf;
  size_t o = 0;
  auto take = [&](size_t b) { const size_t r = o; o = al256(o + b); return r; };
  P->st_w = take(4 * off);
  P->st_m = take(4 * off);
  P->st_v = take(4 * off);
  P->st_bias = take(4 * kLayers * kWidth);
  P->st_wb = take(2 * bf);
  P->st_wtb = take(2 * bf);
  P->st_total = o;
  P->M = M;
  const int64_t Mr = (M + kRowsPerBlock - 1) / kRowsPerBlock * kRowsPerBlock;
  o = 0;
  P->ws_xb = take(2 * Mr * d.kpad);
  for (int l = 0; l < kLayers; ++l) {
    P->ws_z[l] = take(4 * Mr * pdims[l + 1]);
    P->ws_h[l] = take(2 * Mr * pdims[l + 1]);
  }
  P->ws_dz = take(4 * Mr * kWidth);
  P->ws_dzb = take(2 * Mr * kWidth);
  P->ws_dh = take(4 * Mr * kWidth);
  P->ws_dhb = take(2 * Mr * kWidth);
  P->grad_blocks = (int)((M + kGradRows - 1) / kGradRows);
  if (P->grad_blocks < 1) P->grad_blocks = 1;
  P->ws_part = take(4 * (size_t)P->grad_blocks * kWidth * kWidth);
  P->ws_grad = take(4 * off);
  P->ws_lpart = take(8 * 1024);
  P->ws_total = o;
  return true;
}

template <class T>
static T* ptr(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

// Biases padded to 128 floats per layer (the GEMM epilogues read bias[n] for n < pout).
__global__ void mlp_pad_bias_kernel(const float* __restrict__ w, MlpDims d, float* __restrict__ pb) {
  const int l = blockIdx.x, n = threadIdx.x;
  if (l < kLayers && n < kWidth) pb[l * kWidth + n] = n < d.out[l] ? w[d.boff[l] + n] : 0.0f;
}

static hipError_t refresh_copies(const MlpPlan& P, void* state, hipStream_t s) {
  const int64_t nbf = P.d.nbf;
  hipLaunchKernelGGL(mlp_bf16_copies_kernel, dim3((unsigned)((nbf + 255) / 256)), dim3(256), 0, s,
                     ptr<const float>(state, P.st_w), P.d, ptr<uint16_t>(state, P.st_wb), ptr<uint16_t>(state, P.st_wtb));
  hipLaunchKernelGGL(mlp_pad_bias_kernel, dim3(kLayers), dim3(kWidth), 0, s, ptr<const float>(state, P.st_w), P.d,
                     ptr<float>(state, P.st_bias));
  return hipGetLastError();
}

static void launch_rows(int K, int N, int epi, const uint16_t* A, const uint16_t* Bt, const float* bias,
                        const float* Zin, float* Zout, uint16_t* Hout, int64_t M, hipStream_t s) {
  const dim3 grid((unsigned)((M + kRowsPerBlock - 1) / kRowsPerBlock)), blk(256);
#define PK_ROWS(KK, NN, EE)                                                                                    \
  if (K == KK && N == NN && epi == EE) {                                                                       \
    hipLaunchKernelGGL((mlp_rows_kernel<KK, NN, EE>), grid, blk, 0, s, A, Bt, bias, Zin, Zout, Hout, M);       \
    return;                                                                                                    \
  }
  PK_ROWS(32, 128, 0) PK_ROWS(64, 128, 0) PK_ROWS(128, 128, 0) PK_ROWS(128, 32, 1)
  PK_ROWS(128, 128, 2) PK_ROWS(32, 128, 2)
#undef PK_ROWS
}

static void launch_wgrad(int K, int N, const uint16_t* H, const uint16_t* dZ, float* part, int64_t M, int nblk,
                         hipStream_t s) {
#define PK_WG(KK, NN)                                                                                           \
  if (K == KK && N == NN) {                                                                                     \
    hipLaunchKernelGGL((mlp_wgrad_kernel<KK, NN>), dim3(nblk), dim3(256), 0, s, H, dZ, part, M);               \
    return;                                                                                                     \
  }
  PK_WG(32, 128) PK_WG(64, 128) PK_WG(128, 128) PK_WG(128, 32)
#undef PK_WG
}

// Forward pass over M rows; Z and H of every layer stay in the workspace.
static void forward(const MlpPlan& P, void* state, const float* x, void* ws, hipStream_t s) {
  const MlpDims& d = P.d;
  const int64_t M = P.M;
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((unsigned)((M * d.kpad + 255) / 256)), dim3(256), 0, s, x, M, d.din, d.kpad,
                     ptr<uint16_t>(ws, P.ws_xb));
  const uint16_t* hin = ptr<const uint16_t>(ws, P.ws_xb);
  for (int l = 0; l < kLayers; ++l) {
    const bool last = l == kLayers - 1;
    launch_rows(d.pin[l], d.pout[l], last ? 1 : 0, hin, ptr<const uint16_t>(state, P.st_wtb) + d.bfoff[l],
                ptr<const float>(state, P.st_bias) + l * kWidth, nullptr, ptr<float>(ws, P.ws_z[l]),
                ptr<uint16_t>(ws, P.ws_h[l]), M, s);
    hin = ptr<const uint16_t>(ws, P.ws_h[l]);
  }
}

// Backward pass from the output rows; gradients land in ws_grad (master layout).
static void backward(const MlpPlan& P, void* state, const float* t, float* loss, void* ws, hipStream_t s) {
  const MlpDims& d = P.d;
  const int64_t M = P.M;
  const int lb = 256;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(lb), dim3(256), 0, s, ptr<const float>(ws, P.ws_z[kLayers - 1]), t, M,
                     d.dout, ptr<float>(ws, P.ws_dz), ptr<uint16_t>(ws, P.ws_dzb), ptr<double>(ws, P.ws_lpart));
  hipLaunchKernelGGL(mlp_loss_final_kernel, dim3(1), dim3(64), 0, s, ptr<const double>(ws, P.ws_lpart), lb,
                     (int64_t)(M * d.dout), loss);
  float* grad = ptr<float>(ws, P.ws_grad);
  // dz of the current layer: FP32 at ws_dz (for the bias), BF16 at ws_dzb (for the GEMMs)
  for (int l = kLayers - 1; l >= 0; --l) {
    const uint16_t* hprev = l == 0 ? ptr<const uint16_t>(ws, P.ws_xb) : ptr<const uint16_t>(ws, P.ws_h[l - 1]);
    const int K = d.pin[l], N = d.pout[l];
    const float* dzf = ptr<const float>(ws, (l % 2 == (kLayers - 1) % 2) ? P.ws_dz : P.ws_dh);
    const uint16_t* dzb = ptr<const uint16_t>(ws, (l % 2 == (kLayers - 1) % 2) ? P.ws_dzb : P.ws_dhb);
    launch_wgrad(K, N, hprev, dzb, ptr<float>(ws, P.ws_part), M, P.grad_blocks, s);
    // reduce the padded [K, N] partials, then keep the real [in, out] block
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((K * N + 255) / 256), dim3(256), 0, s, ptr<const float>(ws, P.ws_part),
                       P.grad_blocks, K * N, ptr<float>(ws, P.ws_part));
    (void)hipMemcpy2DAsync(grad + d.woff[l], sizeof(float) * d.out[l], ptr<float>(ws, P.ws_part), sizeof(float) * N,
                           sizeof(float) * d.out[l], d.in[l], hipMemcpyDeviceToDevice, s);
    hipLaunchKernelGGL(mlp_colsum_kernel, dim3(d.out[l]), dim3(256), 0, s, dzf, M, N, grad + d.boff[l]);
    if (l > 0) {
      // dh_{l-1} = dz_l W_l^T, then dz_{l-1} = dh_{l-1} silu'(z_{l-1}); W_l rows are B' rows
      const size_t tgt_f = (l % 2 == (kLayers - 1) % 2) ? P.ws_dh : P.ws_dz;
      const size_t tgt_b = (l % 2 == (kLayers - 1) % 2) ? P.ws_dhb : P.ws_dzb;
      launch_rows(N, K, 2, dzb, ptr<const uint16_t>(state, P.st_wb) + d.bfoff[l], nullptr,
                  ptr<const float>(ws, P.ws_z[l - 1]), ptr<float>(ws, tgt_f), ptr<uint16_t>(ws, tgt_b), M, s);
    }
  }
}

// One Adam step (b1 0.9, b2 0.999, eps 1e-8, bias corrections 1 - b^step) of the FP32
// master weights with the gradient vector g (canonical order), then fresh BF16 copies.
static hipError_t adam(const MlpPlan& P, void* state, const float* g, float lr, int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  const int64_t n = P.d.nparams;
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ptr<float>(state, P.st_w),
                     ptr<float>(state, P.st_m), ptr<float>(state, P.st_v), g, n, lr, b1, b2, 1e-8f, c1, c2);
  const hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : refresh_copies(P, state, s);
}

}  // namespace pk

using namespace pk;

extern "C" {

size_t pk_mlp_state_bytes(const pk_mlp_shape* shape) {
  MlpPlan P;
  return mlp_plan(shape, 0, &P) ? P.st_total : 0;
}

size_t pk_mlp_workspace_bytes(const pk_mlp_shape* shape, int64_t rows) {
  MlpPlan P;
  return mlp_plan(shape, rows, &P) ? P.ws_total : 0;
}

int64_t pk_mlp_num_params(const pk_mlp_shape* shape) {
  MlpPlan P;
  return mlp_plan(shape, 0, &P) ? P.d.nparams : -1;
}

pk_status pk_mlp_set_params(const pk_mlp_shape* shape, void* state, const float* d_params, void* hip_stream) {
  MlpPlan P;
  if (!mlp_plan(shape, 0, &P) || !state || !d_params) return PK_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t nb = sizeof(float) * P.d.nparams;
  hipError_t e = hipMemcpyAsync(ptr<float>(state, P.st_w), d_params, nb, hipMemcpyDeviceToDevice, s);
  const unsigned g = (unsigned)((P.d.nparams + 255) / 256);
  if (e == hipSuccess) hipLaunchKernelGGL(mlp_zero_kernel, dim3(g), dim3(256), 0, s, ptr<float>(state, P.st_m), P.d.nparams);
  if (e == hipSuccess) hipLaunchKernelGGL(mlp_zero_kernel, dim3(g), dim3(256), 0, s, ptr<float>(state, P.st_v), P.d.nparams);
  if (e == hipSuccess) e = refresh_copies(P, state, s);
  return e == hipSuccess ? PK_OK : PK_EDEVICE;
}

pk_status pk_mlp_get_params(const pk_mlp_shape* shape, const void* state, float* d_params, void* hip_stream) {
  MlpPlan P;
  if (!mlp_plan(shape, 0, &P) || !state || !d_params) return PK_EINVAL;
  const hipError_t e = hipMemcpyAsync(d_params, ptr<const float>(const_cast<void*>(state), P.st_w),
                                      sizeof(float) * P.d.nparams, hipMemcpyDeviceToDevice, (hipStream_t)hip_stream);
  return e == hipSuccess ? PK_OK : PK_EDEVICE;
}

pk_status pk_mlp_forward(const pk_mlp_shape* shape, const void* state, const float* d_x, int64_t rows, float* d_y,
                         void* workspace, size_t workspace_bytes, void* hip_stream) {
  MlpPlan P;
  if (!mlp_plan(shape, rows, &P) || !state || (rows > 0 && (!d_x || !d_y))) return PK_EINVAL;
  if (!workspace || workspace_bytes < P.ws_total) return PK_EWORKSPACE;
  if (rows == 0) return PK_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  forward(P, const_cast<void*>(state), d_x, workspace, s);
  const hipError_t e = hipMemcpy2DAsync(d_y, sizeof(float) * P.d.dout, ptr<float>(workspace, P.ws_z[kLayers - 1]),
                                        sizeof(float) * kOutPad, sizeof(float) * P.d.dout, rows,
                                        hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return PK_EDEVICE;
  return hipGetLastError() == hipSuccess ? PK_OK : PK_EDEVICE;
}

pk_status pk_mlp_gradients(const pk_mlp_shape* shape, const void* state, const float* d_x, const float* d_t,
                           int64_t rows, float* d_grads, float* d_loss, void* workspace, size_t workspace_bytes,
                           void* hip_stream) {
  MlpPlan P;
  if (!mlp_plan(shape, rows, &P) || rows < 1 || !state || !d_x || !d_t || !d_loss) return PK_EINVAL;
  if (!workspace || workspace_bytes < P.ws_total) return PK_EWORKSPACE;
  hipStream_t s = (hipStream_t)hip_stream;
  forward(P, const_cast<void*>(state), d_x, workspace, s);
  backward(P, const_cast<void*>(state), d_t, d_loss, workspace, s);
  if (d_grads &&
      hipMemcpyAsync(d_grads, ptr<float>(workspace, P.ws_grad), sizeof(float) * P.d.nparams, hipMemcpyDeviceToDevice,
                     s) != hipSuccess)
    return PK_EDEVICE;
  return hipGetLastError() == hipSuccess ? PK_OK : PK_EDEVICE;
}

pk_status pk_mlp_train_step(const pk_mlp_shape* shape, void* state, const float* d_x, const float* d_t, int64_t rows,
                            float lr, int32_t step, float* d_loss, void* workspace, size_t workspace_bytes,
                            void* hip_stream) {
  MlpPlan P;
  if (!mlp_plan(shape, rows, &P) || rows < 1 || !state || !d_x || !d_t || !d_loss || step < 1) return PK_EINVAL;
  if (!workspace || workspace_bytes < P.ws_total) return PK_EWORKSPACE;
  hipStream_t s = (hipStream_t)hip_stream;
  forward(P, state, d_x, workspace, s);
  backward(P, state, d_t, d_loss, workspace, s);
  if (adam(P, state, ptr<const float>(workspace, P.ws_grad), lr, step, s) != hipSuccess) return PK_EDEVICE;
  return hipGetLastError() == hipSuccess ? PK_OK : PK_EDEVICE;
}

pk_status pk_mlp_adam_apply(const pk_mlp_shape* shape, void* state, const float* d_grads, float lr, int32_t step,
                            void* hip_stream) {
  MlpPlan P;
  if (!mlp_plan(shape, 0, &P) || !state || !d_grads || step < 1) return PK_EINVAL;
  if (adam(P, state, d_grads, lr, step, (hipStream_t)hip_stream) != hipSuccess) return PK_EDEVICE;
  return hipGetLastError() == hipSuccess ? PK_OK : PK_EDEVICE;
}

}  // extern "C"
