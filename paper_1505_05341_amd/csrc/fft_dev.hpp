// Device building blocks of the batched FFTs: complex helpers, in-register DFTs of
// size <= 16 and a multi-stage Stockham transform of length N <= 2048 along one axis.
//
// Stockham (self-sorting) formulation: with radices R_0, R_1, ... (product N) and
// Ns = R_0 ... R_{s-1} before stage s, butterfly j (0 <= j < N/R_s) of stage s reads
// D[j + r N/R_s] (r < R_s), multiplies value r by w_{Ns R_s}^{(j mod Ns) r}
// (w_M = exp(-2 pi i / M)), takes the R_s-point DFT, and writes value r to
// D'[(j div Ns) Ns R_s + (j mod Ns) + r Ns]. After the last stage D' holds the DFT in
// natural order. T = N / E threads cooperate on one transform and each holds E values
// in registers (E = the largest radix, so E / R_s butterflies per thread per stage);
// the data cross LDS between stages.
#pragma once
#include <hip/hip_runtime.h>
#include "dft_consts.h"

namespace pk {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// v * exp(-2 pi i k / R) with R | 32 and k a compile-time constant after unrolling.
template <int R>
__device__ __forceinline__ float2 rot(float2 v, int k) {
  const int idx = (k * (32 / R)) & 31;
  if (idx == 0) return v;
  if (idx == 8) return make_float2(v.y, -v.x);
  if (idx == 16) return make_float2(-v.x, -v.y);
  if (idx == 24) return make_float2(-v.y, v.x);
  const float c = kCos32[idx], s = -kSin32[idx];
  return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
}

// In-place DFT of R register values, natural order in and out (radix-2, decimation in time).
template <int R>
struct Dft {
  __device__ __forceinline__ static void run(float2* x) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    Dft<R / 2>::run(e);
    Dft<R / 2>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const float2 t = rot<R>(o[k], k);
      x[k] = cadd(e[k], t);
      x[k + R / 2] = csub(e[k], t);
    }
  }
};
template <>
struct Dft<1> {
  __device__ __forceinline__ static void run(float2*) {}
};
template <>
struct Dft<2> {
  __device__ __forceinline__ static void run(float2* x) {
    const float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

// Radices of each supported length (largest first, so E = radix(0)), for at most EMAX
// values per thread: 16 (fewer, larger stages; fewer threads per transform) or 8 (half
// the registers per thread, twice the threads).
template <int N, int EMAX> struct Radices;
template <> struct Radices<8, 16>    { static constexpr int NS = 2, R0 = 4,  R1 = 2,  R2 = 1, R3 = 1; };
template <> struct Radices<16, 16>   { static constexpr int NS = 2, R0 = 4,  R1 = 4,  R2 = 1, R3 = 1; };
template <> struct Radices<32, 16>   { static constexpr int NS = 2, R0 = 8,  R1 = 4,  R2 = 1, R3 = 1; };
template <> struct Radices<64, 16>   { static constexpr int NS = 2, R0 = 8,  R1 = 8,  R2 = 1, R3 = 1; };
template <> struct Radices<128, 16>  { static constexpr int NS = 2, R0 = 16, R1 = 8,  R2 = 1, R3 = 1; };
template <> struct Radices<256, 16>  { static constexpr int NS = 2, R0 = 16, R1 = 16, R2 = 1, R3 = 1; };
template <> struct Radices<512, 16>  { static constexpr int NS = 3, R0 = 16, R1 = 8,  R2 = 4, R3 = 1; };
template <> struct Radices<1024, 16> { static constexpr int NS = 3, R0 = 16, R1 = 16, R2 = 4, R3 = 1; };
template <> struct Radices<2048, 16> { static constexpr int NS = 3, R0 = 16, R1 = 16, R2 = 8, R3 = 1; };
template <> struct Radices<8, 8>     { static constexpr int NS = 2, R0 = 4,  R1 = 2,  R2 = 1, R3 = 1; };
template <> struct Radices<16, 8>    { static constexpr int NS = 2, R0 = 4,  R1 = 4,  R2 = 1, R3 = 1; };
template <> struct Radices<32, 8>    { static constexpr int NS = 2, R0 = 8,  R1 = 4,  R2 = 1, R3 = 1; };
template <> struct Radices<64, 8>    { static constexpr int NS = 2, R0 = 8,  R1 = 8,  R2 = 1, R3 = 1; };
template <> struct Radices<128, 8>   { static constexpr int NS = 3, R0 = 8,  R1 = 8,  R2 = 2, R3 = 1; };
template <> struct Radices<256, 8>   { static constexpr int NS = 3, R0 = 8,  R1 = 8,  R2 = 4, R3 = 1; };
template <> struct Radices<512, 8>   { static constexpr int NS = 3, R0 = 8,  R1 = 8,  R2 = 8, R3 = 1; };
template <> struct Radices<1024, 8>  { static constexpr int NS = 4, R0 = 8,  R1 = 8,  R2 = 8, R3 = 2; };
template <> struct Radices<2048, 8>  { static constexpr int NS = 4, R0 = 8,  R1 = 8,  R2 = 8, R3 = 4; };

template <int N, int EMAX = 16>
struct Fft {
  using Rd = Radices<N, EMAX>;
  static constexpr int NS = Rd::NS;
  static constexpr int E = Rd::R0;   // values per thread
  static constexpr int T = N / E;    // threads per transform
  static constexpr int radix(int s) { return s == 0 ? Rd::R0 : (s == 1 ? Rd::R1 : (s == 2 ? Rd::R2 : Rd::R3)); }
  static constexpr int span(int s) { return s == 0 ? 1 : radix(s - 1) * span(s - 1); }  // Ns
  static constexpr int RL = radix(NS - 1);

  // Index read by value (q, r) of thread t at stage s.
  template <int S>
  __device__ __forceinline__ static int src_index(int t, int q, int r) {
    return t + T * q + r * (N / radix(S));
  }
  // Index written by value (q, r) of thread t after stage s.
  template <int S>
  __device__ __forceinline__ static int dst_index(int t, int q, int r) {
    constexpr int R = radix(S), Ns = span(S);
    const int j = t + T * q;
    return (j / Ns) * Ns * R + (j % Ns) + r * Ns;
  }
  // Natural index of output value e = q * RL + r after the last stage.
  __device__ __forceinline__ static int out_index(int t, int e) {
    const int q = e / RL, r = e % RL;
    return t + T * q + r * (N / RL);
  }
  // Natural index of input value e (the first stage has one butterfly per thread).
  __device__ __forceinline__ static int in_index(int t, int e) { return t + T * e; }

  // Twiddles and DFTs of stage S on the E register values of thread t.
  template <int S>
  __device__ __forceinline__ static void stage(float2 (&d)[E], int t, const float2* __restrict__ tw) {
    constexpr int R = radix(S), Ns = span(S), NB = E / R;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (S > 0) {
        const int jm = (t + T * q) % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) d[q * R + r] = cmul(d[q * R + r], tw[(jm * r) * (N / (Ns * R))]);
      }
      Dft<R>::run(&d[q * R]);
    }
  }

  // Whole transform of values already loaded in stage-0 order (d[e] = x[in_index(t, e)]).
  // `slot(idx)` maps a natural index of this transform to its LDS float2 slot. Every
  // exchange starts with a barrier, so the area may still be read by other threads on
  // entry; on exit other threads may still read it until the next barrier.
  // Threads with active = false only take part in the barriers.
  template <class Slot>
  __device__ __forceinline__ static void run(float2 (&d)[E], int t, const float2* __restrict__ tw, float2* lds,
                                             Slot slot, bool active = true) {
    if (active) stage<0>(d, t, tw);
    if constexpr (NS > 1) {
      exchange<0>(d, t, lds, slot, active);
      if (active) stage<(NS > 1 ? 1 : 0)>(d, t, tw);
    }
    if constexpr (NS > 2) {
      exchange<(NS > 2 ? 1 : 0)>(d, t, lds, slot, active);
      if (active) stage<(NS > 2 ? 2 : 0)>(d, t, tw);
    }
    if constexpr (NS > 3) {
      exchange<(NS > 3 ? 2 : 0)>(d, t, lds, slot, active);
      if (active) stage<(NS > 3 ? 3 : 0)>(d, t, tw);
    }
  }

  // Writes the outputs of stage S and reads the inputs of stage S + 1.
  template <int S, class Slot>
  __device__ __forceinline__ static void exchange(float2 (&d)[E], int t, float2* lds, Slot slot, bool active) {
    constexpr int R = radix(S), NB = E / R;
    __syncthreads();  // earlier readers of the area are done
    if (active) {
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) lds[slot(dst_index<S>(t, q, r))] = d[q * R + r];
    }
    __syncthreads();
    constexpr int R2 = radix(S + 1 < NS ? S + 1 : S), NB2 = E / R2;
    if (active) {
#pragma unroll
      for (int q = 0; q < NB2; ++q)
#pragma unroll
        for (int r = 0; r < R2; ++r) d[q * R2 + r] = lds[slot(src_index<S + 1 < NS ? S + 1 : S>(t, q, r))];
    }
  }
};

// Signed integer frequency of FFT index k.
template <int N>
__device__ __forceinline__ int signed_freq(int k) { return k < N / 2 ? k : k - N; }

}  // namespace pk
