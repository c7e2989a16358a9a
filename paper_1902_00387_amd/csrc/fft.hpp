// Register/LDS complex FFT building blocks for gfx950 (FP64).
//
// A group of T = N/E lanes (E = 8 or 4) of one wavefront transforms one
// length-N sequence.  Lane j holds E values in registers, v[e] = x[j + T*e]
// ("strided layout").  Each
// pass is a mixed-radix Stockham step: butterfly b gathers x[b + k*N/R]
// (k < R), which for the strided layout are the lane's own registers, so a
// pass needs no load exchange; its outputs go to LDS at their autosorted
// positions and are read back in the strided layout for the next pass.  The
// final read-back leaves the transform in natural order, again strided.
//
// DIR = -1 is the forward transform X_k = sum_n x_n e^{-2 pi i nk/N},
// DIR = +1 the unnormalised inverse.  Twiddles come from a table
// tw[m] = e^{-2 pi i m/N} built on the host in extended precision.
#pragma once
#include <hip/hip_runtime.h>

namespace pd {

struct cplx {
  double re, im;
};

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
__device__ __forceinline__ cplx cmulc(cplx a, cplx b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// multiply by DIR*i  (DIR = -1: by -i, DIR = +1: by +i)
template <int DIR>
__device__ __forceinline__ cplx mul_i(cplx a) {
  if constexpr (DIR < 0) return {a.im, -a.re};
  else return {-a.im, a.re};
}
__device__ __forceinline__ cplx czero() { return {0.0, 0.0}; }

// LDS index padding: one extra 16-byte slot every 2^PAD_SHIFT entries spreads
// the power-of-two strides of the Stockham scatter over the 64 LDS banks
// (every 16 entries for N >= 64, every 8 below; chosen with a bank model of
// the exchange patterns).
template <int N>
struct LdsSpan {
  static constexpr int shift = N >= 64 ? 4 : 3;
  static constexpr int value = N + (N >> shift);
};
template <int N>
__device__ __forceinline__ int lpad(int i) { return i + (i >> LdsSpan<N>::shift); }

// ---- small DFTs in registers ---------------------------------------------
template <int DIR>
__device__ __forceinline__ void dft2(cplx& a, cplx& b) {
  cplx t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR>
__device__ __forceinline__ void dft4(cplx& x0, cplx& x1, cplx& x2, cplx& x3) {
  cplx t0 = cadd(x0, x2), t1 = csub(x0, x2);
  cplx t2 = cadd(x1, x3), t3 = mul_i<DIR>(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

template <int DIR>
__device__ __forceinline__ void dft8(cplx* x) {
  // split into even / odd halves, two radix-4 DFTs, then combine with
  // w8^k = e^{DIR 2 pi i k/8}
  cplx e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  cplx o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  constexpr double h = 0.70710678118654752440;  // sqrt(2)/2
  // w8^1 = h (1 + DIR i), w8^2 = DIR i, w8^3 = h (-1 + DIR i)
  cplx w1o1 = {h * (o1.re - DIR * o1.im), h * (o1.im + DIR * o1.re)};
  cplx w2o2 = mul_i<DIR>(o2);
  cplx w3o3 = {h * (-o3.re - DIR * o3.im), h * (-o3.im + DIR * o3.re)};
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, w1o1);
  x[5] = csub(e1, w1o1);
  x[2] = cadd(e2, w2o2);
  x[6] = csub(e2, w2o2);
  x[3] = cadd(e3, w3o3);
  x[7] = csub(e3, w3o3);
}

template <int R, int DIR>
__device__ __forceinline__ void dftR(cplx* x) {
  if constexpr (R == 2) dft2<DIR>(x[0], x[1]);
  else if constexpr (R == 4) dft4<DIR>(x[0], x[1], x[2], x[3]);
  else dft8<DIR>(x);
}

// Orders the LDS exchange of one transform.  Every transform group lies
// inside one wavefront, whose lanes issue each LDS instruction together and
// whose LDS operations complete in order, so the exchange only has to stop the
// compiler from moving LDS accesses across this point.
__device__ __forceinline__ void group_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One Stockham pass of radix R over sub-transforms of length NS, E values a
// lane.  Lane j owns butterflies b = j + T*q, q < E/R (T = N/E lanes).
// Outputs are scattered to LDS (padded), then the lane reads back its
// strided values.
template <int N, int E, int R, int NS, int DIR>
__device__ __forceinline__ void fft_pass(cplx* v, cplx* s, int j, const cplx* __restrict__ tw) {
  constexpr int T = N / E, Q = E / R;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = j + T * q;
    const int jj = b & (NS - 1);
    cplx x[R];
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = v[q + k * Q];
    if constexpr (NS > 1) {
#pragma unroll
      for (int k = 1; k < R; ++k) {
        const cplx w = tw[jj * k * (N / (NS * R))];
        x[k] = (DIR < 0) ? cmul(x[k], w) : cmulc(x[k], w);
      }
    }
    dftR<R, DIR>(x);
    const int base = (b / NS) * NS * R + jj;
#pragma unroll
    for (int k = 0; k < R; ++k) s[lpad<N>(base + k * NS)] = x[k];
  }
  group_sync();
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = s[lpad<N>(j + T * e)];
  group_sync();
}

// Full length-N transform of the strided register vector v (E values a
// lane, T = N/E lanes, all in one wavefront; see header).  s: this group's
// LDS span (LdsSpan<N>::value entries).
//   E = 8: 16: 8x2   32: 8x4   64: 8x8   128: 8x8x2   256: 8x8x4   512: 8x8x8
//   E = 4: 16: 4x4   32: 4x4x2   64: 4x4x4   128: 4x4x4x2   256: 4x4x4x4
template <int N, int E, int DIR>
__device__ __forceinline__ void fft(cplx* v, cplx* s, int j, const cplx* __restrict__ tw) {
  static_assert(N >= 16 && N <= 512 && (N & (N - 1)) == 0, "N");
  static_assert((E == 8 && N / E <= 64) || (E == 4 && N / E <= 64), "group must fit a wavefront");
  if constexpr (E == 8) {
    fft_pass<N, 8, 8, 1, DIR>(v, s, j, tw);
    if constexpr (N == 16) fft_pass<N, 8, 2, 8, DIR>(v, s, j, tw);
    else if constexpr (N == 32) fft_pass<N, 8, 4, 8, DIR>(v, s, j, tw);
    else {
      fft_pass<N, 8, 8, 8, DIR>(v, s, j, tw);
      if constexpr (N == 128) fft_pass<N, 8, 2, 64, DIR>(v, s, j, tw);
      else if constexpr (N == 256) fft_pass<N, 8, 4, 64, DIR>(v, s, j, tw);
      else if constexpr (N == 512) fft_pass<N, 8, 8, 64, DIR>(v, s, j, tw);
    }
  } else {
    fft_pass<N, 4, 4, 1, DIR>(v, s, j, tw);
    fft_pass<N, 4, 4, 4, DIR>(v, s, j, tw);
    if constexpr (N == 32) fft_pass<N, 4, 2, 16, DIR>(v, s, j, tw);
    else if constexpr (N >= 64) {
      fft_pass<N, 4, 4, 16, DIR>(v, s, j, tw);
      if constexpr (N == 128) fft_pass<N, 4, 2, 64, DIR>(v, s, j, tw);
      else if constexpr (N == 256) fft_pass<N, 4, 4, 64, DIR>(v, s, j, tw);
    }
  }
}

}  // namespace pd
