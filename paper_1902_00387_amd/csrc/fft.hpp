// Register/LDS complex FFT building blocks for gfx950 (FP64, or FP32 for the
// complex64 variant).
//
// A group of T = N/E lanes (E = 8 or 4) of one wavefront transforms one
// length-N sequence.  Lane j holds E values in registers, v[e] = x[j + T*e]
// ("strided layout").  Each
// pass is a mixed-radix Stockham step: butterfly b gathers x[b + k*N/R]
// (k < R), which for the strided layout are the lane's own registers, so a
// pass needs no load exchange; its outputs go to LDS at their autosorted
// positions and are read back in the strided layout for the next pass.  The
// last pass's outputs already sit in the lane's own strided registers, so it
// runs in place without LDS and leaves the transform in natural order,
// strided: a transform of P passes makes P - 1 LDS exchanges.
//
// DIR = -1 is the forward transform X_k = sum_n x_n e^{-2 pi i nk/N},
// DIR = +1 the unnormalised inverse.  Twiddles come from a table
// tw[m] = e^{-2 pi i m/N} built on the host in extended precision.  Every
// function works on complex128 (cplx) or complex64 (cplxf) values.
#pragma once
#include <hip/hip_runtime.h>

namespace pd {

// Complex value of real type R (double: complex128 state, float: the
// complex64 variant); re and im interleaved in memory.
template <class R>
struct cpx {
  R re, im;
};
using cplx = cpx<double>;
using cplxf = cpx<float>;

template <class R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.re * s, a.im * s}; }
template <class R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <class R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// multiply by DIR*i  (DIR = -1: by -i, DIR = +1: by +i)
template <int DIR, class R>
__device__ __forceinline__ cpx<R> mul_i(cpx<R> a) {
  if constexpr (DIR < 0) return {a.im, -a.re};
  else return {-a.im, a.re};
}
__device__ __forceinline__ cplx czero() { return {0.0, 0.0}; }
template <class C>
__device__ __forceinline__ C zero_of() { return {0, 0}; }

// LDS index padding: one extra slot every 8 entries spreads the power-of-two
// strides of the Stockham scatter (consecutive lanes writing 8 entries
// apart in the first pass) over the LDS banks.
template <int N>
struct LdsSpan {
  static constexpr int shift = 3;
  static constexpr int value = N + (N >> shift);
};
template <int N>
__device__ __forceinline__ int lpad(int i) { return i + (i >> LdsSpan<N>::shift); }

// LDS slot of entry i of a transform's span.  A 16-byte access of a
// wavefront is served 16 lanes at a time, conflict-free when the 16 lanes'
// slots differ modulo 16.  The padded layout lpad does that for the
// scatters (lanes 8 entries apart) but leaves one two-way conflict in every
// 16 lanes of the gathers (entries j, j + 1, ... cross a padding slot).  For
// the 512-point transform with 8 values a lane (passes with sub-transform
// lengths 1, 8, 64) the permutation that XORs index bits 0-2 with bits 3-5
// and bit 3 with bit 6 keeps all three patterns conflict-free: the gathers
// j + 64 e (bits 0-3 vary), the first scatter 8 j + k (bits 3-6 vary) and
// the second 64 (j / 8) + 8 k + j % 8 (bits 0-2 and 6 vary) each map their
// 16 lanes onto 16 distinct slots.  Complex64 spans (8-byte entries) keep
// the padded layout.
template <int N, int E, class C>
__device__ __forceinline__ int lidx(int i) {
  if constexpr (N == 512 && E == 8 && sizeof(C) == 16)
    return i ^ ((i >> 3) & 7) ^ (((i >> 6) & 1) << 3);
  else
    return lpad<N>(i);
}

// ---- small DFTs in registers ---------------------------------------------
template <int DIR, class C>
__device__ __forceinline__ void dft2(C& a, C& b) {
  C t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR, class C>
__device__ __forceinline__ void dft4(C& x0, C& x1, C& x2, C& x3) {
  C t0 = cadd(x0, x2), t1 = csub(x0, x2);
  C t2 = cadd(x1, x3), t3 = mul_i<DIR>(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

template <int DIR, class C>
__device__ __forceinline__ void dft8(C* x) {
  using R = decltype(x->re);
  // split into even / odd halves, two radix-4 DFTs, then combine with
  // w8^k = e^{DIR 2 pi i k/8}
  C e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  C o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  constexpr R h = (R)0.70710678118654752440;  // sqrt(2)/2
  // w8^1 = h (1 + DIR i), w8^2 = DIR i, w8^3 = h (-1 + DIR i)
  C w1o1 = {h * (o1.re - DIR * o1.im), h * (o1.im + DIR * o1.re)};
  C w2o2 = mul_i<DIR>(o2);
  C w3o3 = {h * (-o3.re - DIR * o3.im), h * (-o3.im + DIR * o3.re)};
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, w1o1);
  x[5] = csub(e1, w1o1);
  x[2] = cadd(e2, w2o2);
  x[6] = csub(e2, w2o2);
  x[3] = cadd(e3, w3o3);
  x[7] = csub(e3, w3o3);
}

template <int R, int DIR, class C>
__device__ __forceinline__ void dftR(C* x) {
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

// Pass plan of a length-N transform with E values a lane: pass p has radix
// R(p) and combines sub-transforms of length NS(p).
//   E = 8: 16: 8x2   32: 8x4   64: 8x8   128: 8x8x2   256: 8x8x4   512: 8x8x8
//   E = 4: 16: 4x4   32: 4x4x2   64: 4x4x4   128: 4x4x4x2   256: 4x4x4x4
template <int N, int E>
struct Plan {
  static_assert(N >= 16 && N <= 512 && (N & (N - 1)) == 0, "N");
  static_assert((E == 8 && N / E <= 64) || (E == 4 && N / E <= 64), "group must fit a wavefront");
  static constexpr int passes = E == 8 ? (N <= 64 ? 2 : 3) : (N == 16 ? 2 : (N <= 64 ? 3 : 4));
  static constexpr int R(int p) {
    return E == 8 ? (p == 0 ? 8 : p == 1 ? (N == 16 ? 2 : N == 32 ? 4 : 8) : N / 64)
                  : (p <= 1 ? 4 : p == 2 ? (N == 32 ? 2 : 4) : N / 64);
  }
  static constexpr int NS(int p) { return p == 0 ? 1 : p == 1 ? E : p == 2 ? (E == 8 ? 64 : 16) : 64; }
  // twiddles a lane needs in pass p: R - 1 for each of its E/R butterflies
  static constexpr int tw_count(int p) { return NS(p) > 1 ? (E / R(p)) * (R(p) - 1) : 0; }
  static constexpr int tw_total() {
    int t = 0;
    for (int p = 0; p < passes; ++p) t += tw_count(p);
    return t;
  }
};

// The twiddles of every pass of one transform for one lane, read once from
// the table and then kept in registers (forward convention e^{-2 pi i m/N};
// the inverse uses their conjugates).  Loading them ahead keeps global-memory
// latency out of the passes, which the LDS exchange orders.
template <int N, int E, class C = cplx>
struct TwRegs {
  using PL = Plan<N, E>;
  static constexpr int count = PL::tw_total();
  C w[count > 0 ? count : 1];
  __device__ __forceinline__ void load(int j, const C* __restrict__ tw) {
    constexpr int T = N / E;
    int o = 0;
#pragma unroll
    for (int p = 0; p < PL::passes; ++p) {
      const int R = PL::R(p), NS = PL::NS(p);
      if (NS == 1) continue;
#pragma unroll
      for (int q = 0; q < E / R; ++q) {
        const int jj = (j + T * q) & (NS - 1);
#pragma unroll
        for (int k = 1; k < R; ++k) w[o++] = tw[jj * k * (N / (NS * R))];
      }
    }
  }
};

// One Stockham pass of radix R over sub-transforms of length NS, E values a
// lane.  Lane j owns butterflies b = j + T*q, q < E/R (T = N/E lanes); wl
// holds its (E/R) * (R-1) twiddles of this pass.  Outputs are scattered to
// LDS (slots lidx), then the lane reads back its strided values.  In the last
// pass (NS * R = N) output k of butterfly b lands at b + k*NS = j + T*(q +
// Q*k), which is the lane's own strided register q + Q*k: the butterfly runs
// in place in registers and the pass needs no exchange.
template <int N, int E, int R, int NS, int DIR, class C>
__device__ __forceinline__ void fft_pass(C* v, C* s, int j, const C* wl) {
  constexpr int T = N / E, Q = E / R;
  if constexpr (NS * R == N) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      C x[R];
#pragma unroll
      for (int k = 0; k < R; ++k) x[k] = v[q + k * Q];
      if constexpr (NS > 1) {
#pragma unroll
        for (int k = 1; k < R; ++k) {
          const C w = wl[q * (R - 1) + k - 1];
          x[k] = (DIR < 0) ? cmul(x[k], w) : cmulc(x[k], w);
        }
      }
      dftR<R, DIR>(x);
#pragma unroll
      for (int k = 0; k < R; ++k) v[q + k * Q] = x[k];
    }
    return;
  }
  // the swizzled 512-point layout with its slots written out per pattern
  // (the same slots as lidx, with the lane's part computed once)
  constexpr bool SWZ = N == 512 && E == 8 && sizeof(C) == 16;
  static_assert(!SWZ || Q == 1, "one butterfly a lane in the swizzled passes");
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = j + T * q;
    const int jj = b & (NS - 1);
    C x[R];
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = v[q + k * Q];
    if constexpr (NS > 1) {
#pragma unroll
      for (int k = 1; k < R; ++k) {
        const C w = wl[q * (R - 1) + k - 1];
        x[k] = (DIR < 0) ? cmul(x[k], w) : cmulc(x[k], w);
      }
    }
    dftR<R, DIR>(x);
    if constexpr (SWZ && NS == 1) {
      // entries 8 j + k: slot ((8 j) ^ (8 bit3(j))) + (k ^ (j & 7))
      const int hi = (8 * j) ^ (((j >> 3) & 1) << 3), lo = j & 7;
#pragma unroll
      for (int k = 0; k < R; ++k) s[hi + (k ^ lo)] = x[k];
    } else if constexpr (SWZ && NS == 8) {
      // entries 64 (j / 8) + 8 k + j % 8: slot 64 (j / 8) + 8 (k ^ bit3(j)) + ((j & 7) ^ k)
      const int hi = 64 * (j >> 3), c1 = (j >> 3) & 1, lo = j & 7;
#pragma unroll
      for (int k = 0; k < R; ++k) s[hi + 8 * (k ^ c1) + (lo ^ k)] = x[k];
    } else {
      const int base = (b / NS) * NS * R + jj;
#pragma unroll
      for (int k = 0; k < R; ++k) s[lidx<N, E, C>(base + k * NS)] = x[k];
    }
  }
  group_sync();
  if constexpr (SWZ) {
    // entries j + 64 e: slot (j ^ ((j >> 3) & 7) ^ (8 (e & 1))) + 64 e
    const int jg = j ^ ((j >> 3) & 7);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = s[(jg ^ ((e & 1) << 3)) + T * e];
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = s[lidx<N, E, C>(j + T * e)];
  }
  group_sync();
}

template <int N, int E, int P, int DIR, class C>
__device__ __forceinline__ void fft_from(C* v, C* s, int j, const C* w) {
  using PL = Plan<N, E>;
  if constexpr (P < PL::passes) {
    fft_pass<N, E, PL::R(P), PL::NS(P), DIR>(v, s, j, w);
    fft_from<N, E, P + 1, DIR>(v, s, j, w + PL::tw_count(P));
  }
}

// Full length-N transform of the strided register vector v (E values a
// lane, T = N/E lanes, all in one wavefront; see header).  s: this group's
// LDS span (LdsSpan<N>::value entries); t: the lane's twiddles (TwRegs).
template <int N, int E, int DIR, class C>
__device__ __forceinline__ void fft(C* v, C* s, int j, const TwRegs<N, E, C>& t) {
  fft_from<N, E, 0, DIR>(v, s, j, t.w);
}

// Same, reading the lane's twiddles from the table first.
template <int N, int E, int DIR, class C>
__device__ __forceinline__ void fft(C* v, C* s, int j, const C* __restrict__ tw) {
  TwRegs<N, E, C> t;
  t.load(j, tw);
  fft_from<N, E, 0, DIR>(v, s, j, t.w);
}

}  // namespace pd
