// Host-side helpers shared by the C-ABI runtime files (no device code).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "fft.hpp"

namespace pd {
namespace rt {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, n ? n : 16);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = n;
    return hipSuccess;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

inline int box_K(int N) { return (N - 1) / 3; }
inline int box_M(int N) { return 2 * box_K(N) + 1; }
inline bool valid_N(int N) {
  return N == 16 || N == 32 || N == 64 || N == 128 || N == 256 || N == 512;
}

// e^{-2 pi i m/N}, m = 0..N-1.  Angles are reduced to the first octant and
// evaluated in extended precision, so quadrant values are exact and the
// table is symmetric to the last bit.
inline std::vector<cplx> twiddles(int N) {
  std::vector<cplx> tw(N);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  const int n4 = N / 4;
  for (int m = 0; m < N; ++m) {
    const int q = m / n4, r = m % n4;
    long double c, s;
    if (2 * r <= n4) {
      const long double a = two_pi * (long double)r / (long double)N;
      c = cosl(a);
      s = sinl(a);
    } else {
      const long double a = two_pi * (long double)(n4 - r) / (long double)N;
      c = sinl(a);
      s = cosl(a);
    }
    long double cq, sq;  // rotate by q quarter turns
    switch (q) {
      case 0: cq = c; sq = s; break;
      case 1: cq = -s; sq = c; break;
      case 2: cq = -c; sq = -s; break;
      default: cq = s; sq = -c; break;
    }
    tw[m] = {(double)cq, (double)(-sq)};
  }
  return tw;
}

inline bool integer_ratio(double a, double b, int* n) {
  if (!(a > 0) || !(b > 0)) return false;
  const double q = a / b;
  const double r = std::nearbyint(q);
  if (r < 1 || r > 1e9 || std::fabs(q - r) > 1e-9 * r) return false;
  *n = (int)r;
  return true;
}

}  // namespace rt
}  // namespace pd
