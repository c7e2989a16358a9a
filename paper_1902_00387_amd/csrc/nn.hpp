// Internal interface of the learned coarse-propagator correction kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "fft.hpp"

namespace pd {
namespace nn {

constexpr int CH = 32;  // channels of the hidden layers

// Parameter views into one contiguous FP32 vector:
//   W_in [12][CH] | V [L][3][5][CH][CH] | gamma [L][Q][CH] | W_out [CH][6]
struct Net {
  int Q = 0, Mf = 0, L = 0;
  int f32 = 0;  // matrix-core operands: 0 BF16 (rounded from FP32), 1 FP32
  float* W_in = nullptr;
  float* V = nullptr;
  float* gamma = nullptr;
  float* W_out = nullptr;
};
using Grads = Net;

inline size_t param_count(int Q, int L) {
  return (size_t)12 * CH + (size_t)L * 15 * CH * CH + (size_t)L * Q * CH + (size_t)CH * 6;
}
inline Net view(float* base, int Q, int Mf, int L) {
  Net n;
  n.Q = Q;
  n.Mf = Mf;
  n.L = L;
  n.W_in = base;
  n.V = n.W_in + 12 * CH;
  n.gamma = n.V + (size_t)L * 15 * CH * CH;
  n.W_out = n.gamma + (size_t)L * Q * CH;
  return n;
}

struct Work {
  float* dc = nullptr;   // [B][Q][6]
  float* dhA = nullptr;  // [B][Q][CH]
  float* dhB = nullptr;  // [B][Q][CH]
  float* dW = nullptr;   // [B][5][CH][CH]
  float* part = nullptr; // outer-product partials
  const float* wq = nullptr;  // [Q] per-mode loss weights (null: all 1)
};

// x[b][m][12] = (re/im of D, re/im of g) / |D_b| from compact boxes [b][3][Q]
hipError_t features(const cplx* D, const cplx* g, const double* nrm2, float* x, int Q, int B,
                    hipStream_t st);
// r[b][m][6] = (F - g) / |D_b|
hipError_t targets(const cplx* F, const cplx* g, const double* nrm2, float* r, int Q, int B,
                   hipStream_t st);
// forward over batch positions b < B (x, t through bidx when non-null);
// h[0..L], y[0..L-1]: [B][Q][CH] activations; c: [B][Q][6]
hipError_t forward(const Net& net, const float* x, const double* tb, const int* bidx, int B,
                   float* const* h, float* const* y, float* c, hipStream_t st);
// sums[0] = sum w_m (c - r)^2, sums[1] = sum w_m r^2 (r through bidx; w_m the
// per-mode weight, all 1 when wq is null); part: >= 512 doubles
hipError_t loss(const float* c, const float* r, int Q, int B, const int* bidx, const float* wq,
                double* part, double* sums, hipStream_t st);
// gradients of sums[0]/sums[1] with respect to every parameter (weights w.wq)
hipError_t backward(const Net& net, const float* x, const double* tb, const int* bidx, int B,
                    float* const* h, float* const* y, const float* c, const float* r,
                    const double* sums, Grads& gr, Work& w, hipStream_t st);
hipError_t adam(float* p, const float* g, float* m1, float* m2, size_t n, float lr, int step,
                hipStream_t st);
// out = a - b (b null: copy), n complex values
hipError_t sub(const cplx* a, const cplx* b, cplx* out, size_t n, hipStream_t st);
// red[0] = |u - v|^2, red[1] = |u|^2
hipError_t defect(const cplx* u, const cplx* v, size_t n, double* red, hipStream_t st);
// out = (with_F ? F : 0) + g + |D| c for one field (compact box, Q modes)
hipError_t combine(const cplx* F, const cplx* g, const float* c, const double* nrm2, cplx* out,
                   int Q, bool with_F, hipStream_t st);

}  // namespace nn
}  // namespace pd
