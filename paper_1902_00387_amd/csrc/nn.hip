// Learned coarse-propagator correction: forward, backward and Adam kernels
// (gfx950; BF16 MFMA with FP32 accumulation for the channel-mixing layers).
//
// For a slice starting at time t and an input field D with plain coarse
// result g (both on the fine 2/3 box, Q = Mf^2 modes), the correction is
//   c = Net(x),  x[m] = (re/im of D, re/im of g)[m] / |D|   (12 reals a mode)
//   h0 = x W_in;  y_l[m] = sum_s h_l[m + s] W_{l,s}(t);  h_{l+1} = h_l + gamma_l * y_l
//   W_{l,s}(t) = V_{l,0,s} + cos t V_{l,1,s} + sin t V_{l,2,s},  s in {0, +kx, -kx, +ky, -ky}
//   c = h_L W_out  (6 reals = 3 complex a mode)
// and the learned coarse propagator is g + |D| c.  Activations are FP32 in
// memory and rounded to BF16 as MFMA operands (v_mfma_f32_16x16x16_bf16); a
// test mode feeds the same FP32 values unrounded to the FP32 matrix
// instruction (v_mfma_f32_16x16x4_f32, four per BF16 one: the K-slot of lane
// group kb in instruction q is channel 4 kb + q), with the same accumulation.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft.hpp"
#include "nn.hpp"

namespace pd {
namespace nn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ short f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// shift s: 0 (0,0), 1 (0,+1), 2 (0,-1), 3 (+1,0), 4 (-1,0) in (ky, kx); returns
// the mode index of m + sign*s inside the Mf x Mf box, or -1 outside
__device__ __forceinline__ int shifted(int m, int s, int sign, int Mf) {
  int r = m / Mf, c = m - r * Mf;
  const int dy = (s == 3) ? 1 : (s == 4 ? -1 : 0);
  const int dx = (s == 1) ? 1 : (s == 2 ? -1 : 0);
  r += sign * dy;
  c += sign * dx;
  if (r < 0 || r >= Mf || c < 0 || c >= Mf) return -1;
  return r * Mf + c;
}

// ---------------------------------------------------------------------------
// Features: x[b][m][12] from compact fine-box fields D, g ([b][3][Q] complex)
// scaled by 1/|D_b| (0 when D_b = 0).
__global__ void k_features(const cplx* __restrict__ D, const cplx* __restrict__ g,
                           const double* __restrict__ nrm2, float* __restrict__ x, int Q,
                           int B) {
  const size_t total = (size_t)B * Q;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / Q, m = i - b * Q;
    const double n2 = nrm2[b];
    const double sc = n2 > 0 ? 1.0 / sqrt(n2) : 0.0;
    float* xo = x + i * 12;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cplx d = D[(b * 3 + c) * Q + m], gg = g[(b * 3 + c) * Q + m];
      xo[2 * c] = (float)(d.re * sc);
      xo[2 * c + 1] = (float)(d.im * sc);
      xo[6 + 2 * c] = (float)(gg.re * sc);
      xo[6 + 2 * c + 1] = (float)(gg.im * sc);
    }
  }
}

// r[b][m][6] = (F - g)[b][m] / |D_b|
__global__ void k_targets(const cplx* __restrict__ F, const cplx* __restrict__ g,
                          const double* __restrict__ nrm2, float* __restrict__ r, int Q, int B) {
  const size_t total = (size_t)B * Q;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / Q, m = i - b * Q;
    const double n2 = nrm2[b];
    const double sc = n2 > 0 ? 1.0 / sqrt(n2) : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cplx f = F[(b * 3 + c) * Q + m], gg = g[(b * 3 + c) * Q + m];
      r[i * 6 + 2 * c] = (float)((f.re - gg.re) * sc);
      r[i * 6 + 2 * c + 1] = (float)((f.im - gg.im) * sc);
    }
  }
}

// Dense rows: out[row][0..NO) = in[row][0..NI) W[NI][NO] (FP32), row index of
// the input through bidx when given (sample store -> batch position).
template <int NI, int NO>
__global__ __launch_bounds__(256) void k_dense(const float* __restrict__ in, const float* __restrict__ W,
                        float* __restrict__ out, int Q, int B, const int* __restrict__ bidx) {
  __shared__ float w[NI * NO];
  for (int i = threadIdx.x; i < NI * NO; i += blockDim.x) w[i] = W[i];
  __syncthreads();
  const size_t total = (size_t)B * Q;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / Q, m = i - b * Q;
    const size_t src = (bidx ? (size_t)bidx[b] : b) * Q + m;
    float a[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) a[k] = in[src * NI + k];
#pragma unroll 2
    for (int o = 0; o < NO; ++o) {
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < NI; ++k) s = fmaf(a[k], w[k * NO + o], s);
      out[i * NO + o] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Channel-mixing layer, one workgroup = one sample x 64 modes (4 waves of 16).
// FWD:  y[m] = sum_s h[m + s] W_s(t);  out[m] = h[m] + gamma[m] * y[m]
// BWD:  out[m] = dh[m] + sum_s (gamma * dh)[m - s] W_s(t)^T
// W_s(t) is assembled in LDS (BF16) from the FP32 master V of layer l.
// one 16 x 16 x 16 product step on the matrix cores: A[i][k] from lane (i,
// kb) as a[r] = A[i][4 kb + r], B[k][j] as b[r] = B[4 kb + r][j]
template <bool F32>
__device__ __forceinline__ f32x4 mfma16(const float (&a)[4], const float (&b)[4], f32x4 acc) {
  if constexpr (F32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b[q], acc, 0, 0, 0);
    return acc;
  } else {
    bf16x4 ab, bb;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ab[r] = f2bf(a[r]);
      bb[r] = f2bf(b[r]);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ab, bb, acc, 0, 0, 0);
  }
}

template <bool BWD, bool F32>
__global__ __launch_bounds__(256) void k_layer(const float* __restrict__ hin,
                                               const float* __restrict__ V,
                                               const double* __restrict__ tb,
                                               const float* __restrict__ gamma,
                                               float* __restrict__ y_out, float* __restrict__ out,
                                               int Q, int Mf, const int* __restrict__ bidx) {
  constexpr int C = CH;
  __shared__ float ws[5 * C * C];  // [s][k][j] (BWD: transposed), FP32 (rounded at use)
  const int b = blockIdx.y;
  const double t = tb[bidx ? bidx[b] : b];
  const float ct = (float)cos(t), st = (float)sin(t);
  for (int i = threadIdx.x; i < 5 * C * C; i += blockDim.x) {
    const int s = i / (C * C), rem = i - s * C * C;
    const int k = rem / C, j = rem - k * C;
    // V layout [3][5][C][C] = [feature][shift][in][out]
    const int vi = BWD ? (j * C + k) : (k * C + j);
    const float w = V[(0 * 5 + s) * C * C + vi] + ct * V[(1 * 5 + s) * C * C + vi] +
                    st * V[(2 * 5 + s) * C * C + vi];
    ws[i] = w;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mbase = blockIdx.x * 64 + wave * 16;
  const int li = lane & 15, kb = lane >> 4;
  const size_t bo = (size_t)b * Q;
  f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  const int m = mbase + li;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const int ms = (m < Q) ? shifted(m, s, BWD ? -1 : 1, Mf) : -1;
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      float a[4] = {0.f, 0.f, 0.f, 0.f};
      if (ms >= 0) {
        const float4 v = *reinterpret_cast<const float4*>(hin + (bo + ms) * C + 16 * kc + 4 * kb);
        float4 gv = {1.f, 1.f, 1.f, 1.f};
        if (BWD) gv = *reinterpret_cast<const float4*>(gamma + (size_t)ms * C + 16 * kc + 4 * kb);
        a[0] = v.x * gv.x;
        a[1] = v.y * gv.y;
        a[2] = v.z * gv.z;
        a[3] = v.w * gv.w;
      }
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        float bv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) bv[r] = ws[(s * C + 16 * kc + 4 * kb + r) * C + 16 * nt + li];
        acc[nt] = mfma16<F32>(a, bv, acc[nt]);
      }
    }
  }
  // lane holds D[i = 4 kb + r][j = li] of each 16 x 16 output tile
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mo = mbase + 4 * kb + r;
      if (mo >= Q) continue;
      const int ch = 16 * nt + li;
      const size_t o = (bo + mo) * C + ch;
      const float yv = acc[nt][r];
      if (BWD) {
        out[o] = hin[o] + yv;
      } else {
        y_out[o] = yv;
        out[o] = hin[o] + gamma[(size_t)mo * C + ch] * yv;
      }
    }
}

// dW_s(b)[i][o] = sum_m h[b][m + s][i] (gamma * dh)[b][m][o], one workgroup per
// (sample, shift), one wave per 16 x 16 output tile, MFMA over 16-mode chunks.
template <bool F32>
__global__ __launch_bounds__(256) void k_dweight(const float* __restrict__ h,
                                                 const float* __restrict__ dh,
                                                 const float* __restrict__ gamma,
                                                 float* __restrict__ dW, int Q, int Mf) {
  constexpr int C = CH;
  const int b = blockIdx.y, s = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int it = wave >> 1, ot = wave & 1;
  const int li = lane & 15, kb = lane >> 4;
  const size_t bo = (size_t)b * Q;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int m0 = 0; m0 < Q; m0 += 16) {
    float a[4], bv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + 4 * kb + r;
      float av = 0.f, dv = 0.f;
      if (m < Q) {
        const int ms = shifted(m, s, 1, Mf);
        if (ms >= 0) av = h[(bo + ms) * C + 16 * it + li];
        const int o = 16 * ot + li;
        dv = dh[(bo + m) * C + o] * gamma[(size_t)m * C + o];
      }
      a[r] = av;
      bv[r] = dv;
    }
    acc = mfma16<F32>(a, bv, acc);
  }
  float* out = dW + ((size_t)b * 5 + s) * C * C;
#pragma unroll
  for (int r = 0; r < 4; ++r) out[(16 * it + 4 * kb + r) * C + 16 * ot + li] = acc[r];
}

// dV[j][s][i][o] = sum_b phi_j(t_b) dW[b][s][i][o]  (fixed order)
__global__ void k_dV(const float* __restrict__ dW, const double* __restrict__ tb,
                     const int* __restrict__ bidx, float* __restrict__ dV, int B) {
  constexpr int C = CH;
  const int n = 5 * C * C;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    for (int b = 0; b < B; ++b) {
      const double t = tb[bidx ? bidx[b] : b];
      const float w = dW[(size_t)b * n + i];
      a0 += w;
      a1 += (float)cos(t) * w;
      a2 += (float)sin(t) * w;
    }
    dV[i] = a0;
    dV[n + i] = a1;
    dV[2 * n + i] = a2;
  }
}

// dgamma[m][c] = sum_b dh[b][m][c] y[b][m][c]
__global__ void k_dgamma(const float* __restrict__ dh, const float* __restrict__ y,
                         float* __restrict__ dg, int Q, int B) {
  const size_t n = (size_t)Q * CH;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    float a = 0.f;
    for (int b = 0; b < B; ++b) a += dh[(size_t)b * n + i] * y[(size_t)b * n + i];
    dg[i] = a;
  }
}

// Outer-product reduction partials: part[blk][p][q] = sum over this block's
// rows of A[row][p] * Bm[row][q]  (A rows through bidx when given).
template <int NP, int NQ>
__global__ __launch_bounds__(256) void k_outer(const float* __restrict__ A,
                                               const float* __restrict__ Bm,
                                               float* __restrict__ part, int Q, int Bn,
                                               const int* __restrict__ bidx, int rows_per_blk) {
  __shared__ float red[256];
  const size_t total = (size_t)Bn * Q;
  const size_t r0 = (size_t)blockIdx.x * rows_per_blk;
  const size_t r1 = r0 + rows_per_blk < total ? r0 + rows_per_blk : total;
  for (int pq = 0; pq < NP * NQ; ++pq) {
    const int p = pq / NQ, q = pq - p * NQ;
    float s = 0.f;
    for (size_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      const size_t b = r / Q, m = r - b * Q;
      const size_t ar = (bidx ? (size_t)bidx[b] : b) * Q + m;
      s += A[ar * NP + p] * Bm[r * NQ + q];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * NP * NQ + pq] = red[0];
    __syncthreads();
  }
}

__global__ void k_sum_parts(const float* __restrict__ part, int nblk, int n,
                            float* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * n + i];
    out[i] = s;
  }
}

// loss partials of sum (c - r)^2 and sum r^2 (double), r through bidx
__global__ __launch_bounds__(256) void k_loss_part(const float* __restrict__ c,
                                                   const float* __restrict__ r, int Q, int B,
                                                   const int* __restrict__ bidx,
                                                   const float* __restrict__ wq,
                                                   double* __restrict__ part) {
  __shared__ double red[2][256];
  const size_t total = (size_t)B * Q * 6;
  double s0 = 0.0, s1 = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / ((size_t)Q * 6), rem = i - b * Q * 6;
    const size_t ri = (bidx ? (size_t)bidx[b] : b) * Q * 6 + rem;
    const double wm = wq ? (double)wq[rem / 6] : 1.0;
    const double d = (double)c[i] - (double)r[ri];
    s0 += wm * d * d;
    s1 += wm * (double)r[ri] * (double)r[ri];
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_loss_sum(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nblk; ++i) {
      a += part[2 * i];
      b += part[2 * i + 1];
    }
    out[0] = a;
    out[1] = b;
  }
}

// dc = 2 w_m (c - r) / sum w r^2 ; then dh_L = dc W_out^T
__global__ void k_dc_dh(const float* __restrict__ c, const float* __restrict__ r,
                        const double* __restrict__ sums, const float* __restrict__ Wout,
                        float* __restrict__ dc, float* __restrict__ dh, int Q, int B,
                        const int* __restrict__ bidx, const float* __restrict__ wq) {
  const size_t total = (size_t)B * Q;
  const double den = sums[1];
  const float s2 = den > 0 ? (float)(2.0 / den) : 0.f;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / Q, m = i - b * Q;
    const size_t ri = ((bidx ? (size_t)bidx[b] : b) * Q + m) * 6;
    const float sw = wq ? s2 * wq[m] : s2;
    float d[6];
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      d[o] = sw * (c[i * 6 + o] - r[ri + o]);
      dc[i * 6 + o] = d[o];
    }
#pragma unroll 4
    for (int k = 0; k < CH; ++k) {
      float a = 0.f;
#pragma unroll
      for (int o = 0; o < 6; ++o) a = fmaf(d[o], Wout[k * 6 + o], a);
      dh[i * CH + k] = a;
    }
  }
}

// Adam on FP32 master weights (bias-corrected, fixed coefficients)
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  }
}

// U_next = F + g + |D| c   (compact fine box), c as 3 complex a mode
__global__ void k_combine(const cplx* __restrict__ F, const cplx* __restrict__ g,
                          const float* __restrict__ c, const double* __restrict__ nrm2,
                          cplx* __restrict__ out, int Q, int with_F) {
  const double sc = nrm2[0] > 0 ? sqrt(nrm2[0]) : 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 3 * Q; i += gridDim.x * blockDim.x) {
    const int comp = i / Q, m = i - comp * Q;
    const cplx corr = {sc * (double)c[m * 6 + 2 * comp], sc * (double)c[m * 6 + 2 * comp + 1]};
    cplx v = cadd(g[i], corr);
    if (with_F) v = cadd(F[i], v);
    out[i] = v;
  }
}

// out = a - b (n complex values; b may be null: out = a)
__global__ void k_sub(const cplx* __restrict__ a, const cplx* __restrict__ b,
                      cplx* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = b ? csub(a[i], b[i]) : a[i];
}

// red[0] = |u - v|^2, red[1] = |u|^2 (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_defect(const cplx* __restrict__ u,
                                                const cplx* __restrict__ v, size_t n,
                                                double* __restrict__ red) {
  __shared__ double rs[2][256];
  double s0 = 0.0, s1 = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 256) {
    const cplx d = csub(u[i], v[i]);
    s0 += d.re * d.re + d.im * d.im;
    s1 += u[i].re * u[i].re + u[i].im * u[i].im;
  }
  rs[0][threadIdx.x] = s0;
  rs[1][threadIdx.x] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rs[0][threadIdx.x] += rs[0][threadIdx.x + w];
      rs[1][threadIdx.x] += rs[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[0] = rs[0][0];
    red[1] = rs[1][0];
  }
}

// ---------------------------------------------------------------------------
static int grid1(size_t n) {
  size_t g = (n + 255) / 256;
  return (int)(g > 4096 ? 4096 : (g ? g : 1));
}

hipError_t features(const cplx* D, const cplx* g, const double* nrm2, float* x, int Q, int B,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3(grid1((size_t)B * Q)), dim3(256), 0, st, D, g, nrm2, x, Q, B);
  return hipGetLastError();
}

hipError_t targets(const cplx* F, const cplx* g, const double* nrm2, float* r, int Q, int B,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_targets, dim3(grid1((size_t)B * Q)), dim3(256), 0, st, F, g, nrm2, r, Q, B);
  return hipGetLastError();
}

hipError_t forward(const Net& net, const float* x, const double* tb, const int* bidx, int B,
                   float* const* h, float* const* y, float* c, hipStream_t st) {
  const int Q = net.Q;
  hipLaunchKernelGGL((k_dense<12, CH>), dim3(grid1((size_t)B * Q)), dim3(256), 0, st, x,
                     net.W_in, h[0], Q, B, bidx);
  for (int l = 0; l < net.L; ++l) {
    auto kern = net.f32 ? k_layer<false, true> : k_layer<false, false>;
    hipLaunchKernelGGL(kern, dim3((Q + 63) / 64, B), dim3(256), 0, st, h[l],
                       net.V + (size_t)l * 15 * CH * CH, tb, net.gamma + (size_t)l * Q * CH, y[l],
                       h[l + 1], Q, net.Mf, bidx);
  }
  hipLaunchKernelGGL((k_dense<CH, 6>), dim3(grid1((size_t)B * Q)), dim3(256), 0, st, h[net.L],
                     net.W_out, c, Q, B, nullptr);
  return hipGetLastError();
}

hipError_t loss(const float* c, const float* r, int Q, int B, const int* bidx, const float* wq,
                double* part, double* sums, hipStream_t st) {
  const int nblk = 256;
  hipLaunchKernelGGL(k_loss_part, dim3(nblk), dim3(256), 0, st, c, r, Q, B, bidx, wq, part);
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(64), 0, st, part, nblk, sums);
  return hipGetLastError();
}

hipError_t backward(const Net& net, const float* x, const double* tb, const int* bidx, int B,
                    float* const* h, float* const* y, const float* c, const float* r,
                    const double* sums, Grads& gr, Work& w, hipStream_t st) {
  const int Q = net.Q;
  const size_t rows = (size_t)B * Q;
  const int rpb = 4096;
  const int nblk = (int)((rows + rpb - 1) / rpb);
  // output layer
  hipLaunchKernelGGL(k_dc_dh, dim3(grid1(rows)), dim3(256), 0, st, c, r, sums, net.W_out, w.dc,
                     w.dhA, Q, B, bidx, w.wq);
  hipLaunchKernelGGL((k_outer<CH, 6>), dim3(nblk), dim3(256), 0, st, h[net.L], w.dc, w.part, Q,
                     B, nullptr, rpb);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, w.part, nblk, CH * 6, gr.W_out);
  float* dh = w.dhA;
  float* dh2 = w.dhB;
  for (int l = net.L - 1; l >= 0; --l) {
    const float* gam = net.gamma + (size_t)l * Q * CH;
    hipLaunchKernelGGL(k_dgamma, dim3(grid1((size_t)Q * CH)), dim3(256), 0, st, dh, y[l],
                       gr.gamma + (size_t)l * Q * CH, Q, B);
    auto kdw = net.f32 ? k_dweight<true> : k_dweight<false>;
    hipLaunchKernelGGL(kdw, dim3(5, B), dim3(256), 0, st, h[l], dh, gam, w.dW, Q, net.Mf);
    hipLaunchKernelGGL(k_dV, dim3(grid1(5 * CH * CH)), dim3(256), 0, st, w.dW, tb, bidx,
                       gr.V + (size_t)l * 15 * CH * CH, B);
    auto kb = net.f32 ? k_layer<true, true> : k_layer<true, false>;
    hipLaunchKernelGGL(kb, dim3((Q + 63) / 64, B), dim3(256), 0, st, dh,
                       net.V + (size_t)l * 15 * CH * CH, tb, gam, nullptr, dh2, Q, net.Mf, bidx);
    float* tmp = dh;
    dh = dh2;
    dh2 = tmp;
  }
  hipLaunchKernelGGL((k_outer<12, CH>), dim3(nblk), dim3(256), 0, st, x, dh, w.part, Q, B, bidx,
                     rpb);
  hipLaunchKernelGGL(k_sum_parts, dim3(2), dim3(256), 0, st, w.part, nblk, 12 * CH, gr.W_in);
  return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m1, float* m2, size_t n, float lr, int step,
                hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, st, p, g, m1, m2, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t sub(const cplx* a, const cplx* b, cplx* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_sub, dim3(grid1(n)), dim3(256), 0, st, a, b, out, n);
  return hipGetLastError();
}

hipError_t defect(const cplx* u, const cplx* v, size_t n, double* red, hipStream_t st) {
  hipLaunchKernelGGL(k_defect, dim3(1), dim3(256), 0, st, u, v, n, red);
  return hipGetLastError();
}

hipError_t combine(const cplx* F, const cplx* g, const float* c, const double* nrm2, cplx* out,
                   int Q, bool with_F, hipStream_t st) {
  hipLaunchKernelGGL(k_combine, dim3(grid1((size_t)3 * Q)), dim3(256), 0, st, F, g, c, nrm2, out,
                     Q, with_F ? 1 : 0);
  return hipGetLastError();
}

}  // namespace nn
}  // namespace pd
