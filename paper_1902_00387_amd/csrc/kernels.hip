// HIP kernels (gfx950, FP64) for the pseudo-spectral IMEX step of the 2.5D
// induction equation and the Parareal sweep.
//
// Model: db/dt = curl(u x b) - |k|^2/Rm b for b(x, y) e^{i kz z} on the
// 2pi-periodic square (paper Sections 1-2), Fourier collocation (Section 4),
// explicit advection/stretching and implicit diffusion (Section 4), second
// order SBDF restarted with one SBDF1 step in every slice (Section 4 notes
// multistep methods restart per slice), Parareal (Section 3, eq. parareal).
//
// Layouts in device memory (complex128, re/im interleaved):
//   state  B, H   [f][3][M][M]  compact 2/3 box, row ky = r - K, col kx = c - K
//   rows   T1, T2 [f][3][M][N]  for each retained ky, values along x
// with K = floor((N-1)/3), M = 2K + 1, f the field (slice / instance) index.
//
// One fine step of field f is two phases:
//   column phase (T1 -> T2): inverse y-FFT of each x column (M nonzero
//     inputs), physical E = u x b, forward y-FFT, keep the M box rows;
//   row phase (T2 -> B, H, T1): forward x-FFT of each box row, keep the box
//     columns, scale 1/N^2, spectral curl i k x E, SBDF update with the
//     diagonal implicit diffusion solve, inverse x-FFT of the new row.
#include "fft.hpp"
#include "launch.hpp"

namespace pd {

template <int N>
struct Geo {
  static constexpr int K = (N - 1) / 3;
  static constexpr int M = 2 * K + 1;
  static constexpr int T = N / 8;           // lanes per transform
  static constexpr int SPAN = LdsSpan<N>::value;
  // multi-launch shapes: rows per workgroup, columns per workgroup
  static constexpr int RPW = (64 / T) > 0 ? 64 / T : 1;
  static constexpr int TX = N <= 32 ? 16 : (N <= 128 ? 8 : 4);
  // single-workgroup (persistent) shape: FFT groups per 512-lane workgroup
  static constexpr int NG = 512 / T;
};

__device__ __forceinline__ int signed_k(int m, int N) { return m < N / 2 ? m : m - N; }

// Flow u = A (cos(y + py), sin(x + px), cos(x + px) + sin(y + py)) with
// (px, py) = (cos t, sin t) for the Galloway-Proctor CP flow and (0, 0) for
// the steady Roberts flow (Section 2; the paper's GP (y, z, x) relabelled as
// (x, y, z)).  cos/sin of the grid angles come from the twiddle table,
// tw[m] = (cos 2 pi m/N, -sin 2 pi m/N); the phases by angle addition.
struct FlowPhase {
  double amp, cpx, spx, cpy, spy;
};

__device__ __forceinline__ FlowPhase flow_phase(const Problem& pb, double t) {
  FlowPhase f;
  f.amp = pb.amp;
  if (pb.tdep) {
    double px = cos(t), py = sin(t);
    sincos(px, &f.spx, &f.cpx);
    sincos(py, &f.spy, &f.cpy);
  } else {
    f.cpx = 1.0;
    f.spx = 0.0;
    f.cpy = 1.0;
    f.spy = 0.0;
  }
  return f;
}

// ---------------------------------------------------------------------------
// Row phase of one box row r of one field, by one group of T lanes (lane j).
// mode 0: start of a slice (inverse transform of the state only);
// mode 1: SBDF1 update; mode 2: SBDF2 update.  last: skip the inverse.
template <int N>
__device__ __forceinline__ void row_phase(int r, bool active, int j, cplx* s, cplx* __restrict__ B,
                                          cplx* __restrict__ H, const cplx* __restrict__ T2,
                                          cplx* __restrict__ T1, const cplx* __restrict__ tw,
                                          const Problem& pb, int mode, bool last) {
  using G = Geo<N>;
  constexpr int T = G::T, K = G::K, M = G::M;
  cplx w[3][8];
  const int ky = r - K;
  if (mode == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int kx = signed_k(j + T * e, N);
        w[c][e] = (active && kx >= -K && kx <= K) ? B[(c * M + r) * M + kx + K] : czero();
      }
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int e = 0; e < 8; ++e) w[c][e] = active ? T2[(c * M + r) * N + j + T * e] : czero();
      fft<N, -1>(w[c], s, j, tw);
    }
    const double sc = 1.0 / ((double)N * (double)N);
    const double dt = pb.dt, kz = pb.kz;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kx = signed_k(j + T * e, N);
      if (active && kx >= -K && kx <= K) {
        const cplx ex = cscale(w[0][e], sc), ey = cscale(w[1][e], sc), ez = cscale(w[2][e], sc);
        // i k x E with k = (kx, ky, kz)
        const double dkx = kx, dky = ky;
        cplx nl[3];
        nl[0] = mul_i<1>(csub(cscale(ez, dky), cscale(ey, kz)));
        nl[1] = mul_i<1>(csub(cscale(ex, kz), cscale(ez, dkx)));
        nl[2] = mul_i<1>(csub(cscale(ey, dkx), cscale(ex, dky)));
        const double a = dt * (dkx * dkx + dky * dky + kz * kz) / pb.Rm;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int idx = (c * M + r) * M + kx + K;
          const cplx b = B[idx];
          cplx bn;
          if (mode == 1) {
            const double inv = 1.0 / (1.0 + a);
            bn = cscale(cadd(b, cscale(nl[c], dt)), inv);
          } else {
            const double inv = 1.0 / (1.5 + a);
            const cplx h = H[idx];
            bn = cscale(cadd(cadd(cscale(b, 2.0), cscale(nl[c], 2.0 * dt)), h), inv);
          }
          H[idx] = csub(cscale(b, -0.5), cscale(nl[c], dt));
          B[idx] = bn;
          w[c][e] = bn;
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) w[c][e] = czero();
      }
    }
  }
  if (!last) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      fft<N, 1>(w[c], s, j, tw);
      if (active) {
#pragma unroll
        for (int e = 0; e < 8; ++e) T1[(c * M + r) * N + j + T * e] = w[c][e];
      }
    }
  }
}

// Column phase of one grid column x of one field at time t.
template <int N>
__device__ __forceinline__ void col_phase(int x, bool active, int j, cplx* s,
                                          const cplx* __restrict__ T1, cplx* __restrict__ T2,
                                          const cplx* __restrict__ tw, const FlowPhase& fp) {
  using G = Geo<N>;
  constexpr int T = G::T, K = G::K, M = G::M;
  cplx w[3][8];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ky = signed_k(j + T * e, N);
      w[c][e] = (active && ky >= -K && ky <= K) ? T1[(c * M + ky + K) * N + x] : czero();
    }
    fft<N, 1>(w[c], s, j, tw);
  }
  // E = u x b at (x, y_e)
  const int xa = active ? x : 0;
  const double cx = tw[xa].re, sx = -tw[xa].im;
  const double cxp = cx * fp.cpx - sx * fp.spx;   // cos(x + px)
  const double sxp = sx * fp.cpx + cx * fp.spx;   // sin(x + px)
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int m = j + T * e;
    const double cy = tw[m].re, sy = -tw[m].im;
    const double cyp = cy * fp.cpy - sy * fp.spy;  // cos(y + py)
    const double syp = sy * fp.cpy + cy * fp.spy;  // sin(y + py)
    const double ux = fp.amp * cyp, uy = fp.amp * sxp, uz = fp.amp * (cxp + syp);
    const cplx bx = w[0][e], by = w[1][e], bz = w[2][e];
    w[0][e] = csub(cscale(bz, uy), cscale(by, uz));
    w[1][e] = csub(cscale(bx, uz), cscale(bz, ux));
    w[2][e] = csub(cscale(by, ux), cscale(bx, uy));
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    fft<N, -1>(w[c], s, j, tw);
    if (active) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int ky = signed_k(j + T * e, N);
        if (ky >= -K && ky <= K) T2[(c * M + ky + K) * N + x] = w[c][e];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Multi-launch path: one launch per phase over every (field, tile).
template <int N>
__global__ __launch_bounds__(64) void k_rows(FieldBatch fb, Problem pb, int mode, int last) {
  using G = Geo<N>;
  __shared__ cplx sm[G::RPW * G::SPAN];
  const int g = threadIdx.x / G::T, j = threadIdx.x % G::T;
  const int r = blockIdx.x * G::RPW + g;
  const size_t f = blockIdx.y;
  const size_t box = (size_t)3 * G::M * G::M, rows = (size_t)3 * G::M * N;
  row_phase<N>(r, r < G::M, j, sm + g * G::SPAN, fb.B + f * box, fb.H + f * box,
               fb.T2 + f * rows, fb.T1 + f * rows, fb.tw, pb, mode, last != 0);
}

template <int N>
__global__ __launch_bounds__(256) void k_cols(FieldBatch fb, Problem pb, int step) {
  using G = Geo<N>;
  __shared__ cplx sm[G::TX * G::SPAN];
  const int tx = threadIdx.x % G::TX, j = threadIdx.x / G::TX;
  const int x = blockIdx.x * G::TX + tx;
  const size_t f = blockIdx.y;
  const size_t rows = (size_t)3 * G::M * N;
  const FlowPhase fp = flow_phase(pb, fb.t0[f] + step * pb.dt);
  col_phase<N>(x, x < N, j, sm + tx * G::SPAN, fb.T1 + f * rows, fb.T2 + f * rows, fb.tw, fp);
}

// ---------------------------------------------------------------------------
// Single-workgroup path: one 512-lane workgroup owns a field and runs every
// step of the slice; the two phases meet at workgroup barriers, the row
// buffers stay in this workgroup's slice of global memory.
template <int N>
__device__ __forceinline__ void propagate_wg(cplx* sm, cplx* B, cplx* H, cplx* T1, cplx* T2,
                                             const cplx* tw, const Problem& pb, double t0,
                                             int nsteps) {
  using G = Geo<N>;
  constexpr int T = G::T, NG = G::NG, M = G::M;
  const int tid = threadIdx.x;
  const int rg = tid / T, rj = tid % T;   // row phase: lanes of a group adjacent
  const int cg = tid % NG, cj = tid / NG; // column phase: groups adjacent (coalesced x)
  for (int r0 = 0; r0 < M; r0 += NG)
    row_phase<N>(r0 + rg, r0 + rg < M, rj, sm + rg * G::SPAN, B, H, T2, T1, tw, pb, 0, false);
  __syncthreads();
  for (int step = 0; step < nsteps; ++step) {
    const FlowPhase fp = flow_phase(pb, t0 + step * pb.dt);
    for (int x0 = 0; x0 < N; x0 += NG)
      col_phase<N>(x0 + cg, x0 + cg < N, cj, sm + cg * G::SPAN, T1, T2, tw, fp);
    __syncthreads();
    const int mode = step == 0 ? 1 : 2;
    const bool last = step == nsteps - 1;
    for (int r0 = 0; r0 < M; r0 += NG)
      row_phase<N>(r0 + rg, r0 + rg < M, rj, sm + rg * G::SPAN, B, H, T2, T1, tw, pb, mode, last);
    __syncthreads();
  }
}

template <int N>
__global__ __launch_bounds__(512) void k_slice(FieldBatch fb, Problem pb, int nsteps) {
  using G = Geo<N>;
  __shared__ cplx sm[G::NG * G::SPAN];
  const size_t f = blockIdx.x;
  const size_t box = (size_t)3 * G::M * G::M, rows = (size_t)3 * G::M * N;
  propagate_wg<N>(sm, fb.B + f * box, fb.H + f * box, fb.T1 + f * rows, fb.T2 + f * rows, fb.tw,
                  pb, fb.t0[f], nsteps);
}

// ---------------------------------------------------------------------------
// Coarse sweep with the Parareal correction, one workgroup, slices in order
// (Section 3: the coarse correction is serial).  For each slice n:
//   g = prolong(G(restrict(U_n)))
//   mode 0 (initial coarse run):  U_{n+1} = g,                 Gold_n = g
//   mode 1 (correction):          U_{n+1} = F_n + (g - Gold_n), Gold_n = g
// Fine fields are compact [3][M][M]; the coarse box is their central
// [3][Mc][Mc] block, so restriction and zero-padding prolongation are index
// maps.  After the last slice the defect sums |U_P - Uprev_P|^2 and |U_P|^2
// are reduced in a fixed order into red[0], red[1].
template <int NC>
__global__ __launch_bounds__(512) void k_sweep(SweepArgs a, Problem pb) {
  using G = Geo<NC>;
  __shared__ cplx sm[G::NG * G::SPAN];
  __shared__ double rs[2][512];
  constexpr int Mc = G::M, Kc = G::K;
  const int M = a.M, K = (a.M - 1) / 2;
  const size_t fbox = (size_t)3 * M * M;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int n = a.n0; n < a.P; ++n) {
    const cplx* Un = a.U + n * fbox;
    for (int i = tid; i < 3 * Mc * Mc; i += nt) {
      const int c = i / (Mc * Mc), rr = (i / Mc) % Mc, cc = i % Mc;
      a.Bc[i] = Un[(c * M + rr + K - Kc) * M + cc + K - Kc];
    }
    __syncthreads();
    propagate_wg<NC>(sm, a.Bc, a.Hc, a.T1c, a.T2c, a.twc, pb, n * a.dT, a.nsteps);
    cplx* Un1 = a.U + (n + 1) * fbox;
    cplx* Go = a.Gold + n * fbox;
    const cplx* Fn = a.Fo + n * fbox;
    for (int i = tid; i < (int)fbox; i += nt) {
      const int c = i / (M * M), r = (i / M) % M, cc = i % M;
      const int dr = r - K, dc = cc - K;
      cplx g = czero();
      if (dr >= -Kc && dr <= Kc && dc >= -Kc && dc <= Kc) g = a.Bc[(c * Mc + dr + Kc) * Mc + dc + Kc];
      if (a.mode == 0) {
        Un1[i] = g;
      } else {
        Un1[i] = cadd(Fn[i], csub(g, Go[i]));
      }
      Go[i] = g;
    }
    __syncthreads();
  }
  if (a.mode != 0 && a.red != nullptr) {
    const cplx* UP = a.U + (size_t)a.P * fbox;
    double s0 = 0.0, s1 = 0.0;
    for (int i = tid; i < (int)fbox; i += nt) {
      const cplx d = csub(UP[i], a.Uprev[i]);
      s0 += d.re * d.re + d.im * d.im;
      s1 += UP[i].re * UP[i].re + UP[i].im * UP[i].im;
    }
    rs[0][tid] = s0;
    rs[1][tid] = s1;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) {
        rs[0][tid] += rs[0][tid + w];
        rs[1][tid] += rs[1][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      a.red[0] = rs[0][0];
      a.red[1] = rs[1][0];
    }
  }
}

// ---------------------------------------------------------------------------
// Layout conversion, box check, copies, norms.
__global__ void k_pack(const cplx* __restrict__ full, cplx* __restrict__ box, int N, int M,
                       size_t nfields) {
  const int K = (M - 1) / 2;
  const size_t total = nfields * 3 * (size_t)M * M;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t fc = i / ((size_t)M * M);
    const int r = (int)((i / M) % M), c = (int)(i % M);
    const int ky = r - K, kx = c - K;
    box[i] = full[fc * (size_t)N * N + (size_t)((ky + N) % N) * N + (kx + N) % N];
  }
}

__global__ void k_unpack(const cplx* __restrict__ box, cplx* __restrict__ full, int N, int M,
                         size_t nfields) {
  const int K = (M - 1) / 2;
  const size_t total = nfields * 3 * (size_t)N * N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t fc = i / ((size_t)N * N);
    const int my = (int)((i / N) % N), mx = (int)(i % N);
    const int ky = my < N / 2 ? my : my - N, kx = mx < N / 2 ? mx : mx - N;
    cplx v = czero();
    if (ky >= -K && ky <= K && kx >= -K && kx <= K)
      v = box[fc * (size_t)M * M + (size_t)(ky + K) * M + kx + K];
    full[i] = v;
  }
}

// counts nonzero coefficients outside the 2/3 box (any nonzero -> flag = 1)
__global__ void k_check_box(const cplx* __restrict__ full, int N, int K, size_t nfields,
                            int* flag) {
  const size_t total = nfields * 3 * (size_t)N * N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int my = (int)((i / N) % N), mx = (int)(i % N);
    const int ky = my < N / 2 ? my : my - N, kx = mx < N / 2 ? mx : mx - N;
    if (ky < -K || ky > K || kx < -K || kx > K) {
      const cplx v = full[i];
      if (v.re != 0.0 || v.im != 0.0) flag[0] = 1;
    }
  }
}

// per-field squared two-norm, fixed-order reduction (one workgroup a field)
__global__ __launch_bounds__(256) void k_norm2(const cplx* __restrict__ x, size_t len,
                                               double* out) {
  __shared__ double rs[256];
  const cplx* p = x + blockIdx.x * len;
  double s = 0.0;
  for (size_t i = threadIdx.x; i < len; i += 256) s += p[i].re * p[i].re + p[i].im * p[i].im;
  rs[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) rs[threadIdx.x] += rs[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = rs[0];
}

// ---------------------------------------------------------------------------
// Host launchers.
template <int N>
static hipError_t launch_rows(const FieldBatch& fb, const Problem& pb, int nfields, int mode,
                              int last, hipStream_t st) {
  using G = Geo<N>;
  dim3 grid((G::M + G::RPW - 1) / G::RPW, nfields);
  hipLaunchKernelGGL(k_rows<N>, grid, dim3(G::RPW * G::T), 0, st, fb, pb, mode, last);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_cols(const FieldBatch& fb, const Problem& pb, int nfields, int step,
                              hipStream_t st) {
  using G = Geo<N>;
  dim3 grid(N / G::TX, nfields);
  hipLaunchKernelGGL(k_cols<N>, grid, dim3(G::TX * G::T), 0, st, fb, pb, step);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_slice(const FieldBatch& fb, const Problem& pb, int nfields, int nsteps,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_slice<N>, dim3(nfields), dim3(512), 0, st, fb, pb, nsteps);
  return hipGetLastError();
}

template <int N>
static hipError_t propagate_multi(const FieldBatch& fb, const Problem& pb, int nfields,
                                  int nsteps, hipStream_t st) {
  hipError_t e = launch_rows<N>(fb, pb, nfields, 0, 0, st);
  for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
    e = launch_cols<N>(fb, pb, nfields, s, st);
    if (e == hipSuccess) e = launch_rows<N>(fb, pb, nfields, s == 0 ? 1 : 2, s == nsteps - 1, st);
  }
  return e;
}

hipError_t propagate(int N, const FieldBatch& fb, const Problem& pb, int nfields, int nsteps,
                     int path, hipStream_t st) {
  if (nfields <= 0 || nsteps <= 0) return hipSuccess;
  if (path == PATH_SINGLE_WG) {
#define CALL(n) launch_slice<n>(fb, pb, nfields, nsteps, st)
    switch (N) {
      case 16: return CALL(16);
      case 32: return CALL(32);
      case 64: return CALL(64);
      case 128: return CALL(128);
      case 256: return CALL(256);
      case 512: return CALL(512);
      default: return hipErrorInvalidValue;
    }
#undef CALL
  }
#define CALL(n) propagate_multi<n>(fb, pb, nfields, nsteps, st)
  switch (N) {
    case 16: return CALL(16);
    case 32: return CALL(32);
    case 64: return CALL(64);
    case 128: return CALL(128);
    case 256: return CALL(256);
    case 512: return CALL(512);
    default: return hipErrorInvalidValue;
  }
#undef CALL
}

hipError_t rows(int N, const FieldBatch& fb, const Problem& pb, int nfields, int mode, int last,
                hipStream_t st) {
  switch (N) {
    case 16: return launch_rows<16>(fb, pb, nfields, mode, last, st);
    case 32: return launch_rows<32>(fb, pb, nfields, mode, last, st);
    case 64: return launch_rows<64>(fb, pb, nfields, mode, last, st);
    case 128: return launch_rows<128>(fb, pb, nfields, mode, last, st);
    case 256: return launch_rows<256>(fb, pb, nfields, mode, last, st);
    case 512: return launch_rows<512>(fb, pb, nfields, mode, last, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t cols(int N, const FieldBatch& fb, const Problem& pb, int nfields, int step,
                hipStream_t st) {
  switch (N) {
    case 16: return launch_cols<16>(fb, pb, nfields, step, st);
    case 32: return launch_cols<32>(fb, pb, nfields, step, st);
    case 64: return launch_cols<64>(fb, pb, nfields, step, st);
    case 128: return launch_cols<128>(fb, pb, nfields, step, st);
    case 256: return launch_cols<256>(fb, pb, nfields, step, st);
    case 512: return launch_cols<512>(fb, pb, nfields, step, st);
    default: return hipErrorInvalidValue;
  }
}

template <int NC>
static hipError_t launch_sweep(const SweepArgs& a, const Problem& pb, hipStream_t st) {
  hipLaunchKernelGGL(k_sweep<NC>, dim3(1), dim3(512), 0, st, a, pb);
  return hipGetLastError();
}

hipError_t sweep(int Nc, const SweepArgs& a, const Problem& pb, hipStream_t st) {
  switch (Nc) {
    case 16: return launch_sweep<16>(a, pb, st);
    case 32: return launch_sweep<32>(a, pb, st);
    case 64: return launch_sweep<64>(a, pb, st);
    case 128: return launch_sweep<128>(a, pb, st);
    case 256: return launch_sweep<256>(a, pb, st);
    case 512: return launch_sweep<512>(a, pb, st);
    default: return hipErrorInvalidValue;
  }
}

static int grid_for(size_t total) {
  size_t g = (total + 255) / 256;
  if (g > 65535) g = 65535;
  return (int)(g ? g : 1);
}

hipError_t pack(const cplx* full, cplx* box, int N, int M, size_t nfields, hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for(nfields * 3 * (size_t)M * M)), dim3(256), 0, st, full,
                     box, N, M, nfields);
  return hipGetLastError();
}

hipError_t unpack(const cplx* box, cplx* full, int N, int M, size_t nfields, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(nfields * 3 * (size_t)N * N)), dim3(256), 0, st,
                     box, full, N, M, nfields);
  return hipGetLastError();
}

hipError_t check_box(const cplx* full, int N, size_t nfields, int* dflag, hipStream_t st) {
  hipLaunchKernelGGL(k_check_box, dim3(grid_for(nfields * 3 * (size_t)N * N)), dim3(256), 0, st,
                     full, N, (N - 1) / 3, nfields, dflag);
  return hipGetLastError();
}

hipError_t norms2(const cplx* x, size_t len, int nfields, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2, dim3(nfields), dim3(256), 0, st, x, len, out);
  return hipGetLastError();
}

}  // namespace pd
