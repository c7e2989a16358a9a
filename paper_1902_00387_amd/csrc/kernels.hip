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
#include <type_traits>

#include "fft.hpp"
#include "launch.hpp"

namespace pd {

template <int N, int E>
struct Geo {
  static constexpr int K = (N - 1) / 3;
  static constexpr int M = 2 * K + 1;
  static constexpr int T = N / E;           // lanes per transform (one wavefront at most)
  static constexpr int SPAN = LdsSpan<N>::value;
};

// Transform shapes of the launches (values a lane E; rows per 64-lane row
// workgroup; columns per column workgroup; lanes of the single-workgroup path).
template <int N>
struct Shape {
  static constexpr int ER = N == 512 ? 8 : 8;    // row phase, multi-launch path
  static constexpr int EC = N == 512 ? 8 : 4;    // column phase, multi-launch path
  static constexpr int TXC = N <= 64 ? 32 : (N <= 256 ? 16 : 8);  // columns per column workgroup
  static constexpr int ESR = 8;                  // single-workgroup path, rows
  static constexpr int ESC = N == 512 ? 8 : 4;   // single-workgroup path, columns
  static constexpr int LANES = 512;
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
// IMEX Runge-Kutta stages (the ARS pairs of Ascher, Ruuth & Spiteri 1997; the
// paper steps with ARS(4,4,3), its RK443, Section 4): stage i = 1..s+1 at
// time t + c_i dt solves
//   X_i = b_n + dt sum_{j<i} (a_ij N(X_j) + at_ij L X_j) + dt g L X_i,
// L = -|k|^2/Rm; the pairs are stiffly accurate, so b_{n+1} = X_{s+1}.  The
// stage sums R_i (i = 2..s+1) collect the j < i terms as the stages go;
// X_i = R_i / (1 - dt g L).  The tableau comes in the Problem.
__device__ __forceinline__ cplx cdivr(cplx a, double d) { return {a.re / d, a.im / d}; }

// End of stage JS for one mode of one component: X_JS from the state
// (JS = 1) or its stage sum, the contributions of stage JS to the later stage
// sums, and X_{JS+1}; after the last explicit stage, X_{s+1} is the new state.
template <int JS>
__device__ __forceinline__ cplx rk_update(cplx nl, double L, double d, double dt, size_t idx,
                                          size_t rs, cplx* __restrict__ B, cplx* __restrict__ R,
                                          const Problem& pb) {
  const int S = pb.rk_s;
  const cplx X = JS == 1 ? B[idx] : cdivr(R[(JS - 2) * rs + idx], d);
  cplx next = czero();
#pragma unroll
  for (int i = JS + 1; i <= 5; ++i) {
    if (i > S + 1) break;
    const double a = pb.rk_a[i - 1][JS - 1], atl = pb.rk_at[i - 1][JS - 1] * L;
    const cplx base = JS == 1 ? X : R[(i - 2) * rs + idx];
    const cplx term = {a * nl.re + atl * X.re, a * nl.im + atl * X.im};
    const cplx Ri = cadd(base, cscale(term, dt));
    if (i == JS + 1) next = cdivr(Ri, d);
    if (i == S + 1 && JS == S) B[idx] = next;
    else R[(i - 2) * rs + idx] = Ri;
  }
  return next;
}

// ---------------------------------------------------------------------------
// Row phase of one box row r of one field, by one group of T lanes (lane j)
// inside a wavefront; no workgroup barrier.
// mode 0: start of a slice (inverse transform of the state only);
// mode 1: SBDF1 update; mode 2: SBDF2 update; RKS = j > 0 (mode ROW_RK + j):
// end of Runge-Kutta stage j (stage sums in R).  last: skip the inverse.
template <int N, int E, int RKS = 0, bool PF = false, class C = cplx>
__device__ __forceinline__ void row_phase(int r, bool active, int j, C* s, C* __restrict__ B,
                                          C* __restrict__ H, const C* T2, C* T1,
                                          const C* __restrict__ tw,
                                          const Problem& pb, int mode, bool last,
                                          C* __restrict__ R = nullptr) {
  using G = Geo<N, E>;
  using Rl = decltype(C::re);  // FP64, or FP32 for the complex64 variant
  constexpr int T = G::T, K = G::K, M = G::M;
  TwRegs<N, E, C> twr;
  twr.load(j, tw);
  C w[3][E];
  const int ky = r - K;
  if (mode == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int kx = signed_k(j + T * e, N);
        w[c][e] = (active && kx >= -K && kx <= K) ? B[(c * M + r) * M + kx + K] : zero_of<C>();
      }
  } else {
    // all three components' loads are issued before the first transform;
    // with PF (SBDF) also the state and history of the lane's box modes, so
    // the row waits for global memory once (more registers: fewer waves)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) w[c][e] = active ? T2[(c * M + r) * N + j + T * e] : zero_of<C>();
    constexpr bool PRE = PF && RKS == 0;
    C bo[3][PRE ? E : 1], ho[3][PRE ? E : 1];
    if constexpr (PRE) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int kx = signed_k(j + T * e, N);
        const bool in = active && kx >= -K && kx <= K;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int idx = (c * M + r) * M + kx + K;
          bo[c][e] = in ? B[idx] : zero_of<C>();
          ho[c][e] = (in && mode != 1) ? H[idx] : zero_of<C>();
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) fft<N, E, -1>(w[c], s, j, twr);
    const Rl sc = (Rl)(1.0 / ((double)N * (double)N));
    const Rl dt = (Rl)pb.dt, kz = (Rl)pb.kz;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = signed_k(j + T * e, N);
      if (active && kx >= -K && kx <= K) {
        const C ex = cscale(w[0][e], sc), ey = cscale(w[1][e], sc), ez = cscale(w[2][e], sc);
        // i k x E with k = (kx, ky, kz)
        const Rl dkx = kx, dky = ky;
        C nl[3];
        nl[0] = mul_i<1>(csub(cscale(ez, dky), cscale(ey, kz)));
        nl[1] = mul_i<1>(csub(cscale(ex, kz), cscale(ez, dkx)));
        nl[2] = mul_i<1>(csub(cscale(ey, dkx), cscale(ex, dky)));
        if constexpr (RKS > 0) {
          const double L = -(dkx * dkx + dky * dky + kz * kz) / pb.Rm;
          const double d = 1.0 - dt * pb.rk_g * L;
          const size_t rs = (size_t)3 * M * M;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const size_t idx = (size_t)(c * M + r) * M + kx + K;
            w[c][e] = rk_update<RKS>(nl[c], L, d, dt, idx, rs, B, R, pb);
          }
        } else {
          const Rl a = dt * (dkx * dkx + dky * dky + kz * kz) / (Rl)pb.Rm;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int idx = (c * M + r) * M + kx + K;
            const C b = PRE ? bo[c][PRE ? e : 0] : B[idx];
            C bn;
            if (mode == 1) {
              const Rl inv = (Rl)1 / ((Rl)1 + a);
              bn = cscale(cadd(b, cscale(nl[c], dt)), inv);
            } else {
              const Rl inv = (Rl)1 / ((Rl)1.5 + a);
              const C h = PRE ? ho[c][PRE ? e : 0] : H[idx];
              bn = cscale(cadd(cadd(cscale(b, (Rl)2), cscale(nl[c], (Rl)2 * dt)), h), inv);
            }
            H[idx] = csub(cscale(b, (Rl)-0.5), cscale(nl[c], dt));
            B[idx] = bn;
            w[c][e] = bn;
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) w[c][e] = zero_of<C>();
      }
    }
  }
  if (!last) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      fft<N, E, 1>(w[c], s, j, twr);
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) T1[(c * M + r) * N + j + T * e] = w[c][e];
      }
    }
  }
}

// Column phase of the columns [x0, x0 + TX) of one field at time t, by the
// whole workgroup (TX = blockDim / T groups; group g owns column x0 + g).
// The three components' M x TX row blocks are staged through LDS tiles
// (pitch TX + 1) so that global loads and stores run along x and all three
// are in flight at once; once every group holds its column in registers the
// tile memory doubles as the groups' FFT exchange spans.
// (cr, sr) = (cos, sin)(theta + 2 pi e / E) from (c, s) = (cos, sin) theta,
// E = 2, 4 or 8 (e a compile-time index after unrolling): eighth turns are
// sign swaps, odd ones a scaling by sqrt(1/2).
template <int E, class Rl>
__device__ __forceinline__ void turn(int e, Rl c, Rl s, Rl& cr, Rl& sr) {
  static_assert(E == 2 || E == 4 || E == 8, "turns by eighths");
  const Rl h = (Rl)0.70710678118654752440;  // sqrt(1/2)
  switch ((e * (8 / E)) & 7) {
    case 0: cr = c; sr = s; break;
    case 1: cr = h * (c - s); sr = h * (s + c); break;
    case 2: cr = -s; sr = c; break;
    case 3: cr = -h * (c + s); sr = h * (c - s); break;
    case 4: cr = -c; sr = -s; break;
    case 5: cr = h * (s - c); sr = -h * (s + c); break;
    case 6: cr = s; sr = -c; break;
    default: cr = h * (c + s); sr = h * (s - c); break;
  }
}

// `phase()` gives the flow's phases at the step's time; the first wavefront
// evaluates it (three double-precision sincos) once the tile's loads are in
// flight, so its arithmetic overlaps their latency, and leaves it in LDS for
// the others.
template <int N, int E, int LANES, int CH, class C = cplx, class PhaseFn>
__device__ __forceinline__ void col_tile(int x0, C* tile, const C* T1, C* T2,
                                         const C* __restrict__ tw, PhaseFn phase) {
  using G = Geo<N, E>;
  using Rl = decltype(C::re);
  constexpr int T = G::T, K = G::K, M = G::M;
  constexpr int nthr = LANES;
  constexpr int TX = nthr / T < N ? nthr / T : N;
  // Tile rows R = c M + r (component c, box row r), TP slots each.  A
  // 16-byte access is served 16 lanes at a time, conflict-free when their
  // slots differ modulo 16.  Complex128 tiles are unpadded and the column is
  // XOR-swizzled by the row: the staging (16 lanes = 16/TX rows x TX
  // columns, rows aligned) and the column reads (16 consecutive rows, one
  // column) then both meet 16 distinct slots.  Complex64 tiles (8-byte
  // entries) keep one padding slot a row.
  constexpr bool SW = sizeof(C) == 16;
  constexpr int TP = SW ? TX : TX + 1;
  constexpr int RPB = TX >= 16 ? 1 : 16 / TX;  // rows a 16-slot line
  constexpr int FM = (TX < 16 ? TX : 16) - 1;
  const auto tslot = [](int R, int col) { return R * TP + (SW ? (col ^ ((R / RPB) & FM)) : col); };
  const int tid = threadIdx.x;
  const int g = tid / T, j = tid % T;
  const int x = x0 + g;
  const bool active = g < TX && x < N;
  C* s = tile + (g < TX ? g : 0) * G::SPAN;
  TwRegs<N, E, C> twr;
  twr.load(j, tw);
  // each lane issues a chunk of CH tile loads before the chunk's LDS
  // stores, so the workgroup waits for global memory once a chunk, not once
  // per element (CH bounded by register pressure).  The three components'
  // rows are consecutive rows R = c M + r of both T1 and the tile; lane
  // `tid` takes column cc = tid % TX of rows tid / TX + q RPL.
  static_assert((TX & (TX - 1)) == 0 && nthr % TX == 0, "power-of-two tile width");
  constexpr int RPL = nthr / TX;                     // rows a pass
  constexpr int NIT = (3 * M + RPL - 1) / RPL;       // passes
  const int cc = tid % TX, R0 = tid / TX;
  const bool cin = x0 + cc < N;
  __shared__ FlowPhase fsh;
  const auto share_phase = [&] {
    if (tid < 64) {
      const FlowPhase f = phase();
      if (tid == 0) fsh = f;
    }
  };
  if constexpr (SW && TX <= 64) {
    // complex128: global memory straight into LDS (global_load_lds, 16
    // bytes a lane): the 64 lanes of wave w fill the 64 consecutive slots
    // from slot (w 64 / TX + it RPL) TX on, lane l the slot of row R0 + it
    // RPL and swizzled position l % TX, so it loads the column (l % TX) ^
    // f(row) that tslot places there.  No registers, every pass in flight.
    static_assert(N % TX == 0, "whole tiles");
    typedef __attribute__((address_space(3))) void lds_void;
    const int wbase = (tid >> 6) * (64 / TX);
#pragma unroll 1
    for (int it = 0; it < NIT; ++it) {
      const int R = R0 + it * RPL;
      if (R < 3 * M) {
        const int col = cc ^ ((R / RPB) & FM);
        __builtin_amdgcn_global_load_lds(
            static_cast<const void*>(T1 + (size_t)R * N + x0 + col),
            (lds_void*)(tile + (wbase + it * RPL) * TX), 16, 0, 0);
      }
    }
    share_phase();
    __builtin_amdgcn_s_waitcnt(0);
  } else {
    share_phase();
    const C* src = T1 + (size_t)R0 * N + x0 + cc;
#pragma unroll 1
    for (int i0 = 0; i0 < NIT; i0 += CH) {
      C buf[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        const int R = R0 + (i0 + q) * RPL;
        buf[q] = (i0 + q < NIT && R < 3 * M && cin) ? src[(size_t)(i0 + q) * RPL * N] : zero_of<C>();
      }
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        const int R = R0 + (i0 + q) * RPL;
        if (i0 + q < NIT && R < 3 * M) tile[tslot(R, cc)] = buf[q];
      }
    }
  }
  __syncthreads();
  C w[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int ky = signed_k(j + T * e, N);
      w[c][e] = (active && ky >= -K && ky <= K) ? tile[tslot(c * M + ky + K, g)] : zero_of<C>();
    }
  __syncthreads();
  if (g < TX) {
#pragma unroll
    for (int c = 0; c < 3; ++c) fft<N, E, 1>(w[c], s, j, twr);
    // E = u x b at (x, y_e)
    const int xa = active ? x : 0;
    const FlowPhase fp = fsh;
    const Rl fcpx = (Rl)fp.cpx, fspx = (Rl)fp.spx, fcpy = (Rl)fp.cpy, fspy = (Rl)fp.spy;
    const Rl famp = (Rl)fp.amp;
    const Rl cx = tw[xa].re, sx = -tw[xa].im;
    const Rl cxp = cx * fcpx - sx * fspx;   // cos(x + px)
    const Rl sxp = sx * fcpx + cx * fspx;   // sin(x + px)
    // the lane's rows y_m = y_j + 2 pi e / E (m = j + T e): the angle y_j + py
    // once, then turned by the exact rotations through multiples of 2 pi / E
    const Rl cj = tw[j].re, sj = -tw[j].im;
    const Rl cjp = cj * fcpy - sj * fspy;   // cos(y_j + py)
    const Rl sjp = sj * fcpy + cj * fspy;   // sin(y_j + py)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      Rl cyp, syp;                           // cos, sin(y_m + py)
      turn<E>(e, cjp, sjp, cyp, syp);
      const Rl ux = famp * cyp, uy = famp * sxp, uz = famp * (cxp + syp);
      const C bx = w[0][e], by = w[1][e], bz = w[2][e];
      w[0][e] = csub(cscale(bz, uy), cscale(by, uz));
      w[1][e] = csub(cscale(bx, uz), cscale(bz, ux));
      w[2][e] = csub(cscale(by, ux), cscale(bx, uy));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) fft<N, E, -1>(w[c], s, j, twr);
  }
  __syncthreads();
  if (g < TX) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int ky = signed_k(j + T * e, N);
        if (ky >= -K && ky <= K) tile[tslot(c * M + ky + K, g)] = w[c][e];
      }
  }
  __syncthreads();
  C* dst = T2 + (size_t)R0 * N + x0 + cc;
#pragma unroll 1
  for (int i0 = 0; i0 < NIT; i0 += CH) {
    C buf[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int R = R0 + (i0 + q) * RPL;
      buf[q] = (i0 + q < NIT && R < 3 * M) ? tile[tslot(R, cc)] : zero_of<C>();
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int R = R0 + (i0 + q) * RPL;
      if (i0 + q < NIT && R < 3 * M && cin) dst[(size_t)(i0 + q) * RPL * N] = buf[q];
    }
  }
  __syncthreads();
}

// Column groups of a workgroup of `lanes` lanes, and the LDS entries
// col_tile needs: three component tiles, at least as large as the groups'
// FFT spans they double as.
template <int N, int E>
__host__ __device__ constexpr int col_groups(int lanes) {
  return lanes / Geo<N, E>::T < N ? lanes / Geo<N, E>::T : N;
}
template <int N, int E>
__host__ __device__ constexpr int tile_elems(int lanes) {
  const int tx = col_groups<N, E>(lanes);
  const int tiles = 3 * Geo<N, E>::M * (tx + 1);
  const int spans = tx * Geo<N, E>::SPAN;
  return tiles > spans ? tiles : spans;
}

// ---------------------------------------------------------------------------
// Multi-launch path: one launch per phase over every (field, tile).
template <int N, int E, int W, int RKS, bool PF = false, class C = cplx>
__global__ __launch_bounds__(64 * W) void k_rows(FieldBatchT<C> fb, Problem pb, int mode, int last) {
  using G = Geo<N, E>;
  constexpr int RPW = W * 64 / G::T;
  __shared__ C sm[RPW * G::SPAN];
  if (fb.count != nullptr && (int)blockIdx.y >= *fb.count) return;
  const int g = threadIdx.x / G::T, j = threadIdx.x % G::T;
  const int r = blockIdx.x * RPW + g;
  const size_t f = fb.map != nullptr ? (size_t)fb.map[blockIdx.y] : (size_t)blockIdx.y;
  const size_t box = (size_t)3 * G::M * G::M, rows = (size_t)3 * G::M * N;
  Problem p = pb;
  if (fb.fRm != nullptr) p.Rm = fb.fRm[f];
  if (fb.fkz != nullptr) p.kz = fb.fkz[f];
  row_phase<N, E, RKS, PF, C>(r, r < G::M, j, sm + g * G::SPAN, fb.B + f * box, fb.H + f * box,
                       fb.T2 + f * rows, fb.T1 + f * rows, fb.tw, p, mode, last != 0,
                       RKS > 0 ? fb.R + 4 * f * box : nullptr);
}

// Row phase with the three components of one box row on three wavefronts of
// one workgroup (wavefront c transforms component c, T = 64 lanes), so a lane
// holds one component's E values instead of three, and a SIMD holds several
// waves where the one-row kernel above fits one (N = 512).  The spectral curl
// needs all three components of a mode: after its forward transform each
// wave leaves its (unscaled) spectrum in its own LDS span, a barrier, then
// each wave reads the other two components of its lanes' modes and updates
// its own component; a second barrier keeps the spans until every wave has
// read them, before the inverse transforms reuse them.  SBDF modes 0, 1, 2
// only; per mode the same operations as row_phase in the same order.
template <int N, int E, class C = cplx>
__global__ __launch_bounds__(3 * (N / E)) void k_rows_c3(FieldBatchT<C> fb, Problem pb, int mode,
                                                         int last) {
  using G = Geo<N, E>;
  using Rl = decltype(C::re);
  constexpr int T = G::T, K = G::K, M = G::M, SP = G::SPAN;
  static_assert(T == 64, "one wavefront per component");
  __shared__ C sm[3 * SP];
  if (fb.count != nullptr && (int)blockIdx.y >= *fb.count) return;
  const int c = threadIdx.x / T, j = threadIdx.x % T;
  const int r = blockIdx.x;  // one box row a workgroup: the grid is exactly M wide
  const size_t f = fb.map != nullptr ? (size_t)fb.map[blockIdx.y] : (size_t)blockIdx.y;
  const size_t box = (size_t)3 * M * M, rows = (size_t)3 * M * N;
  C* __restrict__ B = fb.B + f * box;
  C* __restrict__ H = fb.H + f * box;
  C* T1 = fb.T1 + f * rows;
  const C* T2 = fb.T2 + f * rows;  // may be T1 itself (see FieldBatchT)
  const Rl Rm = (Rl)(fb.fRm != nullptr ? fb.fRm[f] : pb.Rm);
  const Rl kz = (Rl)(fb.fkz != nullptr ? fb.fkz[f] : pb.kz);
  C* s = sm + c * SP;
  TwRegs<N, E, C> twr;
  twr.load(j, fb.tw);
  C w[E];
  const int ky = r - K;
  if (mode == 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = signed_k(j + T * e, N);
      w[e] = (kx >= -K && kx <= K) ? B[(c * M + r) * M + kx + K] : zero_of<C>();
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) w[e] = T2[(c * M + r) * N + j + T * e];
    fft<N, E, -1>(w, s, j, twr);
#pragma unroll
    for (int e = 0; e < E; ++e) s[j + T * e] = w[e];
    // this wave's own entries of B and H, fetched before the barrier so that
    // their latency overlaps it (no other wave writes them)
    C bq[E], hq[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = signed_k(j + T * e, N);
      if (kx >= -K && kx <= K) {
        const int idx = (c * M + r) * M + kx + K;
        bq[e] = B[idx];
        hq[e] = mode == 1 ? zero_of<C>() : H[idx];
      }
    }
    __syncthreads();
    const C* s1 = sm + ((c + 1) % 3) * SP;  // the next and the one after (cyclic)
    const C* s2 = sm + ((c + 2) % 3) * SP;
    const Rl sc = (Rl)(1.0 / ((double)N * (double)N));
    const Rl dt = (Rl)pb.dt;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = signed_k(j + T * e, N);
      if (kx >= -K && kx <= K) {
        // the curl's component c does not involve E_c itself
        const C o1 = cscale(s1[j + T * e], sc), o2 = cscale(s2[j + T * e], sc);
        const Rl dkx = kx, dky = ky;
        // i k x E, component c only (x: c = 0, y: 1, z: 2)
        C nl;
        if (c == 0)  // (ey, ez) = (o1, o2)
          nl = mul_i<1>(csub(cscale(o2, dky), cscale(o1, kz)));
        else if (c == 1)  // (ez, ex) = (o1, o2)
          nl = mul_i<1>(csub(cscale(o2, kz), cscale(o1, dkx)));
        else  // (ex, ey) = (o1, o2)
          nl = mul_i<1>(csub(cscale(o2, dkx), cscale(o1, dky)));
        const Rl a = dt * (dkx * dkx + dky * dky + kz * kz) / Rm;
        const int idx = (c * M + r) * M + kx + K;
        const C b = bq[e];
        C bn;
        if (mode == 1) {
          const Rl inv = (Rl)1 / ((Rl)1 + a);
          bn = cscale(cadd(b, cscale(nl, dt)), inv);
        } else {
          const Rl inv = (Rl)1 / ((Rl)1.5 + a);
          bn = cscale(cadd(cadd(cscale(b, (Rl)2), cscale(nl, (Rl)2 * dt)), hq[e]), inv);
        }
        H[idx] = csub(cscale(b, (Rl)-0.5), cscale(nl, dt));
        B[idx] = bn;
        w[e] = bn;
      } else {
        w[e] = zero_of<C>();
      }
    }
    __syncthreads();
  }
  if (!last) {
    fft<N, E, 1>(w, s, j, twr);
#pragma unroll
    for (int e = 0; e < E; ++e) T1[(c * M + r) * N + j + T * e] = w[e];
  }
}

// Workgroups are handed to the eight XCDs round-robin by linear block index.
// When a column tile is narrower than a 128-byte line (TX < 8), the GL
// workgroups whose tiles share lines are given block indices b, b + 8, ...,
// so they run on one XCD and the line comes from HBM once (its L2 serves the
// others).  Returns the logical (tile, field row) of this block.
template <int TX>
__device__ __forceinline__ void xcd_tile(int& tile, int& row) {
  constexpr int GL = TX >= 8 ? 1 : 8 / TX;
  const int nx = gridDim.x;
  const int total = nx * gridDim.y;
  const int b = blockIdx.x + blockIdx.y * nx;
  int L = b;
  if constexpr (GL > 1) {
    if (b < total - total % (8 * GL)) {
      const int xcd = b % 8, i = b / 8;
      L = GL * (8 * (i / GL) + xcd) + i % GL;
    }
  }
  tile = L % nx;
  row = L / nx;
}

template <int N, int E, int TX, int MINW, class C = cplx>
__global__ __launch_bounds__(TX * (N / E))
__attribute__((amdgpu_waves_per_eu(MINW))) void k_cols(FieldBatchT<C> fb, Problem pb, int step,
                                                        int stage) {
  using G = Geo<N, E>;
  __shared__ C tile[tile_elems<N, E>(TX * G::T)];
  int xt, row;
  xcd_tile<TX>(xt, row);
  if (fb.count != nullptr && row >= *fb.count) return;
  const size_t f = fb.map != nullptr ? (size_t)fb.map[row] : (size_t)row;
  const size_t rows = (size_t)3 * G::M * N;
  // SBDF steps at t0 + step dt; Runge-Kutta stage `stage` at t0 + step dt + c dt
  const double t = stage == 0 ? fb.t0[f] + step * pb.dt
                              : fb.t0[f] + step * pb.dt + pb.rk_c[stage - 1] * pb.dt;
  col_tile<N, E, TX * G::T, E == 8 ? 8 : 4, C>(xt * TX, tile, fb.T1 + f * rows,
                                            fb.T2 + f * rows, fb.tw,
                                            [&] { return flow_phase(pb, t); });
}

// Persistent column phase: a grid sized to the chip's resident workgroups
// loops over every (field, column tile) of the batch; while the groups
// transform the tile staged in LDS, the lanes' loads of the next tile are
// already in flight (held in registers), so the global-memory latency of one
// tile overlaps the transforms of the previous one instead of adding to them.
// Same arithmetic, in the same order, as col_tile.
template <int N, int E, int TX>
__global__ __launch_bounds__(TX * (N / E)) void k_cols_pf(FieldBatch fb, Problem pb, int step,
                                                        int stage, int nfields) {
  using G = Geo<N, E>;
  constexpr int T = G::T, K = G::K, M = G::M;
  constexpr int LANES = TX * T;
  constexpr int TP = TX + 1, TS = M * TP;
  constexpr int NTX = N / TX;  // column tiles a field
  constexpr int RPL = LANES / TX;                // rows a pass (rows R = c M + r)
  constexpr int NIT = (3 * M + RPL - 1) / RPL;
  static_assert(N % TX == 0 && (TX & (TX - 1)) == 0, "column tiles must cover the grid");
  __shared__ cplx tile[tile_elems<N, E>(LANES)];
  const int nf = fb.count != nullptr ? *fb.count : nfields;
  const int total = nf * NTX;
  const size_t rows = (size_t)3 * M * N;
  const int tid = threadIdx.x;
  const int g = tid / T, j = tid % T;
  cplx* s = tile + g * G::SPAN;
  TwRegs<N, E> twr;
  twr.load(j, fb.tw);
  cplx buf[NIT];
  auto field_of = [&](int t) -> size_t {
    const int row = t / NTX;
    return fb.map != nullptr ? (size_t)fb.map[row] : (size_t)row;
  };
  const int cc0 = tid % TX, R0 = tid / TX;
  auto gload = [&](int t) {
    const cplx* src = fb.T1 + field_of(t) * rows + (t % NTX) * TX + (size_t)R0 * N + cc0;
#pragma unroll
    for (int q = 0; q < NIT; ++q)
      buf[q] = R0 + q * RPL < 3 * M ? src[(size_t)q * RPL * N] : czero();
  };
  int t = blockIdx.x;
  if (t < total) gload(t);
  for (; t < total; t += gridDim.x) {
    const size_t f = field_of(t);
    const int x0 = (t % NTX) * TX;
#pragma unroll
    for (int q = 0; q < NIT; ++q)
      if (R0 + q * RPL < 3 * M) tile[(R0 + q * RPL) * TP + cc0] = buf[q];
    __syncthreads();
    cplx w[3][E];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int ky = signed_k(j + T * e, N);
        w[c][e] = (ky >= -K && ky <= K) ? tile[c * TS + (ky + K) * TP + g] : czero();
      }
    __syncthreads();
    if (t + (int)gridDim.x < total) gload(t + gridDim.x);  // next tile, in flight meanwhile
    // SBDF steps at t0 + step dt; Runge-Kutta stage `stage` at t0 + step dt + c dt
    const double tt = stage == 0 ? fb.t0[f] + step * pb.dt
                                 : fb.t0[f] + step * pb.dt + pb.rk_c[stage - 1] * pb.dt;
    const FlowPhase fp = flow_phase(pb, tt);
#pragma unroll
    for (int c = 0; c < 3; ++c) fft<N, E, 1>(w[c], s, j, twr);
    const int x = x0 + g;
    const double cx = fb.tw[x].re, sx = -fb.tw[x].im;
    const double cxp = cx * fp.cpx - sx * fp.spx;   // cos(x + px)
    const double sxp = sx * fp.cpx + cx * fp.spx;   // sin(x + px)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int m = j + T * e;
      const double cy = fb.tw[m].re, sy = -fb.tw[m].im;
      const double cyp = cy * fp.cpy - sy * fp.spy;  // cos(y + py)
      const double syp = sy * fp.cpy + cy * fp.spy;  // sin(y + py)
      const double ux = fp.amp * cyp, uy = fp.amp * sxp, uz = fp.amp * (cxp + syp);
      const cplx bx = w[0][e], by = w[1][e], bz = w[2][e];
      w[0][e] = csub(cscale(bz, uy), cscale(by, uz));
      w[1][e] = csub(cscale(bx, uz), cscale(bz, ux));
      w[2][e] = csub(cscale(by, ux), cscale(bx, uy));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) fft<N, E, -1>(w[c], s, j, twr);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int ky = signed_k(j + T * e, N);
        if (ky >= -K && ky <= K) tile[c * TS + (ky + K) * TP + g] = w[c][e];
      }
    __syncthreads();
    cplx* dst = fb.T2 + f * rows + x0 + (size_t)R0 * N + cc0;
#pragma unroll
    for (int q = 0; q < NIT; ++q)
      if (R0 + q * RPL < 3 * M) dst[(size_t)q * RPL * N] = tile[(R0 + q * RPL) * TP + cc0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Single-workgroup path: one workgroup owns a field and runs every step of
// the slice; the two phases meet at workgroup barriers, the row buffers stay
// in this workgroup's slice of global memory.
template <int N>
struct SingleLds {
  static constexpr int L = Shape<N>::LANES;
  using GR = Geo<N, Shape<N>::ESR>;
  using GC = Geo<N, Shape<N>::ESC>;
  using G = GR;
  static constexpr int NGR = L / GR::T, NGC = L / GC::T;
  static constexpr int TILE = tile_elems<N, Shape<N>::ESC>(L);
  static constexpr int SPANS = NGR * GR::SPAN;
  // the row phase's spans and the column phase's tiles never coexist
  static constexpr int LDS = TILE > SPANS ? TILE : SPANS;
};

template <int N, bool RK>
__device__ __forceinline__ void propagate_wg(cplx* lds, cplx* B, cplx* H, cplx* T1,
                                             cplx* T2, const cplx* tw, const Problem& pb,
                                             double t0, int nsteps, cplx* R) {
  using S = SingleLds<N>;
  constexpr int ER = Shape<N>::ESR, EC = Shape<N>::ESC;
  constexpr int TR = S::GR::T, M = S::GR::M, NGR = S::NGR, NGC = S::NGC;
  constexpr int TX = NGC < N ? NGC : N;
  const int tid = threadIdx.x;
  const int rg = tid / TR, rj = tid % TR;
  cplx* spans = lds;
  cplx* tile = lds;
  for (int r0 = 0; r0 < M; r0 += NGR)
    row_phase<N, ER>(r0 + rg, r0 + rg < M, rj, spans + rg * S::GR::SPAN, B, H, T2, T1, tw, pb, 0,
                     false);
  __syncthreads();
  if constexpr (RK) {  // IMEX Runge-Kutta: pb.rk_s stages a step
    for (int step = 0; step < nsteps; ++step) {
      auto stage = [&](auto js_c) {
        constexpr int js = decltype(js_c)::value;
        if (js > pb.rk_s) return;
        const FlowPhase fp = flow_phase(pb, t0 + step * pb.dt + pb.rk_c[js - 1] * pb.dt);
        for (int x0 = 0; x0 < N; x0 += TX)
          col_tile<N, EC, S::L, 1>(x0, tile, T1, T2, tw, [&] { return fp; });
        const bool last = step == nsteps - 1 && js == pb.rk_s;
        for (int r0 = 0; r0 < M; r0 += NGR)
          row_phase<N, ER, js>(r0 + rg, r0 + rg < M, rj, spans + rg * S::GR::SPAN, B, H, T2, T1,
                               tw, pb, ROW_RK + js, last, R);
        __syncthreads();
      };
      stage(std::integral_constant<int, 1>{});
      stage(std::integral_constant<int, 2>{});
      stage(std::integral_constant<int, 3>{});
      stage(std::integral_constant<int, 4>{});
    }
  } else {
    for (int step = 0; step < nsteps; ++step) {
      const FlowPhase fp = flow_phase(pb, t0 + step * pb.dt);
      for (int x0 = 0; x0 < N; x0 += TX)
        col_tile<N, EC, S::L, 1>(x0, tile, T1, T2, tw, [&] { return fp; });
      const int mode = step == 0 ? 1 : 2;
      const bool last = step == nsteps - 1;
      for (int r0 = 0; r0 < M; r0 += NGR)
        row_phase<N, ER>(r0 + rg, r0 + rg < M, rj, spans + rg * S::GR::SPAN, B, H, T2, T1, tw, pb,
                         mode, last);
      __syncthreads();
    }
  }
}

template <int N, bool RK>
__global__ __launch_bounds__(Shape<N>::LANES) void k_slice(FieldBatch fb, Problem pb, int nsteps) {
  using S = SingleLds<N>;
  __shared__ cplx lds[S::LDS];
  if (fb.count != nullptr && (int)blockIdx.x >= *fb.count) return;
  const size_t f = fb.map != nullptr ? (size_t)fb.map[blockIdx.x] : (size_t)blockIdx.x;
  const size_t box = (size_t)3 * S::GR::M * S::GR::M, rows = (size_t)3 * S::GR::M * N;
  Problem p = pb;
  if (fb.fRm != nullptr) p.Rm = fb.fRm[f];
  if (fb.fkz != nullptr) p.kz = fb.fkz[f];
  propagate_wg<N, RK>(lds, fb.B + f * box, fb.H + f * box, fb.T1 + f * rows, fb.T2 + f * rows,
                      fb.tw, p, fb.t0[f], nsteps, RK ? fb.R + 4 * f * box : nullptr);
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
template <int NC, bool RK>
__global__ __launch_bounds__(Shape<NC>::LANES) void k_sweep(SweepArgs a, Problem pb) {
  using S = SingleLds<NC>;
  __shared__ cplx lds[S::LDS];
  __shared__ double rs[2][Shape<NC>::LANES];
  constexpr int Mc = S::GR::M, Kc = S::GR::K;
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
    propagate_wg<NC, RK>(lds, a.Bc, a.Hc, a.T1c, a.T2c, a.twc, pb, (a.nbase + n) * a.dT,
                         a.nsteps, a.Rc);
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
// Coarse sweep, spectral-convolution form.  Each flow of Section 2 has only
// four Fourier modes, q = (+-1, 0) and (0, +-1) (ky, kx), so the explicit term
// on the 2/3 box is the exact convolution E_k = sum_q u_q x b_{k-q}: products
// of box modes reach |k| <= K + 1 < N/2 and nothing aliases, hence this
// equals the pseudo-spectral evaluation (transform, multiply, transform,
// truncate) up to rounding.  On the serial coarse path this replaces the two
// transposes of a step by one pass over the box held in LDS.
//
// Flow coefficients (u written as sums of e^{i q.x}, px = cos t, py = sin t
// for Galloway-Proctor, 0 for Roberts):
//   q = (+1, 0): u_q = (A/2) e^{+i py} (1, 0, -i)
//   q = (-1, 0): u_q = (A/2) e^{-i py} (1, 0, +i)
//   q = (0, +1): u_q = (A/2) e^{+i px} (0, -i, 1)
//   q = (0, -1): u_q = (A/2) e^{-i px} (0, +i, 1)
// The four coefficients alpha_+- = (A/2) e^{+-i py}, beta_+- = (A/2) e^{+-i px}.
template <class C = cplx>
struct FlowModesT {
  C ap, am, bp, bm;
};
using FlowModes = FlowModesT<cplx>;

__device__ __forceinline__ FlowModes flow_modes(const Problem& pb, double t) {
  double px = 0.0, py = 0.0;
  if (pb.tdep) {
    px = cos(t);
    py = sin(t);
  }
  double spx, cpx, spy, cpy;
  sincos(px, &spx, &cpx);
  sincos(py, &spy, &cpy);
  const double h = 0.5 * pb.amp;
  FlowModes f;
  f.ap = {h * cpy, h * spy};
  f.am = {h * cpy, -h * spy};
  f.bp = {h * cpx, h * spx};
  f.bm = {h * cpx, -h * spx};
  return f;
}

constexpr int CONV_LANES = 1024;
constexpr int CONV_MMAX = 43;  // widest coarse box held in LDS (N_C = 64)
constexpr int CONV_MPL = (CONV_MMAX * CONV_MMAX + CONV_LANES - 1) / CONV_LANES;  // modes a lane

// dt N = dt i k x E with (dkx, dky, dkz) = dt k: component c is
// i (dk_{c+1} E_{c+2} - dk_{c+2} E_{c+1}).
template <class C, class Rl>
__device__ __forceinline__ void dt_curl(const C e[3], Rl dkx, Rl dky, Rl dkz, C dn[3]) {
  dn[0] = mul_i<1>(csub(cscale(e[2], dky), cscale(e[1], dkz)));
  dn[1] = mul_i<1>(csub(cscale(e[0], dkz), cscale(e[2], dkx)));
  dn[2] = mul_i<1>(csub(cscale(e[1], dkx), cscale(e[0], dky)));
}

// SBDF1 (step 0: b' = (b + dN) inv) or SBDF2 (b' = (2b + 2dN + h) inv) update
// of one component from dN = dt N; h holds the previous step's -b/2 - dN on
// entry and this step's on exit.  inv = 1 / (1 + dt|k|^2/Rm) or
// 1 / (3/2 + dt|k|^2/Rm).
template <class C, class Rl>
__device__ __forceinline__ C sbdf_update(C b, C d, C& h, Rl inv, int step) {
  C bn;
  if (step == 0) {
    bn = {(b.re + d.re) * inv, (b.im + d.im) * inv};
  } else {
    bn = {((Rl)2 * b.re + ((Rl)2 * d.re + h.re)) * inv, ((Rl)2 * b.im + ((Rl)2 * d.im + h.im)) * inv};
  }
  h = {(Rl)-0.5 * b.re - d.re, (Rl)-0.5 * b.im - d.im};
  return bn;
}

// One workgroup runs the coarse sweep of an MC x MC coarse box (a compile-time
// width, so the neighbours' offsets and the index arithmetic are constants);
// lane l owns box modes l + CONV_LANES*m (state and history in registers)
// and reads neighbours from LDS.
template <int MC, class C = cplx>
__device__ __forceinline__ void sweep_conv_lds(const SweepArgsT<C>& a, const Problem& pb, int,
                                               C* bs, double (*rs)[CONV_LANES]) {
  using Rl = decltype(C::re);
  constexpr int Mc = MC;
  constexpr int Kc = (Mc - 1) / 2;
  constexpr int nbox = Mc * Mc;
  const int M = a.M, K = (a.M - 1) / 2;
  const size_t fbox = (size_t)3 * M * M;
  const int tid = threadIdx.x, nt = blockDim.x;
  const Rl kz = (Rl)pb.kz, dt = (Rl)pb.dt, dkz = dt * kz;
  // owned modes and their implicit factors (SBDF1, SBDF2)
  int own[CONV_MPL], oky[CONV_MPL], okx[CONV_MPL];
  Rl inv1[CONV_MPL], inv2[CONV_MPL];
#pragma unroll
  for (int m = 0; m < CONV_MPL; ++m) {
    own[m] = tid + m * nt;
    const int i = own[m] < nbox ? own[m] : 0;
    oky[m] = i / Mc - Kc;
    okx[m] = i % Mc - Kc;
    const Rl kxd = okx[m], kyd = oky[m];
    const Rl aa = dt * (kxd * kxd + kyd * kyd + kz * kz) / (Rl)pb.Rm;
    inv1[m] = (Rl)1 / ((Rl)1 + aa);
    inv2[m] = (Rl)1 / ((Rl)1.5 + aa);
  }
  for (int n = a.n0; n < a.P; ++n) {
    const C* Un = a.U + n * fbox;
    C h[CONV_MPL][3];
#pragma unroll
    for (int m = 0; m < CONV_MPL; ++m)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        h[m][c] = zero_of<C>();
        if (own[m] < nbox) bs[c * nbox + own[m]] = Un[(c * M + oky[m] + K) * M + okx[m] + K];
      }
    __syncthreads();
    const double t0 = (a.nbase + n) * a.dT;
    for (int step = 0; step < a.nsteps; ++step) {
      FlowModesT<C> fm;
      if (a.ftab != nullptr && pb.tdep) {
        const double* ft = a.ftab + 4 * ((size_t)(a.nbase + n) * a.nsteps + step);
        const double h = 0.5 * pb.amp;
        fm.ap = {(Rl)(h * ft[0]), (Rl)(h * ft[1])};
        fm.am = {(Rl)(h * ft[0]), (Rl)(-h * ft[1])};
        fm.bp = {(Rl)(h * ft[2]), (Rl)(h * ft[3])};
        fm.bm = {(Rl)(h * ft[2]), (Rl)(-h * ft[3])};
      } else {
        const FlowModes fd = flow_modes(pb, t0 + step * pb.dt);
        fm.ap = {(Rl)fd.ap.re, (Rl)fd.ap.im};
        fm.am = {(Rl)fd.am.re, (Rl)fd.am.im};
        fm.bp = {(Rl)fd.bp.re, (Rl)fd.bp.im};
        fm.bm = {(Rl)fd.bm.re, (Rl)fd.bm.im};
      }
      C bn[CONV_MPL][3];
#pragma unroll
      for (int m = 0; m < CONV_MPL; ++m) {
        if (own[m] >= nbox) continue;
        // u_q x b_{k-q}, written out for the four u_q above:
        //  q = (+1,0), u = ap (1, 0, -i): ( i ap by, -i ap bx - ap bz,  ap by)
        //  q = (-1,0), u = am (1, 0, +i): (-i am by,  i am bx - am bz,  am by)
        //  q = (0,+1), u = bp (0, -i, 1): (-i bp bz - bp by,  bp bx,  i bp bx)
        //  q = (0,-1), u = bm (0, +i, 1): ( i bm bz - bm by,  bm bx, -i bm bx)
        // with the two-term entries taken as one product, e.g.
        // -i ap bx - ap bz = -ap (i bx + bz): two complex products a neighbour
        C e[3] = {zero_of<C>(), zero_of<C>(), zero_of<C>()};
        const int ky = oky[m], kx = okx[m];
        if (ky - 1 >= -Kc) {
          const int si = (ky - 1 + Kc) * Mc + kx + Kc;
          const C bx = bs[si], by = bs[nbox + si], bz = bs[2 * nbox + si];
          const C aby = cmul(fm.ap, by);
          e[0] = cadd(e[0], mul_i<1>(aby));
          e[1] = csub(e[1], cmul(fm.ap, cadd(mul_i<1>(bx), bz)));
          e[2] = cadd(e[2], aby);
        }
        if (ky + 1 <= Kc) {
          const int si = (ky + 1 + Kc) * Mc + kx + Kc;
          const C bx = bs[si], by = bs[nbox + si], bz = bs[2 * nbox + si];
          const C aby = cmul(fm.am, by);
          e[0] = csub(e[0], mul_i<1>(aby));
          e[1] = cadd(e[1], cmul(fm.am, csub(mul_i<1>(bx), bz)));
          e[2] = cadd(e[2], aby);
        }
        if (kx - 1 >= -Kc) {
          const int si = (ky + Kc) * Mc + kx - 1 + Kc;
          const C bx = bs[si], by = bs[nbox + si], bz = bs[2 * nbox + si];
          const C bbx = cmul(fm.bp, bx);
          e[0] = csub(e[0], cmul(fm.bp, cadd(mul_i<1>(bz), by)));
          e[1] = cadd(e[1], bbx);
          e[2] = cadd(e[2], mul_i<1>(bbx));
        }
        if (kx + 1 <= Kc) {
          const int si = (ky + Kc) * Mc + kx + 1 + Kc;
          const C bx = bs[si], by = bs[nbox + si], bz = bs[2 * nbox + si];
          const C bbx = cmul(fm.bm, bx);
          e[0] = cadd(e[0], cmul(fm.bm, csub(mul_i<1>(bz), by)));
          e[1] = cadd(e[1], bbx);
          e[2] = csub(e[2], mul_i<1>(bbx));
        }
        C dn[3];
        dt_curl(e, dt * (Rl)kx, dt * (Rl)ky, dkz, dn);
        const Rl inv = step == 0 ? inv1[m] : inv2[m];
#pragma unroll
        for (int c = 0; c < 3; ++c) bn[m][c] = sbdf_update(bs[c * nbox + own[m]], dn[c], h[m][c], inv, step);
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < CONV_MPL; ++m)
        if (own[m] < nbox)
#pragma unroll
          for (int c = 0; c < 3; ++c) bs[c * nbox + own[m]] = bn[m][c];
      __syncthreads();
    }
    // correction on the fine box: g = zero-padded coarse result
    C* Un1 = a.U + (n + 1) * fbox;
    C* Go = a.Gold + n * fbox;
    const C* Fn = a.Fo + n * fbox;
    for (int i = tid; i < (int)fbox; i += nt) {
      const int c = i / (M * M), r = (i / M) % M, cc = i % M;
      const int dr = r - K, dc = cc - K;
      C g = zero_of<C>();
      if (dr >= -Kc && dr <= Kc && dc >= -Kc && dc <= Kc) g = bs[c * nbox + (dr + Kc) * Mc + dc + Kc];
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
    const C* UP = a.U + (size_t)a.P * fbox;
    double s0 = 0.0, s1 = 0.0;
    for (int i = tid; i < (int)fbox; i += nt) {
      const C d = csub(UP[i], a.Uprev[i]);
      const double dr = d.re, di = d.im, ur = UP[i].re, ui = UP[i].im;
      s0 += dr * dr + di * di;
      s1 += ur * ur + ui * ui;
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


template <int MC, class C = cplx>
__global__ __launch_bounds__(CONV_LANES) void k_sweep_conv(SweepArgsT<C> a, Problem pb, int Mc) {
  __shared__ C bs[3 * MC * MC];
  __shared__ double rs[2][CONV_LANES];
  sweep_conv_lds<MC, C>(a, pb, Mc, bs, rs);
}

// Defect sums |U_P - Uprev|^2, |U_P|^2 of one sweep, fixed-order tree.
__device__ __forceinline__ void defect_sums(const SweepArgs& a, double (*rs)[CONV_LANES]) {
  const int M = a.M;
  const size_t fbox = (size_t)3 * M * M;
  const int tid = threadIdx.x, nt = blockDim.x;
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

// Coarse sweep for a box too large for LDS: the state is double-buffered in
// the job's global buffers (Bc, T1c) and the history lives in Hc; every lane
// steps the modes i = tid, tid + blockDim, ... of the box, reading the
// neighbours of the previous buffer.  Same arithmetic as sweep_conv_lds.
__device__ __forceinline__ void sweep_conv_global(const SweepArgs& a, const Problem& pb, int Mc,
                                                  double (*rs)[CONV_LANES]) {
  const int Kc = (Mc - 1) / 2;
  const int nbox = Mc * Mc;
  const int M = a.M, K = (a.M - 1) / 2;
  const size_t fbox = (size_t)3 * M * M;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double kz = pb.kz, dt = pb.dt, dkz = dt * kz;
  cplx* buf[2] = {a.Bc, a.T1c};
  cplx* Hg = a.Hc;
  for (int n = a.n0; n < a.P; ++n) {
    const cplx* Un = a.U + n * fbox;
    for (int i = tid; i < 3 * nbox; i += nt) {
      const int c = i / nbox, rem = i - c * nbox;
      const int ky = rem / Mc - Kc, kx = rem % Mc - Kc;
      buf[0][i] = Un[(c * M + ky + K) * M + kx + K];
    }
    __syncthreads();
    const double t0 = (a.nbase + n) * a.dT;
    for (int step = 0; step < a.nsteps; ++step) {
      FlowModes fm;
      if (a.ftab != nullptr && pb.tdep) {
        const double* ft = a.ftab + 4 * ((size_t)(a.nbase + n) * a.nsteps + step);
        const double h = 0.5 * pb.amp;
        fm.ap = {h * ft[0], h * ft[1]};
        fm.am = {h * ft[0], -h * ft[1]};
        fm.bp = {h * ft[2], h * ft[3]};
        fm.bm = {h * ft[2], -h * ft[3]};
      } else {
        fm = flow_modes(pb, t0 + step * dt);
      }
      const cplx* bs = buf[step & 1];
      cplx* bo = buf[(step + 1) & 1];
      for (int i = tid; i < nbox; i += nt) {
        const int ky = i / Mc - Kc, kx = i % Mc - Kc;
        cplx e[3] = {czero(), czero(), czero()};
        if (ky - 1 >= -Kc) {
          const int si = (ky - 1 + Kc) * Mc + kx + Kc;
          const cplx bx = bs[si], by = bs[nbox + si], bz = bs[2 * nbox + si];
          const cplx aby = cmul(fm.ap, by);
          e[0] = cadd(e[0], mul_i<1>(aby));
          e[1] = csub(e[1], cmul(fm.ap, cadd(mul_i<1>(bx), bz)));
          e[2] = cadd(e[2], aby);
        }
        if (ky + 1 <= Kc) {
          const int si = (ky + 1 + Kc) * Mc + kx + Kc;
          const cplx bx = bs[si], by = bs[nbox + si], bz = bs[2 * nbox + si];
          const cplx aby = cmul(fm.am, by);
          e[0] = csub(e[0], mul_i<1>(aby));
          e[1] = cadd(e[1], cmul(fm.am, csub(mul_i<1>(bx), bz)));
          e[2] = cadd(e[2], aby);
        }
        if (kx - 1 >= -Kc) {
          const int si = (ky + Kc) * Mc + kx - 1 + Kc;
          const cplx bx = bs[si], by = bs[nbox + si], bz = bs[2 * nbox + si];
          const cplx bbx = cmul(fm.bp, bx);
          e[0] = csub(e[0], cmul(fm.bp, cadd(mul_i<1>(bz), by)));
          e[1] = cadd(e[1], bbx);
          e[2] = cadd(e[2], mul_i<1>(bbx));
        }
        if (kx + 1 <= Kc) {
          const int si = (ky + Kc) * Mc + kx + 1 + Kc;
          const cplx bx = bs[si], by = bs[nbox + si], bz = bs[2 * nbox + si];
          const cplx bbx = cmul(fm.bm, bx);
          e[0] = cadd(e[0], cmul(fm.bm, csub(mul_i<1>(bz), by)));
          e[1] = cadd(e[1], bbx);
          e[2] = csub(e[2], mul_i<1>(bbx));
        }
        const double kxd = kx, kyd = ky;
        const double aa = dt * (kxd * kxd + kyd * kyd + kz * kz) / pb.Rm;
        cplx dn[3];
        dt_curl(e, dt * kx, dt * ky, dkz, dn);
        const double inv = step == 0 ? 1.0 / (1.0 + aa) : 1.0 / (1.5 + aa);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cplx hc = step == 0 ? czero() : Hg[c * nbox + i];
          bo[c * nbox + i] = sbdf_update(bs[c * nbox + i], dn[c], hc, inv, step);
          Hg[c * nbox + i] = hc;
        }
      }
      __syncthreads();
    }
    const cplx* bfin = buf[a.nsteps & 1];
    cplx* Un1 = a.U + (n + 1) * fbox;
    cplx* Go = a.Gold + n * fbox;
    const cplx* Fn = a.Fo + n * fbox;
    for (int i = tid; i < (int)fbox; i += nt) {
      const int c = i / (M * M), r = (i / M) % M, cc = i % M;
      const int dr = r - K, dc = cc - K;
      cplx g = czero();
      if (dr >= -Kc && dr <= Kc && dc >= -Kc && dc <= Kc) g = bfin[c * nbox + (dr + Kc) * Mc + dc + Kc];
      if (a.mode == 0) {
        Un1[i] = g;
      } else {
        Un1[i] = cadd(Fn[i], csub(g, Go[i]));
      }
      Go[i] = g;
    }
    __syncthreads();
  }
  if (a.mode != 0 && a.red != nullptr) defect_sums(a, rs);
}

template <bool LDS_RESIDENT>
__global__ __launch_bounds__(CONV_LANES) void k_sweep_conv_jobs(const SweepJob* jobs, int njobs) {
  __shared__ double rs[2][CONV_LANES];
  if ((int)blockIdx.x >= njobs) return;
  const SweepJob& jb = jobs[blockIdx.x];
  if (!jb.active) return;
  // keep U^{k-1}_P for the defect before the sweep overwrites it
  if (jb.a.mode != 0 && jb.a.Uprev != nullptr) {
    const size_t fbox = (size_t)3 * jb.a.M * jb.a.M;
    const cplx* UP = jb.a.U + (size_t)jb.a.P * fbox;
    cplx* Up = const_cast<cplx*>(jb.a.Uprev);
    for (int i = threadIdx.x; i < (int)fbox; i += blockDim.x) Up[i] = UP[i];
    __syncthreads();
  }
  if constexpr (LDS_RESIDENT) {
    __shared__ cplx bs[3 * CONV_MMAX * CONV_MMAX];
    // the host puts only the widths conv_lds_width accepts here
    switch (jb.Mc) {
      case 11: sweep_conv_lds<11>(jb.a, jb.pb, jb.Mc, bs, rs); break;
      case 21: sweep_conv_lds<21>(jb.a, jb.pb, jb.Mc, bs, rs); break;
      default: sweep_conv_lds<43>(jb.a, jb.pb, jb.Mc, bs, rs); break;
    }
  } else {
    sweep_conv_global(jb.a, jb.pb, jb.Mc, rs);
  }
}

// ---------------------------------------------------------------------------
// Layout conversion, box check, copies, norms.
template <class C>
__global__ void k_pack(const cplx* __restrict__ full, C* __restrict__ box, int N, int M,
                       size_t nfields) {
  using Rl = decltype(C::re);
  const int K = (M - 1) / 2;
  const size_t total = nfields * 3 * (size_t)M * M;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t fc = i / ((size_t)M * M);
    const int r = (int)((i / M) % M), c = (int)(i % M);
    const int ky = r - K, kx = c - K;
    const cplx v = full[fc * (size_t)N * N + (size_t)((ky + N) % N) * N + (kx + N) % N];
    box[i] = C{(Rl)v.re, (Rl)v.im};
  }
}

template <class C>
__global__ void k_unpack(const C* __restrict__ box, cplx* __restrict__ full, int N, int M,
                         size_t nfields) {
  const int K = (M - 1) / 2;
  const size_t total = nfields * 3 * (size_t)N * N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t fc = i / ((size_t)N * N);
    const int my = (int)((i / N) % N), mx = (int)(i % N);
    const int ky = my < N / 2 ? my : my - N, kx = mx < N / 2 ? mx : mx - N;
    cplx v = czero();
    if (ky >= -K && ky <= K && kx >= -K && kx <= K) {
      const C b = box[fc * (size_t)M * M + (size_t)(ky + K) * M + kx + K];
      v = cplx{(double)b.re, (double)b.im};
    }
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

// Fo[f] = U[uidx[f]] for the active fields f = map[row], row < *count.
__global__ __launch_bounds__(256) void k_gather(const cplx* __restrict__ U, cplx* __restrict__ Fo,
                                                const int* __restrict__ uidx,
                                                const int* __restrict__ map,
                                                const int* __restrict__ count, size_t box) {
  if ((int)blockIdx.y >= *count) return;
  const int f = map[blockIdx.y];
  const cplx* src = U + (size_t)uidx[f] * box;
  cplx* dst = Fo + (size_t)f * box;
  for (size_t i = blockIdx.x * 256 + threadIdx.x; i < box; i += (size_t)gridDim.x * 256)
    dst[i] = src[i];
}

// Multi-launch coarse sweep pieces: restriction of a compact fine box to the
// compact coarse box (its central block), and the Parareal update of one
// slice from the coarse result (zero-padded prolongation):
//   mode 0: U_{n+1} = g,  mode 1: U_{n+1} = F_n + (g - Gold_n);  Gold_n = g.
template <class C>
__global__ __launch_bounds__(256) void k_box_restrict(const C* __restrict__ Un,
                                                      C* __restrict__ Bc, int M, int Mc) {
  const int K = (M - 1) / 2, Kc = (Mc - 1) / 2;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < 3 * Mc * Mc; i += gridDim.x * 256) {
    const int c = i / (Mc * Mc), rr = (i / Mc) % Mc, cc = i % Mc;
    Bc[i] = Un[(c * M + rr + K - Kc) * M + cc + K - Kc];
  }
}

template <class C>
__global__ __launch_bounds__(256) void k_box_correct(const C* __restrict__ Bc,
                                                     const C* __restrict__ Fn,
                                                     C* __restrict__ Go, C* __restrict__ Un1,
                                                     int M, int Mc, int mode) {
  const int K = (M - 1) / 2, Kc = (Mc - 1) / 2;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < 3 * M * M; i += gridDim.x * 256) {
    const int c = i / (M * M), r = (i / M) % M, cc = i % M;
    const int dr = r - K, dc = cc - K;
    C g = zero_of<C>();
    if (dr >= -Kc && dr <= Kc && dc >= -Kc && dc <= Kc) g = Bc[(c * Mc + dr + Kc) * Mc + dc + Kc];
    Un1[i] = mode == 0 ? g : cadd(Fn[i], csub(g, Go[i]));
    Go[i] = g;
  }
}

// per-field squared two-norm, fixed-order reduction (one workgroup a field)
template <class C>
__global__ __launch_bounds__(256) void k_norm2(const C* __restrict__ x, size_t len,
                                               double* out) {
  __shared__ double rs[256];
  const C* p = x + blockIdx.x * len;
  double s = 0.0;
  for (size_t i = threadIdx.x; i < len; i += 256) {
    const double re = p[i].re, im = p[i].im;
    s += re * re + im * im;
  }
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
template <int N, int E, int W, bool PF = false>
static hipError_t launch_rows_v(const FieldBatch& fb, const Problem& pb, int nfields, int mode,
                                int last, hipStream_t st) {
  using G = Geo<N, E>;
  constexpr int RPW = W * 64 / G::T;
  dim3 grid((G::M + RPW - 1) / RPW, nfields);
  // each Runge-Kutta stage (mode ROW_RK + j) runs its own instantiation, so
  // the SBDF kernels keep their register budget
  switch (mode - ROW_RK) {
    case 1: hipLaunchKernelGGL((k_rows<N, E, W, 1>), grid, dim3(64 * W), 0, st, fb, pb, mode, last); break;
    case 2: hipLaunchKernelGGL((k_rows<N, E, W, 2>), grid, dim3(64 * W), 0, st, fb, pb, mode, last); break;
    case 3: hipLaunchKernelGGL((k_rows<N, E, W, 3>), grid, dim3(64 * W), 0, st, fb, pb, mode, last); break;
    case 4: hipLaunchKernelGGL((k_rows<N, E, W, 4>), grid, dim3(64 * W), 0, st, fb, pb, mode, last); break;
    default: hipLaunchKernelGGL((k_rows<N, E, W, 0, PF>), grid, dim3(64 * W), 0, st, fb, pb, mode, last);
  }
  return hipGetLastError();
}

// The component-split row kernel for the SBDF modes; the Runge-Kutta stage
// modes run the one-row kernel.
template <int N, int E>
static hipError_t launch_rows_c3(const FieldBatch& fb, const Problem& pb, int nfields, int mode,
                                 int last, hipStream_t st) {
  if (mode >= ROW_RK) return launch_rows_v<N, E, 1>(fb, pb, nfields, mode, last, st);
  hipLaunchKernelGGL((k_rows_c3<N, E>), dim3(Geo<N, E>::M, nfields), dim3(3 * Geo<N, E>::T), 0, st,
                     fb, pb, mode, last);
  return hipGetLastError();
}

template <int N, int E, int TX, int MINW>
static hipError_t launch_cols_v(const FieldBatch& fb, const Problem& pb, int nfields, int step,
                                int stage, hipStream_t st) {
  constexpr int T = N / E;
  dim3 grid((N + TX - 1) / TX, nfields);
  hipLaunchKernelGGL((k_cols<N, E, TX, MINW>), grid, dim3(TX * T), 0, st, fb, pb, step, stage);
  return hipGetLastError();
}

// Resident workgroups of a kernel on the current device (CUs x blocks a CU),
// the grid of a persistent launch; per device and kernel, looked up once.
template <class KernelT>
static int resident_grid(KernelT kernel, int lanes) {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] > 0) return cached[dev];
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, lanes, 0) != hipSuccess || per < 1)
    per = 1;
  cached[dev] = cus * per;
  return cached[dev];
}

template <int N, int E, int TX>
static hipError_t launch_cols_pf(const FieldBatch& fb, const Problem& pb, int nfields, int step,
                                 int stage, hipStream_t st) {
  constexpr int T = N / E;
  const int tiles = nfields * (N / TX);
  const int res = resident_grid(k_cols_pf<N, E, TX>, TX * T);
  const int grid = tiles < res ? tiles : res;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((k_cols_pf<N, E, TX>), dim3(grid), dim3(TX * T), 0, st, fb, pb, step, stage,
                     nfields);
  return hipGetLastError();
}

// ---- launch-shape variants and the per-size choice (autotuned) -----------
using RowsFn = hipError_t (*)(const FieldBatch&, const Problem&, int, int, int, hipStream_t);
using ColsFn = hipError_t (*)(const FieldBatch&, const Problem&, int, int, int, hipStream_t);
struct RowsVariant {
  int E, W;
  RowsFn fn;
};
struct ColsVariant {
  int E, TX;
  ColsFn fn;
};

// Candidates: rows -- values a lane E (8 or 4), waves a workgroup W, W < 0 for
// the form that loads the state and history with the row (faster on small
// batches, fewer waves), W = 3 for the component-split form (one row a
// workgroup, one component a wave; the default at 512); columns -- values a lane E, columns a workgroup TX
// (lanes <= 1024, LDS <= 160 KB), TX < 0 for the persistent form with |TX|
// columns a tile.
template <int N>
struct Variants;
template <>
struct Variants<16> {
  static constexpr RowsVariant rows[] = {{8, 1, launch_rows_v<16, 8, 1>}};
  static constexpr ColsVariant cols[] = {{4, 16, launch_cols_v<16, 4, 16, 4>}};
};
template <>
struct Variants<32> {
  static constexpr RowsVariant rows[] = {{8, 1, launch_rows_v<32, 8, 1>}};
  static constexpr ColsVariant cols[] = {{4, 16, launch_cols_v<32, 4, 16, 4>}};
};
template <>
struct Variants<64> {
  static constexpr RowsVariant rows[] = {{8, 1, launch_rows_v<64, 8, 1>},
                                         {8, 2, launch_rows_v<64, 8, 2>},
                                         {4, 1, launch_rows_v<64, 4, 1>},
                                         {4, 2, launch_rows_v<64, 4, 2>},
                                         {4, -1, launch_rows_v<64, 4, 1, true>}};
  static constexpr ColsVariant cols[] = {{4, 32, launch_cols_v<64, 4, 32, 4>},
                                         {4, 16, launch_cols_v<64, 4, 16, 4>},
                                         {8, 32, launch_cols_v<64, 8, 32, 2>},
                                         {8, 16, launch_cols_v<64, 8, 16, 2>},
                                         {8, -16, launch_cols_pf<64, 8, 16>},
                                         {4, -16, launch_cols_pf<64, 4, 16>}};
};
template <>
struct Variants<128> {
  static constexpr RowsVariant rows[] = {{8, 1, launch_rows_v<128, 8, 1>},
                                         {8, 2, launch_rows_v<128, 8, 2>},
                                         {4, 1, launch_rows_v<128, 4, 1>},
                                         {4, 2, launch_rows_v<128, 4, 2>},
                                         {4, -1, launch_rows_v<128, 4, 1, true>},
                                         {4, -2, launch_rows_v<128, 4, 2, true>}};
  static constexpr ColsVariant cols[] = {{4, 16, launch_cols_v<128, 4, 16, 4>},
                                         {4, 8, launch_cols_v<128, 4, 8, 4>},
                                         {8, 16, launch_cols_v<128, 8, 16, 2>},
                                         {8, 32, launch_cols_v<128, 8, 32, 2>},
                                         {8, 8, launch_cols_v<128, 8, 8, 2>},
                                         {8, -8, launch_cols_pf<128, 8, 8>},
                                         {8, -16, launch_cols_pf<128, 8, 16>},
                                         {4, -16, launch_cols_pf<128, 4, 16>}};
};
template <>
struct Variants<256> {
  static constexpr RowsVariant rows[] = {{8, 1, launch_rows_v<256, 8, 1>},
                                         {8, 2, launch_rows_v<256, 8, 2>},
                                         {4, 1, launch_rows_v<256, 4, 1>},
                                         {4, -1, launch_rows_v<256, 4, 1, true>},
                                         {4, 3, launch_rows_c3<256, 4>}};
  static constexpr ColsVariant cols[] = {{4, 16, launch_cols_v<256, 4, 16, 4>},
                                         {4, 8, launch_cols_v<256, 4, 8, 4>},
                                         {8, 16, launch_cols_v<256, 8, 16, 2>},
                                         {8, 8, launch_cols_v<256, 8, 8, 2>},
                                         {8, -8, launch_cols_pf<256, 8, 8>},
                                         {4, -8, launch_cols_pf<256, 4, 8>}};
};
template <>
struct Variants<512> {
  static constexpr RowsVariant rows[] = {{8, 3, launch_rows_c3<512, 8>},
                                         {8, 1, launch_rows_v<512, 8, 1>},
                                         {8, 2, launch_rows_v<512, 8, 2>}};
  static constexpr ColsVariant cols[] = {{8, 4, launch_cols_v<512, 8, 4, 2>},
                                         {8, 8, launch_cols_v<512, 8, 8, 2>},
                                         {8, -4, launch_cols_pf<512, 8, 4>}};
};

static int size_slot(int N) {
  switch (N) {
    case 16: return 0;
    case 32: return 1;
    case 64: return 2;
    case 128: return 3;
    case 256: return 4;
    case 512: return 5;
    default: return -1;
  }
}
// chosen variant per size (process-wide; index 0 = default)
static int g_rows_choice[6] = {0, 0, 0, 0, 0, 0};
static int g_cols_choice[6] = {0, 0, 0, 0, 0, 0};

// a batch's own choice (FieldBatch::rows_v / cols_v, if valid) before the
// process-wide one
template <int N>
static hipError_t launch_rows(const FieldBatch& fb, const Problem& pb, int nfields, int mode,
                              int last, hipStream_t st) {
  constexpr int nv = (int)(sizeof(Variants<N>::rows) / sizeof(RowsVariant));
  const int v = fb.rows_v >= 0 && fb.rows_v < nv ? fb.rows_v : g_rows_choice[size_slot(N)];
  return Variants<N>::rows[v].fn(fb, pb, nfields, mode, last, st);
}

template <int N>
static hipError_t launch_cols(const FieldBatch& fb, const Problem& pb, int nfields, int step,
                              hipStream_t st, int stage = 0) {
  constexpr int nv = (int)(sizeof(Variants<N>::cols) / sizeof(ColsVariant));
  const int v = fb.cols_v >= 0 && fb.cols_v < nv ? fb.cols_v : g_cols_choice[size_slot(N)];
  return Variants<N>::cols[v].fn(fb, pb, nfields, step, stage, st);
}

template <int N>
static int nvariants(int kind) {
  return kind == 0 ? (int)(sizeof(Variants<N>::rows) / sizeof(RowsVariant))
                   : (int)(sizeof(Variants<N>::cols) / sizeof(ColsVariant));
}

int variant_count(int N, int kind) {
  switch (N) {
    case 16: return nvariants<16>(kind);
    case 32: return nvariants<32>(kind);
    case 64: return nvariants<64>(kind);
    case 128: return nvariants<128>(kind);
    case 256: return nvariants<256>(kind);
    case 512: return nvariants<512>(kind);
    default: return 0;
  }
}

template <int N>
static void describe(int kind, int v, int* a, int* b) {
  if (kind == 0) {
    *a = Variants<N>::rows[v].E;
    *b = Variants<N>::rows[v].W;
  } else {
    *a = Variants<N>::cols[v].E;
    *b = Variants<N>::cols[v].TX;
  }
}

int variant_describe(int N, int kind, int v, int* a, int* b) {
  if (v < 0 || v >= variant_count(N, kind)) return -1;
  switch (N) {
    case 16: describe<16>(kind, v, a, b); break;
    case 32: describe<32>(kind, v, a, b); break;
    case 64: describe<64>(kind, v, a, b); break;
    case 128: describe<128>(kind, v, a, b); break;
    case 256: describe<256>(kind, v, a, b); break;
    case 512: describe<512>(kind, v, a, b); break;
    default: return -1;
  }
  return 0;
}

int variant_select(int N, int rows_v, int cols_v) {
  const int sl = size_slot(N);
  if (sl < 0 || rows_v < 0 || rows_v >= variant_count(N, 0) || cols_v < 0 ||
      cols_v >= variant_count(N, 1))
    return -1;
  g_rows_choice[sl] = rows_v;
  g_cols_choice[sl] = cols_v;
  return 0;
}

void variant_current(int N, int* rows_v, int* cols_v) {
  const int sl = size_slot(N);
  *rows_v = sl < 0 ? 0 : g_rows_choice[sl];
  *cols_v = sl < 0 ? 0 : g_cols_choice[sl];
}

template <int N>
static hipError_t launch_slice(const FieldBatch& fb, const Problem& pb, int nfields, int nsteps,
                               hipStream_t st) {
  if (pb.scheme == 1)
    hipLaunchKernelGGL((k_slice<N, true>), dim3(nfields), dim3(Shape<N>::LANES), 0, st, fb, pb,
                       nsteps);
  else
    hipLaunchKernelGGL((k_slice<N, false>), dim3(nfields), dim3(Shape<N>::LANES), 0, st, fb, pb,
                       nsteps);
  return hipGetLastError();
}

template <int N>
static hipError_t propagate_multi(const FieldBatch& fb, const Problem& pb, int nfields,
                                  int nsteps, hipStream_t st) {
  hipError_t e = launch_rows<N>(fb, pb, nfields, 0, 0, st);
  if (pb.scheme == 1) {  // Runge-Kutta: one column and one row launch a stage
    for (int s = 0; s < nsteps && e == hipSuccess; ++s)
      for (int j = 1; j <= pb.rk_s && e == hipSuccess; ++j) {
        e = launch_cols<N>(fb, pb, nfields, s, st, j);
        if (e == hipSuccess)
          e = launch_rows<N>(fb, pb, nfields, ROW_RK + j, s == nsteps - 1 && j == pb.rk_s, st);
      }
    return e;
  }
  for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
    e = launch_cols<N>(fb, pb, nfields, s, st);
    if (e == hipSuccess) e = launch_rows<N>(fb, pb, nfields, s == 0 ? 1 : 2, s == nsteps - 1, st);
  }
  return e;
}

// Two halves of the batch on two streams, the second started half a step
// late, so that one half's column phase (transform-heavy) overlaps the
// other half's row phase (memory-heavy).
template <int N>
static hipError_t propagate_multi2(const FieldBatch& fb, const Problem& pb, int nfields,
                                   int nsteps, hipStream_t st, hipStream_t st2, hipEvent_t* ev) {
  const int h = (nfields + 1) / 2;
  FieldBatch fa = fb, fbb = fb;
  const size_t box = (size_t)3 * Geo<N, 8>::M * Geo<N, 8>::M, rows = (size_t)3 * Geo<N, 8>::M * N;
  fbb.B += h * box;
  fbb.H += h * box;
  fbb.T1 += h * rows;
  fbb.T2 += h * rows;
  fbb.t0 += h;
  hipError_t e;
  if ((e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(st2, ev[0], 0)) != hipSuccess) return e;
  if ((e = launch_rows<N>(fa, pb, h, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_cols<N>(fa, pb, h, 0, st)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(st2, ev[1], 0)) != hipSuccess) return e;
  if ((e = launch_rows<N>(fbb, pb, nfields - h, 0, 0, st2)) != hipSuccess) return e;
  for (int s = 0; s < nsteps; ++s) {
    if (s > 0 && (e = launch_cols<N>(fa, pb, h, s, st)) != hipSuccess) return e;
    if ((e = launch_rows<N>(fa, pb, h, s == 0 ? 1 : 2, s == nsteps - 1, st)) != hipSuccess) return e;
    if ((e = launch_cols<N>(fbb, pb, nfields - h, s, st2)) != hipSuccess) return e;
    if ((e = launch_rows<N>(fbb, pb, nfields - h, s == 0 ? 1 : 2, s == nsteps - 1, st2)) != hipSuccess)
      return e;
  }
  if ((e = hipEventRecord(ev[2], st2)) != hipSuccess) return e;
  return hipStreamWaitEvent(st, ev[2], 0);
}

hipError_t propagate2(int N, const FieldBatch& fb, const Problem& pb, int nfields, int nsteps,
                      hipStream_t st, hipStream_t st2, hipEvent_t* ev) {
  if (nfields <= 0 || nsteps <= 0) return hipSuccess;
  if (nfields < 2 || pb.scheme != 0) return propagate(N, fb, pb, nfields, nsteps, PATH_MULTI, st);
  switch (N) {
    case 16: return propagate_multi2<16>(fb, pb, nfields, nsteps, st, st2, ev);
    case 32: return propagate_multi2<32>(fb, pb, nfields, nsteps, st, st2, ev);
    case 64: return propagate_multi2<64>(fb, pb, nfields, nsteps, st, st2, ev);
    case 128: return propagate_multi2<128>(fb, pb, nfields, nsteps, st, st2, ev);
    case 256: return propagate_multi2<256>(fb, pb, nfields, nsteps, st, st2, ev);
    case 512: return propagate_multi2<512>(fb, pb, nfields, nsteps, st, st2, ev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t propagate(int N, const FieldBatch& fb, const Problem& pb, int nfields, int nsteps,
                     int path, hipStream_t st) {
  if (nfields <= 0 || nsteps <= 0) return hipSuccess;
  if (pb.scheme == 1 && (fb.R == nullptr || pb.rk_s < 1 || pb.rk_s > 4))
    return hipErrorInvalidValue;  // stage sums and a tableau needed
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
  if (pb.scheme == 1)
    hipLaunchKernelGGL((k_sweep<NC, true>), dim3(1), dim3(Shape<NC>::LANES), 0, st, a, pb);
  else
    hipLaunchKernelGGL((k_sweep<NC, false>), dim3(1), dim3(Shape<NC>::LANES), 0, st, a, pb);
  return hipGetLastError();
}

hipError_t sweep_conv(int Nc, const SweepArgs& a, const Problem& pb, hipStream_t st) {
  const int Mc = 2 * ((Nc - 1) / 3) + 1;
  if (!conv_lds_width(Mc) || pb.scheme != 0) return hipErrorInvalidValue;  // SBDF2 only
  switch (Mc) {
    case 11: hipLaunchKernelGGL(k_sweep_conv<11>, dim3(1), dim3(CONV_LANES), 0, st, a, pb, Mc); break;
    case 21: hipLaunchKernelGGL(k_sweep_conv<21>, dim3(1), dim3(CONV_LANES), 0, st, a, pb, Mc); break;
    case 43: hipLaunchKernelGGL(k_sweep_conv<43>, dim3(1), dim3(CONV_LANES), 0, st, a, pb, Mc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t sweep_conv_jobs(const SweepJob* d_jobs, int njobs, bool lds_resident, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  if (lds_resident)
    hipLaunchKernelGGL(k_sweep_conv_jobs<true>, dim3(njobs), dim3(CONV_LANES), 0, st, d_jobs, njobs);
  else
    hipLaunchKernelGGL(k_sweep_conv_jobs<false>, dim3(njobs), dim3(CONV_LANES), 0, st, d_jobs, njobs);
  return hipGetLastError();
}

hipError_t sweep(int Nc, const SweepArgs& a, const Problem& pb, hipStream_t st) {
  if (pb.scheme == 1 && (a.Rc == nullptr || pb.rk_s < 1 || pb.rk_s > 4))
    return hipErrorInvalidValue;  // stage sums and a tableau needed
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

hipError_t sweep_multi(int Nc, const SweepArgs& a, const Problem& pb, hipStream_t st) {
  if (pb.scheme == 1 && (a.Rc == nullptr || pb.rk_s < 1 || pb.rk_s > 4)) return hipErrorInvalidValue;
  if (a.t0s == nullptr) return hipErrorInvalidValue;
  const int Mc = 2 * ((Nc - 1) / 3) + 1;
  const size_t fbox = (size_t)3 * a.M * a.M;
  const int gb = (int)((3 * Mc * Mc + 255) / 256), gf = (int)((fbox + 255) / 256);
  FieldBatch fb;
  fb.B = a.Bc;
  fb.H = a.Hc;
  fb.T1 = a.T1c;
  fb.T2 = a.T2c;
  fb.tw = a.twc;
  fb.R = a.Rc;
  for (int n = a.n0; n < a.P; ++n) {
    hipLaunchKernelGGL(k_box_restrict<cplx>, dim3(gb < 1024 ? gb : 1024), dim3(256), 0, st,
                       a.U + n * fbox, a.Bc, a.M, Mc);
    fb.t0 = a.t0s + n;
    hipError_t e = propagate(Nc, fb, pb, 1, a.nsteps, PATH_MULTI, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_box_correct<cplx>, dim3(gf < 1024 ? gf : 1024), dim3(256), 0, st, a.Bc,
                       a.Fo + n * fbox, a.Gold + n * fbox, a.U + (n + 1) * fbox, a.M, Mc, a.mode);
  }
  return hipGetLastError();
}

static int grid_for(size_t total) {
  size_t g = (total + 255) / 256;
  if (g > 65535) g = 65535;
  return (int)(g ? g : 1);
}

hipError_t pack(const cplx* full, cplx* box, int N, int M, size_t nfields, hipStream_t st) {
  hipLaunchKernelGGL(k_pack<cplx>, dim3(grid_for(nfields * 3 * (size_t)M * M)), dim3(256), 0, st, full,
                     box, N, M, nfields);
  return hipGetLastError();
}

hipError_t unpack(const cplx* box, cplx* full, int N, int M, size_t nfields, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack<cplx>, dim3(grid_for(nfields * 3 * (size_t)N * N)), dim3(256), 0, st,
                     box, full, N, M, nfields);
  return hipGetLastError();
}

hipError_t check_box(const cplx* full, int N, size_t nfields, int* dflag, hipStream_t st) {
  hipLaunchKernelGGL(k_check_box, dim3(grid_for(nfields * 3 * (size_t)N * N)), dim3(256), 0, st,
                     full, N, (N - 1) / 3, nfields, dflag);
  return hipGetLastError();
}

hipError_t gather(const cplx* U, cplx* Fo, const int* uidx, const int* map, const int* count,
                  int rows, size_t box, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  dim3 grid((unsigned)((box + 255) / 256 < 64 ? (box + 255) / 256 : 64), rows);
  hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, st, U, Fo, uidx, map, count, box);
  return hipGetLastError();
}

hipError_t norms2(const cplx* x, size_t len, int nfields, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2<cplx>, dim3(nfields), dim3(256), 0, st, x, len, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The complex64 variant: the same kernels on FP32 values (SBDF2 fine and
// coarse steps, the multi-launch path), one launch shape per grid size.
template <int N>
struct ShapeF {
  static constexpr int RE = 8, RW = 1;  // rows: values a lane, waves a workgroup
  static constexpr int CE = N >= 128 ? 8 : 4;
  static constexpr int CTX = N >= 256 ? 8 : (N == 128 ? 16 : (N == 64 ? 32 : 16));
};

template <int N>
static hipError_t launch_rows_f(const FieldBatchF& fb, const Problem& pb, int nfields, int mode,
                                int last, hipStream_t st) {
  constexpr int E = ShapeF<N>::RE, W = ShapeF<N>::RW;
  using G = Geo<N, E>;
  constexpr int RPW = W * 64 / G::T;
  if (mode >= ROW_RK) return hipErrorInvalidValue;  // SBDF2 only
  dim3 grid((G::M + RPW - 1) / RPW, nfields);
  hipLaunchKernelGGL((k_rows<N, E, W, 0, false, cplxf>), grid, dim3(64 * W), 0, st, fb, pb, mode,
                     last);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_cols_f(const FieldBatchF& fb, const Problem& pb, int nfields, int step,
                                hipStream_t st) {
  constexpr int E = ShapeF<N>::CE, TX = ShapeF<N>::CTX, T = N / E;
  dim3 grid((N + TX - 1) / TX, nfields);
  hipLaunchKernelGGL((k_cols<N, E, TX, 4, cplxf>), grid, dim3(TX * T), 0, st, fb, pb, step, 0);
  return hipGetLastError();
}

template <int N>
static hipError_t propagate_f(const FieldBatchF& fb, const Problem& pb, int nfields, int nsteps,
                              hipStream_t st) {
  hipError_t e = launch_rows_f<N>(fb, pb, nfields, 0, 0, st);
  for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
    e = launch_cols_f<N>(fb, pb, nfields, s, st);
    if (e == hipSuccess) e = launch_rows_f<N>(fb, pb, nfields, s == 0 ? 1 : 2, s == nsteps - 1, st);
  }
  return e;
}

#define PD_SIZE_SWITCH(CALL)          \
  switch (N) {                        \
    case 16: return CALL(16);         \
    case 32: return CALL(32);         \
    case 64: return CALL(64);         \
    case 128: return CALL(128);       \
    case 256: return CALL(256);       \
    case 512: return CALL(512);       \
    default: return hipErrorInvalidValue; \
  }

hipError_t propagate(int N, const FieldBatchF& fb, const Problem& pb, int nfields, int nsteps,
                     int, hipStream_t st) {
  if (nfields <= 0 || nsteps <= 0) return hipSuccess;
  if (pb.scheme != 0) return hipErrorInvalidValue;
#define CALL(n) propagate_f<n>(fb, pb, nfields, nsteps, st)
  PD_SIZE_SWITCH(CALL)
#undef CALL
}

hipError_t rows(int N, const FieldBatchF& fb, const Problem& pb, int nfields, int mode, int last,
                hipStream_t st) {
#define CALL(n) launch_rows_f<n>(fb, pb, nfields, mode, last, st)
  PD_SIZE_SWITCH(CALL)
#undef CALL
}

hipError_t cols(int N, const FieldBatchF& fb, const Problem& pb, int nfields, int step,
                hipStream_t st) {
#define CALL(n) launch_cols_f<n>(fb, pb, nfields, step, st)
  PD_SIZE_SWITCH(CALL)
#undef CALL
}
#undef PD_SIZE_SWITCH

hipError_t sweep_conv(int Nc, const SweepArgsF& a, const Problem& pb, hipStream_t st) {
  const int Mc = 2 * ((Nc - 1) / 3) + 1;
  if (!conv_lds_width(Mc) || pb.scheme != 0) return hipErrorInvalidValue;
  switch (Mc) {
    case 11: hipLaunchKernelGGL((k_sweep_conv<11, cplxf>), dim3(1), dim3(CONV_LANES), 0, st, a, pb, Mc); break;
    case 21: hipLaunchKernelGGL((k_sweep_conv<21, cplxf>), dim3(1), dim3(CONV_LANES), 0, st, a, pb, Mc); break;
    case 43: hipLaunchKernelGGL((k_sweep_conv<43, cplxf>), dim3(1), dim3(CONV_LANES), 0, st, a, pb, Mc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t sweep_multi(int Nc, const SweepArgsF& a, const Problem& pb, hipStream_t st) {
  if (pb.scheme != 0 || a.t0s == nullptr) return hipErrorInvalidValue;
  const int Mc = 2 * ((Nc - 1) / 3) + 1;
  const size_t fbox = (size_t)3 * a.M * a.M;
  const int gb = (int)((3 * Mc * Mc + 255) / 256), gf = (int)((fbox + 255) / 256);
  FieldBatchF fb;
  fb.B = a.Bc;
  fb.H = a.Hc;
  fb.T1 = a.T1c;
  fb.T2 = a.T2c;
  fb.tw = a.twc;
  for (int n = a.n0; n < a.P; ++n) {
    hipLaunchKernelGGL(k_box_restrict<cplxf>, dim3(gb < 1024 ? gb : 1024), dim3(256), 0, st,
                       a.U + n * fbox, a.Bc, a.M, Mc);
    fb.t0 = a.t0s + n;
    hipError_t e = propagate(Nc, fb, pb, 1, a.nsteps, PATH_MULTI, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_box_correct<cplxf>, dim3(gf < 1024 ? gf : 1024), dim3(256), 0, st, a.Bc,
                       a.Fo + n * fbox, a.Gold + n * fbox, a.U + (n + 1) * fbox, a.M, Mc, a.mode);
  }
  return hipGetLastError();
}

hipError_t pack(const cplx* full, cplxf* box, int N, int M, size_t nfields, hipStream_t st) {
  hipLaunchKernelGGL(k_pack<cplxf>, dim3(grid_for(nfields * 3 * (size_t)M * M)), dim3(256), 0, st,
                     full, box, N, M, nfields);
  return hipGetLastError();
}

hipError_t unpack(const cplxf* box, cplx* full, int N, int M, size_t nfields, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack<cplxf>, dim3(grid_for(nfields * 3 * (size_t)N * N)), dim3(256), 0,
                     st, box, full, N, M, nfields);
  return hipGetLastError();
}

hipError_t norms2(const cplxf* x, size_t len, int nfields, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2<cplxf>, dim3(nfields), dim3(256), 0, st, x, len, out);
  return hipGetLastError();
}

// red[0] = |u - v|^2, red[1] = |u|^2, one workgroup, fixed order (FP64 sums)
__global__ __launch_bounds__(256) void k_defect_f(const cplxf* __restrict__ u,
                                                  const cplxf* __restrict__ v, size_t n,
                                                  double* __restrict__ red) {
  __shared__ double rs[2][256];
  double s0 = 0.0, s1 = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 256) {
    const double dr = (double)u[i].re - (double)v[i].re, di = (double)u[i].im - (double)v[i].im;
    const double ur = u[i].re, ui = u[i].im;
    s0 += dr * dr + di * di;
    s1 += ur * ur + ui * ui;
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

hipError_t defect2(const cplxf* u, const cplxf* v, size_t n, double* red, hipStream_t st) {
  hipLaunchKernelGGL(k_defect_f, dim3(1), dim3(256), 0, st, u, v, n, red);
  return hipGetLastError();
}

}  // namespace pd
