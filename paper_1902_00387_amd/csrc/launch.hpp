// Internal interface between the C-ABI runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "fft.hpp"

namespace pd {

enum { PATH_MULTI = 0, PATH_SINGLE_WG = 1 };
// row-phase modes: 0 start of a slice, 1 SBDF1, 2 SBDF2, ROW_RK + j end of
// ARS(4,4,3) stage j = 1..4
enum { ROW_RK = 10 };

// Per-launch physical and step parameters.
struct Problem {
  double Rm;   // magnetic Reynolds number
  double kz;   // wavenumber of the e^{i kz z} ansatz
  double dt;   // step size
  double amp;  // flow amplitude: 0 (none), 1 (Roberts), sqrt(3/2) (GP)
  int tdep;    // 1: Galloway-Proctor phases (cos t, sin t); 0: steady
  int scheme = 0;  // 0: SBDF1-started SBDF2; 1: IMEX Runge-Kutta (tableau below)
  // IMEX Runge-Kutta pair with rk_s explicit stages (1, 2 or 4), stiffly
  // accurate: stage i = 1..rk_s+1 at t + rk_c[i-1] dt uses rk_a[i-1][j-1]
  // (explicit) and rk_at[i-1][j-1] (implicit) for j < i and the implicit
  // diagonal rk_g; the new state is stage rk_s + 1
  int rk_s = 0;
  double rk_g = 0.0;
  double rk_c[4] = {0.0, 0.0, 0.0, 0.0};
  double rk_a[5][4] = {};
  double rk_at[5][4] = {};
};

// A batch of fields stepped together (all of grid size N), complex128 (C =
// cplx) or complex64 (C = cplxf).
template <class C>
struct FieldBatchT {
  C* B = nullptr;              // [f][3][M][M] state (in: start value, out: end value)
  C* H = nullptr;              // [f][3][M][M] SBDF2 history workspace
  // [f][3][M][N] row workspaces: the row phase reads T2 and writes T1, the
  // column phase reads T1 and writes T2.  Each phase reads a row (a column
  // tile) before it writes the same row (tile), and no other workgroup touches
  // it, so T2 may be T1 itself: the library's fine buffers work in place,
  // which keeps a slice's buffers a third smaller in the last-level cache.
  C* T1 = nullptr;
  C* T2 = nullptr;
  const double* t0 = nullptr;  // [f] start time of each field's slice
  const C* tw = nullptr;       // [N] twiddles e^{-2 pi i m/N}
  C* R = nullptr;              // [f][4][3][M][M] Runge-Kutta stage sums (scheme 1 only)
  // optional (null: use the Problem's scalars / the identity map)
  const double* fRm = nullptr;  // [f] per-field Rm
  const double* fkz = nullptr;  // [f] per-field kz
  const int* map = nullptr;     // [launch row] field index; rows >= *count exit at once
  const int* count = nullptr;   // device count of active launch rows
  int rows_v = -1, cols_v = -1;  // launch-shape variants for this batch (-1: process-wide choice)
};
using FieldBatch = FieldBatchT<cplx>;
using FieldBatchF = FieldBatchT<cplxf>;

// One serial coarse sweep (complex128, or complex64 with C = cplxf).
template <class C>
struct SweepArgsT {
  C* U = nullptr;               // [P+1][3][M][M] slice-boundary states (fine, compact)
  const C* Fo = nullptr;        // [P][3][M][M] fine results F(U^{k-1}_n)
  C* Gold = nullptr;            // [P][3][M][M] previous coarse results
  const C* Uprev = nullptr;     // [3][M][M] U^{k-1}_P (defect; the batched sweep fills it)
  C *Bc = nullptr, *Hc = nullptr, *T1c = nullptr, *T2c = nullptr;  // coarse workspaces
  C* Rc = nullptr;              // [4][3][Mc][Mc] coarse Runge-Kutta stage sums (scheme 1)
  const double* t0s = nullptr;  // [P] slice start times (multi-launch sweep only)
  const C* twc = nullptr;       // coarse twiddles
  double* red = nullptr;        // [2] defect sums (may be null)
  const double* ftab = nullptr; // [P][nsteps][4] cos(py), sin(py), cos(px), sin(px) of the
                      // flow phases at every coarse step time (time-dependent flow)
  double dT;          // slice length
  int M;              // fine box width
  int P, n0;          // slices, first slice swept
  int nsteps;         // coarse steps per slice
  int mode;           // 0: initial coarse run, 1: correction
  int nbase = 0;      // absolute index of local slice 0 (start time (nbase + n) dT)
};
using SweepArgs = SweepArgsT<cplx>;
using SweepArgsF = SweepArgsT<cplxf>;

struct SweepJob {
  SweepArgs a;
  Problem pb;
  int Mc;      // coarse box width
  int active;  // 0: skip (instance converged)
};

hipError_t propagate(int N, const FieldBatch& fb, const Problem& pb, int nfields, int nsteps,
                     int path, hipStream_t st);
// the complex64 variant: FP32 kernels, SBDF2, the default launch shapes
hipError_t propagate(int N, const FieldBatchF& fb, const Problem& pb, int nfields, int nsteps,
                     int path, hipStream_t st);
hipError_t rows(int N, const FieldBatchF& fb, const Problem& pb, int nfields, int mode, int last,
                hipStream_t st);
hipError_t cols(int N, const FieldBatchF& fb, const Problem& pb, int nfields, int step,
                hipStream_t st);
hipError_t sweep_conv(int Nc, const SweepArgsF& a, const Problem& pb, hipStream_t st);
hipError_t sweep_multi(int Nc, const SweepArgsF& a, const Problem& pb, hipStream_t st);
hipError_t pack(const cplx* full, cplxf* box, int N, int M, size_t nfields, hipStream_t st);
hipError_t unpack(const cplxf* box, cplx* full, int N, int M, size_t nfields, hipStream_t st);
hipError_t norms2(const cplxf* x, size_t len, int nfields, double* out, hipStream_t st);
// red[0] = |u - v|^2, red[1] = |u|^2 (one workgroup, fixed order)
hipError_t defect2(const cplxf* u, const cplxf* v, size_t n, double* red, hipStream_t st);
// single launches of the two phases of the multi-launch path
hipError_t rows(int N, const FieldBatch& fb, const Problem& pb, int nfields, int mode, int last,
                hipStream_t st);
hipError_t cols(int N, const FieldBatch& fb, const Problem& pb, int nfields, int step,
                hipStream_t st);
// the multi-launch path with the batch halved over two streams, the second
// half started half a step later (ev: three events owned by the caller;
// fields must not be remapped: fb.map and fb.count must be null)
hipError_t propagate2(int N, const FieldBatch& fb, const Problem& pb, int nfields, int nsteps,
                      hipStream_t st, hipStream_t st2, hipEvent_t* ev);
hipError_t sweep(int Nc, const SweepArgs& a, const Problem& pb, hipStream_t st);
// Host-driven coarse sweep: per slice a restriction kernel, the multi-launch
// propagator on the coarse grid (one field; SBDF2 or Runge-Kutta) and the
// Parareal update kernel; no defect sums (the caller reduces them)
hipError_t sweep_multi(int Nc, const SweepArgs& a, const Problem& pb, hipStream_t st);
// Launch-shape variants of the two phase kernels (kind 0: rows, 1: columns):
// count, description (rows: values a lane, waves a workgroup; columns: values a
// lane, columns a workgroup), process-wide selection and current choice.
int variant_count(int N, int kind);
int variant_describe(int N, int kind, int v, int* a, int* b);
int variant_select(int N, int rows_v, int cols_v);
void variant_current(int N, int* rows_v, int* cols_v);
// coarse box widths whose convolution-form sweep keeps the box in LDS (a
// compiled width each): those of N_C = 16, 32, 64
inline constexpr bool conv_lds_width(int Mc) { return Mc == 11 || Mc == 21 || Mc == 43; }
// same sweep with the explicit term as the exact spectral convolution with the
// flow's four Fourier modes (N_C <= 64)
hipError_t sweep_conv(int Nc, const SweepArgs& a, const Problem& pb, hipStream_t st);
// many independent coarse sweeps, one workgroup each (convolution form);
// jobs whose width passes conv_lds_width keep the box in LDS, others in their
// Bc/T1c/Hc global buffers (3 Mc^2 values each)
hipError_t sweep_conv_jobs(const SweepJob* d_jobs, int njobs, bool lds_resident, hipStream_t st);
// full layout [f][3][N][N] <-> compact [f][3][M][M] of the |k| <= (M-1)/2 box
// (M < box width of N restricts / zero-pads: Fourier re-sampling)
hipError_t pack(const cplx* full, cplx* box, int N, int M, size_t nfields, hipStream_t st);
hipError_t unpack(const cplx* box, cplx* full, int N, int M, size_t nfields, hipStream_t st);
hipError_t check_box(const cplx* full, int N, size_t nfields, int* dflag, hipStream_t st);
// device address of the static fine-grid workspace on `device` (looked up
// once per device; static_ws.hip)
hipError_t scratch_resolve(int device);
hipError_t norms2(const cplx* x, size_t len, int nfields, double* out, hipStream_t st);
// Fo[f] = U[uidx[f]] for f = map[row], row < *count (rows = launch rows)
hipError_t gather(const cplx* U, cplx* Fo, const int* uidx, const int* map, const int* count,
                  int rows, size_t box, hipStream_t st);

}  // namespace pd
