// Internal interface between the C-ABI runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "fft.hpp"

namespace pd {

enum { PATH_MULTI = 0, PATH_SINGLE_WG = 1 };

// Per-launch physical and step parameters.
struct Problem {
  double Rm;   // magnetic Reynolds number
  double kz;   // wavenumber of the e^{i kz z} ansatz
  double dt;   // step size
  double amp;  // flow amplitude: 0 (none), 1 (Roberts), sqrt(3/2) (GP)
  int tdep;    // 1: Galloway-Proctor phases (cos t, sin t); 0: steady
};

// A batch of fields stepped together (all of grid size N).
struct FieldBatch {
  cplx* B;           // [f][3][M][M] state (in: start value, out: end value)
  cplx* H;           // [f][3][M][M] SBDF2 history workspace
  cplx* T1;          // [f][3][M][N] row workspace
  cplx* T2;          // [f][3][M][N] row workspace
  const double* t0;  // [f] start time of each field's slice
  const cplx* tw;    // [N] twiddles e^{-2 pi i m/N}
};

struct SweepArgs {
  cplx* U;            // [P+1][3][M][M] slice-boundary states (fine, compact)
  const cplx* Fo;     // [P][3][M][M] fine results F(U^{k-1}_n)
  cplx* Gold;         // [P][3][M][M] previous coarse results
  const cplx* Uprev;  // [3][M][M] U^{k-1}_P (defect)
  cplx *Bc, *Hc, *T1c, *T2c;  // coarse workspaces
  const cplx* twc;    // coarse twiddles
  double* red;        // [2] defect sums (may be null)
  const double* ftab; // [P][nsteps][4] cos(py), sin(py), cos(px), sin(px) of the
                      // flow phases at every coarse step time (time-dependent flow)
  double dT;          // slice length
  int M;              // fine box width
  int P, n0;          // slices, first slice swept
  int nsteps;         // coarse steps per slice
  int mode;           // 0: initial coarse run, 1: correction
};

hipError_t propagate(int N, const FieldBatch& fb, const Problem& pb, int nfields, int nsteps,
                     int path, hipStream_t st);
// single launches of the two phases of the multi-launch path
hipError_t rows(int N, const FieldBatch& fb, const Problem& pb, int nfields, int mode, int last,
                hipStream_t st);
hipError_t cols(int N, const FieldBatch& fb, const Problem& pb, int nfields, int step,
                hipStream_t st);
hipError_t sweep(int Nc, const SweepArgs& a, const Problem& pb, hipStream_t st);
// same sweep with the explicit term as the exact spectral convolution with the
// flow's four Fourier modes (N_C <= 64)
hipError_t sweep_conv(int Nc, const SweepArgs& a, const Problem& pb, hipStream_t st);
// full layout [f][3][N][N] <-> compact [f][3][M][M] of the |k| <= (M-1)/2 box
// (M < box width of N restricts / zero-pads: Fourier re-sampling)
hipError_t pack(const cplx* full, cplx* box, int N, int M, size_t nfields, hipStream_t st);
hipError_t unpack(const cplx* box, cplx* full, int N, int M, size_t nfields, hipStream_t st);
hipError_t check_box(const cplx* full, int N, size_t nfields, int* dflag, hipStream_t st);
hipError_t norms2(const cplx* x, size_t len, int nfields, double* out, hipStream_t st);

}  // namespace pd
