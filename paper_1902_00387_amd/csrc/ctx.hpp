// The context of the C ABI (pd_ctx) and the helpers shared by the runtime
// files that implement its calls.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/pitdyn.h"
#include "launch.hpp"
#include "runtime.hpp"

using pd::rt::DevBuf;
using pd::cplx;
using pd::cplxf;

struct pd_ctx {
  int device = 0;
  hipStream_t own = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;      // second stream of the two-stream fine sweep
  hipEvent_t sev[3] = {nullptr, nullptr, nullptr};
  hipStream_t cst = nullptr;       // pipelined Parareal: coarse sweep stream
  hipStream_t fst = nullptr;       // pipelined Parareal: fine streams
  int pipe_spec = 2;               // pipelined: which chunks of the next fine sweep start early
  int pipe_chunks = 2;             // slice chunks of the pipelined Parareal (< 2: off)
  // temporal blocking of fine sweeps on the multi-launch path: groups of blk_g
  // fields run all their steps back to back, dealt round-robin to blk_s
  // streams (blk_g < 0: the grid's default, 0: off)
  int blk_g = -1, blk_s = 0;
  hipEvent_t bev[3] = {nullptr, nullptr, nullptr};  // fork and joins of the blocked sweep
  std::string err;
  int path = PD_PATH_AUTO;
  int coarse_form = PD_COARSE_AUTO;
  int scheme_f = PD_SCHEME_SBDF2;  // time steppers of F and G
  int scheme_c = PD_SCHEME_SBDF2;
  int prec = PD_C128;              // number type of the context's fields and kernels
  int rows_v = -1, cols_v = -1;    // launch-shape variants chosen by pd_autotune (-1: process default)
  int sweep_next = -1;             // pd_fine_sweep_steps: next step of the stepwise fine sweep
  // problem
  bool have_problem = false;
  int flow = PD_FLOW_NONE;
  double Rm = 1, kz = 0;
  int N = 0, K = 0, M = 0;
  // time grid
  bool have_time = false;
  double T = 0, dT = 0, dtf = 0, dtc = 0;
  int P = 0, Nc = 0, Mc = 0, nf = 0, nc = 0;
  bool have_initial = false;
  int resume_k = -1;                   // pd_set_slices: the next pd_parareal goes on after iteration k
  int last_k = -1;                     // iterations the last pd_parareal completed on the current
                                       // state (-1: nothing pd_parareal_continue may go on from)
  bool have_gold = false;              // the resumed state came with the previous coarse values
  // device memory
  DevBuf tw, twc;                      // twiddles (fine, coarse)
  DevBuf twf, twcf;                    // the same in FP32 (complex64 variant)
  DevBuf U, Fo, Gold, Hf, T1f;         // slice buffers (the fine row phases work in place in T1f)
  DevBuf Uprev, t0s;                   // defect copy, slice start times
  DevBuf Bc, Hc, T1c, T2c;             // coarse sweep workspaces
  DevBuf red, flag;                    // reduction outputs, box-check flag
  DevBuf ftab;                         // flow phases at every coarse step time
  DevBuf Rf, Rc, wR;                   // Runge-Kutta stage sums: slices, coarse sweep, propagator calls
  DevBuf wB, wH, wT1, wt0;             // workspaces of the propagator calls
  double* hred = nullptr;              // pinned host copy of red
  // learned coarse propagator (correction network) state
  struct LG {
    bool init = false, enabled = false;
    int L = 0, Q = 0, Mf = 0, step = 0;
    DevBuf params, grads, m1, m2;      // FP32 vectors of nn::param_count values
    int S = 0;                         // stored samples
    DevBuf xs, rs, ts;                 // [S][Q][12] features, [S][Q][6] targets, [S] slice times
    int Bcap = 0;                      // batch capacity of the activation buffers
    DevBuf act, ys, c, dc, dhA, dhB, dW, part, lpart, sums, bidx;
    int* hbidx = nullptr;              // pinned batch indices
    DevBuf Dn, gn, fn, nrm, uold;      // sweep and sample work (compact fine box)
    DevBuf wq;                         // [Q] per-mode loss weights (empty: uniform)
    bool weighted = false;
    int f32ops = 0;                    // matrix-core operands: 0 BF16, 1 FP32 (test mode)
  } lg;

  size_t box_elems() const { return (size_t)3 * M * M; }
  // bytes of one complex value of the context's number type
  size_t esize() const { return prec == PD_C64 ? sizeof(pd::cplxf) : sizeof(pd::cplx); }
  // twiddle tables of the fine and coarse grid in the number type C
  template <class C>
  const C* twid() const {
    if constexpr (sizeof(C) == sizeof(pd::cplxf)) return twf.as<C>();
    else return tw.as<C>();
  }
  template <class C>
  const C* twidc() const {
    if constexpr (sizeof(C) == sizeof(pd::cplxf)) return twcf.as<C>();
    else return twc.as<C>();
  }
  // a batch of fields on the fine grid with this context's launch shapes
  template <class C>
  void shapes(pd::FieldBatchT<C>& fb) const {
    fb.rows_v = rows_v;
    fb.cols_v = cols_v;
  }
  size_t rows_elems() const { return (size_t)3 * M * N; }
};

namespace pd {
namespace ctxh {

pd_status fail(pd_ctx* c, pd_status s, const char* fmt, ...);
pd_status hipfail(pd_ctx* c, hipError_t e, const char* what);

#define PD_HIP(ctx, expr, what)                            \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return hipfail(ctx, e_, what);   \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(d);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

pd::Problem make_problem(const pd_ctx* c, double dt, int scheme = PD_SCHEME_SBDF2);
// fills the report's R_f / R_c and model speed-up from its sweep times
void finish_report(pd_report& r, int P);
pd_status ensure_rk_buffers(pd_ctx* c);
bool use_conv_sweep(const pd_ctx* c);
hipError_t coarse_sweep(pd_ctx* c, pd::SweepArgs& sa, const pd::Problem& pc, hipStream_t st);
int choose_path(const pd_ctx* c, int nfields);
// fields a group (0: unblocked) and streams of the blocked fine sweep for a
// batch of nfields fields
void fine_blocking(const pd_ctx* c, int nfields, int* group, int* streams);
// Enqueue `run(sub_batch, fields, stream)` for consecutive groups of `group`
// fields of fb (fields on the context's fine grid: sub-batches are offset by
// its box and row sizes), dealt round-robin to `streams` streams (st first,
// then the context's idle pipeline streams), forked from and joined back
// into st.
// the streams of a blocked sweep (st first, at most 3) and the fork event
// recorded on st that the others wait for; returns how many there are
int blocking_fork(pd_ctx* c, int streams, hipStream_t st, hipStream_t* out, hipError_t* err);
template <class C, class Fn>
hipError_t over_groups(pd_ctx* c, const pd::FieldBatchT<C>& fb, int nfields, int group,
                       int streams, hipStream_t st, Fn&& run) {
  hipStream_t ss[3];
  hipError_t e = hipSuccess;
  const int n = blocking_fork(c, streams, st, ss, &e);
  if (e != hipSuccess) return e;
  const size_t box = c->box_elems(), rows = c->rows_elems();
  int gi = 0;
  for (int f0 = 0; f0 < nfields; f0 += group, ++gi) {
    const int ng = nfields - f0 < group ? nfields - f0 : group;
    pd::FieldBatchT<C> q = fb;
    q.B += (size_t)f0 * box;
    q.H += (size_t)f0 * box;
    q.T1 += (size_t)f0 * rows;
    q.T2 += (size_t)f0 * rows;
    if (q.R) q.R += (size_t)4 * f0 * box;
    if (q.t0) q.t0 += f0;
    if (q.fRm) q.fRm += f0;
    if (q.fkz) q.fkz += f0;
    e = run(q, ng, ss[gi % n]);
    if (e != hipSuccess) return e;
  }
  // join: later work on st follows every group
  for (int i = 1; i < n; ++i) {
    e = hipEventRecord(c->bev[i], ss[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, c->bev[i], 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t fine_batch(pd_ctx* c, const pd::FieldBatch& fb, const pd::Problem& pb, int nfields,
                      int nsteps, hipStream_t st);
pd_status check_box_dev(pd_ctx* c, const void* d, int N, size_t nfields, hipStream_t st);
pd_status run_propagator(pd_ctx* c, const double* t0, int batch, double dt, int nsteps,
                         int Ngrid, const void* d_in, void* d_out, hipStream_t st, int scheme);
// the same two for a complex64 batch and sweep
hipError_t coarse_sweep(pd_ctx* c, pd::SweepArgsF& sa, const pd::Problem& pc, hipStream_t st);
hipError_t fine_batch(pd_ctx* c, const pd::FieldBatchF& fb, const pd::Problem& pb, int nfields,
                      int nsteps, hipStream_t st);
// upload a host twiddle table (FP64 and its FP32 rounding)
pd_status upload_twiddles(pd_ctx* c, int N, DevBuf& d64, DevBuf& d32, hipStream_t st);
// learned coarse propagator (lg.cpp)
void lg_release(pd_ctx* c);
pd_status lg_sweep(pd_ctx* c, int n0, bool initial, hipStream_t st);
pd_status lg_sweep_range(pd_ctx* c, int a, int b, int n0, bool initial, bool defect,
                         hipStream_t st);
// pipelined Parareal with the plain coarse propagator (pipeline.cpp)
pd_status parareal_pipelined(pd_ctx* c, double tol, int max_iter, int kres, pd_report* rep);

}  // namespace ctxh
}  // namespace pd
