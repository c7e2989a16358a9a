// C-ABI runtime of libpitdyn.so: contexts, device buffers, the Parareal
// driver (Section 3 of Clarke et al., arXiv:1902.00387) and the propagator
// entry points.  Every step of the numerical path runs in the HIP kernels of
// kernels.hip; this file only validates arguments, owns memory and orders
// launches on a stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pitdyn.h"
#include "launch.hpp"
#include "runtime.hpp"
#include "ctx.hpp"
#include "nn.hpp"

using pd::cplx;

using namespace pd::rt;


namespace pd {
namespace ctxh {

pd_status fail(pd_ctx* c, pd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

pd_status hipfail(pd_ctx* c, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory)
    return fail(c, PD_ENOMEM, "%s: out of device memory", what);
  return fail(c, PD_EHIP, "%s: %s", what, hipGetErrorString(e));
}


// Section 3.1, eq. speed_up: R_f from the mean fine sweep (all slices at
// once), R_c from the mean coarse sweep over P (slices one after another).
void finish_report(pd_report& r, int P) {
  r.Rf_over_Rc = 0.0;
  r.model_speedup = 0.0;
  const int sweeps_c = r.iters + (r.t_coarse0_s > 0.0 ? 1 : 0);
  const double tc = r.t_coarse0_s + r.t_coarse_s;
  if (P < 1 || r.iters < 1 || r.t_fine_s <= 0.0 || sweeps_c < 1 || tc <= 0.0) return;
  const double Rf = r.t_fine_s / r.iters, Rc = tc / sweeps_c / P;
  r.Rf_over_Rc = Rf / Rc;
  const double k = r.k_con > 0 ? r.k_con : r.iters;
  r.model_speedup = 1.0 / ((1.0 + k / P) * (Rc / Rf) + k / P);
}

pd::Problem make_problem(const pd_ctx* c, double dt, int scheme) {
  pd::Problem pb;
  pb.Rm = c->Rm;
  pb.kz = c->kz;
  pb.dt = dt;
  pb.amp = c->flow == PD_FLOW_NONE ? 0.0 : (c->flow == PD_FLOW_ROBERTS ? 1.0 : std::sqrt(1.5));
  pb.tdep = c->flow == PD_FLOW_GP ? 1 : 0;
  pb.scheme = scheme == PD_SCHEME_SBDF2 ? 0 : 1;
  // IMEX Runge-Kutta tableaus of Ascher, Ruuth & Spiteri (1997): rows are the
  // stages 2..s+1, columns the stages 1..s they use
  if (scheme == PD_SCHEME_RK443) {  // ARS(4,4,3)
    const double c[4] = {0.0, 0.5, 2.0 / 3.0, 0.5};
    const double a[5][4] = {{0, 0, 0, 0}, {0.5, 0, 0, 0}, {11.0 / 18.0, 1.0 / 18.0, 0, 0},
                            {5.0 / 6.0, -5.0 / 6.0, 0.5, 0}, {0.25, 1.75, 0.75, -1.75}};
    const double at[5][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 1.0 / 6.0, 0, 0},
                             {0, -0.5, 0.5, 0}, {0, 1.5, -1.5, 0.5}};
    pb.rk_s = 4;
    pb.rk_g = 0.5;
    std::memcpy(pb.rk_c, c, sizeof c);
    std::memcpy(pb.rk_a, a, sizeof a);
    std::memcpy(pb.rk_at, at, sizeof at);
  } else if (scheme == PD_SCHEME_RK222) {  // ARS(2,2,2)
    const double g = 1.0 - 1.0 / std::sqrt(2.0), dl = 1.0 - 1.0 / (2.0 * g);
    pb.rk_s = 2;
    pb.rk_g = g;
    pb.rk_c[0] = 0.0;
    pb.rk_c[1] = g;
    pb.rk_a[1][0] = g;
    pb.rk_a[2][0] = dl;
    pb.rk_a[2][1] = 1.0 - dl;
    pb.rk_at[2][1] = 1.0 - g;
  } else if (scheme == PD_SCHEME_RK111) {  // ARS(1,1,1), forward-backward Euler
    pb.rk_s = 1;
    pb.rk_g = 1.0;
    pb.rk_c[0] = 0.0;
    pb.rk_a[1][0] = 1.0;
  }
  return pb;
}

// the convolution form of the coarse sweep steps SBDF2 only
bool use_conv_sweep(const pd_ctx* c) {
  if (c->coarse_form == PD_COARSE_FFT || c->scheme_c != PD_SCHEME_SBDF2) return false;
  return c->Nc <= 64;
}

// The serial coarse sweep in the form the context selects: the exact
// convolution (SBDF2, N_C <= 64), the one-workgroup FFT form, or the
// host-driven multi-launch form (then the defect sums run after it).
hipError_t coarse_sweep(pd_ctx* c, pd::SweepArgs& sa, const pd::Problem& pc, hipStream_t st) {
  if (use_conv_sweep(c)) return pd::sweep_conv(c->Nc, sa, pc, st);
  const bool multi = c->coarse_form == PD_COARSE_MULTI ||
                     (c->coarse_form == PD_COARSE_AUTO);
  if (!multi) return pd::sweep(c->Nc, sa, pc, st);
  if (sa.t0s == nullptr) sa.t0s = c->t0s.as<double>() + sa.nbase;
  hipError_t e = pd::sweep_multi(c->Nc, sa, pc, st);
  if (e == hipSuccess && sa.mode != 0 && sa.red != nullptr)
    e = pd::nn::defect(sa.U + (size_t)sa.P * c->box_elems(), sa.Uprev, c->box_elems(), sa.red, st);
  return e;
}

// stage-sum buffers of the Runge-Kutta steppers for the slice arrays and the
// coarse sweep (none for SBDF2)
pd_status ensure_rk_buffers(pd_ctx* c) {
  if (!c->have_time) return PD_OK;
  if (c->scheme_f != PD_SCHEME_SBDF2)
    PD_HIP(c, c->Rf.ensure((size_t)4 * c->box_elems() * c->P * sizeof(cplx)), "alloc");
  if (c->scheme_c != PD_SCHEME_SBDF2)
    PD_HIP(c, c->Rc.ensure((size_t)4 * 3 * c->Mc * c->Mc * sizeof(cplx)), "alloc");
  return PD_OK;
}

int choose_path(const pd_ctx* c, int nfields) {
  if (c->path == PD_PATH_MULTI || c->path == PD_PATH_SINGLE || c->path == PD_PATH_MULTI2)
    return c->path;
  return nfields >= 512 ? pd::PATH_SINGLE_WG : pd::PATH_MULTI;
}

// Temporal blocking of fine sweeps.  A step of the whole batch streams every
// field's state, history and row buffer through HBM (213 B a grid mode at
// 512^2, about 14 GB a step for 256 fields); a group of a few fields that
// runs all its steps back to back keeps its 19.6 MB a field (512^2: state,
// history, one row buffer used in place) in the 256 MB memory-side
// last-level cache from one step to the next, and the phases of groups on
// different streams overlap.  Defaults measured on MI355X (40 steps of every
// slice, best launch shapes): 512^2 x 256 fields, groups of 4 on 3 streams,
// 2.50 against 3.22 ms a step unblocked; 256^2 x 128, groups of 16 on 3
// streams, 0.322 against 0.387 ms; 128^2 x 64 gains 7 % with groups of 32
// (half its batch: a size that depends on the slice count) and stays
// unblocked by default.
void fine_blocking(const pd_ctx* c, int nfields, int* group, int* streams) {
  int g = c->blk_g, s = c->blk_s;
  if (g < 0) {
    g = c->N >= 512 ? 4 : c->N == 256 ? 16 : 0;
    s = 3;
  }
  if (g >= nfields) g = 0;
  *group = g;
  *streams = g > 0 ? std::max(1, std::min(s, 3)) : 1;
}

int blocking_fork(pd_ctx* c, int streams, hipStream_t st, hipStream_t* out, hipError_t* err) {
  out[0] = st;
  *err = hipSuccess;
  if (streams <= 1) return 1;
  // the pipelined schedule's two extra streams, idle outside it
  for (hipStream_t* p : {&c->fst, &c->cst})
    if (!*p && (*err = hipStreamCreateWithFlags(p, hipStreamNonBlocking)) != hipSuccess) return 1;
  for (auto& ev : c->bev)
    if (!ev && (*err = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return 1;
  int n = 1;
  for (hipStream_t x : {c->fst, c->cst})
    if (n < streams && x != st) out[n++] = x;
  if (n > 1) {
    *err = hipEventRecord(c->bev[0], st);
    for (int i = 1; i < n && *err == hipSuccess; ++i)
      *err = hipStreamWaitEvent(out[i], c->bev[0], 0);
  }
  return n;
}

// Fine propagation of a batch on the context's launch path (blocked in groups
// of fields when the context's blocking says so).
template <class C>
static hipError_t fine_batch_t(pd_ctx* c, const pd::FieldBatchT<C>& fb, const pd::Problem& pb,
                               int nfields, int nsteps, int path, hipStream_t st) {
  int g = 0, ns = 1;
  if (path == pd::PATH_MULTI && fb.map == nullptr) fine_blocking(c, nfields, &g, &ns);
  if (g > 0 && nsteps > 0)
    return over_groups(c, fb, nfields, g, ns, st,
                       [&](const pd::FieldBatchT<C>& q, int ng, hipStream_t x) {
                         return pd::propagate(c->N, q, pb, ng, nsteps, pd::PATH_MULTI, x);
                       });
  return pd::propagate(c->N, fb, pb, nfields, nsteps, path, st);
}

hipError_t fine_batch(pd_ctx* c, const pd::FieldBatch& fb, const pd::Problem& pb, int nfields,
                      int nsteps, hipStream_t st) {
  const int path = choose_path(c, nfields);
  if (path == PD_PATH_MULTI2 && fb.map == nullptr) {
    // the second stream of the two-stream path exists only once it is used:
    // HIP spreads a process's streams over a few hardware queues
    if (c->side == nullptr && hipStreamCreate(&c->side) != hipSuccess) return hipErrorOutOfMemory;
    return pd::propagate2(c->N, fb, pb, nfields, nsteps, st, c->side, c->sev);
  }
  return fine_batch_t(c, fb, pb, nfields, nsteps, path == PD_PATH_MULTI2 ? 0 : path, st);
}

// complex64: the convolution sweep (N_C <= 64) or the multi-launch sweep
// followed by the defect sums
hipError_t coarse_sweep(pd_ctx* c, pd::SweepArgsF& sa, const pd::Problem& pc, hipStream_t st) {
  if (use_conv_sweep(c)) return pd::sweep_conv(c->Nc, sa, pc, st);
  if (sa.t0s == nullptr) sa.t0s = c->t0s.as<double>() + sa.nbase;
  hipError_t e = pd::sweep_multi(c->Nc, sa, pc, st);
  if (e == hipSuccess && sa.mode != 0 && sa.red != nullptr)
    e = pd::defect2(sa.U + (size_t)sa.P * c->box_elems(), sa.Uprev, c->box_elems(), sa.red, st);
  return e;
}

hipError_t fine_batch(pd_ctx* c, const pd::FieldBatchF& fb, const pd::Problem& pb, int nfields,
                      int nsteps, hipStream_t st) {
  return fine_batch_t(c, fb, pb, nfields, nsteps, pd::PATH_MULTI, st);
}

pd_status upload_twiddles(pd_ctx* c, int N, DevBuf& d64, DevBuf& d32, hipStream_t st) {
  const std::vector<cplx> tw = twiddles(N);
  std::vector<cplxf> twf(N);
  for (int m = 0; m < N; ++m) twf[m] = {(float)tw[m].re, (float)tw[m].im};
  PD_HIP(c, d64.ensure(sizeof(cplx) * N), "alloc twiddles");
  PD_HIP(c, d32.ensure(sizeof(cplxf) * N), "alloc twiddles");
  PD_HIP(c, hipMemcpyAsync(d64.p, tw.data(), sizeof(cplx) * N, hipMemcpyHostToDevice, st), "copy");
  PD_HIP(c, hipMemcpyAsync(d32.p, twf.data(), sizeof(cplxf) * N, hipMemcpyHostToDevice, st), "copy");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  return PD_OK;
}

// Validate `nfields` full-layout device fields: zero outside the 2/3 box.
pd_status check_box_dev(pd_ctx* c, const void* d, int N, size_t nfields, hipStream_t st) {
  PD_HIP(c, c->flag.ensure(sizeof(int)), "alloc");
  PD_HIP(c, hipMemsetAsync(c->flag.p, 0, sizeof(int), st), "memset");
  PD_HIP(c, pd::check_box(static_cast<const cplx*>(d), N, nfields, c->flag.as<int>(), st),
         "check_box");
  int h = 0;
  PD_HIP(c, hipMemcpyAsync(&h, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  if (h) return fail(c, PD_EINVAL, "input field has nonzero coefficients outside the 2/3 box");
  return PD_OK;
}

// Propagate `batch` full-layout fields by nsteps steps of dt on grid N (with
// restriction to Ngrid <= N and zero-padding back when Ngrid < N), in the
// context's number type C.
template <class C>
static pd_status run_propagator_t(pd_ctx* c, const double* t0, int batch, double dt, int nsteps,
                                  int Ngrid, const void* d_in, void* d_out, hipStream_t st,
                                  int scheme) {
  pd_status s = check_box_dev(c, d_in, c->N, batch, st);
  if (s != PD_OK) return s;
  const int Mg = box_M(Ngrid);
  const size_t box = (size_t)3 * Mg * Mg, rows = (size_t)3 * Mg * Ngrid;
  PD_HIP(c, c->wB.ensure(box * batch * sizeof(C)), "alloc");
  PD_HIP(c, c->wH.ensure(box * batch * sizeof(C)), "alloc");
  PD_HIP(c, c->wT1.ensure(rows * batch * sizeof(C)), "alloc");
  PD_HIP(c, c->wt0.ensure(sizeof(double) * batch), "alloc");
  PD_HIP(c, hipMemcpyAsync(c->wt0.p, t0, sizeof(double) * batch, hipMemcpyHostToDevice, st),
         "copy t0");
  const C* twg = c->twid<C>();
  if (Ngrid != c->N) {
    s = upload_twiddles(c, Ngrid, c->twc, c->twcf, st);
    if (s != PD_OK) return s;
    twg = c->twidc<C>();
  }
  // full layout on N -> compact box of Ngrid: for Ngrid < N the pack keeps
  // only |k| <= Kg (restriction) and the unpack zero-pads (prolongation)
  PD_HIP(c, pd::pack(static_cast<const cplx*>(d_in), c->wB.as<C>(), c->N, Mg, (size_t)batch, st),
         "pack");
  pd::FieldBatchT<C> fb;
  fb.B = c->wB.as<C>();
  fb.H = c->wH.as<C>();
  fb.T1 = c->wT1.as<C>();
  fb.T2 = fb.T1;  // in place
  fb.t0 = c->wt0.as<double>();
  fb.tw = twg;
  if constexpr (sizeof(C) == sizeof(cplx)) {
    if (scheme != PD_SCHEME_SBDF2) {
      PD_HIP(c, c->wR.ensure(4 * box * batch * sizeof(cplx)), "alloc");
      fb.R = c->wR.as<cplx>();
    }
  }
  const pd::Problem pb = make_problem(c, dt, scheme);
  if (Ngrid == c->N) {
    c->shapes(fb);
    PD_HIP(c, fine_batch(c, fb, pb, batch, nsteps, st), "propagate");
  } else {
    const int path = choose_path(c, batch);
    PD_HIP(c, pd::propagate(Ngrid, fb, pb, batch, nsteps, path == PD_PATH_MULTI2 ? 0 : path, st),
           "propagate");
  }
  PD_HIP(c, pd::unpack(c->wB.as<C>(), static_cast<cplx*>(d_out), c->N, Mg, (size_t)batch, st),
         "unpack");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  return PD_OK;
}

pd_status run_propagator(pd_ctx* c, const double* t0, int batch, double dt, int nsteps,
                         int Ngrid, const void* d_in, void* d_out, hipStream_t st, int scheme) {
  if (!c->have_problem) return fail(c, PD_ESTATE, "pd_set_problem not called");
  if (batch < 0 || batch > 65535) return fail(c, PD_EINVAL, "batch must be in [0, 65535]");
  if (batch == 0) return PD_OK;
  if (!t0 || !d_in || !d_out) return fail(c, PD_EINVAL, "null pointer argument");
  if (nsteps < 1) return fail(c, PD_EINVAL, "n_steps must be >= 1");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(c, PD_EINVAL, "dt must be positive");
  for (int f = 0; f < batch; ++f)
    if (!std::isfinite(t0[f])) return fail(c, PD_EINVAL, "t0 must be finite");
  DeviceGuard dg(c->device);
  if (c->prec == PD_C64) {
    if (scheme != PD_SCHEME_SBDF2) return fail(c, PD_EINVAL, "complex64 steps SBDF2 only");
    return run_propagator_t<cplxf>(c, t0, batch, dt, nsteps, Ngrid, d_in, d_out, st, scheme);
  }
  return run_propagator_t<cplx>(c, t0, batch, dt, nsteps, Ngrid, d_in, d_out, st, scheme);
}

}  // namespace ctxh
}  // namespace pd

using namespace pd::ctxh;

// The plain order of Parareal (Section 3): every fine sweep, then the serial
// coarse sweep with the correction and the defect, on the context's stream,
// in the context's number type C (the learned coarse propagator: complex128).
template <class C>
static pd_status parareal_plain(pd_ctx* c, double tol, int max_iter, int kres, bool learned,
                                pd_report* rep, std::chrono::steady_clock::time_point wall0) {
  hipStream_t st = c->stream;
  const size_t box = c->box_elems(), rows = c->rows_elems();
  const int P = c->P;
  C* U = c->U.as<C>();
  C* Fo = c->Fo.as<C>();
  pd_report r;
  std::memset(&r, 0, sizeof r);
  r.k_con = -1;
  hipEvent_t ev[4];
  for (auto& e : ev) PD_HIP(c, hipEventCreate(&e), "event");
  struct EvFree {
    hipEvent_t* e;
    ~EvFree() { for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]); }
  } evf{ev};

  pd::SweepArgsT<C> sa;
  sa.U = U;
  sa.Fo = Fo;
  sa.Gold = c->Gold.as<C>();
  sa.Uprev = c->Uprev.as<C>();
  sa.Bc = c->Bc.as<C>();
  sa.Hc = c->Hc.as<C>();
  sa.T1c = c->T1c.as<C>();
  sa.T2c = c->T2c.as<C>();
  sa.twc = c->twidc<C>();
  sa.Rc = c->Rc.as<C>();
  sa.red = c->red.as<double>();
  sa.ftab = c->ftab.as<double>();
  sa.dT = c->dT;
  sa.M = c->M;
  sa.P = P;
  sa.nsteps = c->nc;
  const pd::Problem pc = make_problem(c, c->dtc, c->scheme_c),
                    pf = make_problem(c, c->dtf, c->scheme_f);

  // initial coarse run (Section 3: U^0_n from G over [0, T])
  sa.n0 = 0;
  sa.mode = 0;
  PD_HIP(c, hipEventRecord(ev[0], st), "event");
  auto run_sweep = [&]() -> hipError_t {
    return coarse_sweep(c, sa, pc, st);
  };
  if (kres >= 0) {
    // nothing to do: the state of iteration kres was supplied
  } else if (learned) {
    if constexpr (sizeof(C) == sizeof(cplx)) {
      pd_status ls = lg_sweep(c, 0, true, st);
      if (ls != PD_OK) return ls;
    }
  } else {
    PD_HIP(c, run_sweep(), "coarse sweep");
  }
  PD_HIP(c, hipEventRecord(ev[1], st), "event");
  PD_HIP(c, hipEventSynchronize(ev[1]), "sync");
  float ms = 0;
  PD_HIP(c, hipEventElapsedTime(&ms, ev[0], ev[1]), "event");
  r.t_coarse0_s = ms * 1e-3;

  pd_status status = PD_NOT_CONVERGED;
  for (int k = kres >= 0 ? kres + 1 : 1; k <= max_iter; ++k) {
    const int n0 = k - 1 < P - 1 ? k - 1 : P - 1;
    PD_HIP(c, hipMemcpyAsync(c->Uprev.p, U + (size_t)P * box, box * sizeof(C),
                             hipMemcpyDeviceToDevice, st), "copy");
    PD_HIP(c, hipEventRecord(ev[0], st), "event");
    // fine sweep over the slices whose start value can still change
    PD_HIP(c, hipMemcpyAsync(Fo + (size_t)n0 * box, U + (size_t)n0 * box,
                             (size_t)(P - n0) * box * sizeof(C), hipMemcpyDeviceToDevice, st),
           "copy");
    pd::FieldBatchT<C> fb;
    fb.B = Fo + (size_t)n0 * box;
    fb.H = c->Hf.as<C>() + (size_t)n0 * box;
    fb.T1 = c->T1f.as<C>() + (size_t)n0 * rows;
    fb.T2 = fb.T1;
    fb.t0 = c->t0s.as<double>() + n0;
    fb.tw = c->twid<C>();
    c->shapes(fb);
    if constexpr (sizeof(C) == sizeof(cplx))
      if (c->scheme_f != PD_SCHEME_SBDF2) fb.R = c->Rf.as<cplx>() + (size_t)4 * n0 * box;
    PD_HIP(c, fine_batch(c, fb, pf, P - n0, c->nf, st), "fine sweep");
    PD_HIP(c, hipEventRecord(ev[1], st), "event");
    // serial coarse sweep with the correction, then the defect sums
    sa.n0 = n0;
    sa.mode = 1;
    if (learned) {
      if constexpr (sizeof(C) == sizeof(cplx)) {
        pd_status ls = lg_sweep(c, n0, false, st);
        if (ls != PD_OK) return ls;
      }
    } else {
      PD_HIP(c, run_sweep(), "coarse sweep");
    }
    PD_HIP(c, hipEventRecord(ev[2], st), "event");
    PD_HIP(c, hipMemcpyAsync(c->hred, c->red.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
    PD_HIP(c, hipStreamSynchronize(st), "sync");
    float mf = 0, mc = 0;
    PD_HIP(c, hipEventElapsedTime(&mf, ev[0], ev[1]), "event");
    PD_HIP(c, hipEventElapsedTime(&mc, ev[1], ev[2]), "event");
    r.t_fine_s += mf * 1e-3;
    r.t_coarse_s += mc * 1e-3;
    const double num = c->hred[0], den = c->hred[1];
    r.iters = k;
    if (!std::isfinite(num) || !std::isfinite(den)) {
      status = fail(c, PD_EUNSTABLE, "non-finite state at iteration %d (unstable step size?)", k);
      break;
    }
    const double sigma = den > 0 ? std::sqrt(num / den) : (num > 0 ? INFINITY : 0.0);
    r.sigma[k - 1] = sigma;
    if (sigma <= tol) {
      r.k_con = k;
      status = PD_OK;
      break;
    }
  }
  if (max_iter == 0) status = PD_OK;
  c->last_k = status == PD_EUNSTABLE ? -1 : (r.iters > 0 ? r.iters : (kres >= 0 ? kres : 0));
  r.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
  finish_report(r, c->P);
  if (rep) *rep = r;
  return status;
}


template <class C>
static pd_status profile_fine_t(pd_ctx* c, int reps, double* ms) {
  hipStream_t st = c->stream;
  const size_t box = c->box_elems();
  const int P = c->P;
  hipEvent_t ev[2];
  for (auto& e : ev) PD_HIP(c, hipEventCreate(&e), "event");
  struct EvFree {
    hipEvent_t* e;
    ~EvFree() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
  } evf{ev};
  auto fresh = [&]() -> hipError_t {
    return hipMemcpyAsync(c->Fo.p, c->U.p, (size_t)P * box * sizeof(C), hipMemcpyDeviceToDevice, st);
  };
  pd::FieldBatchT<C> fb;
  fb.B = c->Fo.as<C>();
  fb.H = c->Hf.as<C>();
  fb.T1 = c->T1f.as<C>();
  fb.T2 = fb.T1;
  fb.t0 = c->t0s.as<double>();
  fb.tw = c->twid<C>();
  c->shapes(fb);
  const pd::Problem pf = make_problem(c, c->dtf);
  float t = 0;
  // a whole fine sweep (all slices, every step) as Parareal launches it
  PD_HIP(c, fresh(), "copy");
  PD_HIP(c, hipEventRecord(ev[0], st), "event");
  PD_HIP(c, fine_batch(c, fb, pf, P, c->nf, st), "propagate");
  PD_HIP(c, hipEventRecord(ev[1], st), "event");
  PD_HIP(c, hipEventSynchronize(ev[1]), "sync");
  PD_HIP(c, hipEventElapsedTime(&t, ev[0], ev[1]), "event");
  ms[2] = t / c->nf;
  ms[0] = ms[1] = 0.0;
  if (choose_path(c, P) != pd::PATH_SINGLE_WG) {
    // each phase kernel back to back, reps times, over the same batch
    PD_HIP(c, fresh(), "copy");
    PD_HIP(c, pd::rows(c->N, fb, pf, P, 0, 0, st), "rows");
    PD_HIP(c, hipEventRecord(ev[0], st), "event");
    for (int i = 0; i < reps; ++i) PD_HIP(c, pd::cols(c->N, fb, pf, P, 1, st), "cols");
    PD_HIP(c, hipEventRecord(ev[1], st), "event");
    PD_HIP(c, hipEventSynchronize(ev[1]), "sync");
    PD_HIP(c, hipEventElapsedTime(&t, ev[0], ev[1]), "event");
    ms[0] = t / reps;
    PD_HIP(c, hipEventRecord(ev[0], st), "event");
    for (int i = 0; i < reps; ++i) PD_HIP(c, pd::rows(c->N, fb, pf, P, 2, 0, st), "rows");
    PD_HIP(c, hipEventRecord(ev[1], st), "event");
    PD_HIP(c, hipEventSynchronize(ev[1]), "sync");
    PD_HIP(c, hipEventElapsedTime(&t, ev[0], ev[1]), "event");
    ms[1] = t / reps;
  }
  return PD_OK;
}


template <class C>
static pd_status fine_sweep_steps_t(pd_ctx* c, int step0, int n_steps, double* ms) {
  hipStream_t st = c->stream;
  const size_t box = c->box_elems();
  const int P = c->P;
  pd::FieldBatchT<C> fb;
  fb.B = c->Fo.as<C>();
  fb.H = c->Hf.as<C>();
  fb.T1 = c->T1f.as<C>();
  fb.T2 = fb.T1;
  fb.t0 = c->t0s.as<double>();
  fb.tw = c->twid<C>();
  c->shapes(fb);
  const pd::Problem pf = make_problem(c, c->dtf);
  c->sweep_next = -1;
  if (step0 == 0) {
    PD_HIP(c, hipMemcpyAsync(c->Fo.p, c->U.p, (size_t)P * box * sizeof(C),
                             hipMemcpyDeviceToDevice, st), "copy");
    PD_HIP(c, pd::rows(c->N, fb, pf, P, 0, 0, st), "rows");
  }
  std::vector<hipEvent_t> ev;
  struct EvFree {
    std::vector<hipEvent_t>& e;
    ~EvFree() { for (auto x : e) (void)hipEventDestroy(x); }
  } evf{ev};
  int g = 0, ns = 1;
  fine_blocking(c, P, &g, &ns);
  if (g > 0) {
    // blocked: each group of g fields runs all n_steps steps back to back;
    // the phases of different groups overlap, so only the whole is timed
    if (ms) {
      ev.resize(2, nullptr);
      for (auto& e : ev) PD_HIP(c, hipEventCreate(&e), "event");
      PD_HIP(c, hipEventRecord(ev[0], st), "event");
    }
    PD_HIP(c, over_groups(c, fb, P, g, ns, st,
                          [&](const pd::FieldBatchT<C>& q, int ng, hipStream_t x) -> hipError_t {
                            hipError_t e = hipSuccess;
                            for (int s = step0; s < step0 + n_steps && e == hipSuccess; ++s) {
                              e = pd::cols(c->N, q, pf, ng, s, x);
                              if (e == hipSuccess) e = pd::rows(c->N, q, pf, ng, s == 0 ? 1 : 2, 0, x);
                            }
                            return e;
                          }),
           "blocked steps");
    if (ms) PD_HIP(c, hipEventRecord(ev[1], st), "event");
    PD_HIP(c, hipStreamSynchronize(st), "sync");
    if (ms) {
      float all = 0.f;
      PD_HIP(c, hipEventElapsedTime(&all, ev[0], ev[1]), "event");
      ms[0] = ms[1] = -1.0;
      ms[2] = all;
    }
    c->sweep_next = step0 + n_steps;
    return PD_OK;
  }
  if (ms) {
    ev.resize((size_t)2 * n_steps + 1, nullptr);
    for (auto& e : ev) PD_HIP(c, hipEventCreate(&e), "event");
    PD_HIP(c, hipEventRecord(ev[0], st), "event");
  }
  for (int s = step0; s < step0 + n_steps; ++s) {
    const int i = s - step0;
    PD_HIP(c, pd::cols(c->N, fb, pf, P, s, st), "cols");
    if (ms) PD_HIP(c, hipEventRecord(ev[2 * i + 1], st), "event");
    PD_HIP(c, pd::rows(c->N, fb, pf, P, s == 0 ? 1 : 2, 0, st), "rows");
    if (ms) PD_HIP(c, hipEventRecord(ev[2 * i + 2], st), "event");
  }
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  if (ms) {
    double tc = 0.0, tr = 0.0;
    for (int i = 0; i < n_steps; ++i) {
      float a = 0.f, b = 0.f;
      PD_HIP(c, hipEventElapsedTime(&a, ev[2 * i], ev[2 * i + 1]), "event");
      PD_HIP(c, hipEventElapsedTime(&b, ev[2 * i + 1], ev[2 * i + 2]), "event");
      tc += a;
      tr += b;
    }
    float all = 0.f;
    PD_HIP(c, hipEventElapsedTime(&all, ev[0], ev[2 * n_steps]), "event");
    ms[0] = tc;
    ms[1] = tr;
    ms[2] = all;
  }
  c->sweep_next = step0 + n_steps;
  return PD_OK;
}


extern "C" {

pd_status pd_create(pd_ctx** out, int hip_device) {
  if (!out) return PD_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return PD_EINVAL;
  pd_ctx* c = new (std::nothrow) pd_ctx;
  if (!c) return PD_ENOMEM;
  c->device = hip_device;
  DeviceGuard dg(hip_device);
  if (hipStreamCreate(&c->own) != hipSuccess ||
      hipEventCreateWithFlags(&c->sev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->sev[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->sev[2], hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&c->hred, 4 * sizeof(double)) != hipSuccess) {
    delete c;
    return PD_EHIP;
  }
  c->stream = c->own;
  // the static workspace of pd_steps_dev_noalloc: its device address on this
  // device, looked up once per device here (the library's set-up call); a
  // failed lookup is kept and reported by that call alone
  (void)pd::scratch_resolve(hip_device);
  *out = c;
  return PD_OK;
}

void pd_destroy(pd_ctx* c) {
  if (!c) return;
  {
    DeviceGuard dg(c->device);
    if (c->own) {
      (void)hipStreamSynchronize(c->own);
      (void)hipStreamDestroy(c->own);
    }
    if (c->side) {
      (void)hipStreamSynchronize(c->side);
      (void)hipStreamDestroy(c->side);
    }
    for (hipStream_t* p : {&c->cst, &c->fst})
      if (*p) {
        (void)hipStreamSynchronize(*p);
        (void)hipStreamDestroy(*p);
      }
    for (auto& e : c->sev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : c->bev)
      if (e) (void)hipEventDestroy(e);
    if (c->hred) (void)hipHostFree(c->hred);
    lg_release(c);
    c->tw.release(); c->twc.release(); c->twf.release(); c->twcf.release();
    c->U.release(); c->Fo.release(); c->Gold.release();
    c->Hf.release(); c->T1f.release(); c->Uprev.release(); c->t0s.release();
    c->Bc.release(); c->Hc.release(); c->T1c.release(); c->T2c.release(); c->red.release();
    c->ftab.release(); c->Rf.release(); c->Rc.release(); c->wR.release();
    c->flag.release(); c->wB.release(); c->wH.release(); c->wT1.release();
    c->wt0.release();
  }
  delete c;
}

const char* pd_last_error(const pd_ctx* c) { return c ? c->err.c_str() : "null context"; }

pd_status pd_set_stream(pd_ctx* c, void* s) {
  if (!c) return PD_EINVAL;
  c->stream = s ? static_cast<hipStream_t>(s) : c->own;
  return PD_OK;
}

pd_status pd_set_pipeline(pd_ctx* c, int chunks, int speculate) {
  if (!c) return PD_EINVAL;
  if (chunks < 0 || chunks > 64) return fail(c, PD_EINVAL, "chunks must be in [0, 64]");
  if (speculate < 0 || speculate > 2) return fail(c, PD_EINVAL, "speculate must be 0, 1 or 2");
  c->pipe_chunks = chunks;
  c->pipe_spec = speculate;
  return PD_OK;
}

pd_status pd_set_fine_blocking(pd_ctx* c, int group, int streams) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (group < -1) return fail(c, PD_EINVAL, "group must be -1 (default), 0 (off) or positive");
  if (group > 0 && (streams < 1 || streams > 3)) return fail(c, PD_EINVAL, "streams must be in [1, 3]");
  c->blk_g = group;
  c->blk_s = group > 0 ? streams : 0;
  return PD_OK;
}

pd_status pd_get_fine_blocking(pd_ctx* c, int* group, int* streams) {
  if (!c || !group || !streams) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  fine_blocking(c, c->P, group, streams);
  return PD_OK;
}

pd_status pd_set_path(pd_ctx* c, pd_path p) {
  if (!c) return PD_EINVAL;
  if (p != PD_PATH_AUTO && p != PD_PATH_MULTI && p != PD_PATH_SINGLE && p != PD_PATH_MULTI2)
    return fail(c, PD_EINVAL, "unknown path %d", (int)p);
  c->path = p;
  return PD_OK;
}

pd_status pd_set_scheme(pd_ctx* c, pd_scheme fine, pd_scheme coarse) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  for (int v : {(int)fine, (int)coarse})
    if (v < PD_SCHEME_SBDF2 || v > PD_SCHEME_RK111) return fail(c, PD_EINVAL, "unknown scheme %d", v);
  if (coarse != PD_SCHEME_SBDF2 && c->coarse_form == PD_COARSE_CONV)
    return fail(c, PD_EINVAL, "the convolution form of the coarse sweep steps SBDF2 only");
  if (c->prec == PD_C64 && (fine != PD_SCHEME_SBDF2 || coarse != PD_SCHEME_SBDF2))
    return fail(c, PD_EINVAL, "complex64 steps SBDF2 only");
  c->scheme_f = fine;
  c->scheme_c = coarse;
  c->last_k = -1;
  DeviceGuard dg(c->device);
  return ensure_rk_buffers(c);
}

pd_status pd_set_coarse_form(pd_ctx* c, pd_coarse_form f) {
  if (!c) return PD_EINVAL;
  if (f != PD_COARSE_AUTO && f != PD_COARSE_FFT && f != PD_COARSE_CONV && f != PD_COARSE_MULTI)
    return fail(c, PD_EINVAL, "unknown coarse form %d", (int)f);
  if (f == PD_COARSE_CONV && c->scheme_c != PD_SCHEME_SBDF2)
    return fail(c, PD_EINVAL, "the convolution form of the coarse sweep steps SBDF2 only");
  if (f == PD_COARSE_CONV && c->have_time && c->Nc > 64)
    return fail(c, PD_EINVAL, "the convolution coarse sweep needs N_coarse <= 64");
  if (f == PD_COARSE_FFT && c->prec == PD_C64)
    return fail(c, PD_EINVAL, "complex64 has no one-workgroup FFT coarse sweep");
  c->coarse_form = f;
  return PD_OK;
}

pd_status pd_set_precision(pd_ctx* c, pd_prec prec) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (prec != PD_C128 && prec != PD_C64) return fail(c, PD_EINVAL, "unknown precision %d", (int)prec);
  if (prec == PD_C64 && (c->scheme_f != PD_SCHEME_SBDF2 || c->scheme_c != PD_SCHEME_SBDF2))
    return fail(c, PD_EINVAL, "complex64 steps SBDF2 only");
  if (prec == PD_C64 && c->coarse_form == PD_COARSE_FFT)
    return fail(c, PD_EINVAL, "complex64 has no one-workgroup FFT coarse sweep");
  if (prec == c->prec) return PD_OK;
  DeviceGuard dg(c->device);
  c->sweep_next = -1;
  c->have_time = c->have_initial = false;
  c->resume_k = -1;
  c->last_k = -1;
  lg_release(c);
  c->U.release(); c->Fo.release(); c->Gold.release(); c->Hf.release(); c->T1f.release();
  c->Uprev.release(); c->Bc.release(); c->Hc.release(); c->T1c.release();
  c->T2c.release();
  c->prec = prec;
  return PD_OK;
}

pd_status pd_set_problem(pd_ctx* c, pd_flow flow, double Rm, double kz, int N) {
  if (!c) return PD_EINVAL;
  c->sweep_next = -1;
  c->err.clear();
  if (flow != PD_FLOW_NONE && flow != PD_FLOW_ROBERTS && flow != PD_FLOW_GP)
    return fail(c, PD_EINVAL, "unknown flow %d", (int)flow);
  if (!(Rm > 0) || !std::isfinite(Rm)) return fail(c, PD_EINVAL, "Rm must be positive");
  if (!std::isfinite(kz)) return fail(c, PD_EINVAL, "kz must be finite");
  if (!valid_N(N)) return fail(c, PD_EINVAL, "N must be one of 16, 32, 64, 128, 256, 512");
  DeviceGuard dg(c->device);
  c->have_problem = c->have_time = c->have_initial = false;
  c->resume_k = -1;
  c->last_k = -1;
  lg_release(c);
  c->U.release(); c->Fo.release(); c->Gold.release(); c->Hf.release(); c->T1f.release();
  c->Uprev.release();
  c->rows_v = c->cols_v = -1;
  c->flow = flow;
  c->Rm = Rm;
  c->kz = kz;
  c->N = N;
  c->K = box_K(N);
  c->M = box_M(N);
  {
    pd_status ts = upload_twiddles(c, N, c->tw, c->twf, c->stream);
    if (ts != PD_OK) return ts;
  }
  c->have_problem = true;
  return PD_OK;
}

pd_status pd_set_time(pd_ctx* c, double T, int P, double dtf, double dtc, int Nc) {
  if (!c) return PD_EINVAL;
  c->sweep_next = -1;
  c->err.clear();
  if (!c->have_problem) return fail(c, PD_ESTATE, "pd_set_problem not called");
  if (!(T > 0) || !std::isfinite(T)) return fail(c, PD_EINVAL, "T must be positive");
  if (P < 1 || P > 65535) return fail(c, PD_EINVAL, "n_slices must be in [1, 65535]");
  if (Nc == 0) Nc = c->N;
  if (!valid_N(Nc) || Nc > c->N) return fail(c, PD_EINVAL, "N_coarse must be a power of two in [16, N]");
  const double dT = T / P;
  int nf = 0, nc = 0;
  if (!integer_ratio(dT, dtf, &nf)) return fail(c, PD_EINVAL, "slice length is not an integer number of fine steps");
  if (!integer_ratio(dT, dtc, &nc)) return fail(c, PD_EINVAL, "slice length is not an integer number of coarse steps");
  DeviceGuard dg(c->device);
  c->have_time = c->have_initial = false;
  c->resume_k = -1;
  c->last_k = -1;
  lg_release(c);
  c->T = T; c->P = P; c->dT = dT; c->dtf = dtf; c->dtc = dtc; c->Nc = Nc; c->Mc = box_M(Nc);
  c->nf = nf; c->nc = nc;
  if (c->prec == PD_C64 && (c->scheme_f != PD_SCHEME_SBDF2 || c->scheme_c != PD_SCHEME_SBDF2))
    return fail(c, PD_EINVAL, "complex64 steps SBDF2 only");
  if (c->prec == PD_C64 && c->coarse_form == PD_COARSE_FFT)
    return fail(c, PD_EINVAL, "complex64 has no one-workgroup FFT coarse sweep");
  const size_t es = c->esize();
  const size_t box = c->box_elems() * es, rows = c->rows_elems() * es;
  const size_t cbox = (size_t)3 * c->Mc * c->Mc * es, crows = (size_t)3 * c->Mc * Nc * es;
  PD_HIP(c, c->U.ensure(box * (P + 1)), "alloc U");
  PD_HIP(c, c->Fo.ensure(box * P), "alloc F");
  PD_HIP(c, c->Gold.ensure(box * P), "alloc Gold");
  PD_HIP(c, c->Hf.ensure(box * P), "alloc H");
  PD_HIP(c, c->T1f.ensure(rows * P), "alloc T1");
  PD_HIP(c, c->Uprev.ensure(box), "alloc");
  PD_HIP(c, c->Bc.ensure(cbox), "alloc");
  PD_HIP(c, c->Hc.ensure(cbox), "alloc");
  PD_HIP(c, c->T1c.ensure(crows), "alloc");
  PD_HIP(c, c->T2c.ensure(crows), "alloc");
  PD_HIP(c, c->red.ensure(4 * sizeof(double)), "alloc");
  PD_HIP(c, c->t0s.ensure(sizeof(double) * P), "alloc");
  std::vector<double> t0(P);
  for (int n = 0; n < P; ++n) t0[n] = n * dT;
  PD_HIP(c, hipMemcpy(c->t0s.p, t0.data(), sizeof(double) * P, hipMemcpyHostToDevice), "copy");
  {
    pd_status ts = upload_twiddles(c, Nc, c->twc, c->twcf, c->stream);
    if (ts != PD_OK) return ts;
  }
  PD_HIP(c, hipMemset(c->U.p, 0, box * (P + 1)), "memset");
  // phases of the time-dependent flow at the coarse step times t = n dT + j dt_c:
  // (cos py, sin py, cos px, sin px) with px = cos t, py = sin t
  c->ftab.release();
  if ((size_t)P * nc <= ((size_t)1 << 24)) {
    std::vector<double> ft((size_t)4 * P * nc);
    for (int n = 0; n < P; ++n)
      for (int j = 0; j < nc; ++j) {
        const double t = n * dT + j * dtc;
        const double px = std::cos(t), py = std::sin(t);
        double* q = &ft[4 * ((size_t)n * nc + j)];
        q[0] = std::cos(py);
        q[1] = std::sin(py);
        q[2] = std::cos(px);
        q[3] = std::sin(px);
      }
    PD_HIP(c, c->ftab.ensure(ft.size() * sizeof(double)), "alloc");
    PD_HIP(c, hipMemcpy(c->ftab.p, ft.data(), ft.size() * sizeof(double), hipMemcpyHostToDevice), "copy");
  }
  c->have_time = true;
  return ensure_rk_buffers(c);
}

pd_status pd_set_initial_dev(pd_ctx* c, const void* d_b0, void* s) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (!d_b0) return fail(c, PD_EINVAL, "null pointer argument");
  DeviceGuard dg(c->device);
  hipStream_t st = static_cast<hipStream_t>(s);
  pd_status r = check_box_dev(c, d_b0, c->N, 1, st);
  if (r != PD_OK) return r;
  if (c->prec == PD_C64)
    PD_HIP(c, pd::pack(static_cast<const cplx*>(d_b0), c->U.as<cplxf>(), c->N, c->M, 1, st), "pack");
  else
    PD_HIP(c, pd::pack(static_cast<const cplx*>(d_b0), c->U.as<cplx>(), c->N, c->M, 1, st), "pack");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  c->have_initial = true;
  c->resume_k = -1;
  c->last_k = -1;
  return PD_OK;
}

pd_status pd_set_initial(pd_ctx* c, const double* b0) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (!b0) return fail(c, PD_EINVAL, "null pointer argument");
  const int N = c->N, K = c->K;
  for (int comp = 0; comp < 3; ++comp)
    for (int my = 0; my < N; ++my)
      for (int mx = 0; mx < N; ++mx) {
        const int ky = my < N / 2 ? my : my - N, kx = mx < N / 2 ? mx : mx - N;
        const size_t i = 2 * (((size_t)comp * N + my) * N + mx);
        if ((ky < -K || ky > K || kx < -K || kx > K) && (b0[i] != 0.0 || b0[i + 1] != 0.0))
          return fail(c, PD_EINVAL, "initial field has nonzero coefficients outside the 2/3 box");
      }
  DeviceGuard dg(c->device);
  DevBuf tmp;
  const size_t bytes = (size_t)3 * N * N * sizeof(cplx);
  PD_HIP(c, tmp.ensure(bytes), "alloc");
  PD_HIP(c, hipMemcpyAsync(tmp.p, b0, bytes, hipMemcpyHostToDevice, c->stream), "copy");
  if (c->prec == PD_C64)
    PD_HIP(c, pd::pack(tmp.as<cplx>(), c->U.as<cplxf>(), N, c->M, 1, c->stream), "pack");
  else
    PD_HIP(c, pd::pack(tmp.as<cplx>(), c->U.as<cplx>(), N, c->M, 1, c->stream), "pack");
  PD_HIP(c, hipStreamSynchronize(c->stream), "sync");
  c->have_initial = true;
  c->resume_k = -1;
  c->last_k = -1;
  return PD_OK;
}

pd_status pd_steps_dev(pd_ctx* c, const double* t0, int batch, double dt, int n_steps,
                       const void* d_in, void* d_out, void* s) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  return run_propagator(c, t0, batch, dt, n_steps, c->N, d_in, d_out, static_cast<hipStream_t>(s),
                        c->scheme_f);
}

pd_status pd_fine_dev(pd_ctx* c, const double* t0, int batch, const void* d_in, void* d_out,
                      void* s) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  return run_propagator(c, t0, batch, c->dtf, c->nf, c->N, d_in, d_out, static_cast<hipStream_t>(s),
                        c->scheme_f);
}

pd_status pd_coarse_dev(pd_ctx* c, const double* t0, int batch, const void* d_in, void* d_out,
                        void* s) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  return run_propagator(c, t0, batch, c->dtc, c->nc, c->Nc, d_in, d_out, static_cast<hipStream_t>(s),
                        c->scheme_c);
}

pd_status pd_parareal(pd_ctx* c, double tol, int max_iter, pd_report* rep) {
  if (!c) return PD_EINVAL;
  c->sweep_next = -1;
  c->err.clear();
  if (!c->have_initial) return fail(c, PD_ESTATE, "pd_set_initial not called");
  if (max_iter < 0 || max_iter > PD_MAX_ITER) return fail(c, PD_EINVAL, "max_iter must be in [0, %d]", PD_MAX_ITER);
  if (!(tol >= 0)) return fail(c, PD_EINVAL, "tol must be >= 0");
  DeviceGuard dg(c->device);
  const auto wall0 = std::chrono::steady_clock::now();
  // resumed run (pd_set_slices): U holds U^k, Gold holds G(U^k_n)
  const int kres = c->resume_k;
  const bool learned = c->lg.enabled && c->lg.init;
  if (kres >= 0 && !learned && !c->have_gold)
    return fail(c, PD_EINVAL, "resuming plain-G Parareal needs the coarse values (pd_set_slices Gold)");
  if (kres >= 0 && max_iter <= kres)
    return fail(c, PD_EINVAL, "max_iter must exceed the resumed iteration %d", kres);
  c->resume_k = -1;
  c->last_k = -1;
  {
    pd_status rs = ensure_rk_buffers(c);
    if (rs != PD_OK) return rs;
  }
  if (c->pipe_chunks > 1) return parareal_pipelined(c, tol, max_iter, kres, rep);
  if (c->prec == PD_C64) return parareal_plain<cplxf>(c, tol, max_iter, kres, false, rep, wall0);
  return parareal_plain<cplx>(c, tol, max_iter, kres, learned, rep, wall0);
}

pd_status pd_parareal_continue(pd_ctx* c, double tol, int max_iter, pd_report* rep) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_initial || c->last_k < 0)
    return fail(c, PD_ESTATE, "no Parareal run on the current state to continue");
  if (max_iter <= c->last_k || max_iter > PD_MAX_ITER)
    return fail(c, PD_EINVAL, "max_iter must be in (%d, %d]", c->last_k, PD_MAX_ITER);
  if (!(tol >= 0)) return fail(c, PD_EINVAL, "tol must be >= 0");
  // the state after the last completed iteration is in place: U^k, and for
  // the plain coarse propagator G(U^k_n) in Gold
  c->resume_k = c->last_k;
  c->have_gold = true;
  return pd_parareal(c, tol, max_iter, rep);
}

pd_status pd_profile_fine(pd_ctx* c, int reps, double* ms) {
  if (!c) return PD_EINVAL;
  c->sweep_next = -1;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (reps < 1 || !ms) return fail(c, PD_EINVAL, "reps must be >= 1 and ms non-null");
  DeviceGuard dg(c->device);
  return c->prec == PD_C64 ? profile_fine_t<cplxf>(c, reps, ms) : profile_fine_t<cplx>(c, reps, ms);
}

pd_status pd_fine_sweep_steps(pd_ctx* c, int step0, int n_steps, double* ms) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (c->scheme_f != PD_SCHEME_SBDF2) return fail(c, PD_EINVAL, "the fine stepper must be SBDF2");
  if (step0 < 0 || n_steps < 1 || step0 + n_steps > c->nf)
    return fail(c, PD_EINVAL, "steps [%d, %d) outside the slice's %d fine steps", step0,
                step0 + n_steps, c->nf);
  if (step0 > 0 && c->sweep_next != step0)
    return fail(c, PD_ESTATE, "the fine sweep stands at step %d, not %d", c->sweep_next, step0);
  DeviceGuard dg(c->device);
  return c->prec == PD_C64 ? fine_sweep_steps_t<cplxf>(c, step0, n_steps, ms)
                           : fine_sweep_steps_t<cplx>(c, step0, n_steps, ms);
}

// ---- autotuner --------------------------------------------------------------
}  // extern "C"

namespace {

// cache key: gfx architecture, HIP runtime version (launch shapes tuned
// under one runtime and compiler need not suit another), grid, batch
std::string tune_key(int device, int N, int P) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  int rt = 0;
  if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
  return arch + "|hip" + std::to_string(rt) + "|" + std::to_string(N) + "|" + std::to_string(P);
}

// The cache is a flat JSON object {"<arch>|<N>|<batch>": [rows, cols], ...}.
// Cache entries hold [rows, cols] or [rows, cols, group, streams] (the
// fine-sweep blocking); v receives up to four values, the count is returned
// (0: no entry).
int parse_entry(const char* p, int v[4]) {
  const int n = std::sscanf(p, " : [ %d , %d , %d , %d ]", &v[0], &v[1], &v[2], &v[3]);
  return n >= 2 ? n : 0;
}

int cache_lookup(const char* path, const std::string& key, int v[4]) {
  FILE* f = std::fopen(path, "r");
  if (!f) return 0;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  std::fclose(f);
  const std::string q = "\"" + key + "\"";
  const size_t at = text.find(q);
  if (at == std::string::npos) return 0;
  return parse_entry(text.c_str() + at + q.size(), v);
}

void cache_store(const char* path, const std::string& key, const int val[4]) {
  struct Entry {
    std::string k;
    int v[4];
    int n;
  };
  std::vector<Entry> entries;
  FILE* f = std::fopen(path, "r");
  if (f) {
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    size_t pos = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
      const size_t end = text.find('"', pos + 1);
      if (end == std::string::npos) break;
      Entry e;
      e.k = text.substr(pos + 1, end - pos - 1);
      e.n = parse_entry(text.c_str() + end + 1, e.v);
      if (e.n > 0 && e.k != key) entries.push_back(e);
      pos = end + 1;
    }
  }
  Entry mine;
  mine.k = key;
  mine.n = 4;
  for (int i = 0; i < 4; ++i) mine.v[i] = val[i];
  entries.push_back(mine);
  f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < entries.size(); ++i) {
    std::fprintf(f, "  \"%s\": [", entries[i].k.c_str());
    for (int j = 0; j < entries[i].n; ++j) std::fprintf(f, "%s%d", j ? ", " : "", entries[i].v[j]);
    std::fprintf(f, "]%s\n", i + 1 < entries.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  std::fclose(f);
}

}  // namespace

extern "C" {

pd_status pd_variant_info(int N, int kind, int v, int* a, int* b) {
  if (!a || !b || (kind != 0 && kind != 1)) return PD_EINVAL;
  if (v == -1) {
    *a = pd::variant_count(N, kind);
    *b = 0;
    return *a > 0 ? PD_OK : PD_EINVAL;
  }
  return pd::variant_describe(N, kind, v, a, b) == 0 ? PD_OK : PD_EINVAL;
}

pd_status pd_select_variant(int N, int rows_v, int cols_v) {
  return pd::variant_select(N, rows_v, cols_v) == 0 ? PD_OK : PD_EINVAL;
}

pd_status pd_autotune(pd_ctx* c, int reps, const char* cache_path, int* chosen, double* ms) {
  if (!c) return PD_EINVAL;
  c->sweep_next = -1;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (reps < 1) return fail(c, PD_EINVAL, "reps must be >= 1");
  if (c->prec == PD_C64) return fail(c, PD_EINVAL, "complex64 has one launch shape per grid");
  DeviceGuard dg(c->device);
  const int P = c->P;
  const std::string key = tune_key(c->device, c->N, P);
  int cv4[4] = {0, 0, -1, 0};
  const int cn = cache_path ? cache_lookup(cache_path, key, cv4) : 0;
  const int rv = cv4[0], cv = cv4[1];
  if (cn >= 2 && rv >= 0 && rv < pd::variant_count(c->N, 0) && cv >= 0 &&
      cv < pd::variant_count(c->N, 1)) {
    c->rows_v = rv;
    c->cols_v = cv;
    if (cn == 4 && cv4[2] >= 0 && (cv4[2] == 0 || (cv4[3] >= 1 && cv4[3] <= 3))) {
      c->blk_g = cv4[2];
      c->blk_s = cv4[2] > 0 ? cv4[3] : 0;
    }
    if (chosen) {
      chosen[0] = rv;
      chosen[1] = cv;
    }
    if (ms) ms[0] = ms[1] = 0.0;
    return PD_OK;
  }
  hipStream_t st = c->stream;
  const size_t box = c->box_elems();
  hipEvent_t ev[2];
  for (auto& e : ev) PD_HIP(c, hipEventCreate(&e), "event");
  struct EvFree {
    hipEvent_t* e;
    ~EvFree() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
  } evf{ev};
  pd::FieldBatch fb;
  fb.B = c->Fo.as<cplx>();
  fb.H = c->Hf.as<cplx>();
  fb.T1 = c->T1f.as<cplx>();
  fb.T2 = fb.T1;
  fb.t0 = c->t0s.as<double>();
  fb.tw = c->tw.as<cplx>();
  const pd::Problem pf = make_problem(c, c->dtf);
  int cur_r = 0, cur_c = 0;
  pd::variant_current(c->N, &cur_r, &cur_c);
  if (c->rows_v >= 0) cur_r = c->rows_v;
  if (c->cols_v >= 0) cur_c = c->cols_v;
  // launches of the row (kind 0, an SBDF2 step) or column phase over nf
  // fields with batch variants (rows_v, cols_v)
  auto timed = [&](int kind, int nf, int rows_v, int cols_v, float* out) -> hipError_t {
    pd::FieldBatch f = fb;
    f.rows_v = rows_v;
    f.cols_v = cols_v;
    hipError_t e = hipEventRecord(ev[0], st);
    for (int i = 0; i < reps && e == hipSuccess; ++i)
      e = kind == 0 ? pd::rows(c->N, f, pf, nf, 2, 0, st) : pd::cols(c->N, f, pf, nf, 1, st);
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(out, ev[0], ev[1]);
    return e;
  };
  // fastest row variant, then the fastest column variant, on nf fields
  auto tune = [&](int nf, int bestv[2], float best[2]) -> hipError_t {
    best[0] = best[1] = 1e30f;
    bestv[0] = cur_r;
    bestv[1] = cur_c;
    for (int kind = 0; kind < 2; ++kind) {
      const int nv = pd::variant_count(c->N, kind);
      for (int v = 0; v < nv; ++v) {
        const int r = kind == 0 ? v : bestv[0], cc = kind == 1 ? v : cur_c;
        float t = 0;
        hipError_t e = timed(kind, nf, r, cc, &t);  // warm-up
        if (e == hipSuccess) e = timed(kind, nf, r, cc, &t);
        if (e != hipSuccess) return e;
        if (t < best[kind]) {
          best[kind] = t;
          bestv[kind] = v;
        }
      }
    }
    return hipSuccess;
  };
  PD_HIP(c, hipMemcpyAsync(c->Fo.p, c->U.p, (size_t)P * box * sizeof(cplx), hipMemcpyDeviceToDevice, st), "copy");
  PD_HIP(c, pd::rows(c->N, fb, pf, P, 0, 0, st), "rows");
  float best[2];
  int bestv[2];
  PD_HIP(c, tune(P, bestv, best), "autotune");
  c->rows_v = bestv[0];
  c->cols_v = bestv[1];
  if (chosen) {
    chosen[0] = bestv[0];
    chosen[1] = bestv[1];
  }
  if (ms) {
    ms[0] = best[0] / reps;
    ms[1] = best[1] / reps;
  }
  // the fine sweep's blocking (groups of fields that run all their steps back
  // to back, dealt to streams): each candidate runs BLK_STEPS steps of every
  // field in its order with the chosen launch shapes
  {
    constexpr int BLK_STEPS = 12;
    static const int cand[][2] = {{0, 1}, {1, 3}, {2, 3}, {3, 3}, {4, 3}, {8, 3}, {16, 3},
                                  {2, 2}, {4, 2}, {8, 2}, {16, 2}, {32, 2}};
    pd::FieldBatch q = fb;
    q.rows_v = c->rows_v;
    q.cols_v = c->cols_v;
    auto steps = [&](const pd::FieldBatch& x, int ng, hipStream_t s) -> hipError_t {
      hipError_t e = hipSuccess;
      for (int k = 1; k <= BLK_STEPS && e == hipSuccess; ++k) {
        e = pd::cols(c->N, x, pf, ng, k, s);
        if (e == hipSuccess) e = pd::rows(c->N, x, pf, ng, 2, 0, s);
      }
      return e;
    };
    auto sweep = [&](int g, int ns) -> hipError_t {
      return g == 0 ? steps(q, P, st) : over_groups(c, q, P, g, ns, st, steps);
    };
    PD_HIP(c, sweep(0, 1), "autotune");  // warm-up
    float bt = 1e30f;
    int bg = 0, bs = 1;
    for (const auto& cd : cand) {
      if (cd[0] >= P) continue;
      float t = 0;
      PD_HIP(c, hipEventRecord(ev[0], st), "event");
      PD_HIP(c, sweep(cd[0], cd[1]), "autotune");
      PD_HIP(c, hipEventRecord(ev[1], st), "event");
      PD_HIP(c, hipEventSynchronize(ev[1]), "sync");
      PD_HIP(c, hipEventElapsedTime(&t, ev[0], ev[1]), "event");
      if (t < bt) {
        bt = t;
        bg = cd[0];
        bs = cd[1];
      }
    }
    c->blk_g = bg;
    c->blk_s = bg > 0 ? bs : 0;
  }
  if (cache_path) {
    const int val[4] = {bestv[0], bestv[1], c->blk_g, c->blk_g > 0 ? c->blk_s : 1};
    cache_store(cache_path, key, val);
  }
  return PD_OK;
}

pd_status pd_get_slices_dev(const pd_ctx* cc, void* d_out, void* s) {
  pd_ctx* c = const_cast<pd_ctx*>(cc);
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (!d_out) return fail(c, PD_EINVAL, "null pointer argument");
  DeviceGuard dg(c->device);
  hipStream_t st = static_cast<hipStream_t>(s);
  if (c->prec == PD_C64)
    PD_HIP(c, pd::unpack(c->U.as<cplxf>(), static_cast<cplx*>(d_out), c->N, c->M, (size_t)c->P + 1, st), "unpack");
  else
    PD_HIP(c, pd::unpack(c->U.as<cplx>(), static_cast<cplx*>(d_out), c->N, c->M, (size_t)c->P + 1, st), "unpack");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  return PD_OK;
}

pd_status pd_get_fine_states_dev(const pd_ctx* cc, int first, int count, void* d_out, void* s) {
  pd_ctx* c = const_cast<pd_ctx*>(cc);
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (first < 0 || count < 0 || first + count > c->P)
    return fail(c, PD_EINVAL, "slices [%d, %d) outside [0, %d)", first, first + count, c->P);
  if (count == 0) return PD_OK;
  if (!d_out) return fail(c, PD_EINVAL, "null pointer argument");
  DeviceGuard dg(c->device);
  hipStream_t st = static_cast<hipStream_t>(s);
  if (c->prec == PD_C64)
    PD_HIP(c, pd::unpack(c->Fo.as<cplxf>() + (size_t)first * c->box_elems(), static_cast<cplx*>(d_out),
                         c->N, c->M, (size_t)count, st), "unpack");
  else
    PD_HIP(c, pd::unpack(c->Fo.as<cplx>() + (size_t)first * c->box_elems(), static_cast<cplx*>(d_out),
                         c->N, c->M, (size_t)count, st), "unpack");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  return PD_OK;
}

pd_status pd_get_slices(const pd_ctx* cc, double* out) {
  pd_ctx* c = const_cast<pd_ctx*>(cc);
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (!out) return fail(c, PD_EINVAL, "null pointer argument");
  DeviceGuard dg(c->device);
  const size_t full = (size_t)3 * c->N * c->N;
  DevBuf tmp;
  PD_HIP(c, tmp.ensure(full * sizeof(cplx)), "alloc");
  for (int n = 0; n <= c->P; ++n) {
    if (c->prec == PD_C64)
      PD_HIP(c, pd::unpack(c->U.as<cplxf>() + (size_t)n * c->box_elems(), tmp.as<cplx>(), c->N, c->M, 1, c->stream), "unpack");
    else
      PD_HIP(c, pd::unpack(c->U.as<cplx>() + (size_t)n * c->box_elems(), tmp.as<cplx>(), c->N, c->M, 1, c->stream), "unpack");
    PD_HIP(c, hipMemcpyAsync(out + 2 * full * n, tmp.p, full * sizeof(cplx), hipMemcpyDeviceToHost, c->stream), "copy");
  }
  PD_HIP(c, hipStreamSynchronize(c->stream), "sync");
  return PD_OK;
}

pd_status pd_slice_norms(const pd_ctx* cc, double* norms) {
  pd_ctx* c = const_cast<pd_ctx*>(cc);
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (!norms) return fail(c, PD_EINVAL, "null pointer argument");
  DeviceGuard dg(c->device);
  DevBuf d;
  PD_HIP(c, d.ensure(sizeof(double) * (c->P + 1)), "alloc");
  if (c->prec == PD_C64)
    PD_HIP(c, pd::norms2(c->U.as<cplxf>(), c->box_elems(), c->P + 1, d.as<double>(), c->stream), "norms");
  else
    PD_HIP(c, pd::norms2(c->U.as<cplx>(), c->box_elems(), c->P + 1, d.as<double>(), c->stream), "norms");
  PD_HIP(c, hipMemcpyAsync(norms, d.p, sizeof(double) * (c->P + 1), hipMemcpyDeviceToHost, c->stream), "copy");
  PD_HIP(c, hipStreamSynchronize(c->stream), "sync");
  for (int n = 0; n <= c->P; ++n) norms[n] = std::sqrt(norms[n]);
  return PD_OK;
}

pd_status pd_growth_rate(const pd_ctx* cc, double* gamma) {
  pd_ctx* c = const_cast<pd_ctx*>(cc);
  if (!c) return PD_EINVAL;
  if (!gamma) return fail(c, PD_EINVAL, "null pointer argument");
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (c->P < 2) return fail(c, PD_EINVAL, "growth rate needs at least 2 slices");
  std::vector<double> nrm(c->P + 1);
  pd_status s = pd_slice_norms(c, nrm.data());
  if (s != PD_OK) return s;
  const int n0 = (c->P + 1) / 2;
  const int cnt = c->P + 1 - n0;
  double tm = 0, ym = 0;
  std::vector<double> y(cnt), t(cnt);
  for (int i = 0; i < cnt; ++i) {
    if (!(nrm[n0 + i] > 0) || !std::isfinite(nrm[n0 + i]))
      return fail(c, PD_EUNSTABLE, "slice norm is zero or not finite");
    t[i] = (n0 + i) * c->dT;
    y[i] = std::log(nrm[n0 + i]);
    tm += t[i];
    ym += y[i];
  }
  tm /= cnt;
  ym /= cnt;
  double sxy = 0, sxx = 0;
  for (int i = 0; i < cnt; ++i) {
    sxy += (t[i] - tm) * (y[i] - ym);
    sxx += (t[i] - tm) * (t[i] - tm);
  }
  *gamma = sxy / sxx;
  return PD_OK;
}

}  // extern "C"
