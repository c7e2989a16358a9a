// Pipelined Parareal with the plain coarse propagator: the serial coarse
// sweep runs on its own stream, cut into chunks of consecutive slices, and
// the fine sweep of a chunk starts as soon as the coarse sweep has produced
// that chunk's start values (Section 3, eq. parareal: F(U^{k-1}_n) needs only
// U^{k-1}_n, and the sweep of iteration k at slice n needs only F(U^{k-1}_n)
// and U^k_n).  The fine sweeps of iteration k + 1 thus overlap the coarse
// sweep of iteration k, and the one-workgroup coarse kernel shares the chip
// with the fine kernels.  Every slice goes through the same kernels with the
// same inputs as in the unpipelined order, so the iterates are bitwise equal.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.hpp"

using namespace pd::ctxh;

namespace {

struct Events {
  std::vector<hipEvent_t> ev;
  ~Events() {
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  hipError_t make(size_t n) {
    ev.assign(n, nullptr);
    for (auto& e : ev) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  }
};

}  // namespace

namespace pd {
namespace ctxh {

pd_status ensure_pipeline_streams(pd_ctx* c) {
  for (hipStream_t* p : {&c->cst, &c->fst})
    if (!*p) PD_HIP(c, hipStreamCreateWithFlags(p, hipStreamNonBlocking), "stream");
  return PD_OK;
}

// Same contract as pd_parareal (plain coarse propagator only); kres >= 0
// resumes after iteration kres with U and Gold already loaded.  CT: the
// context's complex type (complex128 or complex64).
template <class CT>
static pd_status pipelined_t(pd_ctx* c, double tol, int max_iter, int kres, bool learned,
                             pd_report* rep) {
  const auto wall0 = std::chrono::steady_clock::now();
  pd_status s = ensure_pipeline_streams(c);
  if (s != PD_OK) return s;
  const size_t box = c->box_elems(), rows = c->rows_elems();
  const int P = c->P;
  const int Sc = (P + std::max(1, std::min(c->pipe_chunks, P)) - 1) / std::max(1, std::min(c->pipe_chunks, P));
  const int C = (P + Sc - 1) / Sc;  // chunks of Sc slices, the last one nonempty
  auto lo = [&](int ch) { return std::min(P, ch * Sc); };
  auto hi = [&](int ch) { return std::min(P, (ch + 1) * Sc); };
  CT* U = c->U.as<CT>();
  CT* Fo = c->Fo.as<CT>();
  // two fine streams, the context's own and one more: a chunk's fine launches
  // are latency-bound, so chunks run side by side to keep the chip as busy as
  // one full sweep.  HIP spreads a process's streams over a few hardware
  // queues (four by default); more streams would share a queue and
  // serialise, so the coarse stream, the two fine streams and the caller's
  // default stream are all this schedule uses
  hipStream_t fs[2] = {c->stream, c->fst};
  const int NFS = std::min(C, 2);
  hipStream_t cs = c->cst;

  // per parity of the iteration and chunk: fine start, start values copied,
  // fine end, coarse start, coarse end; then the join events
  Events E;
  PD_HIP(c, E.make((size_t)10 * C + 5), "event");
  auto ev = [&](int kind, int k, int ch) { return E.ev[((size_t)kind * 2 + (k & 1)) * C + ch]; };
  auto Fs = [&](int k, int ch) { return ev(0, k, ch); };
  auto Fc = [&](int k, int ch) { return ev(1, k, ch); };
  auto Fe = [&](int k, int ch) { return ev(2, k, ch); };
  auto Gs = [&](int k, int ch) { return ev(3, k, ch); };
  auto Ge = [&](int k, int ch) { return ev(4, k, ch); };
  hipEvent_t evIn = E.ev[10 * C], evRed = E.ev[10 * C + 1];
  hipEvent_t evJoin[2] = {E.ev[10 * C + 2], E.ev[10 * C + 3]};

  pd::SweepArgsT<CT> sa;
  sa.U = U;
  sa.Fo = Fo;
  sa.Gold = c->Gold.as<CT>();
  sa.Uprev = c->Uprev.as<CT>();
  sa.Bc = c->Bc.as<CT>();
  sa.Hc = c->Hc.as<CT>();
  sa.T1c = c->T1c.as<CT>();
  sa.T2c = c->T2c.as<CT>();
  sa.twc = c->twidc<CT>();
  sa.Rc = c->Rc.as<CT>();
  sa.ftab = c->ftab.as<double>();
  sa.dT = c->dT;
  sa.M = c->M;
  sa.nsteps = c->nc;
  const pd::Problem pc = make_problem(c, c->dtc, c->scheme_c),
                    pf = make_problem(c, c->dtf, c->scheme_f);
  // one run of the serial coarse sweep over slices [sa.n0, sa.P): the plain
  // propagator, or the learned one in difference form (n0 = the first slice
  // the iteration sweeps; defect sums when sa.red is set)
  pd_status lg_status = PD_OK;
  auto sweep_k = [&](int n0) -> hipError_t {
    if constexpr (sizeof(CT) == sizeof(cplx)) {
      if (learned) {
        lg_status = lg_sweep_range(c, sa.n0, sa.P, n0, sa.mode == 0, sa.red != nullptr, cs);
        return lg_status == PD_OK ? hipSuccess : hipErrorUnknown;
      }
    }
    return coarse_sweep(c, sa, pc, cs);
  };

  // everything earlier on the caller's stream comes first
  PD_HIP(c, hipEventRecord(evIn, c->stream), "event");
  PD_HIP(c, hipStreamWaitEvent(cs, evIn, 0), "wait");
  for (int i = 0; i < NFS; ++i) PD_HIP(c, hipStreamWaitEvent(fs[i], evIn, 0), "wait");

  pd_report r;
  std::memset(&r, 0, sizeof r);
  r.k_con = -1;
  // initial coarse run (iteration 0), chunk by chunk
  const int k0 = kres >= 0 ? kres : 0;
  for (int ch = 0; ch < C; ++ch) {
    PD_HIP(c, hipEventRecord(Gs(k0, ch), cs), "event");
    if (kres < 0 && lo(ch) < hi(ch)) {
      sa.mode = 0;
      sa.n0 = lo(ch);
      sa.P = hi(ch);
      sa.red = nullptr;
      const hipError_t e = sweep_k(0);
      if (e != hipSuccess) return lg_status != PD_OK ? lg_status : hipfail(c, e, "coarse sweep");
    }
    PD_HIP(c, hipEventRecord(Ge(k0, ch), cs), "event");
  }

  // fine sweep of iteration k over chunks [c0, c1)
  auto enqueue_fine = [&](int k, int c0, int c1) -> pd_status {
    const int n0 = std::min(k - 1, P - 1);
    for (int ch = c0; ch < c1; ++ch) {
      hipStream_t st = fs[ch % NFS];
      PD_HIP(c, hipStreamWaitEvent(st, Ge(k - 1, ch), 0), "wait");
      PD_HIP(c, hipEventRecord(Fs(k, ch), st), "event");
      const int a = std::max(lo(ch), n0), b = hi(ch);
      if (a < b)
        PD_HIP(c, hipMemcpyAsync(Fo + (size_t)a * box, U + (size_t)a * box,
                                 (size_t)(b - a) * box * sizeof(CT), hipMemcpyDeviceToDevice, st),
               "copy");
      PD_HIP(c, hipEventRecord(Fc(k, ch), st), "event");
      if (a < b) {
        pd::FieldBatchT<CT> fb;
        fb.B = Fo + (size_t)a * box;
        fb.H = c->Hf.as<CT>() + (size_t)a * box;
        fb.T1 = c->T1f.as<CT>() + (size_t)a * rows;
        fb.T2 = fb.T1;
        fb.t0 = c->t0s.as<double>() + a;
        fb.tw = c->twid<CT>();
        c->shapes(fb);
        if constexpr (sizeof(CT) == sizeof(cplx))
          if (c->scheme_f != PD_SCHEME_SBDF2) fb.R = c->Rf.as<cplx>() + (size_t)4 * a * box;
        int path = choose_path(c, b - a);
        if (path == PD_PATH_MULTI2) path = PD_PATH_MULTI;  // the chunks already use two streams
        // blocked in groups on the chunk's own stream, about as many fields
        // in flight as the context's blocking keeps on its streams
        int g = 0, gs = 1;
        if (path == pd::PATH_MULTI) fine_blocking(c, b - a, &g, &gs);
        if (g > 0) g = std::max(1, (g * gs + NFS - 1) / NFS);
        if (g > 0 && g < b - a)
          PD_HIP(c, over_groups(c, fb, b - a, g, 1, st,
                                [&](const pd::FieldBatchT<CT>& q, int ng, hipStream_t x) {
                                  return pd::propagate(c->N, q, pf, ng, c->nf, pd::PATH_MULTI, x);
                                }),
                 "fine sweep");
        else
          PD_HIP(c, pd::propagate(c->N, fb, pf, b - a, c->nf, path, st), "fine sweep");
      }
      PD_HIP(c, hipEventRecord(Fe(k, ch), st), "event");
    }
    return PD_OK;
  };

  auto ms_between = [&](hipEvent_t a, hipEvent_t b) -> double {
    float ms = 0.f;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? ms * 1e-3 : 0.0;
  };

  pd_status status = PD_NOT_CONVERGED;
  int fine_done = 0;  // chunks of the current iteration already enqueued
  const int kfirst = kres >= 0 ? kres + 1 : 1;
  if (kfirst > max_iter) status = PD_OK;
  for (int k = kfirst; k <= max_iter; ++k) {
    const int n0 = std::min(k - 1, P - 1);
    s = enqueue_fine(k, fine_done, C);
    if (s != PD_OK) return s;
    // coarse sweep of iteration k with the correction, chunk by chunk
    PD_HIP(c, hipMemcpyAsync(c->Uprev.p, U + (size_t)P * box, box * sizeof(CT),
                             hipMemcpyDeviceToDevice, cs), "copy");
    for (int ch = 0; ch < C; ++ch) {
      // this chunk's fine results, and the next chunk's start value U^{k-1}
      // read before this chunk's sweep overwrites it with U^k
      PD_HIP(c, hipStreamWaitEvent(cs, Fe(k, ch), 0), "wait");
      if (ch + 1 < C) PD_HIP(c, hipStreamWaitEvent(cs, Fc(k, ch + 1), 0), "wait");
      PD_HIP(c, hipEventRecord(Gs(k, ch), cs), "event");
      const int a = std::max(lo(ch), n0), b = hi(ch);
      if (a < b) {
        sa.mode = 1;
        sa.n0 = a;
        sa.P = b;
        sa.red = ch == C - 1 ? c->red.as<double>() : nullptr;
        const hipError_t e = sweep_k(n0);
        if (e != hipSuccess) return lg_status != PD_OK ? lg_status : hipfail(c, e, "coarse sweep");
      }
      PD_HIP(c, hipEventRecord(Ge(k, ch), cs), "event");
    }
    PD_HIP(c, hipMemcpyAsync(c->hred, c->red.p, 2 * sizeof(double), hipMemcpyDeviceToHost, cs), "copy");
    PD_HIP(c, hipEventRecord(evRed, cs), "event");
    // the next iteration's fine sweeps go ahead chunk by chunk while this
    // iteration's coarse sweep runs: every chunk (speculate 1), all but the
    // last (0), or every chunk unless the defects so far predict that this
    // iteration converges, sigma_{k-1}^2 / sigma_{k-2} <= tol (2)
    fine_done = 0;
    if (k < max_iter && C > 1) {
      int ahead = c->pipe_spec == 0 ? C - 1 : C;
      if (c->pipe_spec == 2 && k >= 3) {
        const double s1 = r.sigma[k - 2], s2 = r.sigma[k - 3];
        if (s2 > 0.0 && s1 * s1 / s2 <= tol) ahead = 0;
      }
      s = enqueue_fine(k + 1, 0, ahead);
      if (s != PD_OK) return s;
      fine_done = ahead;
    }
    PD_HIP(c, hipEventSynchronize(evRed), "sync");
    for (int ch = 0; ch < C; ++ch) {
      r.t_fine_s += ms_between(Fs(k, ch), Fe(k, ch));
      r.t_coarse_s += ms_between(Gs(k, ch), Ge(k, ch));
    }
    if (k == kfirst && kres < 0)
      for (int ch = 0; ch < C; ++ch) r.t_coarse0_s += ms_between(Gs(0, ch), Ge(0, ch));
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
  // join: later work on the caller's stream follows everything above
  // (including fine sweeps of an iteration that was not needed)
  for (int i = 0; i < NFS; ++i) {
    PD_HIP(c, hipEventRecord(evJoin[i], fs[i]), "event");
    PD_HIP(c, hipStreamWaitEvent(c->stream, evJoin[i], 0), "wait");
  }
  PD_HIP(c, hipEventRecord(evRed, cs), "event");
  PD_HIP(c, hipStreamWaitEvent(c->stream, evRed, 0), "wait");
  PD_HIP(c, hipStreamSynchronize(c->stream), "sync");
  c->last_k = status == PD_EUNSTABLE ? -1 : (r.iters > 0 ? r.iters : (kres >= 0 ? kres : 0));
  r.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
  finish_report(r, P);
  if (rep) *rep = r;
  return status;
}

pd_status parareal_pipelined(pd_ctx* c, double tol, int max_iter, int kres, pd_report* rep) {
  const bool learned = c->lg.enabled && c->lg.init;
  return c->prec == PD_C64 ? pipelined_t<cplxf>(c, tol, max_iter, kres, false, rep)
                           : pipelined_t<cplx>(c, tol, max_iter, kres, learned, rep);
}

}  // namespace ctxh
}  // namespace pd
