// Learned coarse propagator for Parareal (C ABI pd_lg_*): sample generation
// with the library's own fine and coarse propagators, training with Adam on
// the GPU (kernels in nn.hip), and the serial coarse sweep in difference form
//   U^k_{n+1} = F(U^{k-1}_n) + G_learned(U^k_n - U^{k-1}_n),
//   G_learned(D) = G(D) + |D| Net(D/|D|, G(D)/|D|; t_n),
// which is the Parareal update of Section 3 (eq. parareal) for a coarse
// propagator linear in its input.  The plain coarse step G stays inside
// G_learned, and the network is zero at D = 0, so converged slices return F
// bitwise.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <vector>

#include "ctx.hpp"
#include "nn.hpp"

using namespace pd::ctxh;

namespace {

// splitmix64 stream: batch selection and parameter initialisation
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
  double normal() {  // Box-Muller
    double u1 = uniform(), u2 = uniform();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

pd::nn::Net net_of(pd_ctx* c, DevBuf& buf) {
  pd::nn::Net n = pd::nn::view(buf.as<float>(), c->lg.Q, c->lg.Mf, c->lg.L);
  n.f32 = c->lg.f32ops;
  return n;
}

// activation pointer tables for a batch of B
void act_ptrs(pd_ctx* c, int B, std::vector<float*>& h, std::vector<float*>& y) {
  auto& g = c->lg;
  const size_t per = (size_t)B * g.Q * pd::nn::CH;
  h.resize(g.L + 1);
  y.resize(g.L);
  for (int l = 0; l <= g.L; ++l) h[l] = g.act.as<float>() + l * per;
  for (int l = 0; l < g.L; ++l) y[l] = g.ys.as<float>() + l * per;
}

pd_status ensure_batch(pd_ctx* c, int B) {
  auto& g = c->lg;
  if (B <= g.Bcap) return PD_OK;
  const size_t per = (size_t)B * g.Q * pd::nn::CH;
  const size_t rows = (size_t)B * g.Q;
  const int nblk = (int)((rows + 4095) / 4096);
  PD_HIP(c, g.act.ensure(sizeof(float) * per * (g.L + 1)), "alloc");
  PD_HIP(c, g.ys.ensure(sizeof(float) * per * g.L), "alloc");
  PD_HIP(c, g.c.ensure(sizeof(float) * rows * 6), "alloc");
  PD_HIP(c, g.dc.ensure(sizeof(float) * rows * 6), "alloc");
  PD_HIP(c, g.dhA.ensure(sizeof(float) * per), "alloc");
  PD_HIP(c, g.dhB.ensure(sizeof(float) * per), "alloc");
  PD_HIP(c, g.dW.ensure(sizeof(float) * B * 5 * pd::nn::CH * pd::nn::CH), "alloc");
  PD_HIP(c, g.part.ensure(sizeof(float) * nblk * 12 * pd::nn::CH), "alloc");
  PD_HIP(c, g.lpart.ensure(sizeof(double) * 512), "alloc");
  PD_HIP(c, g.sums.ensure(sizeof(double) * 2), "alloc");
  PD_HIP(c, g.bidx.ensure(sizeof(int) * B), "alloc");
  if (g.hbidx) (void)hipHostFree(g.hbidx);
  g.hbidx = nullptr;
  PD_HIP(c, hipHostMalloc((void**)&g.hbidx, sizeof(int) * B), "alloc");
  g.Bcap = B;
  return PD_OK;
}

// grow a device buffer to `bytes`, keeping its first `keep` bytes
pd_status grow(pd_ctx* c, DevBuf& b, size_t bytes, size_t keep, hipStream_t st) {
  if (bytes <= b.bytes && b.p) return PD_OK;
  DevBuf nb;
  PD_HIP(c, nb.ensure(bytes), "alloc");
  if (keep) PD_HIP(c, hipMemcpyAsync(nb.p, b.p, keep, hipMemcpyDeviceToDevice, st), "copy");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  b.release();
  b.p = nb.p;
  b.bytes = nb.bytes;
  nb.p = nullptr;
  nb.bytes = 0;
  return PD_OK;
}

// plain coarse propagation of one compact fine field D (slice n) into g:
// the one-workgroup convolution sweep over a single slice
hipError_t coarse_one(pd_ctx* c, const cplx* D, cplx* g, int n, hipStream_t st) {
  auto& L = c->lg;
  (void)L;
  pd::SweepArgs sa;
  // U = [D, g]: the sweep reads U[0] and writes U[1] = g (and Gold[0] = g)
  sa.U = const_cast<cplx*>(D);
  sa.Fo = nullptr;
  sa.Gold = g;
  sa.Uprev = nullptr;
  sa.Bc = c->Bc.as<cplx>();
  sa.Hc = c->Hc.as<cplx>();
  sa.T1c = c->T1c.as<cplx>();
  sa.T2c = c->T2c.as<cplx>();
  sa.twc = c->twc.as<cplx>();
  sa.Rc = c->Rc.as<cplx>();
  sa.red = nullptr;
  sa.ftab = c->ftab.as<double>();
  sa.dT = c->dT;
  sa.M = c->M;
  sa.P = 1;
  sa.n0 = 0;
  sa.nbase = n;
  sa.t0s = c->t0s.as<double>() + n;
  sa.nsteps = c->nc;
  sa.mode = 0;
  const pd::Problem pc = make_problem(c, c->dtc, c->scheme_c);
  return coarse_sweep(c, sa, pc, st);
}

}  // namespace

namespace pd {
namespace ctxh {

void lg_release(pd_ctx* c) {
  auto& g = c->lg;
  if (g.hbidx) (void)hipHostFree(g.hbidx);
  g.hbidx = nullptr;
  g.params.release(); g.grads.release(); g.m1.release(); g.m2.release();
  g.xs.release(); g.rs.release(); g.ts.release();
  g.act.release(); g.ys.release(); g.c.release(); g.dc.release(); g.dhA.release();
  g.dhB.release(); g.dW.release(); g.part.release(); g.lpart.release(); g.sums.release();
  g.bidx.release(); g.Dn.release(); g.gn.release(); g.fn.release(); g.nrm.release();
  g.uold.release(); g.wq.release();
  g.weighted = false;
  g.init = g.enabled = false;
  g.S = 0;
  g.Bcap = 0;
}

// Serial coarse sweep with the learned propagator over slices [a, b).
// initial: U_{n+1} = G_learned(U_n); otherwise the difference form
// U_{n+1} = F_n + G_learned(U_n - Uold_n), with the fine results in Fo and
// the previous iterate in lg.uold: the states this range overwrites, U_{a+1}
// .. U_b (and U_a when a = n0, the first slice swept), are copied there
// first, so the ranges of one sweep may run one after another.  With
// `defect` (after the last range, b = P) the defect sums go to c->red.
pd_status lg_sweep_range(pd_ctx* c, int a, int b, int n0, bool initial, bool defect,
                         hipStream_t st) {
  auto& g = c->lg;
  const size_t box = c->box_elems();
  const int P = c->P;
  cplx* U = c->U.as<cplx>();
  pd_status s = ensure_batch(c, 1);
  if (s != PD_OK) return s;
  PD_HIP(c, g.uold.ensure(sizeof(cplx) * box * (P + 1)), "alloc");
  PD_HIP(c, g.Dn.ensure(sizeof(cplx) * box * 2), "alloc");
  PD_HIP(c, g.gn.ensure(sizeof(cplx) * box), "alloc");
  PD_HIP(c, g.nrm.ensure(sizeof(double) * 2), "alloc");
  if (!initial && a < b) {
    const int lo = a == n0 ? a : a + 1;
    PD_HIP(c, hipMemcpyAsync(g.uold.as<cplx>() + (size_t)lo * box, U + (size_t)lo * box,
                             sizeof(cplx) * box * (b + 1 - lo), hipMemcpyDeviceToDevice, st),
           "copy");
  }
  const pd::nn::Net net = net_of(c, g.params);
  std::vector<float*> h, y;
  act_ptrs(c, 1, h, y);
  float* xw = g.dhA.as<float>();  // features of one field ([Q][12] <= [Q][CH])
  cplx* D = g.Dn.as<cplx>();      // [D, g_scratch]: coarse_one reads D, writes D + box
  for (int n = a; n < b; ++n) {
    PD_HIP(c, pd::nn::sub(U + (size_t)n * box, initial ? nullptr : g.uold.as<cplx>() + (size_t)n * box,
                          D, box, st), "sub");
    PD_HIP(c, pd::norms2(D, box, 1, g.nrm.as<double>(), st), "norm");
    PD_HIP(c, coarse_one(c, D, g.gn.as<cplx>(), n, st), "coarse");
    const cplx* gout = D + box;  // U[1] of the one-slice sweep
    PD_HIP(c, pd::nn::features(D, gout, g.nrm.as<double>(), xw, g.Q, 1, st), "features");
    PD_HIP(c, pd::nn::forward(net, xw, c->t0s.as<double>() + n, nullptr, 1, h.data(), y.data(),
                              g.c.as<float>(), st), "forward");
    PD_HIP(c, pd::nn::combine(c->Fo.as<cplx>() + (size_t)n * box, gout, g.c.as<float>(),
                              g.nrm.as<double>(), U + (size_t)(n + 1) * box, g.Q, !initial, st),
           "combine");
  }
  if (!initial && defect)
    PD_HIP(c, pd::nn::defect(U + (size_t)P * box, g.uold.as<cplx>() + (size_t)P * box, box,
                             c->red.as<double>(), st), "defect");
  return PD_OK;
}

// the whole sweep over slices n0..P-1 in one range
pd_status lg_sweep(pd_ctx* c, int n0, bool initial, hipStream_t st) {
  return lg_sweep_range(c, n0, c->P, n0, initial, true, st);
}

}  // namespace ctxh
}  // namespace pd

extern "C" {

pd_status pd_lg_init(pd_ctx* c, int layers, uint64_t seed) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (layers < 1 || layers > 8) return fail(c, PD_EINVAL, "layers must be in [1, 8]");
  if (c->prec == PD_C64) return fail(c, PD_EINVAL, "the learned coarse propagator is complex128 only");
  DeviceGuard dg(c->device);
  lg_release(c);
  auto& g = c->lg;
  g.L = layers;
  g.Mf = c->M;
  g.Q = c->M * c->M;
  const size_t np = pd::nn::param_count(g.Q, g.L);
  std::vector<float> p(np);
  SplitMix rng{seed};
  pd::nn::Net v = pd::nn::view(p.data(), g.Q, g.Mf, g.L);
  const int C = pd::nn::CH;
  for (int i = 0; i < 12 * C; ++i) v.W_in[i] = (float)(rng.normal() / std::sqrt(12.0));
  for (size_t i = 0; i < (size_t)g.L * 15 * C * C; ++i)
    v.V[i] = (float)(rng.normal() * 0.3 / std::sqrt(5.0 * C));
  for (size_t i = 0; i < (size_t)g.L * g.Q * C; ++i) v.gamma[i] = 1.0f;
  for (int i = 0; i < C * 6; ++i) v.W_out[i] = (float)(rng.normal() * 1e-3 / std::sqrt((double)C));
  PD_HIP(c, g.params.ensure(sizeof(float) * np), "alloc");
  PD_HIP(c, g.grads.ensure(sizeof(float) * np), "alloc");
  PD_HIP(c, g.m1.ensure(sizeof(float) * np), "alloc");
  PD_HIP(c, g.m2.ensure(sizeof(float) * np), "alloc");
  PD_HIP(c, hipMemcpy(g.params.p, p.data(), sizeof(float) * np, hipMemcpyHostToDevice), "copy");
  PD_HIP(c, hipMemset(g.m1.p, 0, sizeof(float) * np), "memset");
  PD_HIP(c, hipMemset(g.m2.p, 0, sizeof(float) * np), "memset");
  g.step = 0;
  g.init = true;
  return PD_OK;
}

pd_status pd_lg_params(pd_ctx* c, float* out, size_t* n) {
  if (!c || !n) return PD_EINVAL;
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  const size_t np = pd::nn::param_count(c->lg.Q, c->lg.L);
  if (out) {
    if (*n < np) return fail(c, PD_EINVAL, "output holds %zu values, %zu needed", *n, np);
    DeviceGuard dg(c->device);
    PD_HIP(c, hipMemcpy(out, c->lg.params.p, sizeof(float) * np, hipMemcpyDeviceToHost), "copy");
  }
  *n = np;
  return PD_OK;
}

pd_status pd_lg_add_parareal_samples(pd_ctx* c, int iters, int* n_stored) {
  if (!c) return PD_EINVAL;
  c->sweep_next = -1;
  c->err.clear();
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  if (!c->have_initial) return fail(c, PD_ESTATE, "pd_set_initial not called");
  if (iters < 0 || iters >= c->P) return fail(c, PD_EINVAL, "iters must be in [0, n_slices)");
  c->last_k = -1;
  c->resume_k = -1;
  DeviceGuard dg(c->device);
  hipStream_t st = c->stream;
  const size_t box = c->box_elems(), rows = c->rows_elems(), full = (size_t)3 * c->N * c->N;
  const int P = c->P;
  cplx* U = c->U.as<cplx>();
  DevBuf prev, dfull, dc;
  PD_HIP(c, prev.ensure(sizeof(cplx) * box * (P + 1)), "alloc");
  PD_HIP(c, dfull.ensure(sizeof(cplx) * full * P), "alloc");
  PD_HIP(c, dc.ensure(sizeof(cplx) * box * P), "alloc");
  std::vector<double> t0(P);
  pd::SweepArgs sa;
  sa.U = U;
  sa.Fo = c->Fo.as<cplx>();
  sa.Gold = c->Gold.as<cplx>();
  sa.Uprev = c->Uprev.as<cplx>();
  sa.Bc = c->Bc.as<cplx>();
  sa.Hc = c->Hc.as<cplx>();
  sa.T1c = c->T1c.as<cplx>();
  sa.T2c = c->T2c.as<cplx>();
  sa.twc = c->twc.as<cplx>();
  sa.Rc = c->Rc.as<cplx>();
  sa.red = c->red.as<double>();
  sa.ftab = c->ftab.as<double>();
  sa.dT = c->dT;
  sa.M = c->M;
  sa.P = P;
  sa.nsteps = c->nc;
  const pd::Problem pc = make_problem(c, c->dtc, c->scheme_c),
                    pf = make_problem(c, c->dtf, c->scheme_f);
  {
    pd_status rs = ensure_rk_buffers(c);
    if (rs != PD_OK) return rs;
  }
  auto sweep = [&]() {
    return coarse_sweep(c, sa, pc, st);
  };
  // the inputs the coarse propagator sees: U^0_n in the initial run, then the
  // changes U^k_n - U^{k-1}_n of every later iteration (plain-G trajectory)
  sa.n0 = 0;
  sa.mode = 0;
  PD_HIP(c, sweep(), "coarse sweep");
  for (int k = 0; k <= iters; ++k) {
    const int first = k;  // U^k_n = U^{k-1}_n for n < k
    const int cnt = P - first;
    if (k == 0) {
      PD_HIP(c, hipMemcpyAsync(dc.p, U, sizeof(cplx) * box * P, hipMemcpyDeviceToDevice, st), "copy");
    } else {
      PD_HIP(c, hipMemcpyAsync(prev.p, U, sizeof(cplx) * box * (P + 1), hipMemcpyDeviceToDevice, st), "copy");
      const int n0 = k - 1;
      PD_HIP(c, hipMemcpyAsync(c->Uprev.p, U + (size_t)P * box, sizeof(cplx) * box, hipMemcpyDeviceToDevice, st), "copy");
      PD_HIP(c, hipMemcpyAsync(c->Fo.as<cplx>() + (size_t)n0 * box, U + (size_t)n0 * box,
                               sizeof(cplx) * box * (P - n0), hipMemcpyDeviceToDevice, st), "copy");
      pd::FieldBatch fb;
      fb.B = c->Fo.as<cplx>() + (size_t)n0 * box;
      fb.H = c->Hf.as<cplx>() + (size_t)n0 * box;
      fb.T1 = c->T1f.as<cplx>() + (size_t)n0 * rows;
      fb.T2 = fb.T1;
      fb.t0 = c->t0s.as<double>() + n0;
      fb.tw = c->tw.as<cplx>();
      c->shapes(fb);
      if (c->scheme_f != PD_SCHEME_SBDF2) fb.R = c->Rf.as<cplx>() + (size_t)4 * n0 * box;
      PD_HIP(c, fine_batch(c, fb, pf, P - n0, c->nf, st), "fine sweep");
      sa.n0 = n0;
      sa.mode = 1;
      PD_HIP(c, sweep(), "coarse sweep");
      PD_HIP(c, pd::nn::sub(U + (size_t)first * box, prev.as<cplx>() + (size_t)first * box, dc.as<cplx>(),
                            box * cnt, st), "sub");
    }
    PD_HIP(c, pd::unpack(dc.as<cplx>(), dfull.as<cplx>(), c->N, c->M, cnt, st), "unpack");
    PD_HIP(c, hipStreamSynchronize(st), "sync");
    for (int i = 0; i < cnt; ++i) t0[i] = (first + i) * c->dT;
    pd_status s = pd_lg_add_samples(c, cnt, t0.data(), dfull.p, st);
    if (s != PD_OK) return s;
  }
  if (n_stored) *n_stored = c->lg.S;
  return PD_OK;
}

pd_status pd_lg_set_params(pd_ctx* c, const float* in, size_t n) {
  if (!c || !in) return PD_EINVAL;
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  const size_t np = pd::nn::param_count(c->lg.Q, c->lg.L);
  if (n != np) return fail(c, PD_EINVAL, "expected %zu values, got %zu", np, n);
  DeviceGuard dg(c->device);
  PD_HIP(c, hipMemcpy(c->lg.params.p, in, sizeof(float) * np, hipMemcpyHostToDevice), "copy");
  PD_HIP(c, hipMemset(c->lg.m1.p, 0, sizeof(float) * np), "memset");
  PD_HIP(c, hipMemset(c->lg.m2.p, 0, sizeof(float) * np), "memset");
  c->lg.step = 0;
  return PD_OK;
}

pd_status pd_lg_add_samples(pd_ctx* c, int n, const double* t0, const void* d_D, void* stream) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  if (n < 1 || n > 4096 || !t0 || !d_D) return fail(c, PD_EINVAL, "need 1..4096 fields and t0");
  DeviceGuard dg(c->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto& g = c->lg;
  const size_t box = c->box_elems(), full = (size_t)3 * c->N * c->N;
  // F(D) and G(D) on the full layout through the library's propagators
  DevBuf fF, fG;
  PD_HIP(c, fF.ensure(sizeof(cplx) * full * n), "alloc");
  PD_HIP(c, fG.ensure(sizeof(cplx) * full * n), "alloc");
  pd_status s = run_propagator(c, t0, n, c->dtf, c->nf, c->N, d_D, fF.p, st, c->scheme_f);
  if (s != PD_OK) return s;
  s = run_propagator(c, t0, n, c->dtc, c->nc, c->Nc, d_D, fG.p, st, c->scheme_c);
  if (s != PD_OK) return s;
  PD_HIP(c, g.Dn.ensure(sizeof(cplx) * box * (n > 2 ? n : 2)), "alloc");
  PD_HIP(c, g.fn.ensure(sizeof(cplx) * box * n), "alloc");
  PD_HIP(c, g.gn.ensure(sizeof(cplx) * box * n), "alloc");
  PD_HIP(c, g.nrm.ensure(sizeof(double) * (n > 2 ? n : 2)), "alloc");
  PD_HIP(c, pd::pack(static_cast<const cplx*>(d_D), g.Dn.as<cplx>(), c->N, c->M, n, st), "pack");
  PD_HIP(c, pd::pack(fF.as<cplx>(), g.fn.as<cplx>(), c->N, c->M, n, st), "pack");
  PD_HIP(c, pd::pack(fG.as<cplx>(), g.gn.as<cplx>(), c->N, c->M, n, st), "pack");
  PD_HIP(c, pd::norms2(g.Dn.as<cplx>(), box, n, g.nrm.as<double>(), st), "norms");
  const size_t xq = (size_t)g.Q * 12, rq = (size_t)g.Q * 6;
  s = grow(c, g.xs, sizeof(float) * xq * (g.S + n), sizeof(float) * xq * g.S, st);
  if (s != PD_OK) return s;
  s = grow(c, g.rs, sizeof(float) * rq * (g.S + n), sizeof(float) * rq * g.S, st);
  if (s != PD_OK) return s;
  s = grow(c, g.ts, sizeof(double) * (g.S + n), sizeof(double) * g.S, st);
  if (s != PD_OK) return s;
  PD_HIP(c, pd::nn::features(g.Dn.as<cplx>(), g.gn.as<cplx>(), g.nrm.as<double>(),
                             g.xs.as<float>() + xq * g.S, g.Q, n, st), "features");
  PD_HIP(c, pd::nn::targets(g.fn.as<cplx>(), g.gn.as<cplx>(), g.nrm.as<double>(),
                            g.rs.as<float>() + rq * g.S, g.Q, n, st), "targets");
  PD_HIP(c, hipMemcpyAsync(g.ts.as<double>() + g.S, t0, sizeof(double) * n, hipMemcpyHostToDevice, st),
         "copy");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  g.S += n;
  return PD_OK;
}

pd_status pd_lg_add_feature_samples(pd_ctx* c, int n, const float* x, const float* r,
                                    const double* t, int* n_stored) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  if (n < 1 || n > 65536 || !x || !r || !t) return fail(c, PD_EINVAL, "need 1..65536 samples and x, r, t");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(t[i])) return fail(c, PD_EINVAL, "t must be finite");
  DeviceGuard dg(c->device);
  hipStream_t st = c->stream;
  auto& g = c->lg;
  const size_t xq = (size_t)g.Q * 12, rq = (size_t)g.Q * 6;
  pd_status s = grow(c, g.xs, sizeof(float) * xq * (g.S + n), sizeof(float) * xq * g.S, st);
  if (s != PD_OK) return s;
  s = grow(c, g.rs, sizeof(float) * rq * (g.S + n), sizeof(float) * rq * g.S, st);
  if (s != PD_OK) return s;
  s = grow(c, g.ts, sizeof(double) * (g.S + n), sizeof(double) * g.S, st);
  if (s != PD_OK) return s;
  PD_HIP(c, hipMemcpyAsync(g.xs.as<float>() + xq * g.S, x, sizeof(float) * xq * n,
                           hipMemcpyHostToDevice, st), "copy");
  PD_HIP(c, hipMemcpyAsync(g.rs.as<float>() + rq * g.S, r, sizeof(float) * rq * n,
                           hipMemcpyHostToDevice, st), "copy");
  PD_HIP(c, hipMemcpyAsync(g.ts.as<double>() + g.S, t, sizeof(double) * n, hipMemcpyHostToDevice, st),
         "copy");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  g.S += n;
  if (n_stored) *n_stored = g.S;
  return PD_OK;
}

pd_status pd_lg_set_operands(pd_ctx* c, int fp32) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (fp32 != 0 && fp32 != 1) return fail(c, PD_EINVAL, "operand type must be 0 (BF16) or 1 (FP32)");
  c->lg.f32ops = fp32;
  return PD_OK;
}

// one forward (+ optional backward) over the samples idx[0..B)
static pd_status lg_pass(pd_ctx* c, const int* idx, int B, bool grad, double* sums_host) {
  auto& g = c->lg;
  hipStream_t st = c->stream;
  pd_status s = ensure_batch(c, B);
  if (s != PD_OK) return s;
  std::memcpy(g.hbidx, idx, sizeof(int) * B);
  PD_HIP(c, hipMemcpyAsync(g.bidx.p, g.hbidx, sizeof(int) * B, hipMemcpyHostToDevice, st), "copy");
  const pd::nn::Net net = net_of(c, g.params);
  std::vector<float*> h, y;
  act_ptrs(c, B, h, y);
  PD_HIP(c, pd::nn::forward(net, g.xs.as<float>(), g.ts.as<double>(), g.bidx.as<int>(), B,
                            h.data(), y.data(), g.c.as<float>(), st), "forward");
  const float* wq = g.weighted ? g.wq.as<float>() : nullptr;
  PD_HIP(c, pd::nn::loss(g.c.as<float>(), g.rs.as<float>(), g.Q, B, g.bidx.as<int>(), wq,
                         g.lpart.as<double>(), g.sums.as<double>(), st), "loss");
  if (grad) {
    pd::nn::Grads gr = net_of(c, g.grads);
    pd::nn::Work w;
    w.dc = g.dc.as<float>();
    w.dhA = g.dhA.as<float>();
    w.dhB = g.dhB.as<float>();
    w.dW = g.dW.as<float>();
    w.part = g.part.as<float>();
    w.wq = wq;
    PD_HIP(c, pd::nn::backward(net, g.xs.as<float>(), g.ts.as<double>(), g.bidx.as<int>(), B,
                               h.data(), y.data(), g.c.as<float>(), g.rs.as<float>(),
                               g.sums.as<double>(), gr, w, st), "backward");
  }
  PD_HIP(c, hipMemcpyAsync(sums_host, g.sums.p, sizeof(double) * 2, hipMemcpyDeviceToHost, st), "copy");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  return PD_OK;
}

pd_status pd_lg_train(pd_ctx* c, int first, int count, int steps, int batch, double lr,
                      uint64_t seed, double* losses) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  auto& g = c->lg;
  if (g.S < 1) return fail(c, PD_ESTATE, "no samples (pd_lg_add_samples)");
  if (first < 0 || count < 1 || first + count > g.S) return fail(c, PD_EINVAL, "sample range");
  if (steps < 0 || batch < 1 || batch > count || !(lr >= 0)) return fail(c, PD_EINVAL, "bad steps, batch or lr");
  DeviceGuard dg(c->device);
  SplitMix rng{seed};
  std::vector<int> perm(count), idx(batch);
  for (int i = 0; i < count; ++i) perm[i] = first + i;
  const size_t np = pd::nn::param_count(g.Q, g.L);
  for (int it = 0; it < steps; ++it) {
    for (int i = 0; i < batch; ++i) {  // partial Fisher-Yates: batch distinct samples
      const int j = i + (int)(rng.next() % (uint64_t)(count - i));
      std::swap(perm[i], perm[j]);
      idx[i] = perm[i];
    }
    double sums[2];
    pd_status s = lg_pass(c, idx.data(), batch, true, sums);
    if (s != PD_OK) return s;
    if (losses) losses[it] = sums[1] > 0 ? sums[0] / sums[1] : 0.0;
    g.step += 1;
    PD_HIP(c, pd::nn::adam(g.params.as<float>(), g.grads.as<float>(), g.m1.as<float>(),
                           g.m2.as<float>(), np, (float)lr, g.step, c->stream), "adam");
  }
  PD_HIP(c, hipStreamSynchronize(c->stream), "sync");
  return PD_OK;
}

pd_status pd_lg_loss(pd_ctx* c, int first, int count, double* loss) {
  if (!c || !loss) return PD_EINVAL;
  c->err.clear();
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  if (first < 0 || count < 1 || first + count > c->lg.S) return fail(c, PD_EINVAL, "sample range");
  DeviceGuard dg(c->device);
  double num = 0.0, den = 0.0;
  const int chunk = 32;
  std::vector<int> idx(chunk);
  for (int a = first; a < first + count; a += chunk) {
    const int B = first + count - a < chunk ? first + count - a : chunk;
    for (int i = 0; i < B; ++i) idx[i] = a + i;
    double sums[2];
    pd_status s = lg_pass(c, idx.data(), B, false, sums);
    if (s != PD_OK) return s;
    num += sums[0];
    den += sums[1];
  }
  *loss = den > 0 ? num / den : 0.0;
  return PD_OK;
}

pd_status pd_lg_gradients(pd_ctx* c, int first, int count, float* grads, double* loss) {
  if (!c || !grads) return PD_EINVAL;
  c->err.clear();
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  if (first < 0 || count < 1 || first + count > c->lg.S) return fail(c, PD_EINVAL, "sample range");
  DeviceGuard dg(c->device);
  std::vector<int> idx(count);
  for (int i = 0; i < count; ++i) idx[i] = first + i;
  double sums[2];
  pd_status s = lg_pass(c, idx.data(), count, true, sums);
  if (s != PD_OK) return s;
  if (loss) *loss = sums[1] > 0 ? sums[0] / sums[1] : 0.0;
  const size_t np = pd::nn::param_count(c->lg.Q, c->lg.L);
  PD_HIP(c, hipMemcpy(grads, c->lg.grads.p, sizeof(float) * np, hipMemcpyDeviceToHost), "copy");
  return PD_OK;
}

pd_status pd_lg_sample(pd_ctx* c, int i, float* x, float* r, double* t) {
  if (!c) return PD_EINVAL;
  if (!c->lg.init || i < 0 || i >= c->lg.S) return fail(c, PD_EINVAL, "no sample %d", i);
  DeviceGuard dg(c->device);
  const size_t xq = (size_t)c->lg.Q * 12, rq = (size_t)c->lg.Q * 6;
  if (x) PD_HIP(c, hipMemcpy(x, c->lg.xs.as<float>() + xq * i, sizeof(float) * xq, hipMemcpyDeviceToHost), "copy");
  if (r) PD_HIP(c, hipMemcpy(r, c->lg.rs.as<float>() + rq * i, sizeof(float) * rq, hipMemcpyDeviceToHost), "copy");
  if (t) PD_HIP(c, hipMemcpy(t, c->lg.ts.as<double>() + i, sizeof(double), hipMemcpyDeviceToHost), "copy");
  return PD_OK;
}

pd_status pd_lg_forward_sample(pd_ctx* c, int i, float* out) {
  if (!c || !out) return PD_EINVAL;
  if (!c->lg.init || i < 0 || i >= c->lg.S) return fail(c, PD_EINVAL, "no sample %d", i);
  DeviceGuard dg(c->device);
  double sums[2];
  pd_status s = lg_pass(c, &i, 1, false, sums);
  if (s != PD_OK) return s;
  PD_HIP(c, hipMemcpy(out, c->lg.c.p, sizeof(float) * c->lg.Q * 6, hipMemcpyDeviceToHost), "copy");
  return PD_OK;
}

pd_status pd_lg_set_loss_decay(pd_ctx* c, double beta) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  if (!(beta >= 0) || !std::isfinite(beta)) return fail(c, PD_EINVAL, "beta must be finite and >= 0");
  auto& g = c->lg;
  if (beta == 0.0) {
    g.weighted = false;
    return PD_OK;
  }
  // w_m = exp(-beta |k_m|^2 dT / Rm): the factor by which diffusion alone
  // damps mode m over beta slices
  const int Mf = g.Mf, K = (Mf - 1) / 2;
  std::vector<float> w((size_t)g.Q);
  for (int r = 0; r < Mf; ++r)
    for (int q = 0; q < Mf; ++q) {
      const double ky = r - K, kx = q - K;
      const double k2 = kx * kx + ky * ky + c->kz * c->kz;
      w[(size_t)r * Mf + q] = (float)std::exp(-beta * k2 * c->dT / c->Rm);
    }
  DeviceGuard dg(c->device);
  PD_HIP(c, g.wq.ensure(sizeof(float) * g.Q), "alloc");
  PD_HIP(c, hipMemcpy(g.wq.p, w.data(), sizeof(float) * g.Q, hipMemcpyHostToDevice), "copy");
  g.weighted = true;
  return PD_OK;
}

pd_status pd_set_coarse(pd_ctx* c, int learned) {
  if (!c) return PD_EINVAL;
  if (learned && !c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  // switching to the plain propagator: the coarse values of the learned
  // iterates are not there, so the state cannot be continued; the learned
  // difference form needs only U^k, so switching to it keeps it continuable
  if (!learned && c->lg.enabled) c->last_k = -1;
  c->lg.enabled = learned != 0;
  return PD_OK;
}

}  // extern "C"
