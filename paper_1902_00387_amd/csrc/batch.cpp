// Batched Parareal over many independent (flow, Rm, kz, N) instances of
// uneven size on one GPU (C ABI pd_batch_*).
//
// Instances are grouped into classes of equal (flow, N, fine steps per slice);
// every class keeps the slice buffers of all its instances side by side, so one
// fine sweep of a class is one multi-launch batch over its active slices (an
// active-field map selects them; per-field Rm and kz).  The serial coarse
// sweeps of all instances run concurrently, one workgroup per instance.  One
// Parareal iteration of the whole batch -- the class fine sweeps on forked
// streams, then the coarse sweeps with the correction and defect -- is captured
// once in a HIP graph and replayed every iteration; between replays only the
// small device tables (active maps, sweep jobs) change.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pitdyn.h"
#include "launch.hpp"
#include "runtime.hpp"

using pd::cplx;
using namespace pd::rt;

namespace {

struct Inst {
  int flow;
  double Rm, kz;
  int N, Nc, P, nf, nc;
  double T, dT, dtf, dtc;
  int cls = -1, f0 = 0, u0 = 0;  // class, first field, first U index in the class
  bool lds_job = true;
  int job = -1;                  // index in its job list
  size_t ftab_off = 0;
  std::vector<double> b0;        // full layout, host
  pd_report rep;
  bool done = false;
};

struct Cls {
  int N = 0, flow = 0, nf = 0;
  double dtf = 0;
  int nfields = 0, nU = 0;
  std::vector<int> finst, fslice;  // instance and slice of each field
  DevBuf U, Fo, Gold, H, T1, t0, fRm, fkz, uidx, map, count, tw;
  int* hmap = nullptr;  // pinned host staging: [nfields] map then [1] count
  hipStream_t side = nullptr;
  hipEvent_t done_ev = nullptr;
};

}  // namespace

struct pd_batch {
  int device = 0;
  hipStream_t st = nullptr;
  hipEvent_t fork_ev = nullptr;
  std::string err;
  std::vector<Inst> inst;
  std::deque<Cls> cls;
  bool built = false;
  std::vector<pd::SweepJob> jobsL, jobsG;  // LDS-resident / global coarse sweeps
  DevBuf djobsL, djobsG;
  pd::SweepJob* hjobs = nullptr;           // pinned staging for both lists
  DevBuf cws, uprev, red, ftab;
  double* hred = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  double t_total = 0;
};

namespace {

pd_status bfail(pd_batch* b, pd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) b->err = buf;
  return s;
}

pd_status bhip(pd_batch* b, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return bfail(b, PD_ENOMEM, "%s: out of device memory", what);
  return bfail(b, PD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define PB_HIP(b, expr, what)                           \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return bhip(b, e_, what);     \
  } while (0)

double flow_amp(int flow) {
  return flow == PD_FLOW_NONE ? 0.0 : (flow == PD_FLOW_ROBERTS ? 1.0 : std::sqrt(1.5));
}

pd::Problem problem_of(const Inst& in, double dt) {
  pd::Problem pb;
  pb.Rm = in.Rm;
  pb.kz = in.kz;
  pb.dt = dt;
  pb.amp = flow_amp(in.flow);
  pb.tdep = in.flow == PD_FLOW_GP ? 1 : 0;
  return pb;
}

void free_all(pd_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  for (auto& c : b->cls) {
    if (c.hmap) (void)hipHostFree(c.hmap);
    if (c.side) (void)hipStreamDestroy(c.side);
    if (c.done_ev) (void)hipEventDestroy(c.done_ev);
    c.hmap = nullptr;
    c.side = nullptr;
    c.done_ev = nullptr;
  }
  b->cls.clear();
  if (b->hjobs) (void)hipHostFree(b->hjobs);
  b->hjobs = nullptr;
  b->built = false;
}

// Group instances into classes and allocate every device buffer.
pd_status build(pd_batch* b) {
  free_all(b);
  std::map<std::tuple<int, int, int, double>, int> key2cls;
  for (auto& in : b->inst) {
    auto key = std::make_tuple(in.flow, in.N, in.nf, in.dtf);
    auto it = key2cls.find(key);
    int ci;
    if (it == key2cls.end()) {
      ci = (int)b->cls.size();
      key2cls[key] = ci;
      b->cls.emplace_back();
      Cls& c = b->cls.back();
      c.N = in.N;
      c.flow = in.flow;
      c.nf = in.nf;
      c.dtf = in.dtf;
    } else {
      ci = it->second;
    }
    Cls& c = b->cls[ci];
    in.cls = ci;
    in.f0 = c.nfields;
    in.u0 = c.nU;
    c.nfields += in.P;
    c.nU += in.P + 1;
  }
  for (auto& c : b->cls)
    if (c.nfields > 65535) return bfail(b, PD_EINVAL, "too many slices of grid %d in one batch", c.N);
  size_t ftab_total = 0, cws_total = 0, uprev_total = 0;
  b->jobsL.clear();
  b->jobsG.clear();
  for (auto& in : b->inst) {
    const int Mc = box_M(in.Nc);
    in.lds_job = pd::conv_lds_width(Mc);
    in.ftab_off = ftab_total;
    if (in.flow == PD_FLOW_GP) ftab_total += (size_t)4 * in.P * in.nc;
    if (!in.lds_job) cws_total += (size_t)9 * Mc * Mc;
    uprev_total += (size_t)3 * box_M(in.N) * box_M(in.N);
  }
  PB_HIP(b, b->ftab.ensure(sizeof(double) * (ftab_total ? ftab_total : 1)), "alloc");
  PB_HIP(b, b->cws.ensure(sizeof(cplx) * (cws_total ? cws_total : 1)), "alloc");
  PB_HIP(b, b->uprev.ensure(sizeof(cplx) * uprev_total), "alloc");
  PB_HIP(b, b->red.ensure(sizeof(double) * 2 * b->inst.size()), "alloc");
  PB_HIP(b, hipHostMalloc((void**)&b->hjobs, sizeof(pd::SweepJob) * b->inst.size()), "alloc");
  std::vector<double> ft(ftab_total);
  for (auto& in : b->inst)
    if (in.flow == PD_FLOW_GP)
      for (int n = 0; n < in.P; ++n)
        for (int j = 0; j < in.nc; ++j) {
          const double t = n * in.dT + j * in.dtc;
          const double px = std::cos(t), py = std::sin(t);
          double* q = &ft[in.ftab_off + 4 * ((size_t)n * in.nc + j)];
          q[0] = std::cos(py);
          q[1] = std::sin(py);
          q[2] = std::cos(px);
          q[3] = std::sin(px);
        }
  if (ftab_total)
    PB_HIP(b, hipMemcpy(b->ftab.p, ft.data(), ft.size() * sizeof(double), hipMemcpyHostToDevice), "copy");
  // classes
  for (auto& c : b->cls) {
    const int M = box_M(c.N);
    const size_t box = (size_t)3 * M * M, rows = (size_t)3 * M * c.N;
    PB_HIP(b, c.U.ensure(sizeof(cplx) * box * c.nU), "alloc U");
    PB_HIP(b, c.Fo.ensure(sizeof(cplx) * box * c.nfields), "alloc F");
    PB_HIP(b, c.Gold.ensure(sizeof(cplx) * box * c.nfields), "alloc Gold");
    PB_HIP(b, c.H.ensure(sizeof(cplx) * box * c.nfields), "alloc H");
    PB_HIP(b, c.T1.ensure(sizeof(cplx) * rows * c.nfields), "alloc T1");
    PB_HIP(b, c.t0.ensure(sizeof(double) * c.nfields), "alloc");
    PB_HIP(b, c.fRm.ensure(sizeof(double) * c.nfields), "alloc");
    PB_HIP(b, c.fkz.ensure(sizeof(double) * c.nfields), "alloc");
    PB_HIP(b, c.uidx.ensure(sizeof(int) * c.nfields), "alloc");
    PB_HIP(b, c.map.ensure(sizeof(int) * c.nfields), "alloc");
    PB_HIP(b, c.count.ensure(sizeof(int)), "alloc");
    PB_HIP(b, hipHostMalloc((void**)&c.hmap, sizeof(int) * (c.nfields + 1)), "alloc");
    PB_HIP(b, hipStreamCreate(&c.side), "stream");
    PB_HIP(b, hipEventCreateWithFlags(&c.done_ev, hipEventDisableTiming), "event");
    std::vector<cplx> tw = twiddles(c.N);
    PB_HIP(b, c.tw.ensure(sizeof(cplx) * c.N), "alloc");
    PB_HIP(b, hipMemcpy(c.tw.p, tw.data(), sizeof(cplx) * c.N, hipMemcpyHostToDevice), "copy");
    c.finst.assign(c.nfields, 0);
    c.fslice.assign(c.nfields, 0);
  }
  for (size_t i = 0; i < b->inst.size(); ++i) {
    Inst& in = b->inst[i];
    Cls& c = b->cls[in.cls];
    for (int n = 0; n < in.P; ++n) {
      c.finst[in.f0 + n] = (int)i;
      c.fslice[in.f0 + n] = n;
    }
  }
  for (auto& c : b->cls) {
    std::vector<double> t0(c.nfields), rm(c.nfields), kz(c.nfields);
    std::vector<int> ui(c.nfields);
    for (int f = 0; f < c.nfields; ++f) {
      const Inst& in = b->inst[c.finst[f]];
      t0[f] = c.fslice[f] * in.dT;
      rm[f] = in.Rm;
      kz[f] = in.kz;
      ui[f] = in.u0 + c.fslice[f];
    }
    PB_HIP(b, hipMemcpy(c.t0.p, t0.data(), sizeof(double) * c.nfields, hipMemcpyHostToDevice), "copy");
    PB_HIP(b, hipMemcpy(c.fRm.p, rm.data(), sizeof(double) * c.nfields, hipMemcpyHostToDevice), "copy");
    PB_HIP(b, hipMemcpy(c.fkz.p, kz.data(), sizeof(double) * c.nfields, hipMemcpyHostToDevice), "copy");
    PB_HIP(b, hipMemcpy(c.uidx.p, ui.data(), sizeof(int) * c.nfields, hipMemcpyHostToDevice), "copy");
  }
  // coarse sweep jobs (static pointers; n0 / mode / active change per iteration)
  size_t cws_off = 0, up_off = 0;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    Inst& in = b->inst[i];
    Cls& c = b->cls[in.cls];
    const int M = box_M(in.N), Mc = box_M(in.Nc);
    const size_t box = (size_t)3 * M * M;
    pd::SweepJob jb;
    std::memset(&jb, 0, sizeof jb);
    jb.a.U = c.U.as<cplx>() + (size_t)in.u0 * box;
    jb.a.Fo = c.Fo.as<cplx>() + (size_t)in.f0 * box;
    jb.a.Gold = c.Gold.as<cplx>() + (size_t)in.f0 * box;
    jb.a.Uprev = b->uprev.as<cplx>() + up_off;
    up_off += box;
    if (!in.lds_job) {
      const size_t cb = (size_t)3 * Mc * Mc;
      cplx* w = b->cws.as<cplx>() + cws_off;
      jb.a.Bc = w;
      jb.a.T1c = w + cb;
      jb.a.Hc = w + 2 * cb;
      cws_off += 3 * cb;
    }
    jb.a.red = b->red.as<double>() + 2 * i;
    jb.a.ftab = in.flow == PD_FLOW_GP ? b->ftab.as<double>() + in.ftab_off : nullptr;
    jb.a.dT = in.dT;
    jb.a.M = M;
    jb.a.P = in.P;
    jb.a.nsteps = in.nc;
    jb.pb = problem_of(in, in.dtc);
    jb.Mc = Mc;
    jb.active = 1;
    if (in.lds_job) {
      in.job = (int)b->jobsL.size();
      b->jobsL.push_back(jb);
    } else {
      in.job = (int)b->jobsG.size();
      b->jobsG.push_back(jb);
    }
  }
  PB_HIP(b, b->djobsL.ensure(sizeof(pd::SweepJob) * (b->jobsL.size() + 1)), "alloc");
  PB_HIP(b, b->djobsG.ensure(sizeof(pd::SweepJob) * (b->jobsG.size() + 1)), "alloc");
  b->built = true;
  return PD_OK;
}

// Upload the jobs (both lists) through the pinned staging buffer.
pd_status upload_jobs(pd_batch* b) {
  const size_t nl = b->jobsL.size(), ng = b->jobsG.size();
  std::memcpy(b->hjobs, b->jobsL.data(), sizeof(pd::SweepJob) * nl);
  std::memcpy(b->hjobs + nl, b->jobsG.data(), sizeof(pd::SweepJob) * ng);
  if (nl)
    PB_HIP(b, hipMemcpyAsync(b->djobsL.p, b->hjobs, sizeof(pd::SweepJob) * nl, hipMemcpyHostToDevice, b->st), "copy");
  if (ng)
    PB_HIP(b, hipMemcpyAsync(b->djobsG.p, b->hjobs + nl, sizeof(pd::SweepJob) * ng, hipMemcpyHostToDevice, b->st), "copy");
  return PD_OK;
}

// One Parareal iteration's launches (what the graph holds): per class, on its
// side stream, gather the start values of the active slices and run the fine
// sweep; then, on the main stream, the coarse sweeps with the correction.
hipError_t enqueue_iteration(pd_batch* b) {
  hipError_t e = hipEventRecord(b->fork_ev, b->st);
  if (e != hipSuccess) return e;
  for (auto& c : b->cls) {
    if ((e = hipStreamWaitEvent(c.side, b->fork_ev, 0)) != hipSuccess) return e;
    const int M = box_M(c.N);
    const size_t box = (size_t)3 * M * M;
    e = pd::gather(c.U.as<cplx>(), c.Fo.as<cplx>(), c.uidx.as<int>(), c.map.as<int>(),
                   c.count.as<int>(), c.nfields, box, c.side);
    if (e != hipSuccess) return e;
    pd::FieldBatch fb;
    fb.B = c.Fo.as<cplx>();
    fb.H = c.H.as<cplx>();
    fb.T1 = c.T1.as<cplx>();
    fb.T2 = fb.T1;  // in place
    fb.t0 = c.t0.as<double>();
    fb.tw = c.tw.as<cplx>();
    fb.fRm = c.fRm.as<double>();
    fb.fkz = c.fkz.as<double>();
    fb.map = c.map.as<int>();
    fb.count = c.count.as<int>();
    pd::Problem pb;
    pb.Rm = 1.0;
    pb.kz = 0.0;
    pb.dt = c.dtf;
    pb.amp = flow_amp(c.flow);
    pb.tdep = c.flow == PD_FLOW_GP ? 1 : 0;
    e = pd::propagate(c.N, fb, pb, c.nfields, c.nf, pd::PATH_MULTI, c.side);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(c.done_ev, c.side)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(b->st, c.done_ev, 0)) != hipSuccess) return e;
  }
  if ((e = pd::sweep_conv_jobs(b->djobsL.as<pd::SweepJob>(), (int)b->jobsL.size(), true, b->st)) != hipSuccess)
    return e;
  return pd::sweep_conv_jobs(b->djobsG.as<pd::SweepJob>(), (int)b->jobsG.size(), false, b->st);
}

}  // namespace

extern "C" {

pd_status pd_batch_create(pd_batch** out, int hip_device) {
  if (!out) return PD_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return PD_EINVAL;
  pd_batch* b = new (std::nothrow) pd_batch;
  if (!b) return PD_ENOMEM;
  b->device = hip_device;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(hip_device);
  if (hipStreamCreate(&b->st) != hipSuccess ||
      hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&b->hred, 2 * sizeof(double) * 4096) != hipSuccess) {
    (void)hipSetDevice(prev);
    delete b;
    return PD_EHIP;
  }
  (void)hipSetDevice(prev);
  *out = b;
  return PD_OK;
}

void pd_batch_destroy(pd_batch* b) {
  if (!b) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->st);
  free_all(b);
  b->djobsL.release(); b->djobsG.release(); b->cws.release(); b->uprev.release();
  b->red.release(); b->ftab.release();
  if (b->hred) (void)hipHostFree(b->hred);
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  if (b->st) (void)hipStreamDestroy(b->st);
  (void)hipSetDevice(prev);
  delete b;
}

const char* pd_batch_last_error(const pd_batch* b) { return b ? b->err.c_str() : "null batch"; }

pd_status pd_batch_add(pd_batch* b, pd_flow flow, double Rm, double kz, int N, double T,
                       int n_slices, double dt_fine, double dt_coarse, int N_coarse,
                       const double* b0, int* id) {
  if (!b) return PD_EINVAL;
  b->err.clear();
  if (b->inst.size() >= 4096) return bfail(b, PD_EINVAL, "at most 4096 instances");
  if (flow != PD_FLOW_NONE && flow != PD_FLOW_ROBERTS && flow != PD_FLOW_GP)
    return bfail(b, PD_EINVAL, "unknown flow %d", (int)flow);
  if (!(Rm > 0) || !std::isfinite(Rm) || !std::isfinite(kz)) return bfail(b, PD_EINVAL, "bad Rm or kz");
  if (!valid_N(N)) return bfail(b, PD_EINVAL, "N must be one of 16, 32, 64, 128, 256, 512");
  if (!(T > 0) || n_slices < 1 || n_slices > 65535) return bfail(b, PD_EINVAL, "bad T or n_slices");
  if (N_coarse == 0) N_coarse = N;
  if (!valid_N(N_coarse) || N_coarse > N) return bfail(b, PD_EINVAL, "N_coarse must be a power of two in [16, N]");
  if (!b0) return bfail(b, PD_EINVAL, "null initial field");
  Inst in;
  in.flow = flow;
  in.Rm = Rm;
  in.kz = kz;
  in.N = N;
  in.Nc = N_coarse;
  in.P = n_slices;
  in.T = T;
  in.dT = T / n_slices;
  in.dtf = dt_fine;
  in.dtc = dt_coarse;
  if (!integer_ratio(in.dT, dt_fine, &in.nf)) return bfail(b, PD_EINVAL, "slice is not an integer number of fine steps");
  if (!integer_ratio(in.dT, dt_coarse, &in.nc)) return bfail(b, PD_EINVAL, "slice is not an integer number of coarse steps");
  const int K = box_K(N);
  for (int c = 0; c < 3; ++c)
    for (int my = 0; my < N; ++my)
      for (int mx = 0; mx < N; ++mx) {
        const int ky = my < N / 2 ? my : my - N, kx = mx < N / 2 ? mx : mx - N;
        const size_t i = 2 * (((size_t)c * N + my) * N + mx);
        if ((ky < -K || ky > K || kx < -K || kx > K) && (b0[i] != 0.0 || b0[i + 1] != 0.0))
          return bfail(b, PD_EINVAL, "initial field has nonzero coefficients outside the 2/3 box");
      }
  in.b0.assign(b0, b0 + (size_t)6 * N * N);
  std::memset(&in.rep, 0, sizeof in.rep);
  in.rep.k_con = -1;
  b->inst.push_back(std::move(in));
  b->built = false;
  if (id) *id = (int)b->inst.size() - 1;
  return PD_OK;
}

pd_status pd_batch_run(pd_batch* b, double tol, int max_iter, int use_graph) {
  if (!b) return PD_EINVAL;
  b->err.clear();
  if (b->inst.empty()) return bfail(b, PD_ESTATE, "no instances");
  if (max_iter < 0 || max_iter > PD_MAX_ITER) return bfail(b, PD_EINVAL, "max_iter must be in [0, %d]", PD_MAX_ITER);
  if (!(tol >= 0)) return bfail(b, PD_EINVAL, "tol must be >= 0");
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(b->device);
  struct Restore {
    int d;
    ~Restore() { (void)hipSetDevice(d); }
  } restore{prev};
  const auto w0 = std::chrono::steady_clock::now();
  if (!b->built) {
    pd_status s = build(b);
    if (s != PD_OK) return s;
  }
  // initial fields
  {
    DevBuf tmp;
    for (auto& in : b->inst) {
      Cls& c = b->cls[in.cls];
      const size_t full = (size_t)3 * in.N * in.N;
      PB_HIP(b, tmp.ensure(sizeof(cplx) * full), "alloc");
      PB_HIP(b, hipMemcpyAsync(tmp.p, in.b0.data(), sizeof(cplx) * full, hipMemcpyHostToDevice, b->st), "copy");
      const int M = box_M(in.N);
      PB_HIP(b, pd::pack(tmp.as<cplx>(), c.U.as<cplx>() + (size_t)in.u0 * 3 * M * M, in.N, M, 1, b->st), "pack");
      PB_HIP(b, hipStreamSynchronize(b->st), "sync");
      std::memset(&in.rep, 0, sizeof in.rep);
      in.rep.k_con = -1;
      in.done = false;
    }
  }
  // initial coarse run of every instance
  for (auto* jl : {&b->jobsL, &b->jobsG})
    for (auto& jb : *jl) {
      jb.a.n0 = 0;
      jb.a.mode = 0;
      jb.active = 1;
    }
  pd_status s = upload_jobs(b);
  if (s != PD_OK) return s;
  PB_HIP(b, pd::sweep_conv_jobs(b->djobsL.as<pd::SweepJob>(), (int)b->jobsL.size(), true, b->st), "sweep");
  PB_HIP(b, pd::sweep_conv_jobs(b->djobsG.as<pd::SweepJob>(), (int)b->jobsG.size(), false, b->st), "sweep");
  PB_HIP(b, hipStreamSynchronize(b->st), "sync");

  pd_status status = PD_OK;
  bool all_done = max_iter == 0;
  for (int k = 1; k <= max_iter && !all_done; ++k) {
    // active fields of every class, sweep jobs of every instance
    for (auto& c : b->cls) {
      int cnt = 0;
      for (int f = 0; f < c.nfields; ++f) {
        const Inst& in = b->inst[c.finst[f]];
        const int n0 = k - 1 < in.P - 1 ? k - 1 : in.P - 1;
        if (!in.done && c.fslice[f] >= n0) c.hmap[cnt++] = f;
      }
      c.hmap[c.nfields] = cnt;
      PB_HIP(b, hipMemcpyAsync(c.map.p, c.hmap, sizeof(int) * c.nfields, hipMemcpyHostToDevice, b->st), "copy");
      PB_HIP(b, hipMemcpyAsync(c.count.p, c.hmap + c.nfields, sizeof(int), hipMemcpyHostToDevice, b->st), "copy");
    }
    for (auto& in : b->inst) {
      pd::SweepJob& jb = in.lds_job ? b->jobsL[in.job] : b->jobsG[in.job];
      jb.a.n0 = k - 1 < in.P - 1 ? k - 1 : in.P - 1;
      jb.a.mode = 1;
      jb.active = in.done ? 0 : 1;
    }
    s = upload_jobs(b);
    if (s != PD_OK) return s;
    if (use_graph) {
      if (!b->gexec) {
        PB_HIP(b, hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal), "capture");
        hipError_t e = enqueue_iteration(b);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->st, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          return bhip(b, e != hipSuccess ? e : e2, "graph capture");
        }
        b->graph = g;
        PB_HIP(b, hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0), "graph instantiate");
      }
      PB_HIP(b, hipGraphLaunch(b->gexec, b->st), "graph launch");
    } else {
      PB_HIP(b, enqueue_iteration(b), "iteration");
    }
    PB_HIP(b, hipMemcpyAsync(b->hred, b->red.p, sizeof(double) * 2 * b->inst.size(), hipMemcpyDeviceToHost, b->st), "copy");
    PB_HIP(b, hipStreamSynchronize(b->st), "sync");
    all_done = true;
    for (size_t i = 0; i < b->inst.size(); ++i) {
      Inst& in = b->inst[i];
      if (in.done) continue;
      const double num = b->hred[2 * i], den = b->hred[2 * i + 1];
      in.rep.iters = k;
      if (!std::isfinite(num) || !std::isfinite(den)) {
        in.done = true;
        status = bfail(b, PD_EUNSTABLE, "instance %zu: non-finite state at iteration %d", i, k);
        continue;
      }
      const double sigma = den > 0 ? std::sqrt(num / den) : (num > 0 ? INFINITY : 0.0);
      in.rep.sigma[k - 1] = sigma;
      if (sigma <= tol) {
        in.rep.k_con = k;
        in.done = true;
      } else {
        all_done = false;
      }
    }
  }
  if (status == PD_OK && !all_done) status = PD_NOT_CONVERGED;
  b->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
  for (auto& in : b->inst) in.rep.t_total_s = b->t_total;
  return status;
}

pd_status pd_batch_result(const pd_batch* cb, int id, pd_report* rep, double* gamma) {
  pd_batch* b = const_cast<pd_batch*>(cb);
  if (!b) return PD_EINVAL;
  if (id < 0 || id >= (int)b->inst.size()) return bfail(b, PD_EINVAL, "unknown instance %d", id);
  if (!b->built) return bfail(b, PD_ESTATE, "pd_batch_run not called");
  Inst& in = b->inst[id];
  if (rep) *rep = in.rep;
  if (gamma) {
    if (in.P < 2) return bfail(b, PD_EINVAL, "growth rate needs at least 2 slices");
    const int M = box_M(in.N);
    const size_t box = (size_t)3 * M * M;
    Cls& c = b->cls[in.cls];
    DevBuf d;
    std::vector<double> nrm(in.P + 1);
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    PB_HIP(b, d.ensure(sizeof(double) * (in.P + 1)), "alloc");
    PB_HIP(b, pd::norms2(c.U.as<cplx>() + (size_t)in.u0 * box, box, in.P + 1, d.as<double>(), b->st), "norms");
    PB_HIP(b, hipMemcpyAsync(nrm.data(), d.p, sizeof(double) * (in.P + 1), hipMemcpyDeviceToHost, b->st), "copy");
    PB_HIP(b, hipStreamSynchronize(b->st), "sync");
    (void)hipSetDevice(prev);
    const int n0 = (in.P + 1) / 2, cnt = in.P + 1 - n0;
    double tm = 0, ym = 0;
    std::vector<double> t(cnt), y(cnt);
    for (int i = 0; i < cnt; ++i) {
      const double v = std::sqrt(nrm[n0 + i]);
      if (!(v > 0) || !std::isfinite(v)) return bfail(b, PD_EUNSTABLE, "slice norm is zero or not finite");
      t[i] = (n0 + i) * in.dT;
      y[i] = std::log(v);
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
  }
  return PD_OK;
}

pd_status pd_batch_get_slices(const pd_batch* cb, int id, double* out) {
  pd_batch* b = const_cast<pd_batch*>(cb);
  if (!b) return PD_EINVAL;
  if (id < 0 || id >= (int)b->inst.size()) return bfail(b, PD_EINVAL, "unknown instance %d", id);
  if (!b->built) return bfail(b, PD_ESTATE, "pd_batch_run not called");
  if (!out) return bfail(b, PD_EINVAL, "null pointer argument");
  Inst& in = b->inst[id];
  Cls& c = b->cls[in.cls];
  const int M = box_M(in.N);
  const size_t box = (size_t)3 * M * M, full = (size_t)3 * in.N * in.N;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(b->device);
  DevBuf tmp;
  PB_HIP(b, tmp.ensure(sizeof(cplx) * full * (in.P + 1)), "alloc");
  PB_HIP(b, pd::unpack(c.U.as<cplx>() + (size_t)in.u0 * box, tmp.as<cplx>(), in.N, M, (size_t)in.P + 1, b->st), "unpack");
  PB_HIP(b, hipMemcpyAsync(out, tmp.p, sizeof(cplx) * full * (in.P + 1), hipMemcpyDeviceToHost, b->st), "copy");
  PB_HIP(b, hipStreamSynchronize(b->st), "sync");
  (void)hipSetDevice(prev);
  return PD_OK;
}

pd_status pd_batch_time(const pd_batch* b, double* seconds) {
  if (!b || !seconds) return PD_EINVAL;
  *seconds = b->t_total;
  return PD_OK;
}

}  // extern "C"
