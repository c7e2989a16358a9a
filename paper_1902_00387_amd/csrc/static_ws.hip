// Fine-grid propagation without device allocation: the workspace of
// pd_steps_dev (compact state, SBDF history, the two row buffers, the start
// times, the box-check flag, Runge-Kutta stage sums) lives in one static
// device array per GPU instead of buffers the context allocates.
//
// The array's name is only a host-side stand-in for the symbol; its device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) when the first context on the device is created, and only that
// address is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/pitdyn.h"
#include "ctx.hpp"
#include "launch.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB a device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

// zero-fills n ints (a kernel, not a memset, so the call stays capturable)
__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace pd {

// Device address of this device's workspace; resolved once per device with
// that device current.  Returns the HIP status of the lookup.
hipError_t scratch_resolve(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[device]) {
    int prev = -1;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev >= 0) (void)hipSetDevice(prev);
    g_err[device] = e;
    g_ptr[device] = e == hipSuccess ? p : nullptr;
    g_done[device] = true;
  }
  return g_err[device];
}

}  // namespace pd

using namespace pd::ctxh;

extern "C" {

pd_status pd_steps_dev_noalloc(pd_ctx* c, const double* t0, int batch, double dt, int n_steps,
                               const void* d_in, void* d_out, void* s) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_problem) return fail(c, PD_ESTATE, "pd_set_problem not called");
  if (batch < 0 || batch > 65535) return fail(c, PD_EINVAL, "batch must be in [0, 65535]");
  if (batch == 0) return PD_OK;
  if (!t0 || !d_in || !d_out) return fail(c, PD_EINVAL, "null pointer argument");
  if (c->prec == PD_C64) return fail(c, PD_EINVAL, "the static-workspace call is complex128 only");
  if (n_steps < 1) return fail(c, PD_EINVAL, "n_steps must be >= 1");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(c, PD_EINVAL, "dt must be positive");
  for (int f = 0; f < batch; ++f)
    if (!std::isfinite(t0[f])) return fail(c, PD_EINVAL, "t0 must be finite");
  const int N = c->N, M = c->M;
  const bool rk = c->scheme_f != PD_SCHEME_SBDF2;
  const size_t box = (size_t)3 * M * M * sizeof(cplx), rows = (size_t)3 * M * N * sizeof(cplx);
  // layout: flag | t0[batch] | B | H | T1 | T2 | R (Runge-Kutta only)
  const size_t o_t0 = 256, o_B = o_t0 + align256(sizeof(double) * batch);
  const size_t o_H = o_B + align256(box * batch), o_T1 = o_H + align256(box * batch);
  const size_t o_T2 = o_T1 + align256(rows * batch), o_R = o_T2 + align256(rows * batch);
  const size_t need = rk ? o_R + 4 * box * batch : o_R;
  if (need > kScratchBytes)
    return fail(c, PD_EINVAL,
                "batch of %d fields on %d^2 needs %zu bytes of workspace; the static workspace "
                "holds %zu",
                batch, N, need, kScratchBytes);
  DeviceGuard dg(c->device);
  hipError_t le = pd::scratch_resolve(c->device);
  if (le != hipSuccess) return hipfail(c, le, "static workspace address");
  unsigned char* base = static_cast<unsigned char*>(g_ptr[c->device]);
  hipStream_t st = static_cast<hipStream_t>(s);
  int* flag = reinterpret_cast<int*>(base);
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, flag, 1);
  PD_HIP(c, hipGetLastError(), "zero flag");
  PD_HIP(c, pd::check_box(static_cast<const cplx*>(d_in), N, batch, flag, st), "check_box");
  int h = 0;
  PD_HIP(c, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  if (h) return fail(c, PD_EINVAL, "input field has nonzero coefficients outside the 2/3 box");
  double* dt0 = reinterpret_cast<double*>(base + o_t0);
  PD_HIP(c, hipMemcpyAsync(dt0, t0, sizeof(double) * batch, hipMemcpyHostToDevice, st), "copy t0");
  pd::FieldBatch fb;
  fb.B = reinterpret_cast<cplx*>(base + o_B);
  fb.H = reinterpret_cast<cplx*>(base + o_H);
  fb.T1 = reinterpret_cast<cplx*>(base + o_T1);
  fb.T2 = reinterpret_cast<cplx*>(base + o_T2);
  fb.R = rk ? reinterpret_cast<cplx*>(base + o_R) : nullptr;
  fb.t0 = dt0;
  fb.tw = c->tw.as<cplx>();
  c->shapes(fb);
  PD_HIP(c, pd::pack(static_cast<const cplx*>(d_in), fb.B, N, M, (size_t)batch, st), "pack");
  const pd::Problem pb = make_problem(c, dt, c->scheme_f);
  // the two-stream path would create a stream: run its one-stream form
  int path = choose_path(c, batch);
  if (path == PD_PATH_MULTI2) path = pd::PATH_MULTI;
  PD_HIP(c, pd::propagate(N, fb, pb, batch, n_steps, path, st), "propagate");
  PD_HIP(c, pd::unpack(fb.B, static_cast<cplx*>(d_out), N, M, (size_t)batch, st), "unpack");
  PD_HIP(c, hipStreamSynchronize(st), "sync");
  return PD_OK;
}

}  // extern "C"
