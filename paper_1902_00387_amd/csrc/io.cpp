// Host-array propagator calls, Parareal checkpoint / resume, and the file
// format of the learned coarse propagator's parameters (C ABI).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ctx.hpp"
#include "nn.hpp"

using namespace pd::ctxh;

namespace {

// F or G over one slice on host arrays [batch][3][N][N] (interleaved re, im)
pd_status step_host(pd_ctx* c, const double* t0, int batch, const double* in, double* out,
                    bool fine) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (batch < 0 || batch > 65535) return fail(c, PD_EINVAL, "batch must be in [0, 65535]");
  if (batch == 0) return PD_OK;
  if (!t0 || !in || !out) return fail(c, PD_EINVAL, "null pointer argument");
  DeviceGuard dg(c->device);
  const size_t bytes = (size_t)batch * 3 * c->N * c->N * sizeof(cplx);
  DevBuf d;
  PD_HIP(c, d.ensure(bytes), "alloc");
  PD_HIP(c, hipMemcpyAsync(d.p, in, bytes, hipMemcpyHostToDevice, c->stream), "copy");
  pd_status s = fine ? run_propagator(c, t0, batch, c->dtf, c->nf, c->N, d.p, d.p, c->stream,
                                      c->scheme_f)
                     : run_propagator(c, t0, batch, c->dtc, c->nc, c->Nc, d.p, d.p, c->stream,
                                      c->scheme_c);
  if (s != PD_OK) return s;
  PD_HIP(c, hipMemcpyAsync(out, d.p, bytes, hipMemcpyDeviceToHost, c->stream), "copy");
  PD_HIP(c, hipStreamSynchronize(c->stream), "sync");
  return PD_OK;
}

// host full-layout fields [n][3][N][N] -> compact boxes at dst (checked)
pd_status host_to_box(pd_ctx* c, const double* src, size_t n, cplx* dst) {
  const size_t full = (size_t)3 * c->N * c->N;
  DevBuf tmp;
  PD_HIP(c, tmp.ensure(full * n * sizeof(cplx)), "alloc");
  PD_HIP(c, hipMemcpyAsync(tmp.p, src, full * n * sizeof(cplx), hipMemcpyHostToDevice, c->stream),
         "copy");
  pd_status s = check_box_dev(c, tmp.p, c->N, n, c->stream);
  if (s != PD_OK) return s;
  PD_HIP(c, pd::pack(tmp.as<cplx>(), dst, c->N, c->M, n, c->stream), "pack");
  PD_HIP(c, hipStreamSynchronize(c->stream), "sync");
  return PD_OK;
}

constexpr char kMagic[8] = {'P', 'D', 'L', 'G', 'N', 'E', 'T', '1'};

struct FileCloser {
  FILE* f;
  ~FileCloser() {
    if (f) std::fclose(f);
  }
};

}  // namespace

extern "C" {

pd_status pd_step_fine(pd_ctx* c, const double* t0, int batch, const double* in, double* out) {
  return step_host(c, t0, batch, in, out, true);
}

pd_status pd_step_coarse(pd_ctx* c, const double* t0, int batch, const double* in, double* out) {
  return step_host(c, t0, batch, in, out, false);
}

pd_status pd_get_coarse_values(const pd_ctx* cc, double* out) {
  pd_ctx* c = const_cast<pd_ctx*>(cc);
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (!out) return fail(c, PD_EINVAL, "null pointer argument");
  if (c->prec == PD_C64) return fail(c, PD_EINVAL, "checkpoints are complex128 only");
  DeviceGuard dg(c->device);
  const size_t full = (size_t)3 * c->N * c->N;
  DevBuf tmp;
  PD_HIP(c, tmp.ensure(full * c->P * sizeof(cplx)), "alloc");
  PD_HIP(c, pd::unpack(c->Gold.as<cplx>(), tmp.as<cplx>(), c->N, c->M, (size_t)c->P, c->stream), "unpack");
  PD_HIP(c, hipMemcpyAsync(out, tmp.p, full * c->P * sizeof(cplx), hipMemcpyDeviceToHost, c->stream),
         "copy");
  PD_HIP(c, hipStreamSynchronize(c->stream), "sync");
  return PD_OK;
}

pd_status pd_set_slices(pd_ctx* c, const double* U, const double* Gold, int k) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (!U) return fail(c, PD_EINVAL, "null pointer argument");
  if (k < 0 || k >= PD_MAX_ITER) return fail(c, PD_EINVAL, "k must be in [0, %d)", PD_MAX_ITER);
  if (c->prec == PD_C64) return fail(c, PD_EINVAL, "checkpoints are complex128 only");
  DeviceGuard dg(c->device);
  pd_status s = host_to_box(c, U, (size_t)c->P + 1, c->U.as<cplx>());
  if (s != PD_OK) return s;
  c->have_gold = Gold != nullptr;
  if (Gold) {
    s = host_to_box(c, Gold, (size_t)c->P, c->Gold.as<cplx>());
    if (s != PD_OK) return s;
  }
  c->have_initial = true;
  c->resume_k = k;
  c->last_k = -1;
  return PD_OK;
}

pd_status pd_lg_save(const pd_ctx* cc, const char* path) {
  pd_ctx* c = const_cast<pd_ctx*>(cc);
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->lg.init) return fail(c, PD_ESTATE, "pd_lg_init not called");
  if (!path) return fail(c, PD_EINVAL, "null pointer argument");
  const size_t np = pd::nn::param_count(c->lg.Q, c->lg.L);
  std::vector<float> p(np);
  DeviceGuard dg(c->device);
  PD_HIP(c, hipMemcpy(p.data(), c->lg.params.p, sizeof(float) * np, hipMemcpyDeviceToHost), "copy");
  FileCloser fc{std::fopen(path, "wb")};
  if (!fc.f) return fail(c, PD_EINVAL, "cannot open %s for writing", path);
  const int32_t hdr[4] = {c->N, c->lg.Mf, c->lg.L, pd::nn::CH};
  const uint64_t n64 = np;
  bool ok = std::fwrite(kMagic, 1, 8, fc.f) == 8 && std::fwrite(hdr, sizeof hdr, 1, fc.f) == 1 &&
            std::fwrite(&n64, sizeof n64, 1, fc.f) == 1 &&
            std::fwrite(p.data(), sizeof(float), np, fc.f) == np;
  ok = (std::fclose(fc.f) == 0) && ok;
  fc.f = nullptr;
  if (!ok) return fail(c, PD_EINVAL, "write to %s failed", path);
  return PD_OK;
}

pd_status pd_lg_load(pd_ctx* c, const char* path) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return fail(c, PD_ESTATE, "pd_set_time not called");
  if (!path) return fail(c, PD_EINVAL, "null pointer argument");
  FileCloser fc{std::fopen(path, "rb")};
  if (!fc.f) return fail(c, PD_EINVAL, "cannot open %s", path);
  char magic[8];
  int32_t hdr[4];
  uint64_t n64 = 0;
  if (std::fread(magic, 1, 8, fc.f) != 8 || std::memcmp(magic, kMagic, 8) != 0 ||
      std::fread(hdr, sizeof hdr, 1, fc.f) != 1 || std::fread(&n64, sizeof n64, 1, fc.f) != 1)
    return fail(c, PD_EINVAL, "%s is not a learned-propagator parameter file", path);
  if (hdr[0] != c->N || hdr[1] != c->M || hdr[3] != pd::nn::CH || hdr[2] < 1 || hdr[2] > 8)
    return fail(c, PD_EINVAL, "%s holds a network for N=%d (box %d, width %d), context has N=%d",
                path, hdr[0], hdr[1], hdr[3], c->N);
  const size_t np = pd::nn::param_count(c->M * c->M, hdr[2]);
  if (n64 != np) return fail(c, PD_EINVAL, "%s: %llu values, %zu expected", path,
                             (unsigned long long)n64, np);
  std::vector<float> p(np);
  if (std::fread(p.data(), sizeof(float), np, fc.f) != np)
    return fail(c, PD_EINVAL, "%s is truncated", path);
  const bool enabled = c->lg.enabled;
  pd_status s = pd_lg_init(c, hdr[2], 0);
  if (s != PD_OK) return s;
  s = pd_lg_set_params(c, p.data(), np);
  if (s != PD_OK) return s;
  c->lg.enabled = enabled;
  return PD_OK;
}

}  // extern "C"
