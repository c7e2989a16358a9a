// Seeded initial field on the host (the paper's random initial perturbation,
// Section 4), reproducing the test suite's generator bit for bit: every
// coefficient is drawn from a counter-based generator written from its
// published definitions, so no generator state has to be shared.
//
//   Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011), key = the 64-bit
//   seed, counter = (kx mod 2^32, ky mod 2^32, component, 0);
//   two 53-bit uniforms u1 = (j1 + 1) 2^-53, u2 = j2 2^-53 with
//   j = (w_a >> 5) 2^26 + (w_b >> 6) from the words (w0, w1) and (w2, w3);
//   Box-Muller (Box & Muller 1958): r = sqrt(-2 ln u1), re = r cos(2 pi u2),
//   im = r sin(2 pi u2), each times amp;
//   kept for modes inside the 2/3 box with kx^2 + ky^2 <= kmax^2, then made
//   solenoidal for k = (kx, ky, kz): b <- b - k (k . b)/|k|^2 (|k| = 0 left).
//
// Every floating-point step is one IEEE double operation in a fixed order
// (contraction into fused multiply-adds is switched off below) and the
// logarithm, sine and cosine are the C library's, so the result is the same
// bits as the reference generator on the same host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/pitdyn.h"
#include "ctx.hpp"

namespace {

struct W4 {
  uint32_t w[4];
};

W4 philox4x32_10(W4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   // round multipliers
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   // Weyl key increments
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c.w[0], p1 = (uint64_t)M1 * c.w[2];
    W4 o;
    o.w[0] = (uint32_t)(p1 >> 32) ^ c.w[1] ^ k0;
    o.w[1] = (uint32_t)p1;
    o.w[2] = (uint32_t)(p0 >> 32) ^ c.w[3] ^ k1;
    o.w[3] = (uint32_t)p0;
    c = o;
  }
  return c;
}

// fills out[3][N][N] (complex, interleaved) -- see the file comment
void seed_field(int N, double kz, uint64_t seed, double amp, double kmax, double* out) {
#pragma clang fp contract(off)
  const int K = (N - 1) / 3;
  const double two_pi = 6.283185307179586;  // the double nearest 2 pi
  const double two_m53 = 1.0 / 9007199254740992.0;
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  for (size_t i = 0; i < (size_t)6 * N * N; ++i) out[i] = 0.0;
  for (int my = 0; my < N; ++my)
    for (int mx = 0; mx < N; ++mx) {
      const int ky = my < N / 2 ? my : my - N, kx = mx < N / 2 ? mx : mx - N;
      const double dkx = kx, dky = ky;
      if (kx < -K || kx > K || ky < -K || ky > K) continue;
      if (!(dkx * dkx + dky * dky <= kmax * kmax)) continue;
      double re[3], im[3];
      for (int c = 0; c < 3; ++c) {
        W4 ctr = {{(uint32_t)kx, (uint32_t)ky, (uint32_t)c, 0u}};
        const W4 w = philox4x32_10(ctr, k0, k1);
        const uint64_t j1 = (uint64_t)(w.w[0] >> 5) * 67108864ull + (w.w[1] >> 6);
        const uint64_t j2 = (uint64_t)(w.w[2] >> 5) * 67108864ull + (w.w[3] >> 6);
        const double u1 = (double)(j1 + 1) * two_m53, u2 = (double)j2 * two_m53;
        const double r = std::sqrt(-2.0 * std::log(u1));
        const double th = two_pi * u2;
        re[c] = r * std::cos(th) * amp;
        im[c] = r * std::sin(th) * amp;
      }
      const double k2 = dkx * dkx + dky * dky + kz * kz;
      double sr = 0.0, si = 0.0;
      if (k2 > 0) {
        sr = (dkx * re[0] + dky * re[1] + kz * re[2]) / k2;
        si = (dkx * im[0] + dky * im[1] + kz * im[2]) / k2;
      }
      const double kv[3] = {dkx, dky, kz};
      for (int c = 0; c < 3; ++c) {
        const size_t o = 2 * (((size_t)c * N + my) * N + mx);
        out[o] = re[c] - kv[c] * sr;
        out[o + 1] = im[c] - kv[c] * si;
      }
    }
}

}  // namespace

extern "C" {

pd_status pd_seed_field(int N, double kz, uint64_t seed, double amp, double kmax, double* out) {
  if (!out || !pd::rt::valid_N(N) || !std::isfinite(kz) || !std::isfinite(amp) ||
      !(kmax >= 0) || !std::isfinite(kmax))
    return PD_EINVAL;
  seed_field(N, kz, seed, amp, kmax, out);
  return PD_OK;
}

pd_status pd_seed_initial(pd_ctx* c, uint64_t seed, double amp, double kmax) {
  if (!c) return PD_EINVAL;
  c->err.clear();
  if (!c->have_time) return pd::ctxh::fail(c, PD_ESTATE, "pd_set_time not called");
  if (!std::isfinite(amp) || !(kmax >= 0) || !std::isfinite(kmax))
    return pd::ctxh::fail(c, PD_EINVAL, "amp must be finite and kmax finite and >= 0");
  std::vector<double> b((size_t)6 * c->N * c->N);
  seed_field(c->N, c->kz, seed, amp, kmax, b.data());
  return pd_set_initial(c, b.data());
}

}  // extern "C"
