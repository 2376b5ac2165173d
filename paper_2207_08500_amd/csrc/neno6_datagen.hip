// Seeded classifier-training samples generated on the device (the synthetic
// stand-in for the training data of Sec. 3.2: smooth functions and functions
// with a jump or a kink, each six-point stencil labelled per candidate).
//
// Sample i is a pure function of (seed, i): its uniforms come from
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011) with the counters
// (lo(i), hi(i), b, 0x43355331), b = 0..4, and the key (lo(seed),
// hi(seed)); a 32-bit word w gives (w + 1/2) 2^-32.  Every value is formed in
// FP64 with separately rounded operations (this file is compiled without
// contraction), so the positions and the labels are exactly reproducible on
// the host; exp and sin come from the device math library.
#include "neno6_device.h"
#include "neno6_fast.h"

namespace n6 {

namespace {

constexpr uint32_t PM0 = 0xD2511F53u, PM1 = 0xCD9E8D57u;  // round multipliers
constexpr uint32_t PW0 = 0x9E3779B9u, PW1 = 0xBB67AE85u;  // key increments
constexpr uint32_t C5_STREAM = 0x43355331u;

struct U4 {
  uint32_t v[4];
};

N6_DEV U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                        uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += PW0;
      k1 += PW1;
    }
    const uint64_t p0 = (uint64_t)PM0 * c0, p1 = (uint64_t)PM1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  return U4{{c0, c1, c2, c3}};
}

N6_DEV double unit(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

__global__ void __launch_bounds__(256) k_classifier_samples(uint64_t seed, int64_t first, int64_t n,
                                                            float *__restrict__ s,
                                                            uint8_t *__restrict__ y) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint64_t i = (uint64_t)(first + t);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  double u[5][4];
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const U4 w = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), (uint32_t)b, C5_STREAM, k0, k1);
#pragma unroll
    for (int q = 0; q < 4; ++q) u[b][q] = unit(w.v[q]);
  }
  const double N = u[0][0] < 0.4 ? 50.0 : (u[0][0] < 0.8 ? 100.0 : 200.0);
  const double dx = 2.0 / N;
  const double xc = -1.0 + 2.0 * u[0][1];
  const bool smooth = u[0][2] < 0.5;
  const bool kind = u[0][3] >= 0.5;  // smooth: sine / polynomial; jump: kink / step
  double xs[6], tt[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    tt[j] = (double)(j - 2) * dx;
    xs[j] = xc + tt[j];
  }
  double f[6];
  uint8_t lab = 0;
  if (smooth && !kind) {  // polynomial of degree 0..5 in t, Horner
    const double deg = fmin(floor(6.0 * u[1][0]), 5.0);
    const double cu[6] = {u[2][0], u[2][1], u[2][2], u[2][3], u[3][0], u[3][1]};
    double coef[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) coef[d] = (double)d <= deg ? -1.0 + 2.0 * cu[d] : 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double p = 0.0;
#pragma unroll
      for (int d = 5; d >= 0; --d) p = p * tt[j] + coef[d];
      f[j] = p;
    }
  } else if (smooth) {  // A sin(w x + phi)
    const double w = 0.5 + 19.5 * u[1][1];
    const double phi = 0x1.921fb54442d18p+2 * u[1][2];
    const double lo = -0x1.26bb1bbb55515p+2, hi = 0x1.26bb1bbb55516p+2;
    const double A = exp(lo + u[1][3] * (hi - lo));
#pragma unroll
    for (int j = 0; j < 6; ++j) f[j] = A * sin(w * xs[j] + phi);
  } else {  // a jump at x_d: step or kink, amplitude ratio r across it
    const double xd = xs[0] + u[3][2] * (xs[5] - xs[0]);
    const double a = (0.1 + 0.9 * u[3][3]) * (u[4][0] < 0.5 ? -1.0 : 1.0);
    const double lo = -0x1.ba18a998fffa0p+2, hi = 0x1.ba18a998fffa0p+2;
    const double r = exp(lo + u[4][1] * (hi - lo));
    const double ar = a * r;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const double amp = xs[j] > xd ? ar : a;
      f[j] = kind ? amp * (xs[j] - xd) : amp;
    }
    // candidate k is crossed when x_d lies strictly inside its span
    const int span[4][2] = {{1, 3}, {2, 4}, {0, 2}, {2, 5}};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (xd > xs[span[k][0]] && xd < xs[span[k][1]]) lab |= (uint8_t)(1u << k);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) s[6 * t + j] = (float)f[j];
  y[t] = lab;
}

}  // namespace

hipError_t launch_classifier_samples(uint64_t seed, int64_t first, int64_t n, float *s, uint8_t *y,
                                     hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_classifier_samples, dim3((unsigned)blocks), dim3(256), 0, st, seed, first, n,
                     s, y);
  return hipGetLastError();
}

}  // namespace n6
