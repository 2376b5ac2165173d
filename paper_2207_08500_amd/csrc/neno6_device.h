// Device helpers of the NENO6 kernels (gfx950).  Internal to libneno6.
//
// Everything here is written for one stencil at a time in registers; the
// kernels decide how stencils map to lanes.  The templates are instantiated
// for double (the plain FP64 path, compiled without FP contraction so that
// the written fma order is the one executed) and float (fast paths).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "neno6_internal.h"
#include "neno6_teno_tables.h"

#define N6_DEV __device__ __forceinline__

namespace n6 {

// Status codes mirrored from the public header.
constexpr int32_t ST_NONPHYSICAL = -4;

// Linear weights of TENO6-opt, also NENO6's (Sec. 2.2 / Sec. 4).
template <typename T> struct Lin;
template <> struct Lin<double> {
  static constexpr double d0 = 0.4294317718960898, d1 = 0.1727270875843552,
                          d2 = 0.0855682281039113, d3 = 0.312272912415645;
};
template <> struct Lin<float> {
  static constexpr float d0 = 0.4294317718960898f, d1 = 0.1727270875843552f,
                         d2 = 0.0855682281039113f, d3 = 0.312272912415645f;
};

template <typename T> N6_DEV T fma_(T a, T b, T c);
template <> N6_DEV double fma_<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> N6_DEV float fma_<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Candidate interface values at x_{i+1/2} (eq. approximatepolynomial with
// eq. definitionEq: cell averages of the candidate polynomial reproduce the
// stencil values).  s[0..5] = values at cells i-2..i+3.  Each sum is an fma
// chain from zero in ascending stencil position.
template <typename T>
N6_DEV void candidates(const T s[6], T &q0, T &q1, T &q2, T &q3) {
  const T z = T(0);
  // S0 = {i-1, i, i+1}
  q0 = fma_<T>(T(1) / T(3), s[3], fma_<T>(T(5) / T(6), s[2], fma_<T>(T(-1) / T(6), s[1], z)));
  // S1 = {i, i+1, i+2}
  q1 = fma_<T>(T(-1) / T(6), s[4], fma_<T>(T(5) / T(6), s[3], fma_<T>(T(1) / T(3), s[2], z)));
  // S2 = {i-2, i-1, i}
  q2 = fma_<T>(T(11) / T(6), s[2], fma_<T>(T(-7) / T(6), s[1], fma_<T>(T(1) / T(3), s[0], z)));
  // S3 = {i, i+1, i+2, i+3}
  q3 = fma_<T>(T(1) / T(12), s[5],
               fma_<T>(T(-5) / T(12), s[4], fma_<T>(T(13) / T(12), s[3], fma_<T>(T(1) / T(4), s[2], z))));
}

// Re-normalised convex combination of the kept candidates (eq. convex,
// eq. TENOweight_renormalize); with nothing kept, the first-order upwind
// value s[2] (Alg. 2, step 4).  Canonical order: D summed over kept k in k
// order, w_k = d_k / D, fma chain over kept k from zero.
template <typename T>
N6_DEV T combine_canonical(const T s[6], unsigned sel) {
  T q0, q1, q2, q3;
  candidates<T>(s, q0, q1, q2, q3);
  if ((sel & 15u) == 0u) return s[2];
  T D = T(0);
  if (sel & 1u) D = D + Lin<T>::d0;
  if (sel & 2u) D = D + Lin<T>::d1;
  if (sel & 4u) D = D + Lin<T>::d2;
  if (sel & 8u) D = D + Lin<T>::d3;
  T h = T(0);
  if (sel & 1u) h = fma_<T>(Lin<T>::d0 / D, q0, h);
  if (sel & 2u) h = fma_<T>(Lin<T>::d1 / D, q1, h);
  if (sel & 4u) h = fma_<T>(Lin<T>::d2 / D, q2, h);
  if (sel & 8u) h = fma_<T>(Lin<T>::d3 / D, q3, h);
  return h;
}

// Branch-free combine for the fast paths (same weights, FP32, one reciprocal).
// No implicit contraction here or in combine_pair: a face whose flux is
// computed in two kernels (or twice in one) gives the same bits both times.
N6_DEV float combine_fast(const float s[6], unsigned sel) {
#pragma clang fp contract(off)
  float q0, q1, q2, q3;
  candidates<float>(s, q0, q1, q2, q3);
  const float w0 = (sel & 1u) ? Lin<float>::d0 : 0.f;
  const float w1 = (sel & 2u) ? Lin<float>::d1 : 0.f;
  const float w2 = (sel & 4u) ? Lin<float>::d2 : 0.f;
  const float w3 = (sel & 8u) ? Lin<float>::d3 : 0.f;
  const float D = (w0 + w1) + (w2 + w3);
  const float num = fmaf(w3, q3, fmaf(w2, q2, fmaf(w1, q1, w0 * q0)));
  return (sel & 15u) ? num * __builtin_amdgcn_rcpf(D) : s[2];
}

// h+ + h- of one characteristic field (the two split fluxes' reconstructions).
N6_DEV float combine_pair(const float sp[6], unsigned selp, const float sm[6], unsigned selm) {
#pragma clang fp contract(off)
  return combine_fast(sp, selp) + combine_fast(sm, selm);
}

// The re-normalised combination as one linear stencil per selection: with
// the candidates in sel kept, h = sum_j c_j(sel) s_j, where c(sel) is the
// combination of the unit stencils (sel = 0: the fallback s_2).  The
// weights of every selection sum to one, so h = s_2 + sum_{j != 2} c_j
// (s_j - s_2): the form the fused Euler kernels evaluate, whose rounding
// scales with the stencil's variation rather than its size (a constant
// stencil gives s_2 exactly).  They hold the 16 x 6 table in LDS,
// coefficient j of selection m at [j][m] (lanes with different selections
// read different banks, lanes with the same one the same word), and take
// five differences and five products per reconstruction instead of four
// candidates and their weights.
struct CombTab {
  float c[6][16];
};
// The candidates' coefficients on cells i-2..i+3 (those of candidates()) and
// the table, both evaluated at compile time: entry [j][m] is the FP64
// combination of the unit stencil e_j, rounded to FP32.
constexpr double kCand[4][6] = {{0.0, -1.0 / 6, 5.0 / 6, 1.0 / 3, 0.0, 0.0},
                                {0.0, 0.0, 1.0 / 3, 5.0 / 6, -1.0 / 6, 0.0},
                                {1.0 / 3, -7.0 / 6, 11.0 / 6, 0.0, 0.0, 0.0},
                                {0.0, 0.0, 1.0 / 4, 13.0 / 12, -5.0 / 12, 1.0 / 12}};
constexpr CombTab make_comb_tab() {
  const double d[4] = {Lin<double>::d0, Lin<double>::d1, Lin<double>::d2, Lin<double>::d3};
  CombTab t{};
  for (int m = 0; m < 16; ++m) {
    double D = 0.0;
    for (int k = 0; k < 4; ++k)
      if (m >> k & 1) D += d[k];
    for (int j = 0; j < 6; ++j) {
      double c = m == 0 && j == 2 ? 1.0 : 0.0;
      for (int k = 0; k < 4; ++k)
        if (m >> k & 1) c += d[k] / D * kCand[k][j];
      t.c[j][m] = (float)c;
    }
  }
  return t;
}
// Copies the table into LDS; every thread of the workgroup calls it (it
// ends with a barrier).
N6_DEV void comb_fill(CombTab &t) {
  constexpr CombTab k = make_comb_tab();
  for (int i = (int)threadIdx.x; i < 96; i += (int)blockDim.x) t.c[i >> 4][i & 15] = k.c[i >> 4][i & 15];
  __syncthreads();
}
// sel < 16 (a selection).
N6_DEV float comb_tab(const CombTab &t, const float s[6], unsigned sel) {
  float d = t.c[0][sel] * (s[0] - s[2]);
  d = fmaf(t.c[1][sel], s[1] - s[2], d);
  d = fmaf(t.c[3][sel], s[3] - s[2], d);
  d = fmaf(t.c[4][sel], s[4] - s[2], d);
  d = fmaf(t.c[5][sel], s[5] - s[2], d);
  return s[2] + d;
}
N6_DEV float comb_pair_tab(const CombTab &t, const float sp[6], unsigned selp, const float sm[6], unsigned selm) {
  return comb_tab(t, sp, selp) + comb_tab(t, sm, selm);
}

// Input scaling of the classifier (eq. normalizainput): divide by
// max(|s_0|, ..., |s_5|, 1).
template <typename T>
N6_DEV void features(const T s[6], T x[6]) {
  T M = T(1);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T a = s[j] < T(0) ? -s[j] : s[j];
    M = a > M ? a : M;
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) x[j] = s[j] / M;
}

// Parameter block offsets (row-major [out][in] weights then biases).
constexpr int OW1 = 0, OB1 = 384, OW2 = 448, OB2 = 2496, OW3 = 2528, OB3 = 3040, OW4 = 3056,
              OB4 = 3184, OW5 = 3192, OB5 = 3224, NPARAM = 3228;

// Dense layer with the canonical fma order (bias first, inputs ascending).
template <typename T, int NIN, int NOUT, bool RELU>
N6_DEV void dense(const T *__restrict__ W, const T *__restrict__ b, const T *x, T *y) {
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    T acc = b[o];
#pragma unroll
    for (int i = 0; i < NIN; ++i) acc = fma_<T>(W[o * NIN + i], x[i], acc);
    y[o] = RELU ? (acc > T(0) ? acc : T(0)) : acc;
  }
}

// The 6-64-32-16-8-4 network (eq. reconstuction, activationfunction) up to
// the output logits.  P: parameter block in type T (uniform across lanes, so
// the weights come in through scalar loads).
template <typename T>
N6_DEV void mlp_logits(const T *__restrict__ P, const T x0[6], T z[4]) {
  T a1[64], a2[32], a3[16], a4[8];
  dense<T, 6, 64, true>(P + OW1, P + OB1, x0, a1);
  dense<T, 64, 32, true>(P + OW2, P + OB2, a1, a2);
  dense<T, 32, 16, true>(P + OW3, P + OB3, a2, a3);
  dense<T, 16, 8, true>(P + OW4, P + OB4, a3, a4);
  dense<T, 8, 4, false>(P + OW5, P + OB5, a4, z);
}

// Kept mask: candidate k discarded iff logit > 0 (sigmoid > 1/2).
template <typename T>
N6_DEV unsigned mask_from_logits(const T z[4]) {
  unsigned m = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) m |= (z[k] > T(0)) ? 0u : (1u << k);
  return m;
}

template <typename T>
N6_DEV unsigned classify(const T *__restrict__ P, const T s[6]) {
  T x[6], z[4];
  features<T>(s, x);
  mlp_logits<T>(P, x, z);
  return mask_from_logits<T>(z);
}

// Ghost cells: periodic wrap, or zero-gradient copy of the nearest cell.
N6_DEV int64_t ghost(int64_t c, int64_t n, int bc) {
  if (bc == 0) {
    int64_t r = c % n;
    return r < 0 ? r + n : r;
  }
  return c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
}

// The same in 32-bit arithmetic for indices within one line (c in
// [-3, n + 2]); the periodic wrap needs at most three corrections.
N6_DEV int ghost32(int c, int n, int bc) {
  if (bc == 0) {
    while (c < 0) c += n;
    while (c >= n) c -= n;
    return c;
  }
  return c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
}

// Largest p with offsets[p] + p*extra <= g (problems are non-empty).
N6_DEV int find_problem(const int64_t *__restrict__ offsets, int np, int64_t g, int extra) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offsets[mid] + (int64_t)mid * extra <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Line of face g: one load from the face map when it was built for this
// call, else a binary search over the offsets.
N6_DEV int line_of_face(const Line1D &ln, int64_t g) {
  return ln.fmap ? ln.fmap[g] : find_problem(ln.offsets, ln.np, g, 1);
}

template <typename T> N6_DEV T sqrt_(T x);
template <> N6_DEV double sqrt_<double>(double x) { return __builtin_sqrt(x); }
template <> N6_DEV float sqrt_<float>(float x) { return __builtin_sqrtf(x); }
template <typename T> N6_DEV T abs_(T x) { return x < T(0) ? -x : x; }

// ---- 1D Euler (Sec. 4.4), state (rho, rho u, E) ----------------------------
template <typename T>
N6_DEV void prim1d(const T q[3], T gamma, T &u, T &p, T &c) {
  u = q[1] / q[0];
  const T t = q[1] * u;
  const T ke = T(0.5) * t;
  p = (gamma - T(1)) * (q[2] - ke);
  c = sqrt_<T>((gamma * p) / q[0]);
}

template <typename T>
N6_DEV void flux1d(const T q[3], T u, T p, T F[3]) {
  F[0] = q[1];
  F[1] = q[1] * u + p;
  F[2] = (q[2] + p) * u;
}

// Roe-averaged eigenvectors of the 1D flux Jacobian: columns of R (and rows
// of L = R^-1) are the fields of speed u-c, u, u+c.
template <typename T>
N6_DEV void roe1d(const T qL[3], const T qR[3], T gamma, T L[3][3], T R[3][3]) {
  T uL, pL, cL, uR, pR, cR;
  prim1d<T>(qL, gamma, uL, pL, cL);
  prim1d<T>(qR, gamma, uR, pR, cR);
  const T sL = sqrt_<T>(qL[0]), sR = sqrt_<T>(qR[0]);
  const T HL = (qL[2] + pL) / qL[0], HR = (qR[2] + pR) / qR[0];
  const T den = sL + sR;
  const T ut = (sL * uL + sR * uR) / den;
  const T Ht = (sL * HL + sR * HR) / den;
  const T q2 = T(0.5) * (ut * ut);
  const T c2 = (gamma - T(1)) * (Ht - q2);
  const T ct = sqrt_<T>(c2);
  const T b1 = (gamma - T(1)) / c2;
  const T b2 = b1 * q2;
  const T uc = ut / ct;
  const T ic = T(1) / ct;
  R[0][0] = T(1);         R[0][1] = T(1); R[0][2] = T(1);
  R[1][0] = ut - ct;      R[1][1] = ut;   R[1][2] = ut + ct;
  R[2][0] = Ht - ut * ct; R[2][1] = q2;   R[2][2] = Ht + ut * ct;
  L[0][0] = T(0.5) * (b2 + uc); L[0][1] = T(-0.5) * (b1 * ut + ic); L[0][2] = T(0.5) * b1;
  L[1][0] = T(1) - b2;          L[1][1] = b1 * ut;                  L[1][2] = -b1;
  L[2][0] = T(0.5) * (b2 - uc); L[2][1] = T(-0.5) * (b1 * ut - ic); L[2][2] = T(0.5) * b1;
}

// ---- 2D Euler, state (rho, rho u, rho v, E); dir 0 = x, 1 = y -------------
template <typename T>
N6_DEV void prim2d(const T q[4], T gamma, T &u, T &v, T &p, T &c) {
  u = q[1] / q[0];
  v = q[2] / q[0];
  const T t1 = q[1] * u;
  const T t2 = q[2] * v;
  const T ke = T(0.5) * (t1 + t2);
  p = (gamma - T(1)) * (q[3] - ke);
  c = sqrt_<T>((gamma * p) / q[0]);
}

template <typename T>
N6_DEV void flux2d(const T q[4], T u, T v, T p, int dir, T F[4]) {
  if (dir == 0) {
    F[0] = q[1];
    F[1] = q[1] * u + p;
    F[2] = q[2] * u;
    F[3] = (q[3] + p) * u;
  } else {
    F[0] = q[2];
    F[1] = q[1] * v;
    F[2] = q[2] * v + p;
    F[3] = (q[3] + p) * v;
  }
}

// Roe eigenvectors for the sweep direction.  Fields: u_n - c, u_n, shear
// (tangential velocity, passive), u_n + c.
template <typename T>
N6_DEV void roe2d(const T qL[4], const T qR[4], T gamma, int dir, T L[4][4], T R[4][4]) {
  T uL, vL, pL, cL, uR, vR, pR, cR;
  prim2d<T>(qL, gamma, uL, vL, pL, cL);
  prim2d<T>(qR, gamma, uR, vR, pR, cR);
  const T sL = sqrt_<T>(qL[0]), sR = sqrt_<T>(qR[0]);
  const T HL = (qL[3] + pL) / qL[0], HR = (qR[3] + pR) / qR[0];
  const T den = sL + sR;
  const T ut = (sL * uL + sR * uR) / den;
  const T vt = (sL * vL + sR * vR) / den;
  const T Ht = (sL * HL + sR * HR) / den;
  const T q2 = T(0.5) * (ut * ut + vt * vt);
  const T c2 = (gamma - T(1)) * (Ht - q2);
  const T ct = sqrt_<T>(c2);
  const T b1 = (gamma - T(1)) / c2;
  const T b2 = b1 * q2;
  const T ic = T(1) / ct;
  const T un = dir == 0 ? ut : vt;
  const T us = dir == 0 ? vt : ut;
  const T nc = un / ct;
  // rows/cols in the variable order (rho, rho u_n, rho u_s, E)
  const T Rn[4][4] = {{T(1), T(1), T(0), T(1)},
                      {un - ct, un, T(0), un + ct},
                      {us, us, T(1), us},
                      {Ht - un * ct, q2, us, Ht + un * ct}};
  const T Ln[4][4] = {{T(0.5) * (b2 + nc), T(-0.5) * (b1 * un + ic), T(-0.5) * (b1 * us), T(0.5) * b1},
                      {T(1) - b2, b1 * un, b1 * us, -b1},
                      {-us, T(0), T(1), T(0)},
                      {T(0.5) * (b2 - nc), T(-0.5) * (b1 * un - ic), T(-0.5) * (b1 * us), T(0.5) * b1}};
  const int vn = dir == 0 ? 1 : 2, vs = dir == 0 ? 2 : 1;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    R[0][m] = Rn[0][m];
    R[vn][m] = Rn[1][m];
    R[vs][m] = Rn[2][m];
    R[3][m] = Rn[3][m];
    L[m][0] = Ln[m][0];
    L[m][vn] = Ln[m][1];
    L[m][vs] = Ln[m][2];
    L[m][3] = Ln[m][3];
  }
}

// RK3 stage update (Sec. 4.4, SSP-RK3):
//   stage 1: u1 = u0 + dt L(u0)
//   stage 2: u2 = 3/4 u0 + 1/4 (u1 + dt L(u1))
//   stage 3: u  = 1/3 u0 + 2/3 (u2 + dt L(u2))
template <typename T>
N6_DEV T rk3(int stage, T us, T u0, T L, T dt) {
  if (stage == 1) return fma_<T>(dt, L, us);
  const T t = fma_<T>(dt, L, us);
  if (stage == 2) return fma_<T>(T(0.25), t, T(0.75) * u0);
  return fma_<T>(T(2) / T(3), t, (T(1) / T(3)) * u0);
}

template <typename T>
N6_DEV bool physical(T rho, T p) {
  return rho > T(0) && p > T(0) && __builtin_isfinite(rho) && __builtin_isfinite(p);
}

// ---- classifier on the vector units, weights staged in LDS ------------------
// LDS image of the parameters (values of type T):
//   W1b [64][8]  (W1 row, b1, pad)   W2T [64][32]  b2 [32]
//   W3T [32][16] b3 [16]   W4T [16][8] b4 [8]   W5T [8][4] b5 [4]
constexpr int S_W1 = 0, S_W2 = 512, S_B2 = 2560, S_W3 = 2592, S_B3 = 3104, S_W4 = 3120,
              S_B4 = 3248, S_W5 = 3256, S_B5 = 3288, S_SIZE = 3292;

template <typename T>
N6_DEV void stage_params(const T *__restrict__ P, T *S) {
  for (int t = threadIdx.x; t < S_SIZE; t += blockDim.x) {
    T v = T(0);
    if (t < S_W2) {
      const int o = t >> 3, k = t & 7;
      v = k < 6 ? P[OW1 + o * 6 + k] : (k == 6 ? P[OB1 + o] : T(0));
    } else if (t < S_B2) {
      const int i = (t - S_W2) >> 5, o = (t - S_W2) & 31;
      v = P[OW2 + o * 64 + i];
    } else if (t < S_W3) {
      v = P[OB2 + t - S_B2];
    } else if (t < S_B3) {
      const int i = (t - S_W3) >> 4, o = (t - S_W3) & 15;
      v = P[OW3 + o * 32 + i];
    } else if (t < S_W4) {
      v = P[OB3 + t - S_B3];
    } else if (t < S_B4) {
      const int i = (t - S_W4) >> 3, o = (t - S_W4) & 7;
      v = P[OW4 + o * 16 + i];
    } else if (t < S_W5) {
      v = P[OB4 + t - S_B4];
    } else if (t < S_B5) {
      const int i = (t - S_W5) >> 2, o = (t - S_W5) & 3;
      v = P[OW5 + o * 8 + i];
    } else {
      v = P[OB5 + t - S_B5];
    }
    S[t] = v;
  }
}

// The 6-64-32-16-8-4 network up to the logits, input-stationary (the loop
// over a layer's inputs is outermost, all of the layer's accumulators
// advance together), with the same per-accumulator operation sequence as the
// output-stationary form: bias, then fma over the inputs in ascending order;
// ReLU as "x > 0 ? x : 0".
template <typename T>
N6_DEV void mlp_lean(const T *S, const T x0[6], T z[4]) {
  T acc2[32];
#pragma unroll
  for (int o = 0; o < 32; ++o) acc2[o] = S[S_B2 + o];
#pragma unroll 2
  for (int i = 0; i < 64; ++i) {
    T a = S[S_W1 + i * 8 + 6];
#pragma unroll
    for (int k = 0; k < 6; ++k) a = fma_<T>(S[S_W1 + i * 8 + k], x0[k], a);
    a = a > T(0) ? a : T(0);
#pragma unroll
    for (int o = 0; o < 32; ++o) acc2[o] = fma_<T>(S[S_W2 + i * 32 + o], a, acc2[o]);
  }
  T acc3[16];
#pragma unroll
  for (int o = 0; o < 16; ++o) acc3[o] = S[S_B3 + o];
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const T a = acc2[i] > T(0) ? acc2[i] : T(0);
#pragma unroll
    for (int o = 0; o < 16; ++o) acc3[o] = fma_<T>(S[S_W3 + i * 16 + o], a, acc3[o]);
  }
  T acc4[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) acc4[o] = S[S_B4 + o];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const T a = acc3[i] > T(0) ? acc3[i] : T(0);
#pragma unroll
    for (int o = 0; o < 8; ++o) acc4[o] = fma_<T>(S[S_W4 + i * 8 + o], a, acc4[o]);
  }
#pragma unroll
  for (int o = 0; o < 4; ++o) z[o] = S[S_B5 + o];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const T a = acc4[i] > T(0) ? acc4[i] : T(0);
#pragma unroll
    for (int o = 0; o < 4; ++o) z[o] = fma_<T>(S[S_W5 + i * 4 + o], a, z[o]);
  }
}

template <typename T>
N6_DEV unsigned classify_lean(const T *S, const T s[6]) {
  T x[6], z[4];
  features<T>(s, x);
  mlp_lean<T>(S, x, z);
  return mask_from_logits<T>(z);
}

// ---- TENO6-opt selection (Sec. 2.2 and 2.3) ---------------------------------
// Smoothness indicators (eq. measureTENO) in the Jiang-Shu form, written over
// differences of neighbouring values so constant data give exactly zero;
// sixth-order reference tau_6 (eq. taukTENO); normalisation (eq. normalize)
// and the sharp cut-off C_T (eq. cut-off); C = 1, q = 6, eps = 1e-40,
// C_T = 1e-6.  Evaluated in FP64 in every mode, from the stencil values
// promoted exactly, in this fixed order (no contraction):
//   d_a = s[first+a+1] - s[first+a]; t_a = fma over b ascending of D[a][b] d_b
//   from 0; beta = fma over a ascending of d_a t_a from 0;
//   tau = |beta6 - ((beta1 + beta2) + 4 beta0) / 6|;
//   x_k = 1 + tau / (beta_k + eps); gamma_k = (x^2 x^2) x^2;
//   chi_k = gamma_k / (((gamma0 + gamma1) + gamma2) + gamma3);
//   candidate k kept unless chi_k < C_T.
template <int FIRST, int N>
N6_DEV double teno_beta(const double (&D)[N][N], const double s[6]) {
#pragma clang fp contract(off)
  double d[N];
#pragma unroll
  for (int a = 0; a < N; ++a) d[a] = s[FIRST + a + 1] - s[FIRST + a];
  double beta = 0.0;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) t = __builtin_fma(D[a][b], d[b], t);
    beta = __builtin_fma(d[a], t, beta);
  }
  return beta;
}

N6_DEV unsigned teno_mask(const double s[6]) {
#pragma clang fp contract(off)
  const double bk[4] = {teno_beta<TENO_FIRST_S0>(TENO_D_S0, s), teno_beta<TENO_FIRST_S1>(TENO_D_S1, s),
                        teno_beta<TENO_FIRST_S2>(TENO_D_S2, s), teno_beta<TENO_FIRST_S3>(TENO_D_S3, s)};
  const double b6 = teno_beta<TENO_FIRST_S6>(TENO_D_S6, s);
  const double tau = __builtin_fabs(b6 - ((bk[1] + bk[2]) + 4.0 * bk[0]) / 6.0);
  double g[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double x = 1.0 + tau / (bk[k] + 1e-40);
    const double x2 = x * x;
    g[k] = (x2 * x2) * x2;
  }
  const double sum = ((g[0] + g[1]) + g[2]) + g[3];
  unsigned m = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double chi = g[k] / sum;
    if (!(chi < 1e-6)) m |= 1u << k;
  }
  return m;
}

template <typename T>
N6_DEV unsigned teno_mask_of(const T s[6]) {
  double sd[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) sd[j] = (double)s[j];
  return teno_mask(sd);
}

}  // namespace n6
