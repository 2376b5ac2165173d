// Plain NENO6 kernels: the classifier on the vector units with the canonical
// fma order, one lane per classifier evaluation.
//
// Instantiated for double -- the FP64 path, whose classification labels and
// values are bit-identical to the FP64 reference implementation because this
// file is compiled with -ffp-contract=off and every fma is written out -- and
// for float (the FP32 vector-unit path).
//
// Face fluxes of the Euler equations take two kernels: k_evals_* gives one
// lane to each (face, characteristic field, split sign) -- the field and sign
// are uniform across a block -- which reconstructs that one stencil; k_back_*
// adds the two signs of every field and back-projects with R.  The classifier
// weights are staged once per block in LDS, transposed so that the network
// runs input-stationary: the loop over a layer's inputs is outermost and all
// of the layer's accumulators advance together, which keeps ~100 FP64
// registers live while every accumulator still sees bias first and then its
// inputs in ascending order.
#include "neno6_device.h"
#include "neno6_internal.h"

namespace n6 {

namespace {

constexpr int TPB = 256;

template <typename T>
N6_DEV unsigned select_mask(int selector, const T *S, const T s[6], unsigned mask_in) {
  switch (selector) {
  case 0: return classify_lean<T>(S, s);
  case 1: return 15u;
  case 2: return 0u;
  case 4: return teno_mask_of<T>(s);
  default: return mask_in & 15u;
  }
}

template <typename T>
__global__ void __launch_bounds__(TPB)
k_reconstruct(const T *__restrict__ P, const T *__restrict__ f, int64_t n_faces, int sign,
              int selector, const uint8_t *__restrict__ min, T *__restrict__ fhat,
              uint8_t *__restrict__ mout) {
  __shared__ T S[S_SIZE];
  if (selector == 0) {
    stage_params<T>(P, S);
    __syncthreads();
  }
  const int64_t k = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (k >= n_faces) return;
  T s[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) s[j] = sign > 0 ? f[k + j] : f[k + 5 - j];
  const unsigned sel = select_mask<T>(selector, S, s, min ? min[k] : 0u);
  fhat[k] = combine_canonical<T>(s, sel);
  if (mout) mout[k] = (uint8_t)sel;
}

template <typename T>
__global__ void __launch_bounds__(TPB)
k_mlp_logits(const T *__restrict__ P, const T *__restrict__ sten, int64_t n, T *__restrict__ z,
             uint8_t *__restrict__ masks) {
  __shared__ T S[S_SIZE];
  stage_params<T>(P, S);
  __syncthreads();
  const int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (e >= n) return;
  T s[6], x[6], zz[4];
#pragma unroll
  for (int j = 0; j < 6; ++j) s[j] = sten[6 * e + j];
  features<T>(s, x);
  mlp_lean<T>(S, x, zz);
#pragma unroll
  for (int k = 0; k < 4; ++k) z[4 * e + k] = zz[k];
  if (masks) masks[e] = (uint8_t)mask_from_logits<T>(zz);
}

// Scalar advection, f = u, unit speed: the '+' split flux (f + u)/2 equals u
// exactly and the '-' split flux is identically zero, so the face flux is the
// '+' reconstruction of u.
template <typename T>
__global__ void __launch_bounds__(TPB)
k_faces_advection(Line1D ln, const T *__restrict__ P, int selector, const T *__restrict__ u,
                  const uint8_t *__restrict__ min, T *__restrict__ Fh, uint8_t *__restrict__ mout) {
  __shared__ T S[S_SIZE];
  if (selector == 0) {
    stage_params<T>(P, S);
    __syncthreads();
  }
  const int64_t g = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (g >= ln.faces()) return;
  const int p = line_of_face(ln, g);
  const int64_t o = ln.offsets[p], n = ln.offsets[p + 1] - o, k = g - o - p;
  T s[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) s[j] = u[o + ghost(k - 3 + j, n, ln.bc)];
  const unsigned sel = select_mask<T>(selector, S, s, min ? min[g] : 0u);
  Fh[g] = combine_canonical<T>(s, sel);
  if (mout) mout[g] = (uint8_t)sel;
}

// Burgers (Sec. 4.3): f = u^2/2, Rusanov speed alpha = max |u| over the six
// cells, f+- = (f +- alpha u)/2; '+' on cells i-2..i+3, '-' mirrored; the face
// flux is the sum of both reconstructions.
template <typename T>
__global__ void __launch_bounds__(TPB)
k_faces_burgers(Line1D ln, const T *__restrict__ P, int selector, const T *__restrict__ u,
                const uint8_t *__restrict__ min, T *__restrict__ Fh, uint8_t *__restrict__ mout) {
  __shared__ T S[S_SIZE];
  if (selector == 0) {
    stage_params<T>(P, S);
    __syncthreads();
  }
  const int64_t g = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (g >= ln.faces()) return;
  const int p = line_of_face(ln, g);
  const int64_t o = ln.offsets[p], n = ln.offsets[p + 1] - o, k = g - o - p;
  T us[6], alpha = T(0);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    us[j] = u[o + ghost(k - 3 + j, n, ln.bc)];
    const T a = abs_<T>(us[j]);
    alpha = a > alpha ? a : alpha;
  }
  T sp[6], sm[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T f = T(0.5) * (us[j] * us[j]);
    const T t = alpha * us[j];
    sp[j] = T(0.5) * (f + t);
    sm[5 - j] = T(0.5) * (f - t);
  }
  const unsigned mi = min ? min[g] : 0u;
  const unsigned selp = select_mask<T>(selector, S, sp, mi & 15u);
  const unsigned selm = select_mask<T>(selector, S, sm, (mi >> 4) & 15u);
  Fh[g] = combine_canonical<T>(sp, selp) + combine_canonical<T>(sm, selm);
  if (mout) mout[g] = (uint8_t)(selp | (selm << 4));
}

// Split stencil of characteristic field M and sign sgn ('-' mirrored) of a
// 1D Euler face from its six cells: Roe eigenvectors of cells i, i+1,
// projection of the six states and fluxes, Rusanov speed alpha_M =
// max_j |lambda_M(q_j)|, s = (g +- alpha v)/2.
template <typename T, int M>
N6_DEV void stencil1d(const T qs[6][3], T gamma, int sgn, T s[6]) {
  T L[3][3], R[3][3];
  roe1d<T>(qs[2], qs[3], gamma, L, R);
  T v[6], gg[6], alpha = T(0);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    T u, pr, c, F[3];
    prim1d<T>(qs[j], gamma, u, pr, c);
    flux1d<T>(qs[j], u, pr, F);
    const T lam = M == 0 ? u - c : (M == 1 ? u : u + c);
    const T a = abs_<T>(lam);
    alpha = a > alpha ? a : alpha;
    T av = T(0), ag = T(0);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      av = fma_<T>(L[M][r], qs[j][r], av);
      ag = fma_<T>(L[M][r], F[r], ag);
    }
    v[j] = av;
    gg[j] = ag;
  }
  T sp[6], sm[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T t = alpha * v[j];
    sp[j] = T(0.5) * (gg[j] + t);
    sm[5 - j] = T(0.5) * (gg[j] - t);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) s[j] = sgn ? sm[j] : sp[j];
}

// Same for field M of a 2D sweep in direction dir (fields: u_n - c, u_n,
// shear, u_n + c).
template <typename T, int M>
N6_DEV void stencil2d(const T qs[6][4], T gamma, int dir, int sgn, T s[6]) {
  T L[4][4], R[4][4];
  roe2d<T>(qs[2], qs[3], gamma, dir, L, R);
  T v[6], gg[6], alpha = T(0);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    T u, vv, pr, c, F[4];
    prim2d<T>(qs[j], gamma, u, vv, pr, c);
    flux2d<T>(qs[j], u, vv, pr, dir, F);
    const T un = dir == 0 ? u : vv;
    const T lam = M == 0 ? un - c : (M == 3 ? un + c : un);
    const T a = abs_<T>(lam);
    alpha = a > alpha ? a : alpha;
    T av = T(0), ag = T(0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      av = fma_<T>(L[M][r], qs[j][r], av);
      ag = fma_<T>(L[M][r], F[r], ag);
    }
    v[j] = av;
    gg[j] = ag;
  }
  T sp[6], sm[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T t = alpha * v[j];
    sp[j] = T(0.5) * (gg[j] + t);
    sm[5 - j] = T(0.5) * (gg[j] - t);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) s[j] = sgn ? sm[j] : sp[j];
}

// One evaluation of a 1D Euler face (Sec. 4.4): Roe eigenvectors of cells i,
// i+1; projection of the six states and fluxes on field m; Rusanov split with
// alpha_m = max_j |lambda_m(q_j)|; stencil of sign sgn (the '-' one mirrored);
// classifier; re-normalised combine.  Writes h and the kept mask.
template <typename T>
__global__ void __launch_bounds__(TPB)
k_evals_euler1d(Line1D ln, const T *__restrict__ P, int selector, const T *__restrict__ q,
                const uint8_t *__restrict__ min, int64_t tfpad, T *__restrict__ hbuf,
                uint8_t *__restrict__ sbuf) {
  __shared__ T S[S_SIZE];
  if (selector == 0) {
    stage_params<T>(P, S);
    __syncthreads();
  }
  const int64_t idx = blockIdx.x * (int64_t)TPB + threadIdx.x;
  const int e = (int)(idx / tfpad);
  const int64_t g = idx - e * tfpad;
  const int64_t tf = ln.faces();
  if (e >= 6 || g >= tf) return;
  const int m = e >> 1, sgn = e & 1;
  const int p = line_of_face(ln, g);
  const int64_t o = ln.offsets[p], n = ln.offsets[p + 1] - o, k = g - o - p;
  const T gamma = (T)ln.gamma;
  T qs[6][3];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int64_t ci = o + ghost(k - 3 + j, n, ln.bc);
#pragma unroll
    for (int r = 0; r < 3; ++r) qs[j][r] = q[r * ln.total + ci];
  }
  T s[6];
  switch (m) {  // block-uniform: each case sees its field index at compile time
  case 0: stencil1d<T, 0>(qs, gamma, sgn, s); break;
  case 1: stencil1d<T, 1>(qs, gamma, sgn, s); break;
  default: stencil1d<T, 2>(qs, gamma, sgn, s); break;
  }
  const unsigned in = min ? (min[m * tf + g] >> (4 * sgn)) & 15u : 0u;
  const unsigned sel = select_mask<T>(selector, S, s, in);
  hbuf[e * tf + g] = combine_canonical<T>(s, sel);
  sbuf[e * tf + g] = (uint8_t)sel;
}

// Sum of the two signs per field and back-projection R (h+ + h-).
template <typename T>
__global__ void __launch_bounds__(TPB)
k_back_euler1d(Line1D ln, const T *__restrict__ q, const T *__restrict__ hbuf,
               const uint8_t *__restrict__ sbuf, T *__restrict__ Fh, uint8_t *__restrict__ mout) {
  const int64_t tf = ln.faces();
  const int64_t g = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (g >= tf) return;
  const int p = line_of_face(ln, g);
  const int64_t o = ln.offsets[p], n = ln.offsets[p + 1] - o, k = g - o - p;
  T qL[3], qR[3];
  const int64_t cL = o + ghost(k - 1, n, ln.bc), cR = o + ghost(k, n, ln.bc);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    qL[r] = q[r * ln.total + cL];
    qR[r] = q[r * ln.total + cR];
  }
  T L[3][3], R[3][3];
  roe1d<T>(qL, qR, (T)ln.gamma, L, R);
  T hs[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    hs[m] = hbuf[(2 * m) * tf + g] + hbuf[(2 * m + 1) * tf + g];
    if (mout) mout[m * tf + g] = (uint8_t)(sbuf[(2 * m) * tf + g] | (sbuf[(2 * m + 1) * tf + g] << 4));
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < 3; ++m) acc = fma_<T>(R[r][m], hs[m], acc);
    Fh[r * tf + g] = acc;
  }
}

// 2D: faces of one sweep, dir 0: [ny][nx+1], dir 1: [ny+1][nx].
template <typename T>
N6_DEV void load_stencil2d(const Grid2D &gd, int dir, const T *__restrict__ q, int64_t f,
                           T qs[6][4]) {
  const int64_t cells = gd.nx * gd.ny;
  if (dir == 0) {
    const int64_t y = f / (gd.nx + 1), k = f % (gd.nx + 1);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int64_t ci = y * gd.nx + ghost(k - 3 + j, gd.nx, gd.bc);
#pragma unroll
      for (int r = 0; r < 4; ++r) qs[j][r] = q[r * cells + ci];
    }
  } else {
    const int64_t k = f / gd.nx, x = f % gd.nx;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int64_t ci = ghost(k - 3 + j, gd.ny, gd.bc) * gd.nx + x;
#pragma unroll
      for (int r = 0; r < 4; ++r) qs[j][r] = q[r * cells + ci];
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(TPB)
k_evals_euler2d(Grid2D gd, int dir, const T *__restrict__ P, int selector, const T *__restrict__ q,
                const uint8_t *__restrict__ min, int64_t nfpad, T *__restrict__ hbuf,
                uint8_t *__restrict__ sbuf) {
  __shared__ T S[S_SIZE];
  if (selector == 0) {
    stage_params<T>(P, S);
    __syncthreads();
  }
  const int64_t nf = dir == 0 ? (gd.nx + 1) * gd.ny : gd.nx * (gd.ny + 1);
  const int64_t idx = blockIdx.x * (int64_t)TPB + threadIdx.x;
  const int e = (int)(idx / nfpad);
  const int64_t f = idx - e * nfpad;
  if (e >= 8 || f >= nf) return;
  const int m = e >> 1, sgn = e & 1;
  const T gamma = (T)gd.gamma;
  T qs[6][4];
  load_stencil2d<T>(gd, dir, q, f, qs);
  T s[6];
  switch (m) {  // block-uniform: each case sees its field index at compile time
  case 0: stencil2d<T, 0>(qs, gamma, dir, sgn, s); break;
  case 1: stencil2d<T, 1>(qs, gamma, dir, sgn, s); break;
  case 2: stencil2d<T, 2>(qs, gamma, dir, sgn, s); break;
  default: stencil2d<T, 3>(qs, gamma, dir, sgn, s); break;
  }
  const unsigned in = min ? (min[m * nf + f] >> (4 * sgn)) & 15u : 0u;
  const unsigned sel = select_mask<T>(selector, S, s, in);
  hbuf[e * nf + f] = combine_canonical<T>(s, sel);
  sbuf[e * nf + f] = (uint8_t)sel;
}

template <typename T>
__global__ void __launch_bounds__(TPB)
k_back_euler2d(Grid2D gd, int dir, const T *__restrict__ q, const T *__restrict__ hbuf,
               const uint8_t *__restrict__ sbuf, T *__restrict__ Fh, uint8_t *__restrict__ mout) {
  const int64_t nf = dir == 0 ? (gd.nx + 1) * gd.ny : gd.nx * (gd.ny + 1);
  const int64_t f = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (f >= nf) return;
  const int64_t cells = gd.nx * gd.ny;
  int64_t cL, cR;
  if (dir == 0) {
    const int64_t y = f / (gd.nx + 1), k = f % (gd.nx + 1);
    cL = y * gd.nx + ghost(k - 1, gd.nx, gd.bc);
    cR = y * gd.nx + ghost(k, gd.nx, gd.bc);
  } else {
    const int64_t k = f / gd.nx, x = f % gd.nx;
    cL = ghost(k - 1, gd.ny, gd.bc) * gd.nx + x;
    cR = ghost(k, gd.ny, gd.bc) * gd.nx + x;
  }
  T qL[4], qR[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    qL[r] = q[r * cells + cL];
    qR[r] = q[r * cells + cR];
  }
  T L[4][4], R[4][4];
  roe2d<T>(qL, qR, (T)gd.gamma, dir, L, R);
  T hs[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    hs[m] = hbuf[(2 * m) * nf + f] + hbuf[(2 * m + 1) * nf + f];
    if (mout) mout[m * nf + f] = (uint8_t)(sbuf[(2 * m) * nf + f] | (sbuf[(2 * m + 1) * nf + f] << 4));
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < 4; ++m) acc = fma_<T>(R[r][m], hs[m], acc);
    Fh[r * nf + f] = acc;
  }
}

template <typename T>
__global__ void __launch_bounds__(TPB)
k_diff1d(Line1D ln, int equation, const T *__restrict__ Fh, const T *__restrict__ q,
         T *__restrict__ rhs, Stage st, int has_stage, int32_t *__restrict__ status_out,
         uint32_t *__restrict__ zero_after) {
  if (zero_after && blockIdx.x == 0 && threadIdx.x < QCOUNTERS) zero_after[threadIdx.x] = 0u;
  // one lane per face g; the face to the left of cell i of line p is i + p,
  // and the last face of every line has no cell to its right
  const int64_t tf = ln.faces();
  const int64_t g = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (g >= tf) return;
  const int p = line_of_face(ln, g);
  const int64_t i = g - p;
  if (i >= ln.offsets[p + 1]) return;
  const T dx = (T)ln.dx[p];
  const int nvar = equation == 2 ? 3 : 1;
  if (status_out && equation == 2) {
    const T qc[3] = {q[i], q[ln.total + i], q[2 * ln.total + i]};
    T u, pr, c;
    prim1d<T>(qc, (T)ln.gamma, u, pr, c);
    if (!physical<T>(qc[0], pr)) status_out[p] = ST_NONPHYSICAL;
  } else if (status_out && equation == 1 && !__builtin_isfinite(q[i])) {
    status_out[p] = ST_NONPHYSICAL;
  }
  for (int r = 0; r < nvar; ++r) {
    const T L = (Fh[r * tf + g] - Fh[r * tf + g + 1]) / dx;
    if (!has_stage) {
      rhs[r * ln.total + i] = L;
    } else {
      const T *us = (const T *)st.us;
      const T *u0 = (const T *)st.u0;
      T *out = (T *)st.out;
      const int64_t idx = r * ln.total + i;
      out[idx] = st.status[p] != 0 ? u0[idx] : rk3<T>(st.stage, us[idx], u0[idx], L, (T)st.dt[p]);
    }
  }
}

// Time step of each line at the start of an RK3 step: one 1024-thread block
// per line (enough loads in flight per line), wave-level max by shuffles.
constexpr int CFL_TPB = 1024;

template <typename T>
__global__ void __launch_bounds__(CFL_TPB)
k_cfl1d(Line1D ln, int equation, const T *__restrict__ q, double cfl, double *__restrict__ dt,
        int32_t *__restrict__ status, double *__restrict__ t, uint32_t *__restrict__ zero_after) {
  // the step's first stage starts with empty re-check queues
  if (zero_after && blockIdx.x == 0 && threadIdx.x < QCOUNTERS) zero_after[threadIdx.x] = 0u;
  const int p = blockIdx.x;
  const int64_t o = ln.offsets[p], n = ln.offsets[p + 1] - o;
  double smax = 0.0;
  int b = 0;
  if (equation == 2) {
    for (int64_t i = threadIdx.x; i < n; i += CFL_TPB) {
      const T qc[3] = {q[o + i], q[ln.total + o + i], q[2 * ln.total + o + i]};
      T u, pr, c;
      prim1d<T>(qc, (T)ln.gamma, u, pr, c);
      if (!physical<T>(qc[0], pr)) b = 1;
      const double sp = (double)(abs_<T>(u) + c);
      smax = sp > smax ? sp : smax;
    }
  } else if (equation == 1) {  // Burgers: wave speed |u|
    for (int64_t i = threadIdx.x; i < n; i += CFL_TPB) {
      const T v = q[o + i];
      if (!__builtin_isfinite(v)) b = 1;
      const double sp = (double)abs_<T>(v);
      smax = sp > smax ? sp : smax;
    }
  }
  // the maximum of the (non-NaN) speeds and the OR of the flags do not depend
  // on the reduction order
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const double o2 = __shfl_xor(smax, d);
    smax = o2 > smax ? o2 : smax;
    b |= __shfl_xor(b, d);
  }
  __shared__ double red[CFL_TPB / 64];
  __shared__ int bad[CFL_TPB / 64];
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = smax;
    bad[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < CFL_TPB / 64; ++w) {
      red[0] = red[w] > red[0] ? red[w] : red[0];
      bad[0] |= bad[w];
    }
  }
  if (threadIdx.x == 0) {
    if (status[p] != 0) {
      dt[p] = 0.0;
      return;
    }
    if (bad[0]) {
      status[p] = ST_NONPHYSICAL;
      dt[p] = 0.0;
      return;
    }
    // advection: unit speed; Burgers with u identically 0: the advection step
    const double d = (equation == 2 || (equation == 1 && red[0] > 0.0)) ? (cfl * ln.dx[p]) / red[0]
                                                                         : cfl * ln.dx[p];
    dt[p] = d;
    t[p] = t[p] + d;
  }
}

template <typename T>
__global__ void __launch_bounds__(TPB)
k_diff2d(Grid2D gd, const T *__restrict__ Fx, const T *__restrict__ Gy, const T *__restrict__ q,
         T *__restrict__ rhs, Stage st, int has_stage, int32_t *__restrict__ status_out,
         uint32_t *__restrict__ zero_after) {
  if (zero_after && blockIdx.x == 0 && threadIdx.x < QCOUNTERS) zero_after[threadIdx.x] = 0u;
  const int64_t cells = gd.nx * gd.ny;
  const int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (i >= cells) return;
  const int64_t y = i / gd.nx, x = i % gd.nx;
  const int64_t nfx = (gd.nx + 1) * gd.ny, nfy = gd.nx * (gd.ny + 1);
  const int64_t fx = y * (gd.nx + 1) + x, fy = y * gd.nx + x;
  if (status_out) {
    const T qc[4] = {q[i], q[cells + i], q[2 * cells + i], q[3 * cells + i]};
    T u, v, pr, c;
    prim2d<T>(qc, (T)gd.gamma, u, v, pr, c);
    if (!physical<T>(qc[0], pr)) status_out[0] = ST_NONPHYSICAL;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const T a = (Fx[r * nfx + fx] - Fx[r * nfx + fx + 1]) / (T)gd.dx;
    const T b = (Gy[r * nfy + fy] - Gy[r * nfy + fy + gd.nx]) / (T)gd.dy;
    const T L = a + b;
    const int64_t idx = r * cells + i;
    if (!has_stage) {
      rhs[idx] = L;
    } else {
      const T *us = (const T *)st.us;
      const T *u0 = (const T *)st.u0;
      T *out = (T *)st.out;
      out[idx] = st.status[0] != 0 ? u0[idx] : rk3<T>(st.stage, us[idx], u0[idx], L, (T)st.dt[0]);
    }
  }
}

constexpr int CFL2D_BLOCKS = 1024;

template <typename T>
__global__ void __launch_bounds__(TPB)
k_cfl2d_partial(Grid2D gd, const T *__restrict__ q, double *__restrict__ part) {
  const int64_t cells = gd.nx * gd.ny;
  __shared__ double rx[TPB], ry[TPB], rb[TPB];
  double sx = 0.0, sy = 0.0, bad = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < cells;
       i += (int64_t)gridDim.x * TPB) {
    const T qc[4] = {q[i], q[cells + i], q[2 * cells + i], q[3 * cells + i]};
    T u, v, pr, c;
    prim2d<T>(qc, (T)gd.gamma, u, v, pr, c);
    if (!physical<T>(qc[0], pr)) bad = 1.0;
    const double a = (double)(abs_<T>(u) + c), b = (double)(abs_<T>(v) + c);
    sx = a > sx ? a : sx;
    sy = b > sy ? b : sy;
  }
  rx[threadIdx.x] = sx;
  ry[threadIdx.x] = sy;
  rb[threadIdx.x] = bad;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rx[threadIdx.x] = rx[threadIdx.x + w] > rx[threadIdx.x] ? rx[threadIdx.x + w] : rx[threadIdx.x];
      ry[threadIdx.x] = ry[threadIdx.x + w] > ry[threadIdx.x] ? ry[threadIdx.x + w] : ry[threadIdx.x];
      rb[threadIdx.x] = rb[threadIdx.x + w] > rb[threadIdx.x] ? rb[threadIdx.x + w] : rb[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = rx[0];
    part[3 * blockIdx.x + 1] = ry[0];
    part[3 * blockIdx.x + 2] = rb[0];
  }
}

__global__ void __launch_bounds__(TPB)
k_cfl2d_final(Grid2D gd, int nparts, const double *__restrict__ part, double cfl,
              double *__restrict__ dt, int32_t *__restrict__ status, double *__restrict__ t) {
  __shared__ double rx[TPB], ry[TPB], rb[TPB];
  double sx = 0.0, sy = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < nparts; i += TPB) {
    sx = part[3 * i] > sx ? part[3 * i] : sx;
    sy = part[3 * i + 1] > sy ? part[3 * i + 1] : sy;
    bad = part[3 * i + 2] > bad ? part[3 * i + 2] : bad;
  }
  rx[threadIdx.x] = sx;
  ry[threadIdx.x] = sy;
  rb[threadIdx.x] = bad;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rx[threadIdx.x] = rx[threadIdx.x + w] > rx[threadIdx.x] ? rx[threadIdx.x + w] : rx[threadIdx.x];
      ry[threadIdx.x] = ry[threadIdx.x + w] > ry[threadIdx.x] ? ry[threadIdx.x + w] : ry[threadIdx.x];
      rb[threadIdx.x] = rb[threadIdx.x + w] > rb[threadIdx.x] ? rb[threadIdx.x + w] : rb[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (status[0] != 0) {
      dt[0] = 0.0;
      return;
    }
    if (rb[0] != 0.0) {
      status[0] = ST_NONPHYSICAL;
      dt[0] = 0.0;
      return;
    }
    const double d = cfl / (rx[0] / gd.dx + ry[0] / gd.dy);
    dt[0] = d;
    t[0] = t[0] + d;
  }
}

__global__ void __launch_bounds__(TPB) k_params_to_f32(const double *__restrict__ P, float *__restrict__ P32) {
  const int i = blockIdx.x * TPB + threadIdx.x;
  if (i < NPARAM) P32[i] = (float)P[i];
}

// Fixed-mask adjoint of the advection rhs on one line (gather form).
// Forward: h_k = sum_j a_{k,j} u_{c(k,j)}, c(k,j) = ghost(k-3+j); rhs_i =
// (h_i - h_{i+1})/dx.  Adjoint: hbar_k = (rbar_k [k<n] - rbar_{k-1} [k>0])/dx,
// ubar_c = sum over faces k and stencil slots j with c(k,j) = c of a_{k,j} hbar_k.
template <typename T>
N6_DEV void face_coeffs(unsigned sel, T a[6]) {
  T e[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
#pragma unroll
    for (int i = 0; i < 6; ++i) e[i] = i == j ? T(1) : T(0);
    a[j] = combine_canonical<T>(e, sel);
  }
}

template <typename T>
N6_DEV void adj_face(int64_t k, int j, int64_t n, T dx, const uint8_t *__restrict__ masks,
                     const T *__restrict__ rbar, T &acc) {
  T a[6];
  face_coeffs<T>(masks[k] & 15u, a);
  const T hb = ((k < n ? rbar[k] : T(0)) - (k > 0 ? rbar[k - 1] : T(0))) / dx;
  acc = fma_<T>(a[j], hb, acc);
}

template <typename T>
__global__ void __launch_bounds__(TPB)
k_adjoint_advection(int64_t n, const double *__restrict__ dxp, int bc,
                    const uint8_t *__restrict__ masks, const T *__restrict__ rbar,
                    T *__restrict__ ubar) {
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= n) return;
  const T dx = (T)dxp[0];
  T acc = T(0);
  if (bc == 0) {
    // face k reads cell (k - 3 + j) mod n; faces 0 and n read the same cells
    for (int j = 0; j < 6; ++j) {
      const int64_t k0 = ((c + 3 - j) % n + n) % n;
      adj_face<T>(k0, j, n, dx, masks, rbar, acc);
      if (k0 == 0) adj_face<T>(n, j, n, dx, masks, rbar, acc);
    }
  } else {
    const int64_t k_lo = c - 3 < 0 ? 0 : c - 3, k_hi = c + 3 > n ? n : c + 3;
    for (int64_t k = k_lo; k <= k_hi; ++k)
      for (int j = 0; j < 6; ++j)
        if (ghost(k - 3 + j, n, bc) == c) adj_face<T>(k, j, n, dx, masks, rbar, acc);
  }
  ubar[c] = acc;
}

// ---- vector-Jacobian products of the right-hand side at fixed labels --------
// With the labels of every evaluation held fixed, the face flux is a smooth
// function of the six stencil states (away from ties in the Rusanov speed
// max), and rhs_i = (F_i - F_{i+1}) / dx.  The adjoint runs per face in
// reverse through back-projection, the fixed-weight combine, the split
// g +- alpha v, the projections, the Rusanov speed (into the cell that
// attains the max) and the Roe average; per-face contributions to the six
// stencil cells are then gathered per cell in a fixed order.

// Reverse of the 1D Euler face flux: Fb = dL/dFhat, qb[j][r] += dL/dq_j.
template <typename T>
N6_DEV void face_vjp_euler1d(const T qs[6][3], T gamma, const uint8_t msk[3], const T Fb[3],
                             T qb[6][3]) {
  const T g1 = gamma - T(1);
  T u[6], p[6], c[6], F[6][3];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    prim1d<T>(qs[j], gamma, u[j], p[j], c[j]);
    flux1d<T>(qs[j], u[j], p[j], F[j]);
  }
  // Roe average of cells 2, 3 and the eigenvectors (as in roe1d)
  const T sL = sqrt_<T>(qs[2][0]), sR = sqrt_<T>(qs[3][0]);
  const T HL = (qs[2][2] + p[2]) / qs[2][0], HR = (qs[3][2] + p[3]) / qs[3][0];
  const T den = sL + sR;
  const T ut = (sL * u[2] + sR * u[3]) / den;
  const T Ht = (sL * HL + sR * HR) / den;
  const T q2 = T(0.5) * (ut * ut);
  const T c2 = g1 * (Ht - q2);
  const T ct = sqrt_<T>(c2);
  const T b1 = g1 / c2, b2 = b1 * q2, uc = ut / ct, ic = T(1) / ct;
  const T L[3][3] = {{T(0.5) * (b2 + uc), T(-0.5) * (b1 * ut + ic), T(0.5) * b1},
                     {T(1) - b2, b1 * ut, -b1},
                     {T(0.5) * (b2 - uc), T(-0.5) * (b1 * ut - ic), T(0.5) * b1}};
  const T R[3][3] = {{T(1), T(1), T(1)}, {ut - ct, ut, ut + ct}, {Ht - ut * ct, q2, Ht + ut * ct}};
  // forward values needed by the reverse sweep
  T v[6][3], alpha[3], hs[3];
  int am[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    alpha[m] = T(0);
    am[m] = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const T lam = m == 0 ? u[j] - c[j] : (m == 1 ? u[j] : u[j] + c[j]);
      const T a = abs_<T>(lam);
      if (a > alpha[m]) {
        alpha[m] = a;
        am[m] = j;
      }
    }
  }
  T sp[3][6], sm[3][6];
#pragma unroll
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      v[j][m] = L[m][0] * qs[j][0] + L[m][1] * qs[j][1] + L[m][2] * qs[j][2];
      const T g = L[m][0] * F[j][0] + L[m][1] * F[j][1] + L[m][2] * F[j][2];
      sp[m][j] = T(0.5) * (g + alpha[m] * v[j][m]);
      sm[m][5 - j] = T(0.5) * (g - alpha[m] * v[j][m]);
    }
  T Wp[3][6], Wm[3][6];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    face_coeffs<T>(msk[m] & 15u, Wp[m]);
    face_coeffs<T>((msk[m] >> 4) & 15u, Wm[m]);
    T h = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) h = h + Wp[m][j] * sp[m][j] + Wm[m][j] * sm[m][j];
    hs[m] = h;
  }
  // ---- reverse ----
  T hsb[3], Rb[3][3], Lb[3][3] = {}, ub[6] = {}, pb[6] = {}, cb[6] = {}, Fcb[6][3] = {};
#pragma unroll
  for (int m = 0; m < 3; ++m) hsb[m] = R[0][m] * Fb[0] + R[1][m] * Fb[1] + R[2][m] * Fb[2];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int m = 0; m < 3; ++m) Rb[r][m] = Fb[r] * hs[m];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    T ab = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const T spb = Wp[m][j] * hsb[m], smb = Wm[m][5 - j] * hsb[m];
      const T gb = T(0.5) * (spb + smb);
      const T vb = T(0.5) * alpha[m] * (spb - smb);
      ab = ab + T(0.5) * v[j][m] * (spb - smb);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Lb[m][r] = Lb[m][r] + vb * qs[j][r] + gb * F[j][r];
        qb[j][r] = qb[j][r] + L[m][r] * vb;
        Fcb[j][r] = Fcb[j][r] + L[m][r] * gb;
      }
    }
    // Rusanov speed: |lambda_m| of the cell that attains the max
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j == am[m]) {
        const T lam = m == 0 ? u[j] - c[j] : (m == 1 ? u[j] : u[j] + c[j]);
        const T sb = lam < T(0) ? -ab : ab;
        ub[j] = ub[j] + sb;
        if (m == 0) cb[j] = cb[j] - sb;
        if (m == 2) cb[j] = cb[j] + sb;
      }
  }
  // Roe quantities
  const T b2b = T(0.5) * Lb[0][0] - Lb[1][0] + T(0.5) * Lb[2][0];
  const T ucb = T(0.5) * Lb[0][0] - T(0.5) * Lb[2][0];
  T b1b = T(-0.5) * ut * Lb[0][1] + T(0.5) * Lb[0][2] + ut * Lb[1][1] - Lb[1][2] -
          T(0.5) * ut * Lb[2][1] + T(0.5) * Lb[2][2];
  T utb = T(-0.5) * b1 * Lb[0][1] + b1 * Lb[1][1] - T(0.5) * b1 * Lb[2][1];
  const T icb = T(-0.5) * Lb[0][1] + T(0.5) * Lb[2][1];
  utb = utb + Rb[1][0] + Rb[1][1] + Rb[1][2] - ct * Rb[2][0] + ct * Rb[2][2];
  T ctb = -Rb[1][0] + Rb[1][2] - ut * Rb[2][0] + ut * Rb[2][2];
  T Htb = Rb[2][0] + Rb[2][2];
  T q2b = Rb[2][1];
  b1b = b1b + q2 * b2b;
  q2b = q2b + b1 * b2b;
  utb = utb + ucb / ct;
  ctb = ctb - ucb * ut / (ct * ct) - icb / (ct * ct);
  T c2b = -b1b * g1 / (c2 * c2) + ctb / (T(2) * ct);
  Htb = Htb + g1 * c2b;
  q2b = q2b - g1 * c2b;
  utb = utb + ut * q2b;
  const T sLb = (u[2] - ut) / den * utb + (HL - Ht) / den * Htb;
  const T sRb = (u[3] - ut) / den * utb + (HR - Ht) / den * Htb;
  ub[2] = ub[2] + sL / den * utb;
  ub[3] = ub[3] + sR / den * utb;
  const T HLb = sL / den * Htb, HRb = sR / den * Htb;
  qb[2][2] = qb[2][2] + HLb / qs[2][0];
  pb[2] = pb[2] + HLb / qs[2][0];
  qb[2][0] = qb[2][0] - HLb * HL / qs[2][0] + sLb / (T(2) * sL);
  qb[3][2] = qb[3][2] + HRb / qs[3][0];
  pb[3] = pb[3] + HRb / qs[3][0];
  qb[3][0] = qb[3][0] - HRb * HR / qs[3][0] + sRb / (T(2) * sR);
  // cell fluxes and primitives
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T m_ = qs[j][1], E = qs[j][2], rho = qs[j][0];
    qb[j][1] = qb[j][1] + Fcb[j][0] + u[j] * Fcb[j][1];
    ub[j] = ub[j] + m_ * Fcb[j][1] + (E + p[j]) * Fcb[j][2];
    pb[j] = pb[j] + Fcb[j][1] + u[j] * Fcb[j][2];
    qb[j][2] = qb[j][2] + u[j] * Fcb[j][2];
    // c = sqrt(gamma p / rho)
    const T wb = cb[j] / (T(2) * c[j]);
    pb[j] = pb[j] + gamma / rho * wb;
    qb[j][0] = qb[j][0] - gamma * p[j] / (rho * rho) * wb;
    // p = g1 (E - m u / 2)
    qb[j][2] = qb[j][2] + g1 * pb[j];
    qb[j][1] = qb[j][1] - T(0.5) * g1 * u[j] * pb[j];
    ub[j] = ub[j] - T(0.5) * g1 * m_ * pb[j];
    // u = m / rho
    qb[j][1] = qb[j][1] + ub[j] / rho;
    qb[j][0] = qb[j][0] - ub[j] * u[j] / rho;
  }
}

// Reverse of the Burgers face flux (f = u^2/2, alpha = max |u| over the cells).
template <typename T>
N6_DEV void face_vjp_burgers(const T us[6], uint8_t msk, T Fb, T qb[6][3]) {
  T alpha = T(0);
  int am = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T a = abs_<T>(us[j]);
    if (a > alpha) {
      alpha = a;
      am = j;
    }
  }
  T Wp[6], Wm[6];
  face_coeffs<T>(msk & 15u, Wp);
  face_coeffs<T>((msk >> 4) & 15u, Wm);
  T ab = T(0);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T spb = Wp[j] * Fb, smb = Wm[5 - j] * Fb;
    // s+_j = (f + alpha u)/2, s-_{5-j} = (f - alpha u)/2, f' = u
    qb[j][0] = qb[j][0] + T(0.5) * (us[j] * (spb + smb) + alpha * (spb - smb));
    ab = ab + T(0.5) * us[j] * (spb - smb);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j)
    if (j == am) qb[j][0] = qb[j][0] + (us[j] < T(0) ? -ab : ab);
}

// Per face: contributions cb[(j * nv + r) * tf + g] to the six stencil cells.
// Reverse of one 2D Euler face flux in sweep direction dir (the forward is
// stencil2d for every field and sign, then the back-projection with R):
// fixed combination weights from the labels; Roe average of cells 2, 3 and
// its eigenvectors in the (rho, m_n, m_s, E) frame; Rusanov speeds
// alpha_m = max_j |lambda_m| (lambda = u_n - c, u_n, u_n, u_n + c) into the
// cell that attains the max.  Fb: cotangent of the face flux; qb[6][4] is
// accumulated.
template <typename T>
N6_DEV void face_vjp_euler2d(const T qs[6][4], T gamma, int dir, const uint8_t msk[4],
                             const T Fb[4], T qb[6][4]) {
  const T g1 = gamma - T(1);
  const int vn = dir == 0 ? 1 : 2, vs = dir == 0 ? 2 : 1;
  T u[6], w[6], p[6], c[6], F[6][4];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    prim2d<T>(qs[j], gamma, u[j], w[j], p[j], c[j]);
    flux2d<T>(qs[j], u[j], w[j], p[j], dir, F[j]);
  }
  // Roe average of cells 2, 3 (as in roe2d)
  const T sL = sqrt_<T>(qs[2][0]), sR = sqrt_<T>(qs[3][0]);
  const T HL = (qs[2][3] + p[2]) / qs[2][0], HR = (qs[3][3] + p[3]) / qs[3][0];
  const T den = sL + sR;
  const T ut = (sL * u[2] + sR * u[3]) / den;
  const T vt = (sL * w[2] + sR * w[3]) / den;
  const T Ht = (sL * HL + sR * HR) / den;
  const T q2 = T(0.5) * (ut * ut + vt * vt);
  const T c2 = g1 * (Ht - q2);
  const T ct = sqrt_<T>(c2);
  const T b1 = g1 / c2, b2 = b1 * q2, ic = T(1) / ct;
  const T un = dir == 0 ? ut : vt, us = dir == 0 ? vt : ut, nc = un / ct;
  T L[4][4], R[4][4];
  roe2d<T>(qs[2], qs[3], gamma, dir, L, R);
  // forward values needed by the reverse sweep
  T v[6][4], alpha[4], hs[4];
  int am[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    alpha[m] = T(0);
    am[m] = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const T unj = dir == 0 ? u[j] : w[j];
      const T lam = m == 0 ? unj - c[j] : (m == 3 ? unj + c[j] : unj);
      const T a = abs_<T>(lam);
      if (a > alpha[m]) {
        alpha[m] = a;
        am[m] = j;
      }
    }
  }
  T Wp[4][6], Wm[4][6];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    face_coeffs<T>(msk[m] & 15u, Wp[m]);
    face_coeffs<T>((msk[m] >> 4) & 15u, Wm[m]);
    T h = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      T av = T(0), ag = T(0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        av = av + L[m][r] * qs[j][r];
        ag = ag + L[m][r] * F[j][r];
      }
      v[j][m] = av;
      h = h + Wp[m][j] * (T(0.5) * (ag + alpha[m] * av)) + Wm[m][5 - j] * (T(0.5) * (ag - alpha[m] * av));
    }
    hs[m] = h;
  }
  // ---- reverse ----
  T hsb[4], Lb[4][4] = {}, Rb[4][4], ub[6] = {}, wb[6] = {}, pb[6] = {}, cb[6] = {};
  T Fcb[6][4] = {};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    hsb[m] = T(0);
#pragma unroll
    for (int r = 0; r < 4; ++r) hsb[m] = hsb[m] + R[r][m] * Fb[r];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int m = 0; m < 4; ++m) Rb[r][m] = Fb[r] * hs[m];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    T ab = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const T spb = Wp[m][j] * hsb[m], smb = Wm[m][5 - j] * hsb[m];
      const T gb = T(0.5) * (spb + smb);
      const T vb = T(0.5) * alpha[m] * (spb - smb);
      ab = ab + T(0.5) * v[j][m] * (spb - smb);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Lb[m][r] = Lb[m][r] + vb * qs[j][r] + gb * F[j][r];
        qb[j][r] = qb[j][r] + L[m][r] * vb;
        Fcb[j][r] = Fcb[j][r] + L[m][r] * gb;
      }
    }
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j == am[m]) {
        const T unj = dir == 0 ? u[j] : w[j];
        const T lam = m == 0 ? unj - c[j] : (m == 3 ? unj + c[j] : unj);
        const T sb = lam < T(0) ? -ab : ab;
        if (dir == 0) ub[j] = ub[j] + sb;
        else wb[j] = wb[j] + sb;
        if (m == 0) cb[j] = cb[j] - sb;
        if (m == 3) cb[j] = cb[j] + sb;
      }
  }
  // to the (rho, m_n, m_s, E) frame
  T Lnb[4][4], Rnb[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    Lnb[m][0] = Lb[m][0];
    Lnb[m][1] = Lb[m][vn];
    Lnb[m][2] = Lb[m][vs];
    Lnb[m][3] = Lb[m][3];
    Rnb[0][m] = Rb[0][m];
    Rnb[1][m] = Rb[vn][m];
    Rnb[2][m] = Rb[vs][m];
    Rnb[3][m] = Rb[3][m];
  }
  const T b2b = T(0.5) * Lnb[0][0] - Lnb[1][0] + T(0.5) * Lnb[3][0];
  const T ncb = T(0.5) * Lnb[0][0] - T(0.5) * Lnb[3][0];
  T b1b = T(-0.5) * un * Lnb[0][1] - T(0.5) * us * Lnb[0][2] + T(0.5) * Lnb[0][3] +
          un * Lnb[1][1] + us * Lnb[1][2] - Lnb[1][3] - T(0.5) * un * Lnb[3][1] -
          T(0.5) * us * Lnb[3][2] + T(0.5) * Lnb[3][3];
  T unb = T(-0.5) * b1 * Lnb[0][1] + b1 * Lnb[1][1] - T(0.5) * b1 * Lnb[3][1];
  T usb = T(-0.5) * b1 * Lnb[0][2] + b1 * Lnb[1][2] - Lnb[2][0] - T(0.5) * b1 * Lnb[3][2];
  const T icb = T(-0.5) * Lnb[0][1] + T(0.5) * Lnb[3][1];
  unb = unb + Rnb[1][0] + Rnb[1][1] + Rnb[1][3] - ct * Rnb[3][0] + ct * Rnb[3][3];
  T ctb = -Rnb[1][0] + Rnb[1][3] - un * Rnb[3][0] + un * Rnb[3][3];
  usb = usb + Rnb[2][0] + Rnb[2][1] + Rnb[2][3] + Rnb[3][2];
  T Htb = Rnb[3][0] + Rnb[3][3];
  T q2b = Rnb[3][1];
  b1b = b1b + q2 * b2b;
  q2b = q2b + b1 * b2b;
  unb = unb + ncb / ct;
  ctb = ctb - ncb * un / (ct * ct) - icb / (ct * ct);
  const T c2b = -b1b * g1 / (c2 * c2) + ctb / (T(2) * ct);
  Htb = Htb + g1 * c2b;
  q2b = q2b - g1 * c2b;
  T utb = ut * q2b, vtb = vt * q2b;
  if (dir == 0) {
    utb = utb + unb;
    vtb = vtb + usb;
  } else {
    vtb = vtb + unb;
    utb = utb + usb;
  }
  const T sLb = (u[2] - ut) / den * utb + (w[2] - vt) / den * vtb + (HL - Ht) / den * Htb;
  const T sRb = (u[3] - ut) / den * utb + (w[3] - vt) / den * vtb + (HR - Ht) / den * Htb;
  ub[2] = ub[2] + sL / den * utb;
  ub[3] = ub[3] + sR / den * utb;
  wb[2] = wb[2] + sL / den * vtb;
  wb[3] = wb[3] + sR / den * vtb;
  const T HLb = sL / den * Htb, HRb = sR / den * Htb;
  qb[2][3] = qb[2][3] + HLb / qs[2][0];
  pb[2] = pb[2] + HLb / qs[2][0];
  qb[2][0] = qb[2][0] - HLb * HL / qs[2][0] + sLb / (T(2) * sL);
  qb[3][3] = qb[3][3] + HRb / qs[3][0];
  pb[3] = pb[3] + HRb / qs[3][0];
  qb[3][0] = qb[3][0] - HRb * HR / qs[3][0] + sRb / (T(2) * sR);
  // cell fluxes and primitives
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T rho = qs[j][0], mu = qs[j][1], mv = qs[j][2], E = qs[j][3];
    if (dir == 0) {  // F = (m_u, m_u u + p, m_v u, (E + p) u)
      qb[j][1] = qb[j][1] + Fcb[j][0] + u[j] * Fcb[j][1];
      qb[j][2] = qb[j][2] + u[j] * Fcb[j][2];
      qb[j][3] = qb[j][3] + u[j] * Fcb[j][3];
      ub[j] = ub[j] + mu * Fcb[j][1] + mv * Fcb[j][2] + (E + p[j]) * Fcb[j][3];
      pb[j] = pb[j] + Fcb[j][1] + u[j] * Fcb[j][3];
    } else {  // G = (m_v, m_u v, m_v v + p, (E + p) v)
      qb[j][2] = qb[j][2] + Fcb[j][0] + w[j] * Fcb[j][2];
      qb[j][1] = qb[j][1] + w[j] * Fcb[j][1];
      qb[j][3] = qb[j][3] + w[j] * Fcb[j][3];
      wb[j] = wb[j] + mu * Fcb[j][1] + mv * Fcb[j][2] + (E + p[j]) * Fcb[j][3];
      pb[j] = pb[j] + Fcb[j][2] + w[j] * Fcb[j][3];
    }
    // c = sqrt(gamma p / rho)
    const T zb = cb[j] / (T(2) * c[j]);
    pb[j] = pb[j] + gamma / rho * zb;
    qb[j][0] = qb[j][0] - gamma * p[j] / (rho * rho) * zb;
    // p = g1 (E - (m_u u + m_v v) / 2)
    qb[j][3] = qb[j][3] + g1 * pb[j];
    const T keb = -g1 * pb[j];
    qb[j][1] = qb[j][1] + T(0.5) * u[j] * keb;
    ub[j] = ub[j] + T(0.5) * mu * keb;
    qb[j][2] = qb[j][2] + T(0.5) * w[j] * keb;
    wb[j] = wb[j] + T(0.5) * mv * keb;
    // u = m_u / rho, v = m_v / rho
    qb[j][1] = qb[j][1] + ub[j] / rho;
    qb[j][2] = qb[j][2] + wb[j] / rho;
    qb[j][0] = qb[j][0] - (ub[j] * u[j] + wb[j] * w[j]) / rho;
  }
}

// 2D: per face of sweep dir, the 24 contributions (cell j of the stencil,
// variable r) at cb[(j * 4 + r) * nf + f].
template <typename T>
__global__ void __launch_bounds__(TPB)
k_vjp_faces2d(Grid2D gd, int dir, const T *__restrict__ q, const uint8_t *__restrict__ masks,
              const T *__restrict__ rbar, T *__restrict__ cb) {
  const int64_t nf = dir == 0 ? (gd.nx + 1) * gd.ny : gd.nx * (gd.ny + 1);
  const int64_t f = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (f >= nf) return;
  const int64_t cells = gd.nx * gd.ny;
  // cotangent of the face flux: d rhs(right cell) / dF = 1/h, d rhs(left) / dF = -1/h
  int64_t cl = -1, cr = -1;
  T h;
  if (dir == 0) {
    const int64_t y = f / (gd.nx + 1), k = f % (gd.nx + 1);
    if (k > 0) cl = y * gd.nx + k - 1;
    if (k < gd.nx) cr = y * gd.nx + k;
    h = (T)gd.dx;
  } else {
    const int64_t k = f / gd.nx, x = f % gd.nx;
    if (k > 0) cl = (k - 1) * gd.nx + x;
    if (k < gd.ny) cr = k * gd.nx + x;
    h = (T)gd.dy;
  }
  T Fb[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const T right = cr >= 0 ? rbar[r * cells + cr] : T(0);
    const T left = cl >= 0 ? rbar[r * cells + cl] : T(0);
    Fb[r] = (right - left) / h;
  }
  T qs[6][4];
  load_stencil2d<T>(gd, dir, q, f, qs);
  uint8_t msk[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) msk[m] = masks[m * nf + f];
  T qb[6][4] = {};
  face_vjp_euler2d<T>(qs, (T)gd.gamma, dir, msk, Fb, qb);
#pragma unroll
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) cb[(int64_t)(j * 4 + r) * nf + f] = qb[j][r];
}

// Per cell: the x-sweep then the y-sweep contributions, each in a fixed order
// (direct stencil positions by ascending face, then ghost positions).
template <typename T>
__global__ void __launch_bounds__(TPB)
k_vjp_gather2d(Grid2D gd, const T *__restrict__ cbx, const T *__restrict__ cby, T *__restrict__ qbar) {
  const int64_t cells = gd.nx * gd.ny;
  const int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (i >= cells) return;
  const int64_t y = i / gd.nx, x = i % gd.nx;
  const int64_t nfx = (gd.nx + 1) * gd.ny, nfy = gd.nx * (gd.ny + 1);
  for (int r = 0; r < 4; ++r) {
    T acc = T(0);
    for (int d = 0; d < 2; ++d) {
      const T *cb = d == 0 ? cbx : cby;
      const int64_t n = d == 0 ? gd.nx : gd.ny, c = d == 0 ? x : y;
      const int64_t nf = d == 0 ? nfx : nfy;
      // face k of this row (x) / column (y)
      auto face = [&](int64_t k) { return d == 0 ? y * (gd.nx + 1) + k : k * gd.nx + x; };
      for (int64_t k = c - 2; k <= c + 3; ++k) {
        if (k < 0 || k > n) continue;
        const int j = (int)(c - k + 3);
        acc = acc + cb[(int64_t)(j * 4 + r) * nf + face(k)];
      }
      if (c < 3 || c > n - 4) {
        for (int64_t k = 0; k <= n; ++k) {
          if (k > 5 && k < n - 5) continue;
          for (int j = 0; j < 6; ++j) {
            const int64_t cc = k - 3 + j;
            if (cc >= 0 && cc < n) continue;
            if (ghost(cc, n, gd.bc) == c) acc = acc + cb[(int64_t)(j * 4 + r) * nf + face(k)];
          }
        }
      }
    }
    qbar[r * cells + i] = acc;
  }
}

template <typename T>
__global__ void __launch_bounds__(TPB)
k_vjp_faces1d(Line1D ln, int equation, const T *__restrict__ q, const uint8_t *__restrict__ masks,
              const T *__restrict__ rbar, T *__restrict__ cb) {
  const int64_t tf = ln.faces();
  const int64_t g = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (g >= tf) return;
  const int p = line_of_face(ln, g);
  const int64_t o = ln.offsets[p], n = ln.offsets[p + 1] - o, k = g - o - p;
  const T dx = (T)ln.dx[p];
  const int nv = equation == 2 ? 3 : 1;
  T qb[6][3] = {};
  T Fb[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    if (r >= nv) break;
    const T right = k < n ? rbar[r * ln.total + o + k] : T(0);
    const T left = k > 0 ? rbar[r * ln.total + o + k - 1] : T(0);
    Fb[r] = (right - left) / dx;
  }
  if (equation == 2) {
    T qs[6][3];
    uint8_t msk[3];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int64_t ci = o + ghost(k - 3 + j, n, ln.bc);
#pragma unroll
      for (int r = 0; r < 3; ++r) qs[j][r] = q[r * ln.total + ci];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) msk[m] = masks[m * tf + g];
    face_vjp_euler1d<T>(qs, (T)ln.gamma, msk, Fb, qb);
  } else {
    T us[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) us[j] = q[o + ghost(k - 3 + j, n, ln.bc)];
    face_vjp_burgers<T>(us, masks[g], Fb[0], qb);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j)
    for (int r = 0; r < nv; ++r) cb[(int64_t)(j * nv + r) * tf + g] = qb[j][r];
}

// Per cell: sum of the face contributions that read it, in a fixed order
// (direct stencil positions by ascending face, then ghost positions).
template <typename T>
__global__ void __launch_bounds__(TPB)
k_vjp_gather1d(Line1D ln, int nv, const T *__restrict__ cb, T *__restrict__ qbar) {
  const int64_t tf = ln.faces();
  const int64_t gidx = blockIdx.x * (int64_t)TPB + threadIdx.x;  // face index = left face of the cell
  if (gidx >= tf) return;
  const int p = line_of_face(ln, gidx);
  const int64_t o = ln.offsets[p], n = ln.offsets[p + 1] - o, c = gidx - o - p;
  if (c >= n) return;
  const int64_t f0 = o + p;  // global index of face 0 of the line
  for (int r = 0; r < nv; ++r) {
    T acc = T(0);
    // direct: face k reads cell k - 3 + j
    for (int64_t k = c - 2; k <= c + 3; ++k) {
      if (k < 0 || k > n) continue;
      const int j = (int)(c - k + 3);
      acc = acc + cb[(int64_t)(j * nv + r) * tf + f0 + k];
    }
    // ghost positions that map onto cell c
    if (c < 3 || c > n - 4) {
      for (int64_t k = 0; k <= n; ++k) {
        if (k > 5 && k < n - 5) continue;
        for (int j = 0; j < 6; ++j) {
          const int64_t cc = k - 3 + j;
          if (cc >= 0 && cc < n) continue;
          if (ghost(cc, n, ln.bc) == c) acc = acc + cb[(int64_t)(j * nv + r) * tf + f0 + k];
        }
      }
    }
    qbar[r * ln.total + o + c] = acc;
  }
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }
inline int64_t pad_to_block(int64_t n) { return (n + TPB - 1) / TPB * TPB; }

// Face-flux scratch of the plain Euler path: h per evaluation, mask per
// evaluation (NE x faces each).
struct EvalBufs {
  void *h;
  uint8_t *sel;
};

}  // namespace

size_t plain_eval_bytes(int nevals, int64_t faces, size_t elem) {
  const size_t h = ((size_t)nevals * faces * elem + 255) & ~(size_t)255;
  return h + (((size_t)nevals * faces + 255) & ~(size_t)255);
}

// ---- launchers --------------------------------------------------------------
template <typename T>
hipError_t launch_reconstruct(const T *P, const T *f, int64_t n_faces, int sign, int selector,
                              const uint8_t *masks_in, T *fhat, uint8_t *masks_out,
                              hipStream_t s) {
  if (n_faces == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reconstruct<T>, dim3(nblocks(n_faces)), dim3(TPB), 0, s, P, f, n_faces,
                     sign, selector, masks_in, fhat, masks_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mlp_logits(const T *P, const T *sten, int64_t n, T *z, uint8_t *masks,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_logits<T>, dim3(nblocks(n)), dim3(TPB), 0, s, P, sten, n, z, masks);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_faces_advection(const Line1D &ln, const T *P, int selector, const T *u,
                                  const uint8_t *masks_in, T *Fhat, uint8_t *masks_out,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_faces_advection<T>, dim3(nblocks(ln.faces())), dim3(TPB), 0, s, ln, P,
                     selector, u, masks_in, Fhat, masks_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_faces_burgers(const Line1D &ln, const T *P, int selector, const T *u,
                                const uint8_t *masks_in, T *Fhat, uint8_t *masks_out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_faces_burgers<T>, dim3(nblocks(ln.faces())), dim3(TPB), 0, s, ln, P,
                     selector, u, masks_in, Fhat, masks_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_faces_euler1d(const Line1D &ln, const T *P, int selector, const T *q,
                                const uint8_t *masks_in, T *Fhat, uint8_t *masks_out,
                                void *evals, hipStream_t s) {
  const int64_t tf = ln.faces(), tfpad = pad_to_block(tf);
  T *h = (T *)evals;
  uint8_t *sel = (uint8_t *)evals + ((6 * tf * sizeof(T) + 255) & ~(size_t)255);
  hipLaunchKernelGGL(k_evals_euler1d<T>, dim3((unsigned)(6 * tfpad / TPB)), dim3(TPB), 0, s, ln, P,
                     selector, q, masks_in, tfpad, h, sel);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_back_euler1d<T>, dim3(nblocks(tf)), dim3(TPB), 0, s, ln, q, h, sel, Fhat,
                     masks_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_diff1d(const Line1D &ln, int equation, const T *Fhat, const T *q, T *rhs,
                         const Stage *st, int32_t *status_out, hipStream_t s,
                         uint32_t *zero_after) {
  Stage sv{};
  if (st) sv = *st;
  hipLaunchKernelGGL(k_diff1d<T>, dim3(nblocks(ln.faces())), dim3(TPB), 0, s, ln, equation, Fhat, q,
                     rhs, sv, st ? 1 : 0, status_out, zero_after);
  return hipGetLastError();
}

// Face -> line map: one block per line writes the line index of its faces.
__global__ void __launch_bounds__(TPB) k_build_fmap(Line1D ln, int32_t *__restrict__ fmap) {
  const int p = blockIdx.x;
  const int64_t a = ln.offsets[p] + p, b = ln.offsets[p + 1] + p + 1;
  for (int64_t g = a + threadIdx.x; g < b; g += TPB) fmap[g] = p;
}

hipError_t launch_build_fmap(const Line1D &ln, int32_t *fmap, hipStream_t s) {
  hipLaunchKernelGGL(k_build_fmap, dim3(ln.np), dim3(TPB), 0, s, ln, fmap);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cfl1d(const Line1D &ln, int equation, const T *q, double cfl, double *dt,
                        int32_t *status, double *t, hipStream_t s, uint32_t *zero_after) {
  hipLaunchKernelGGL(k_cfl1d<T>, dim3(ln.np), dim3(CFL_TPB), 0, s, ln, equation, q, cfl, dt,
                     status, t, zero_after);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_faces_euler2d(const Grid2D &g, const T *P, int selector, const T *q,
                                const uint8_t *mx_in, const uint8_t *my_in, T *Fx, T *Gy,
                                uint8_t *mx_out, uint8_t *my_out, void *evals, hipStream_t s) {
  const int64_t nfx = (g.nx + 1) * g.ny, nfy = g.nx * (g.ny + 1);
  const int64_t nmax = nfx > nfy ? nfx : nfy;
  T *h = (T *)evals;
  uint8_t *sel = (uint8_t *)evals + ((8 * nmax * sizeof(T) + 255) & ~(size_t)255);
  for (int dir = 0; dir < 2; ++dir) {
    const int64_t nf = dir == 0 ? nfx : nfy, nfpad = pad_to_block(nf);
    hipLaunchKernelGGL(k_evals_euler2d<T>, dim3((unsigned)(8 * nfpad / TPB)), dim3(TPB), 0, s, g,
                       dir, P, selector, q, dir == 0 ? mx_in : my_in, nfpad, h, sel);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_back_euler2d<T>, dim3(nblocks(nf)), dim3(TPB), 0, s, g, dir, q, h, sel,
                       dir == 0 ? Fx : Gy, dir == 0 ? mx_out : my_out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_diff2d(const Grid2D &g, const T *Fx, const T *Gy, const T *q, T *rhs,
                         const Stage *st, int32_t *status_out, hipStream_t s,
                         uint32_t *zero_after) {
  Stage sv{};
  if (st) sv = *st;
  hipLaunchKernelGGL(k_diff2d<T>, dim3(nblocks(g.nx * g.ny)), dim3(TPB), 0, s, g, Fx, Gy, q, rhs,
                     sv, st ? 1 : 0, status_out, zero_after);
  return hipGetLastError();
}

int cfl2d_parts() { return CFL2D_BLOCKS; }

template <typename T>
hipError_t launch_cfl2d(const Grid2D &g, const T *q, double cfl, double *part, double *dt,
                        int32_t *status, double *t, hipStream_t s) {
  hipLaunchKernelGGL(k_cfl2d_partial<T>, dim3(CFL2D_BLOCKS), dim3(TPB), 0, s, g, q, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cfl2d_final, dim3(1), dim3(TPB), 0, s, g, CFL2D_BLOCKS, part, cfl, dt,
                     status, t);
  return hipGetLastError();
}

hipError_t launch_adjoint_advection(const Line1D &ln, const uint8_t *masks, const void *rbar,
                                    void *ubar, int is_fp64, hipStream_t s) {
  if (is_fp64)
    hipLaunchKernelGGL(k_adjoint_advection<double>, dim3(nblocks(ln.total)), dim3(TPB), 0, s,
                       ln.total, ln.dx, ln.bc, masks, (const double *)rbar, (double *)ubar);
  else
    hipLaunchKernelGGL(k_adjoint_advection<float>, dim3(nblocks(ln.total)), dim3(TPB), 0, s,
                       ln.total, ln.dx, ln.bc, masks, (const float *)rbar, (float *)ubar);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vjp1d(const Line1D &ln, int equation, const T *q, const uint8_t *masks,
                        const T *rbar, T *qbar, T *scratch, hipStream_t s) {
  hipLaunchKernelGGL(k_vjp_faces1d<T>, dim3(nblocks(ln.faces())), dim3(TPB), 0, s, ln, equation, q,
                     masks, rbar, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vjp_gather1d<T>, dim3(nblocks(ln.faces())), dim3(TPB), 0, s, ln,
                     equation == 2 ? 3 : 1, scratch, qbar);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vjp2d(const Grid2D &g, const T *q, const uint8_t *masks, const T *rbar, T *qbar,
                        T *scratch, hipStream_t s) {
  const int64_t nfx = (g.nx + 1) * g.ny, nfy = g.nx * (g.ny + 1);
  T *cbx = scratch, *cby = scratch + 24 * nfx;
  hipLaunchKernelGGL(k_vjp_faces2d<T>, dim3(nblocks(nfx)), dim3(TPB), 0, s, g, 0, q, masks, rbar,
                     cbx);
  hipLaunchKernelGGL(k_vjp_faces2d<T>, dim3(nblocks(nfy)), dim3(TPB), 0, s, g, 1, q,
                     masks + 4 * nfx, rbar, cby);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vjp_gather2d<T>, dim3(nblocks(g.nx * g.ny)), dim3(TPB), 0, s, g, cbx, cby,
                     qbar);
  return hipGetLastError();
}

hipError_t launch_params_to_f32(const double *P, float *P32, hipStream_t s) {
  hipLaunchKernelGGL(k_params_to_f32, dim3(nblocks(NPARAM)), dim3(TPB), 0, s, P, P32);
  return hipGetLastError();
}

#define N6_INST(T)                                                                               \
  template hipError_t launch_reconstruct<T>(const T *, const T *, int64_t, int, int,              \
                                            const uint8_t *, T *, uint8_t *, hipStream_t);       \
  template hipError_t launch_mlp_logits<T>(const T *, const T *, int64_t, T *, uint8_t *,        \
                                           hipStream_t);                                         \
  template hipError_t launch_faces_advection<T>(const Line1D &, const T *, int, const T *,       \
                                                const uint8_t *, T *, uint8_t *, hipStream_t);   \
  template hipError_t launch_faces_burgers<T>(const Line1D &, const T *, int, const T *,         \
                                              const uint8_t *, T *, uint8_t *, hipStream_t);     \
  template hipError_t launch_faces_euler1d<T>(const Line1D &, const T *, int, const T *,         \
                                              const uint8_t *, T *, uint8_t *, void *,           \
                                              hipStream_t);                                      \
  template hipError_t launch_diff1d<T>(const Line1D &, int, const T *, const T *, T *,           \
                                       const Stage *, int32_t *, hipStream_t, uint32_t *);       \
  template hipError_t launch_cfl1d<T>(const Line1D &, int, const T *, double, double *,          \
                                      int32_t *, double *, hipStream_t, uint32_t *);             \
  template hipError_t launch_faces_euler2d<T>(const Grid2D &, const T *, int, const T *,         \
                                              const uint8_t *, const uint8_t *, T *, T *,        \
                                              uint8_t *, uint8_t *, void *, hipStream_t);        \
  template hipError_t launch_diff2d<T>(const Grid2D &, const T *, const T *, const T *, T *,     \
                                       const Stage *, int32_t *, hipStream_t, uint32_t *);       \
  template hipError_t launch_cfl2d<T>(const Grid2D &, const T *, double, double *, double *,     \
                                      int32_t *, double *, hipStream_t);                         \
  template hipError_t launch_vjp1d<T>(const Line1D &, int, const T *, const uint8_t *, const T *, \
                                      T *, T *, hipStream_t);                                    \
  template hipError_t launch_vjp2d<T>(const Grid2D &, const T *, const uint8_t *, const T *, T *,  \
                                      T *, hipStream_t);

N6_INST(double)
N6_INST(float)

}  // namespace n6
