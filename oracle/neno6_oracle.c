/*
 * NENO6 oracle -- plain, slow, obviously correct FP64 CPU implementation of
 * the six-point neuron-based ENO scheme of Li, Fu & Adams (arXiv 2207.08500)
 * and of the Lax-Friedrichs flux-split, SSP-RK3 finite-difference solver it
 * sits in.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never includes, links or
 * loads this file.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 *
 * Canonical operation order (the GPU FP64 path writes the same order on its
 * own, so classification labels can be compared bit for bit):
 *   - dot products:   acc = init; for i ascending: acc = fma(a_i, x_i, acc)
 *   - MLP layer:      init = bias, W row-major [out][in]
 *   - candidates:     init = 0, stencil points in ascending position
 *   - weights:        D = sum of the kept d_k in k order, w_k = d_k / D,
 *                     h = fma chain over kept k from 0
 *   - max and fabs are exact; '/' and sqrt are IEEE correctly rounded.
 *
 * Paper parity status of each part is stated where the part is defined.
 * NENO6 with the authors' trained network (the NENO6 columns of the advection
 * accuracy table and the F1 table): parity unpinned, the weights are not
 * published in the text.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NPARAM 3228
#define SEL_MLP 0
#define SEL_ALL_SMOOTH 1
#define SEL_ALL_DISCARD 2
#define SEL_MASKS_IN 3
#define SEL_TENO 4
#define BC_PERIODIC 0
#define BC_TRANSMISSIVE 1
#define ST_OK 0
#define ST_BAD_ARG (-1)
#define ST_NONPHYSICAL (-4)

/* ------------------------------------------------------------------------ */
/* Linear weights of TENO6-opt, reused unchanged by NENO6 (Sec. 2.2 and the  */
/* opening paragraph of Sec. 4).                                             */
/* ------------------------------------------------------------------------ */
static const double LINW[4] = {0.4294317718960898, 0.1727270875843552,
                               0.0855682281039113, 0.312272912415645};

/* Candidate fluxes (eq. convex / approximatepolynomial / definitionEq).
 * Positions 0..5 of the six-point stencil are cells i-2 .. i+3.  Each
 * candidate is the degree r_k-1 polynomial whose cell averages reproduce f
 * on its stencil, evaluated at x_{i+1/2}; the rationals below are that
 * evaluation (a test re-derives them exactly from the cell-average system).
 *   S0 = {i-1,i,i+1}, S1 = {i,i+1,i+2}, S2 = {i-2,i-1,i}, S3 = {i,..,i+3}.
 * The assignment of S0..S2 is the one for which the printed d_k give a
 * fourth-order linear scheme (Fig. 1 is missing from the text). */
static const int CAND_FIRST[4] = {1, 2, 0, 2};
static const int CAND_LEN[4] = {3, 3, 3, 4};
static const double CAND_C[4][4] = {
    {-1.0 / 6.0, 5.0 / 6.0, 1.0 / 3.0, 0.0},
    {1.0 / 3.0, 5.0 / 6.0, -1.0 / 6.0, 0.0},
    {1.0 / 3.0, -7.0 / 6.0, 11.0 / 6.0, 0.0},
    {1.0 / 4.0, 13.0 / 12.0, -5.0 / 12.0, 1.0 / 12.0}};

static const int WIDTH[6] = {6, 64, 32, 16, 8, 4};

void oracle_linear_weights(double *out) {
  for (int k = 0; k < 4; ++k) out[k] = LINW[k];
}

/* out[k*6 + j]: coefficient of stencil position j in candidate k. */
void oracle_candidate_coeffs(double *out) {
  for (int k = 0; k < 4; ++k) {
    for (int j = 0; j < 6; ++j) out[k * 6 + j] = 0.0;
    for (int t = 0; t < CAND_LEN[k]; ++t) out[k * 6 + CAND_FIRST[k] + t] = CAND_C[k][t];
  }
}

int oracle_nparam(void) { return NPARAM; }

/* ------------------------------------------------------------------------ */
/* Per-stencil reconstruction: candidates, re-normalised weights, fallback.  */
/* ------------------------------------------------------------------------ */
static void candidates(const double s[6], double q[4]) {
  for (int k = 0; k < 4; ++k) {
    double acc = 0.0;
    for (int t = 0; t < CAND_LEN[k]; ++t) acc = fma(CAND_C[k][t], s[CAND_FIRST[k] + t], acc);
    q[k] = acc;
  }
}

/* sel bit k = delta_k (1 = candidate kept).  eq. TENOweight_renormalize and
 * eq. convex; if every candidate is discarded the first-order upwind value
 * (stencil position 2, cell i for the '+' orientation) is used (Alg. 2,
 * step 4). */
static double combine(const double s[6], unsigned sel) {
  double q[4];
  candidates(s, q);
  if ((sel & 15u) == 0u) return s[2];
  double D = 0.0;
  for (int k = 0; k < 4; ++k)
    if ((sel >> k) & 1u) D = D + LINW[k];
  double h = 0.0;
  for (int k = 0; k < 4; ++k)
    if ((sel >> k) & 1u) {
      double w = LINW[k] / D;
      h = fma(w, q[k], h);
    }
  return h;
}

/* ------------------------------------------------------------------------ */
/* Classifier (Sec. 3.1): input scaling eq. normalizainput, affine layers     */
/* eq. reconstuction, ReLU eq. activationfunction, sigmoid output read as a  */
/* sign test on the logit (probability > 1/2  <=>  logit > 0).               */
/* Parameter block, FP64, row-major [out][in]:                               */
/*   W1[64][6] b1[64] W2[32][64] b2[32] W3[16][32] b3[16] W4[8][16] b4[8]     */
/*   W5[4][8] b5[4]   (3228 values)                                          */
/* ------------------------------------------------------------------------ */
static void features(const double s[6], double x[6]) {
  double M = 1.0;
  for (int j = 0; j < 6; ++j) {
    double a = fabs(s[j]);
    if (a > M) M = a;
  }
  for (int j = 0; j < 6; ++j) x[j] = s[j] / M;
}

static void mlp_logits(const double *P, const double x0[6], double z[4]) {
  double a[64], b[64];
  int nin = 6;
  for (int i = 0; i < 6; ++i) a[i] = x0[i];
  const double *p = P;
  for (int l = 0; l < 5; ++l) {
    int nout = WIDTH[l + 1];
    const double *W = p;
    const double *bias = p + nout * nin;
    p = bias + nout;
    for (int o = 0; o < nout; ++o) {
      double acc = bias[o];
      for (int i = 0; i < nin; ++i) acc = fma(W[o * nin + i], a[i], acc);
      b[o] = (l < 4) ? (acc > 0.0 ? acc : 0.0) : acc;
    }
    for (int o = 0; o < nout; ++o) a[o] = b[o];
    nin = nout;
  }
  for (int k = 0; k < 4; ++k) z[k] = a[k];
}

/* Candidate k is discarded iff its logit is > 0; returns the kept mask. */
static unsigned classify(const double *P, const double s[6]) {
  double x[6], z[4];
  features(s, x);
  mlp_logits(P, x, z);
  unsigned sel = 0;
  for (int k = 0; k < 4; ++k)
    if (!(z[k] > 0.0)) sel |= 1u << k;
  return sel;
}

/* ------------------------------------------------------------------------ */
/* TENO6-opt stencil selection (Sec. 2.2 and 2.3): smoothness indicators     */
/* (eq. measureTENO) with the sixth-order reference tau_6 (eq. taukTENO),    */
/* normalisation (eq. normalize) and sharp cut-off (eq. cut-off).  The beta  */
/* quadratic forms follow the Jiang-Shu definition the paper points to; see  */
/* gen_teno_beta.py.  Canonical order:                                        */
/*   d_a   = s[first+a+1] - s[first+a], a = 0 .. len-2 (differences, so    */
/*           constant data give beta = 0 exactly);                            */
/*   beta  = fma chain over a ascending of d_a * t_a, t_a = fma chain over   */
/*           b ascending of D[a][b] * d_b (both from 0);                     */
/*   tau   = |beta6 - ((beta1 + beta2) + 4 beta0) / 6|;                      */
/*   x_k   = C + tau / (beta_k + eps); gamma_k = (x^2)^2 * x^2;              */
/*   chi_k = gamma_k / (((gamma0 + gamma1) + gamma2) + gamma3);              */
/*   delta_k = 0 if chi_k < C_T else 1 (bit k of the mask).                  */
/* Constants as printed: C = 1, q = 6, eps = 1e-40, C_T = 1e-6.              */
/* Pins: the three-point forms equal the Jiang-Shu closed forms; every form  */
/* gives the exact derivative integrals of cell-averaged monomials; tau_6 is */
/* sixth order on smooth data; a step removes exactly the candidates that    */
/* cross it.                                                                 */
/* ------------------------------------------------------------------------ */
#include "teno_beta.h"

static const double TENO_C = 1.0, TENO_EPS = 1e-40, TENO_CT = 1e-6;

static double beta_form(const double D[5][5], int first, int len, const double s[6]) {
  double d[5];
  for (int a = 0; a < len - 1; ++a) d[a] = s[first + a + 1] - s[first + a];
  double beta = 0.0;
  for (int a = 0; a < len - 1; ++a) {
    double t = 0.0;
    for (int b = 0; b < len - 1; ++b) t = fma(D[a][b], d[b], t);
    beta = fma(d[a], t, beta);
  }
  return beta;
}

/* beta[0..3] of the candidates S0..S3, beta[4] of the full stencil. */
static unsigned teno_indicators(const double s[6], double beta[5], double *tau, double chi[4]) {
  beta[0] = beta_form(TENO_D_S0, 1, 3, s);
  beta[1] = beta_form(TENO_D_S1, 2, 3, s);
  beta[2] = beta_form(TENO_D_S2, 0, 3, s);
  beta[3] = beta_form(TENO_D_S3, 2, 4, s);
  beta[4] = beta_form(TENO_D_S6, 0, 6, s);
  const double t = fabs(beta[4] - ((beta[1] + beta[2]) + 4.0 * beta[0]) / 6.0);
  double g[4];
  for (int k = 0; k < 4; ++k) {
    const double x = TENO_C + t / (beta[k] + TENO_EPS);
    const double x2 = x * x;
    g[k] = (x2 * x2) * x2;
  }
  const double sum = ((g[0] + g[1]) + g[2]) + g[3];
  unsigned sel = 0;
  for (int k = 0; k < 4; ++k) {
    chi[k] = g[k] / sum;
    if (!(chi[k] < TENO_CT)) sel |= 1u << k;
  }
  *tau = t;
  return sel;
}

static unsigned teno_select(const double s[6]) {
  double beta[5], tau, chi[4];
  return teno_indicators(s, beta, &tau, chi);
}

/* The TENO6-opt quantities for n stencils s[n][6]: beta[n][5], tau[n],
 * chi[n][4], masks[n] (bit k = candidate k kept). */
int oracle_teno(const double *s, int64_t n, double *beta, double *tau, double *chi,
                uint8_t *masks) {
  for (int64_t e = 0; e < n; ++e)
    masks[e] = (uint8_t)teno_indicators(s + 6 * e, beta + 5 * e, tau + e, chi + 4 * e);
  return ST_OK;
}

static unsigned select_mask(int selector, const double *P, const double s[6], unsigned mask_in) {
  switch (selector) {
  case SEL_MLP: return classify(P, s);
  case SEL_ALL_SMOOTH: return 15u;
  case SEL_ALL_DISCARD: return 0u;
  case SEL_TENO: return teno_select(s);
  default: return mask_in & 15u;
  }
}

/* Features and logits for n stencils s[n][6] (the classifier on its own). */
int oracle_mlp_logits(const double *P, const double *s, int64_t n, double *x_out, double *z_out) {
  for (int64_t e = 0; e < n; ++e) {
    double x[6], z[4];
    features(s + 6 * e, x);
    mlp_logits(P, x, z);
    if (x_out)
      for (int j = 0; j < 6; ++j) x_out[6 * e + j] = x[j];
    for (int k = 0; k < 4; ++k) z_out[4 * e + k] = z[k];
  }
  return ST_OK;
}

/* Logits for n already-normalised feature vectors x[n][6]. */
int oracle_mlp_logits_raw(const double *P, const double *x, int64_t n, double *z_out) {
  for (int64_t e = 0; e < n; ++e) mlp_logits(P, x + 6 * e, z_out + 4 * e);
  return ST_OK;
}

/* Scalar reconstruction at n_faces faces from f[n_faces + 5]: face k uses
 * f[k .. k+5] (cells i-2 .. i+3 for the '+' orientation).  sign = -1 uses
 * the mirrored stencil f[k+5], ..., f[k] (cells i+3 .. i-2), i.e. the
 * reconstruction of the left-going flux at the same face. */
int oracle_reconstruct(const double *f, int64_t n_faces, int32_t sign, const double *P,
                       int32_t selector, const uint8_t *masks_in, double *fhat,
                       uint8_t *masks_out) {
  if (n_faces < 0 || (sign != 1 && sign != -1) || selector < 0 || selector > 4) return ST_BAD_ARG;
  if (selector == SEL_MASKS_IN && !masks_in) return ST_BAD_ARG;
  if (selector == SEL_MLP && !P) return ST_BAD_ARG;
  for (int64_t k = 0; k < n_faces; ++k) {
    double s[6];
    for (int j = 0; j < 6; ++j) s[j] = (sign > 0) ? f[k + j] : f[k + 5 - j];
    unsigned sel = select_mask(selector, P, s, masks_in ? masks_in[k] : 0u);
    fhat[k] = combine(s, sel);
    if (masks_out) masks_out[k] = (uint8_t)sel;
  }
  return ST_OK;
}

/* ------------------------------------------------------------------------ */
/* Ghost cells: three per side.  Periodic wraps, transmissive copies the     */
/* nearest interior cell (zero gradient).                                    */
/* ------------------------------------------------------------------------ */
static int64_t ghost_index(int64_t c, int64_t n, int bc) {
  if (bc == BC_PERIODIC) {
    int64_t r = c % n;
    return r < 0 ? r + n : r;
  }
  if (c < 0) return 0;
  if (c > n - 1) return n - 1;
  return c;
}

/* ------------------------------------------------------------------------ */
/* Scalar linear advection u_t + u_x = 0 (Sec. 4.2).  Flux f = u, signal     */
/* speed 1, Lax-Friedrichs split f+- = (f +- alpha u)/2 with alpha = 1.      */
/* f- is identically zero, so its reconstruction is zero for every mask and  */
/* the face flux is the '+' reconstruction alone.  Masks: '+' mask per face. */
/* ------------------------------------------------------------------------ */
int oracle_advection_rhs(const double *u, int64_t n, double dx, int32_t bc, const double *P,
                         int32_t selector, const uint8_t *masks_in, double *rhs,
                         uint8_t *masks_out) {
  if (n < 1 || !(dx > 0.0) || (bc != 0 && bc != 1)) return ST_BAD_ARG;
  double *fp = (double *)malloc(sizeof(double) * (size_t)(n + 6));
  double *fh = (double *)malloc(sizeof(double) * (size_t)(n + 1));
  const double alpha = 1.0;
  for (int64_t j = 0; j < n + 6; ++j) {
    double uj = u[ghost_index(j - 3, n, bc)];
    double fj = uj;
    fp[j] = 0.5 * (fj + alpha * uj);
  }
  int st = oracle_reconstruct(fp, n + 1, 1, P, selector, masks_in, fh, masks_out);
  if (st == ST_OK)
    for (int64_t i = 0; i < n; ++i) rhs[i] = (fh[i] - fh[i + 1]) / dx;
  free(fp);
  free(fh);
  return st;
}

/* SSP-RK3 (Sec. 4.4): u1 = u + dt L(u); u2 = 3/4 u + 1/4 (u1 + dt L(u1));
 * u^{n+1} = 1/3 u + 2/3 (u2 + dt L(u2)). */
int oracle_advection_step(double *u, int64_t n, double dx, double dt, int32_t n_steps, int32_t bc,
                          const double *P, int32_t selector, const uint8_t *masks_in) {
  if (n < 1 || n_steps < 0) return ST_BAD_ARG;
  size_t sz = sizeof(double) * (size_t)n;
  double *L = (double *)malloc(sz), *u1 = (double *)malloc(sz), *u2 = (double *)malloc(sz);
  int st = ST_OK;
  for (int32_t it = 0; it < n_steps && st == ST_OK; ++it) {
    st = oracle_advection_rhs(u, n, dx, bc, P, selector, masks_in, L, NULL);
    for (int64_t i = 0; i < n; ++i) u1[i] = fma(dt, L[i], u[i]);
    if (st == ST_OK) st = oracle_advection_rhs(u1, n, dx, bc, P, selector, masks_in, L, NULL);
    for (int64_t i = 0; i < n; ++i) {
      double t = fma(dt, L[i], u1[i]);
      u2[i] = fma(0.25, t, 0.75 * u[i]);
    }
    if (st == ST_OK) st = oracle_advection_rhs(u2, n, dx, bc, P, selector, masks_in, L, NULL);
    for (int64_t i = 0; i < n; ++i) {
      double t = fma(dt, L[i], u2[i]);
      u[i] = fma(2.0 / 3.0, t, (1.0 / 3.0) * u[i]);
    }
  }
  free(L);
  free(u1);
  free(u2);
  return st;
}

/* Adjoint of the advection right-hand side with respect to u at fixed '+'
 * masks.  At fixed masks the map u -> rhs is linear (the classifier only
 * chooses the weights); the oracle assembles its matrix A column by column
 * by applying the right-hand side to unit vectors and returns A^T rbar.
 * n is limited to 8192 (dense matrix). */
int oracle_advection_rhs_adjoint(const uint8_t *masks, int64_t n, double dx, int32_t bc,
                                 const double *rbar, double *ubar) {
  if (n < 1 || n > 8192) return ST_BAD_ARG;
  double *e = (double *)calloc((size_t)n, sizeof(double));
  double *col = (double *)malloc(sizeof(double) * (size_t)n);
  int st = ST_OK;
  for (int64_t c = 0; c < n && st == ST_OK; ++c) {
    e[c] = 1.0;
    st = oracle_advection_rhs(e, n, dx, bc, NULL, SEL_MASKS_IN, masks, col, NULL);
    e[c] = 0.0;
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc = fma(col[i], rbar[i], acc);
    ubar[c] = acc;
  }
  free(e);
  free(col);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Euler equations, gamma-law gas (Sec. 4.4).                                */
/* Characteristic decomposition with Roe-averaged eigenvectors, Rusanov      */
/* (local Lax-Friedrichs) splitting, NENO6 per characteristic field and      */
/* sign, back-projection, conservative flux difference.                      */
/* Reading of the Rusanov speed: alpha_m = max over the six stencil cells of */
/* |lambda_m| evaluated from each cell's own state.                          */
/* ------------------------------------------------------------------------ */

/* 1D: state (rho, rho u, E). */
static void prim1d(const double q[3], double gamma, double *u, double *p, double *c) {
  *u = q[1] / q[0];
  double t = q[1] * (*u);
  double ke = 0.5 * t;
  *p = (gamma - 1.0) * (q[2] - ke);
  *c = sqrt((gamma * (*p)) / q[0]);
}

static void flux1d(const double q[3], double u, double p, double F[3]) {
  F[0] = q[1];
  F[1] = q[1] * u + p;
  F[2] = (q[2] + p) * u;
}

/* Roe-averaged left (L) and right (R) eigenvector matrices of the 1D flux
 * Jacobian; R columns are the fields of speeds u-c, u, u+c. */
static void roe1d(const double qL[3], const double qR[3], double gamma, double L[3][3],
                  double R[3][3]) {
  double uL, pL, cL, uR, pR, cR;
  prim1d(qL, gamma, &uL, &pL, &cL);
  prim1d(qR, gamma, &uR, &pR, &cR);
  double sL = sqrt(qL[0]), sR = sqrt(qR[0]);
  double HL = (qL[2] + pL) / qL[0], HR = (qR[2] + pR) / qR[0];
  double den = sL + sR;
  double ut = (sL * uL + sR * uR) / den;
  double Ht = (sL * HL + sR * HR) / den;
  double q2 = 0.5 * (ut * ut);
  double c2 = (gamma - 1.0) * (Ht - q2);
  double ct = sqrt(c2);
  double b1 = (gamma - 1.0) / c2;
  double b2 = b1 * q2;
  double uc = ut / ct;
  double ic = 1.0 / ct;
  R[0][0] = 1.0;          R[0][1] = 1.0; R[0][2] = 1.0;
  R[1][0] = ut - ct;      R[1][1] = ut;  R[1][2] = ut + ct;
  R[2][0] = Ht - ut * ct; R[2][1] = q2;  R[2][2] = Ht + ut * ct;
  L[0][0] = 0.5 * (b2 + uc); L[0][1] = -0.5 * (b1 * ut + ic); L[0][2] = 0.5 * b1;
  L[1][0] = 1.0 - b2;        L[1][1] = b1 * ut;               L[1][2] = -b1;
  L[2][0] = 0.5 * (b2 - uc); L[2][1] = -0.5 * (b1 * ut - ic); L[2][2] = 0.5 * b1;
}

void oracle_euler1d_eigen(const double *qL, const double *qR, double gamma, double *L, double *R) {
  double Lm[3][3], Rm[3][3];
  roe1d(qL, qR, gamma, Lm, Rm);
  memcpy(L, Lm, sizeof Lm);
  memcpy(R, Rm, sizeof Rm);
}

void oracle_euler1d_flux(const double *q, double gamma, double *F) {
  double u, p, c;
  prim1d(q, gamma, &u, &p, &c);
  flux1d(q, u, p, F);
}

/* Validity of a cell state: rho > 0, p > 0 and finite. */
static int physical(double rho, double p) { return rho > 0.0 && p > 0.0 && isfinite(rho) && isfinite(p); }

/* Face flux of a 1D Euler line between cells i and i+1 from the six cells
 * i-2..i+3 given in qs[j][var] (j = 0..5), and its masks.
 * mask byte per field: low nibble '+', high nibble '-'. */
/* Characteristic Rusanov split of the six cells: the '+' and '-' stencils of
 * every field m (the '-' one mirrored), and the Roe eigenvectors R. */
static void euler1d_split(const double qs[6][3], double gamma, double spl[3][6], double smi[3][6],
                          double R[3][3]) {
  double L[3][3];
  roe1d(qs[2], qs[3], gamma, L, R);
  double v[6][3], g[6][3], lam[6][3];
  for (int j = 0; j < 6; ++j) {
    double u, p, c, F[3];
    prim1d(qs[j], gamma, &u, &p, &c);
    flux1d(qs[j], u, p, F);
    lam[j][0] = u - c;
    lam[j][1] = u;
    lam[j][2] = u + c;
    for (int m = 0; m < 3; ++m) {
      double av = 0.0, ag = 0.0;
      for (int r = 0; r < 3; ++r) {
        av = fma(L[m][r], qs[j][r], av);
        ag = fma(L[m][r], F[r], ag);
      }
      v[j][m] = av;
      g[j][m] = ag;
    }
  }
  for (int m = 0; m < 3; ++m) {
    double alpha = 0.0;
    for (int j = 0; j < 6; ++j) {
      double a = fabs(lam[j][m]);
      if (a > alpha) alpha = a;
    }
    for (int j = 0; j < 6; ++j) {
      double t = alpha * v[j][m];
      spl[m][j] = 0.5 * (g[j][m] + t);
      smi[m][5 - j] = 0.5 * (g[j][m] - t);
    }
  }
}

static void euler1d_face(const double qs[6][3], double gamma, const double *P, int selector,
                         const uint8_t *min, double Fhat[3], uint8_t *mout) {
  double sp[3][6], sm[3][6], R[3][3];
  euler1d_split(qs, gamma, sp, sm, R);
  double hs[3];
  for (int m = 0; m < 3; ++m) {
    unsigned mi = min ? min[m] : 0u;
    unsigned selp = select_mask(selector, P, sp[m], mi & 15u);
    unsigned selm = select_mask(selector, P, sm[m], (mi >> 4) & 15u);
    double hp = combine(sp[m], selp);
    double hm = combine(sm[m], selm);
    hs[m] = hp + hm;
    if (mout) mout[m] = (uint8_t)(selp | (selm << 4));
  }
  for (int r = 0; r < 3; ++r) {
    double acc = 0.0;
    for (int m = 0; m < 3; ++m) acc = fma(R[r][m], hs[m], acc);
    Fhat[r] = acc;
  }
}

/* Right-hand side for a batch of independent 1D Euler lines.
 * q: SoA [3][total] with problem p occupying cells offsets[p]..offsets[p+1]-1.
 * masks (in or out): [3][total + n_problems], faces of problem p at
 * offsets[p] + p + k, k = 0..N_p (face k lies between cells k-1 and k).
 * status[p] is set to -4 if a cell of problem p is not physical. */
int oracle_euler1d_rhs(const double *q, const int64_t *offsets, int32_t n_problems,
                       const double *dx, double gamma, int32_t bc, const double *P,
                       int32_t selector, const uint8_t *masks_in, double *rhs,
                       uint8_t *masks_out, int32_t *status) {
  if (n_problems < 0 || (bc != 0 && bc != 1) || selector < 0 || selector > 4) return ST_BAD_ARG;
  const int64_t total = offsets[n_problems];
  const int64_t tf = total + n_problems;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int32_t pb = 0; pb < n_problems; ++pb) {
    const int64_t o = offsets[pb];
    const int64_t n = offsets[pb + 1] - o;
    if (n < 1) {
      bad = 1;
      continue;
    }
    double(*Fh)[3] = (double(*)[3])malloc(sizeof(double) * 3 * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) {
      double qc[3] = {q[o + i], q[total + o + i], q[2 * total + o + i]};
      double u, p, c;
      prim1d(qc, gamma, &u, &p, &c);
      if (!physical(qc[0], p) && status) status[pb] = ST_NONPHYSICAL;
    }
    for (int64_t k = 0; k <= n; ++k) {
      double qs[6][3];
      for (int j = 0; j < 6; ++j) {
        int64_t ci = ghost_index(k - 3 + j, n, bc);
        for (int r = 0; r < 3; ++r) qs[j][r] = q[r * total + o + ci];
      }
      uint8_t mi[3] = {0, 0, 0}, mo[3];
      const int64_t fidx = o + pb + k;
      if (masks_in)
        for (int m = 0; m < 3; ++m) mi[m] = masks_in[m * tf + fidx];
      euler1d_face(qs, gamma, P, selector, masks_in ? mi : NULL, Fh[k], mo);
      if (masks_out)
        for (int m = 0; m < 3; ++m) masks_out[m * tf + fidx] = mo[m];
    }
    for (int64_t i = 0; i < n; ++i)
      for (int r = 0; r < 3; ++r) rhs[r * total + o + i] = (Fh[i][r] - Fh[i + 1][r]) / dx[pb];
    free(Fh);
  }
  return bad ? ST_BAD_ARG : ST_OK;
}

/* The six split stencils of every face of a batch of 1D Euler lines (the
 * classifier inputs of the rhs): out[face][e][6], e = 2 m + sign, faces
 * numbered as the masks of oracle_euler1d_rhs. */
int oracle_euler1d_stencils(const double *q, const int64_t *offsets, int32_t n_problems,
                            double gamma, int32_t bc, double *out) {
  if (n_problems < 0 || (bc != 0 && bc != 1)) return ST_BAD_ARG;
  const int64_t total = offsets[n_problems];
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int32_t pb = 0; pb < n_problems; ++pb) {
    const int64_t o = offsets[pb];
    const int64_t n = offsets[pb + 1] - o;
    if (n < 1) {
      bad = 1;
      continue;
    }
    for (int64_t k = 0; k <= n; ++k) {
      double qs[6][3], sp[3][6], sm[3][6], R[3][3];
      for (int j = 0; j < 6; ++j) {
        int64_t ci = ghost_index(k - 3 + j, n, bc);
        for (int r = 0; r < 3; ++r) qs[j][r] = q[r * total + o + ci];
      }
      euler1d_split(qs, gamma, sp, sm, R);
      double *dst = out + (o + pb + k) * 36;
      for (int m = 0; m < 3; ++m)
        for (int j = 0; j < 6; ++j) {
          dst[(2 * m) * 6 + j] = sp[m][j];
          dst[(2 * m + 1) * 6 + j] = sm[m][j];
        }
    }
  }
  return bad ? ST_BAD_ARG : ST_OK;
}

/* Time step of each problem: dt = cfl*dx / max_i(|u_i| + c_i); problems with
 * a cell that is not physical get status -4 and are not advanced. */
static void euler1d_dt(const double *q, int64_t total, int64_t o, int64_t n, double gamma,
                       double cfl, double dx, double *dt, int32_t *st) {
  double smax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double qc[3] = {q[o + i], q[total + o + i], q[2 * total + o + i]};
    double u, p, c;
    prim1d(qc, gamma, &u, &p, &c);
    if (!physical(qc[0], p)) {
      *st = ST_NONPHYSICAL;
      return;
    }
    double s = fabs(u) + c;
    if (s > smax) smax = s;
  }
  *dt = (cfl * dx) / smax;
}

/* n_steps SSP-RK3 steps of every problem with status 0, each with its own
 * CFL time step taken at the start of the step; t[p] advances by that dt. */
int oracle_euler1d_step(double *q, const int64_t *offsets, int32_t n_problems, const double *dx,
                        double gamma, int32_t bc, double cfl, int32_t n_steps, const double *P,
                        int32_t selector, double *t, int32_t *status) {
  if (n_problems < 0 || n_steps < 0 || (bc != 0 && bc != 1)) return ST_BAD_ARG;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int32_t pb = 0; pb < n_problems; ++pb) {
    const int64_t n = offsets[pb + 1] - offsets[pb];
    if (n < 1) {
      bad = 1;
      continue;
    }
    const size_t sz = sizeof(double) * 3 * (size_t)n;
    double *u0 = (double *)malloc(sz), *u1 = (double *)malloc(sz), *u2 = (double *)malloc(sz),
           *L = (double *)malloc(sz);
    const int64_t off1[2] = {0, n};
    for (int r = 0; r < 3; ++r)
      for (int64_t i = 0; i < n; ++i) u0[r * n + i] = q[r * offsets[n_problems] + offsets[pb] + i];
    for (int32_t it = 0; it < n_steps; ++it) {
      if (status[pb] != 0) break;
      double dt = 0.0;
      euler1d_dt(u0, n, 0, n, gamma, cfl, dx[pb], &dt, &status[pb]);
      if (status[pb] != 0) break;
      int32_t dummy = 0;
      oracle_euler1d_rhs(u0, off1, 1, &dx[pb], gamma, bc, P, selector, NULL, L, NULL, &dummy);
      for (int64_t i = 0; i < 3 * n; ++i) u1[i] = fma(dt, L[i], u0[i]);
      oracle_euler1d_rhs(u1, off1, 1, &dx[pb], gamma, bc, P, selector, NULL, L, NULL, &dummy);
      for (int64_t i = 0; i < 3 * n; ++i) {
        double tt = fma(dt, L[i], u1[i]);
        u2[i] = fma(0.25, tt, 0.75 * u0[i]);
      }
      oracle_euler1d_rhs(u2, off1, 1, &dx[pb], gamma, bc, P, selector, NULL, L, NULL, &dummy);
      for (int64_t i = 0; i < 3 * n; ++i) {
        double tt = fma(dt, L[i], u2[i]);
        u0[i] = fma(2.0 / 3.0, tt, (1.0 / 3.0) * u0[i]);
      }
      t[pb] = t[pb] + dt;
    }
    for (int r = 0; r < 3; ++r)
      for (int64_t i = 0; i < n; ++i) q[r * offsets[n_problems] + offsets[pb] + i] = u0[r * n + i];
    free(u0);
    free(u1);
    free(u2);
    free(L);
  }
  return bad ? ST_BAD_ARG : ST_OK;
}

/* ------------------------------------------------------------------------ */
/* Inviscid Burgers equation (Sec. 4.3, eq. Burgers): f(u) = u^2/2,          */
/* f'(u) = u.  Rusanov / Lax-Friedrichs splitting f+- = (f +- alpha u)/2 with */
/* alpha the largest |u| over the six stencil cells (the same local reading */
/* as the Euler splitting); f+ is reconstructed on cells i-2..i+3, f- on the */
/* mirrored stencil, and the face flux is their sum.  Open boundaries are   */
/* the transmissive ghost cells.  Order: f = 0.5 * (u * u), t = alpha * u,   */
/* s+ = 0.5 * (f + t), s- = 0.5 * (f - t).                                   */
/* Pins: conservation on periodic grids, the characteristic solution before */
/* shock formation (order of accuracy), the Rankine-Hugoniot shock speed,   */
/* the rarefaction fan, and the u(x) -> -u(-x) symmetry of the equation.    */
/* ------------------------------------------------------------------------ */
static void burgers_face(const double us[6], const double *P, int selector, unsigned mi,
                         double *Fh, uint8_t *mout) {
  double alpha = 0.0;
  for (int j = 0; j < 6; ++j) {
    double a = fabs(us[j]);
    if (a > alpha) alpha = a;
  }
  double sp[6], sm[6];
  for (int j = 0; j < 6; ++j) {
    double f = 0.5 * (us[j] * us[j]);
    double t = alpha * us[j];
    sp[j] = 0.5 * (f + t);
    sm[5 - j] = 0.5 * (f - t);
  }
  unsigned selp = select_mask(selector, P, sp, mi & 15u);
  unsigned selm = select_mask(selector, P, sm, (mi >> 4) & 15u);
  *Fh = combine(sp, selp) + combine(sm, selm);
  if (mout) *mout = (uint8_t)(selp | (selm << 4));
}

/* Right-hand side of a batch of independent Burgers lines: u[total], masks
 * [total + n_problems] (faces as for Euler), status -4 for a line with a
 * non-finite value. */
int oracle_burgers_rhs(const double *u, const int64_t *offsets, int32_t n_problems,
                       const double *dx, int32_t bc, const double *P, int32_t selector,
                       const uint8_t *masks_in, double *rhs, uint8_t *masks_out,
                       int32_t *status) {
  if (n_problems < 0 || (bc != 0 && bc != 1) || selector < 0 || selector > 4) return ST_BAD_ARG;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int32_t pb = 0; pb < n_problems; ++pb) {
    const int64_t o = offsets[pb];
    const int64_t n = offsets[pb + 1] - o;
    if (n < 1) {
      bad = 1;
      continue;
    }
    double *Fh = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i)
      if (!isfinite(u[o + i]) && status) status[pb] = ST_NONPHYSICAL;
    for (int64_t k = 0; k <= n; ++k) {
      double us[6];
      for (int j = 0; j < 6; ++j) us[j] = u[o + ghost_index(k - 3 + j, n, bc)];
      const int64_t fidx = o + pb + k;
      uint8_t mo;
      burgers_face(us, P, selector, masks_in ? masks_in[fidx] : 0u, &Fh[k], &mo);
      if (masks_out) masks_out[fidx] = mo;
    }
    for (int64_t i = 0; i < n; ++i) rhs[o + i] = (Fh[i] - Fh[i + 1]) / dx[pb];
    free(Fh);
  }
  return bad ? ST_BAD_ARG : ST_OK;
}

/* dt = cfl*dx / max|u| (cfl*dx when u is identically 0); a line with a
 * non-finite value gets status -4 and is not advanced. */
static void burgers_dt(const double *u, int64_t n, double cfl, double dx, double *dt, int32_t *st) {
  double smax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!isfinite(u[i])) {
      *st = ST_NONPHYSICAL;
      return;
    }
    double a = fabs(u[i]);
    if (a > smax) smax = a;
  }
  *dt = smax > 0.0 ? (cfl * dx) / smax : cfl * dx;
}

int oracle_burgers_step(double *u, const int64_t *offsets, int32_t n_problems, const double *dx,
                        int32_t bc, double cfl, int32_t n_steps, const double *P, int32_t selector,
                        double *t, int32_t *status) {
  if (n_problems < 0 || n_steps < 0 || (bc != 0 && bc != 1)) return ST_BAD_ARG;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int32_t pb = 0; pb < n_problems; ++pb) {
    const int64_t o = offsets[pb], n = offsets[pb + 1] - o;
    if (n < 1) {
      bad = 1;
      continue;
    }
    const size_t sz = sizeof(double) * (size_t)n;
    double *u0 = (double *)malloc(sz), *u1 = (double *)malloc(sz), *u2 = (double *)malloc(sz),
           *L = (double *)malloc(sz);
    const int64_t off1[2] = {0, n};
    memcpy(u0, u + o, sz);
    for (int32_t it = 0; it < n_steps; ++it) {
      if (status[pb] != 0) break;
      double dt = 0.0;
      burgers_dt(u0, n, cfl, dx[pb], &dt, &status[pb]);
      if (status[pb] != 0) break;
      int32_t dummy = 0;
      oracle_burgers_rhs(u0, off1, 1, &dx[pb], bc, P, selector, NULL, L, NULL, &dummy);
      for (int64_t i = 0; i < n; ++i) u1[i] = fma(dt, L[i], u0[i]);
      oracle_burgers_rhs(u1, off1, 1, &dx[pb], bc, P, selector, NULL, L, NULL, &dummy);
      for (int64_t i = 0; i < n; ++i) {
        double tt = fma(dt, L[i], u1[i]);
        u2[i] = fma(0.25, tt, 0.75 * u0[i]);
      }
      oracle_burgers_rhs(u2, off1, 1, &dx[pb], bc, P, selector, NULL, L, NULL, &dummy);
      for (int64_t i = 0; i < n; ++i) {
        double tt = fma(dt, L[i], u2[i]);
        u0[i] = fma(2.0 / 3.0, tt, (1.0 / 3.0) * u0[i]);
      }
      t[pb] = t[pb] + dt;
    }
    memcpy(u + o, u0, sz);
    free(u0);
    free(u1);
    free(u2);
    free(L);
  }
  return bad ? ST_BAD_ARG : ST_OK;
}

/* 2D: state (rho, rho u, rho v, E); dimension-by-dimension application.
 * dir 0 = x (normal velocity u), dir 1 = y (normal velocity v). */
static void prim2d(const double q[4], double gamma, double *u, double *v, double *p, double *c) {
  *u = q[1] / q[0];
  *v = q[2] / q[0];
  double t1 = q[1] * (*u);
  double t2 = q[2] * (*v);
  double ke = 0.5 * (t1 + t2);
  *p = (gamma - 1.0) * (q[3] - ke);
  *c = sqrt((gamma * (*p)) / q[0]);
}

static void flux2d(const double q[4], double u, double v, double p, int dir, double F[4]) {
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

static void roe2d(const double qL[4], const double qR[4], double gamma, int dir, double L[4][4],
                  double R[4][4]) {
  double uL, vL, pL, cL, uR, vR, pR, cR;
  prim2d(qL, gamma, &uL, &vL, &pL, &cL);
  prim2d(qR, gamma, &uR, &vR, &pR, &cR);
  double sL = sqrt(qL[0]), sR = sqrt(qR[0]);
  double HL = (qL[3] + pL) / qL[0], HR = (qR[3] + pR) / qR[0];
  double den = sL + sR;
  double ut = (sL * uL + sR * uR) / den;
  double vt = (sL * vL + sR * vR) / den;
  double Ht = (sL * HL + sR * HR) / den;
  double q2 = 0.5 * (ut * ut + vt * vt);
  double c2 = (gamma - 1.0) * (Ht - q2);
  double ct = sqrt(c2);
  double b1 = (gamma - 1.0) / c2;
  double b2 = b1 * q2;
  double ic = 1.0 / ct;
  /* n = normal velocity, s = tangential velocity */
  double un = dir == 0 ? ut : vt;
  double us = dir == 0 ? vt : ut;
  double nc = un / ct;
  /* Written in the ordering (rho, rho u_n, rho u_s, E), then permuted. */
  double Rn[4][4] = {{1.0, 1.0, 0.0, 1.0},
                     {un - ct, un, 0.0, un + ct},
                     {us, us, 1.0, us},
                     {Ht - un * ct, q2, us, Ht + un * ct}};
  double Ln[4][4] = {{0.5 * (b2 + nc), -0.5 * (b1 * un + ic), -0.5 * (b1 * us), 0.5 * b1},
                     {1.0 - b2, b1 * un, b1 * us, -b1},
                     {-us, 0.0, 1.0, 0.0},
                     {0.5 * (b2 - nc), -0.5 * (b1 * un - ic), -0.5 * (b1 * us), 0.5 * b1}};
  /* variable index of (rho, rho u_n, rho u_s, E) in (rho, rho u, rho v, E) */
  int perm[4] = {0, dir == 0 ? 1 : 2, dir == 0 ? 2 : 1, 3};
  for (int a = 0; a < 4; ++a)
    for (int m = 0; m < 4; ++m) {
      R[perm[a]][m] = Rn[a][m];
      L[m][perm[a]] = Ln[m][a];
    }
}

void oracle_euler2d_eigen(const double *qL, const double *qR, double gamma, int32_t dir, double *L,
                          double *R) {
  double Lm[4][4], Rm[4][4];
  roe2d(qL, qR, gamma, dir, Lm, Rm);
  memcpy(L, Lm, sizeof Lm);
  memcpy(R, Rm, sizeof Rm);
}

void oracle_euler2d_flux(const double *q, double gamma, int32_t dir, double *F) {
  double u, v, p, c;
  prim2d(q, gamma, &u, &v, &p, &c);
  flux2d(q, u, v, p, dir, F);
}

static void euler2d_face(const double qs[6][4], double gamma, int dir, const double *P,
                         int selector, const uint8_t *min, double Fhat[4], uint8_t *mout) {
  double L[4][4], R[4][4];
  roe2d(qs[2], qs[3], gamma, dir, L, R);
  double v[6][4], g[6][4], lam[6][4];
  for (int j = 0; j < 6; ++j) {
    double u, vv, p, c, F[4];
    prim2d(qs[j], gamma, &u, &vv, &p, &c);
    flux2d(qs[j], u, vv, p, dir, F);
    double un = dir == 0 ? u : vv;
    lam[j][0] = un - c;
    lam[j][1] = un;
    lam[j][2] = un;
    lam[j][3] = un + c;
    for (int m = 0; m < 4; ++m) {
      double av = 0.0, ag = 0.0;
      for (int r = 0; r < 4; ++r) {
        av = fma(L[m][r], qs[j][r], av);
        ag = fma(L[m][r], F[r], ag);
      }
      v[j][m] = av;
      g[j][m] = ag;
    }
  }
  double hs[4];
  for (int m = 0; m < 4; ++m) {
    double alpha = 0.0;
    for (int j = 0; j < 6; ++j) {
      double a = fabs(lam[j][m]);
      if (a > alpha) alpha = a;
    }
    double sp[6], sm[6];
    for (int j = 0; j < 6; ++j) {
      double t = alpha * v[j][m];
      sp[j] = 0.5 * (g[j][m] + t);
      sm[5 - j] = 0.5 * (g[j][m] - t);
    }
    unsigned mi = min ? min[m] : 0u;
    unsigned selp = select_mask(selector, P, sp, mi & 15u);
    unsigned selm = select_mask(selector, P, sm, (mi >> 4) & 15u);
    double hp = combine(sp, selp);
    double hm = combine(sm, selm);
    hs[m] = hp + hm;
    if (mout) mout[m] = (uint8_t)(selp | (selm << 4));
  }
  for (int r = 0; r < 4; ++r) {
    double acc = 0.0;
    for (int m = 0; m < 4; ++m) acc = fma(R[r][m], hs[m], acc);
    Fhat[r] = acc;
  }
}

/* 2D right-hand side on an nx x ny grid.  q, rhs: SoA [4][ny][nx] (x fastest).
 * masks_x: [4][ny][nx+1] (x-face k of row y between cells k-1 and k);
 * masks_y: [4][ny+1][nx] (y-face k of column x between rows k-1 and k).
 * rhs = (Fx_{k} - Fx_{k+1})/dx + (Gy_{k} - Gy_{k+1})/dy. */
int oracle_euler2d_rhs(const double *q, int64_t nx, int64_t ny, double dx, double dy, double gamma,
                       int32_t bc, const double *P, int32_t selector, const uint8_t *mx_in,
                       const uint8_t *my_in, double *rhs, uint8_t *mx_out, uint8_t *my_out,
                       int32_t *status) {
  if (nx < 1 || ny < 1 || (bc != 0 && bc != 1) || selector < 0 || selector > 4) return ST_BAD_ARG;
  if (selector == SEL_MASKS_IN && (!mx_in || !my_in)) return ST_BAD_ARG;
  const int64_t cells = nx * ny;
  const int64_t nfx = (nx + 1) * ny, nfy = nx * (ny + 1);
  double *ax = (double *)malloc(sizeof(double) * 4 * (size_t)cells);
  int flag = 0;
  for (int64_t i = 0; i < cells; ++i) {
    double qc[4] = {q[i], q[cells + i], q[2 * cells + i], q[3 * cells + i]};
    double u, v, p, c;
    prim2d(qc, gamma, &u, &v, &p, &c);
    if (!physical(qc[0], p)) flag = 1;
  }
  if (flag && status) status[0] = ST_NONPHYSICAL;
  /* x sweep */
#pragma omp parallel for schedule(static)
  for (int64_t y = 0; y < ny; ++y) {
    double(*Fh)[4] = (double(*)[4])malloc(sizeof(double) * 4 * (size_t)(nx + 1));
    for (int64_t k = 0; k <= nx; ++k) {
      double qs[6][4];
      for (int j = 0; j < 6; ++j) {
        int64_t ci = ghost_index(k - 3 + j, nx, bc);
        for (int r = 0; r < 4; ++r) qs[j][r] = q[r * cells + y * nx + ci];
      }
      uint8_t mi[4], mo[4];
      const int64_t fidx = y * (nx + 1) + k;
      if (mx_in)
        for (int m = 0; m < 4; ++m) mi[m] = mx_in[m * nfx + fidx];
      euler2d_face(qs, gamma, 0, P, selector, mx_in ? mi : NULL, Fh[k], mo);
      if (mx_out)
        for (int m = 0; m < 4; ++m) mx_out[m * nfx + fidx] = mo[m];
    }
    for (int64_t x = 0; x < nx; ++x)
      for (int r = 0; r < 4; ++r) ax[r * cells + y * nx + x] = (Fh[x][r] - Fh[x + 1][r]) / dx;
    free(Fh);
  }
  /* y sweep */
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < nx; ++x) {
    double(*Gh)[4] = (double(*)[4])malloc(sizeof(double) * 4 * (size_t)(ny + 1));
    for (int64_t k = 0; k <= ny; ++k) {
      double qs[6][4];
      for (int j = 0; j < 6; ++j) {
        int64_t ci = ghost_index(k - 3 + j, ny, bc);
        for (int r = 0; r < 4; ++r) qs[j][r] = q[r * cells + ci * nx + x];
      }
      uint8_t mi[4], mo[4];
      const int64_t fidx = k * nx + x;
      if (my_in)
        for (int m = 0; m < 4; ++m) mi[m] = my_in[m * nfy + fidx];
      euler2d_face(qs, gamma, 1, P, selector, my_in ? mi : NULL, Gh[k], mo);
      if (my_out)
        for (int m = 0; m < 4; ++m) my_out[m * nfy + fidx] = mo[m];
    }
    for (int64_t y = 0; y < ny; ++y)
      for (int r = 0; r < 4; ++r) {
        double b = (Gh[y][r] - Gh[y + 1][r]) / dy;
        rhs[r * cells + y * nx + x] = ax[r * cells + y * nx + x] + b;
      }
    free(Gh);
  }
  free(ax);
  return ST_OK;
}

/* n_steps SSP-RK3 steps, dt = cfl / (max(|u|+c)/dx + max(|v|+c)/dy) taken at
 * the start of every step.  A grid with a cell that is not physical gets
 * status -4 and is not advanced. */
int oracle_euler2d_step(double *q, int64_t nx, int64_t ny, double dx, double dy, double gamma,
                        int32_t bc, double cfl, int32_t n_steps, const double *P, int32_t selector,
                        double *t, int32_t *status) {
  if (nx < 1 || ny < 1 || n_steps < 0) return ST_BAD_ARG;
  const int64_t cells = nx * ny;
  const size_t sz = sizeof(double) * 4 * (size_t)cells;
  double *u1 = (double *)malloc(sz), *u2 = (double *)malloc(sz), *L = (double *)malloc(sz);
  for (int32_t it = 0; it < n_steps; ++it) {
    if (status[0] != 0) break;
    double sx = 0.0, sy = 0.0;
    for (int64_t i = 0; i < cells; ++i) {
      double qc[4] = {q[i], q[cells + i], q[2 * cells + i], q[3 * cells + i]};
      double u, v, p, c;
      prim2d(qc, gamma, &u, &v, &p, &c);
      if (!physical(qc[0], p)) {
        status[0] = ST_NONPHYSICAL;
        break;
      }
      double a = fabs(u) + c, b = fabs(v) + c;
      if (a > sx) sx = a;
      if (b > sy) sy = b;
    }
    if (status[0] != 0) break;
    double dt = cfl / (sx / dx + sy / dy);
    int32_t dummy = 0;
    oracle_euler2d_rhs(q, nx, ny, dx, dy, gamma, bc, P, selector, NULL, NULL, L, NULL, NULL, &dummy);
    for (int64_t i = 0; i < 4 * cells; ++i) u1[i] = fma(dt, L[i], q[i]);
    oracle_euler2d_rhs(u1, nx, ny, dx, dy, gamma, bc, P, selector, NULL, NULL, L, NULL, NULL, &dummy);
    for (int64_t i = 0; i < 4 * cells; ++i) {
      double tt = fma(dt, L[i], u1[i]);
      u2[i] = fma(0.25, tt, 0.75 * q[i]);
    }
    oracle_euler2d_rhs(u2, nx, ny, dx, dy, gamma, bc, P, selector, NULL, NULL, L, NULL, NULL, &dummy);
    for (int64_t i = 0; i < 4 * cells; ++i) {
      double tt = fma(dt, L[i], u2[i]);
      q[i] = fma(2.0 / 3.0, tt, (1.0 / 3.0) * q[i]);
    }
    t[0] = t[0] + dt;
  }
  free(u1);
  free(u2);
  free(L);
  return ST_OK;
}

/* ------------------------------------------------------------------------ */
/* Classifier training (Sec. 3.3): binary cross entropy averaged over the    */
/* S = 4 outputs and the mini-batch (eq. Crossentropy), Adam (Kingma & Ba).  */
/* Labels y_k = eta_k (1 = candidate crossed by a discontinuity).            */
/* ------------------------------------------------------------------------ */
static double softplus(double x) { return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x)); }
static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Loss of one sample and, if g != NULL, accumulation of scale * d(loss)/dP. */
static double sample_grad(const double *P, const double x0[6], unsigned y, double scale,
                          double *g) {
  double act[6][64];  /* act[0] = input, act[l] = post-ReLU output of layer l */
  double pre[6][64];  /* pre-activations */
  const double *Wl[5], *bl[5];
  const double *p = P;
  for (int l = 0; l < 5; ++l) {
    Wl[l] = p;
    bl[l] = p + WIDTH[l + 1] * WIDTH[l];
    p = bl[l] + WIDTH[l + 1];
  }
  for (int i = 0; i < 6; ++i) act[0][i] = x0[i];
  for (int l = 0; l < 5; ++l) {
    int nin = WIDTH[l], nout = WIDTH[l + 1];
    for (int o = 0; o < nout; ++o) {
      double acc = bl[l][o];
      for (int i = 0; i < nin; ++i) acc = fma(Wl[l][o * nin + i], act[l][i], acc);
      pre[l + 1][o] = acc;
      act[l + 1][o] = (l < 4) ? (acc > 0.0 ? acc : 0.0) : acc;
    }
  }
  double loss = 0.0;
  for (int k = 0; k < 4; ++k) {
    double z = pre[5][k];
    double yk = (double)((y >> k) & 1u);
    loss += yk * softplus(-z) + (1.0 - yk) * softplus(z);
  }
  loss = loss / 4.0;
  if (!g) return loss;
  double delta[64], dprev[64];
  for (int k = 0; k < 4; ++k) {
    double yk = (double)((y >> k) & 1u);
    delta[k] = scale * (sigmoid(pre[5][k]) - yk) / 4.0;
  }
  double *gp[5], *gb[5];
  double *q = g;
  for (int l = 0; l < 5; ++l) {
    gp[l] = q;
    gb[l] = q + WIDTH[l + 1] * WIDTH[l];
    q = gb[l] + WIDTH[l + 1];
  }
  for (int l = 4; l >= 0; --l) {
    int nin = WIDTH[l], nout = WIDTH[l + 1];
    for (int o = 0; o < nout; ++o) {
      gb[l][o] += delta[o];
      for (int i = 0; i < nin; ++i) gp[l][o * nin + i] += delta[o] * act[l][i];
    }
    if (l == 0) break;
    for (int i = 0; i < nin; ++i) {
      double acc = 0.0;
      for (int o = 0; o < nout; ++o) acc += Wl[l][o * nin + i] * delta[o];
      dprev[i] = pre[l][i] > 0.0 ? acc : 0.0;
    }
    for (int i = 0; i < nin; ++i) delta[i] = dprev[i];
  }
  return loss;
}

/* Mean loss and its gradient over n raw stencils s[n][6] (scaled here by
 * eq. normalizainput before entering the network), labels y[n] (bit k =
 * eta_k). */
int oracle_bce_grad(const double *P, const double *s, const uint8_t *y, int64_t n, double *loss,
                    double *grad) {
  if (n < 1) return ST_BAD_ARG;
  if (grad) memset(grad, 0, sizeof(double) * NPARAM);
  double acc = 0.0;
  for (int64_t e = 0; e < n; ++e) {
    double x[6];
    features(s + 6 * e, x);
    acc += sample_grad(P, x, y[e], 1.0 / (double)n, grad);
  }
  *loss = acc / (double)n;
  return ST_OK;
}

/* One Adam update: t is the step count after this update (1-based). */
static void adam(double *P, double *m, double *v, const double *g, int64_t t, double lr,
                 double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int i = 0; i < NPARAM; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    P[i] = P[i] - lr * mh / (sqrt(vh) + eps);
  }
}

/* Raw stencils s[n][6] are scaled by eq. normalizainput before entering the
 * network.  Trains over the samples idx[0..n_idx) in that order, in mini-batches of
 * `batch` (the last one may be shorter), one Adam step per mini-batch.
 * m, v: Adam moments [3228]; *t: steps taken so far (updated).
 * loss_out: mean loss over the samples, each taken before its batch's step. */
int oracle_train(double *P, double *m, double *v, int64_t *t, const double *s, const uint8_t *y,
                 const int64_t *idx, int64_t n_idx, int32_t batch, double lr, double b1, double b2,
                 double eps, double *loss_out) {
  if (n_idx < 1 || batch < 1) return ST_BAD_ARG;
  double *g = (double *)malloc(sizeof(double) * NPARAM);
  double total = 0.0;
  for (int64_t s0 = 0; s0 < n_idx; s0 += batch) {
    int64_t mb = n_idx - s0 < batch ? n_idx - s0 : batch;
    memset(g, 0, sizeof(double) * NPARAM);
    for (int64_t e = 0; e < mb; ++e) {
      int64_t i = idx[s0 + e];
      double x[6];
      features(s + 6 * i, x);
      total += sample_grad(P, x, y[i], 1.0 / (double)mb, g);
    }
    *t = *t + 1;
    adam(P, m, v, g, *t, lr, b1, b2, eps);
  }
  if (loss_out) *loss_out = total / (double)n_idx;
  free(g);
  return ST_OK;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel loops over independent problems (timing only; the
 * results do not depend on it). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
