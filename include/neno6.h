/*
 * neno6.h -- C ABI of libneno6.so: the six-point neuron-based ENO (NENO6)
 * reconstruction of Li, Fu & Adams (arXiv 2207.08500) and the Lax-Friedrichs
 * flux-split, SSP-RK3 finite-difference solver around it, as HIP kernels for
 * gfx950 (MI355X).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers marked [dev] are device pointers, [host] host pointers.  The
 *    caller owns all memory; the library never allocates.  Scratch space is a
 *    caller-provided device workspace of at least the size the matching
 *    neno6_*_workspace_size() call returns.
 *  - All work is enqueued on `stream` and is asynchronous; nothing
 *    synchronises the device, so every call can be captured into a HIP graph.
 *    Argument errors are detected on the host and returned before anything is
 *    enqueued.  Conditions found on the device (a state that is not physical)
 *    are written to caller-provided status words, read after a sync.
 *  - Return value: NENO6_OK (0) or a negative neno6_status.
 *  - Stencil orientation (Sec. 2, eq. implicitEq / approximateEq): the face
 *    x_{i+1/2} lies between cells i and i+1.  The '+' (right-going) flux uses
 *    cells i-2..i+3 in that order; the '-' (left-going) flux uses the mirrored
 *    stencil i+3..i-2.
 *  - Candidate mask (one nibble per reconstruction): bit k set = candidate
 *    sub-stencil S_k kept (delta_k = 1, Sec. 2.2).  S0 = {i-1,i,i+1},
 *    S1 = {i,i+1,i+2}, S2 = {i-2,i-1,i}, S3 = {i,i+1,i+2,i+3}.  Mask bytes
 *    carry '+' in the low nibble and '-' in the high nibble.
 *  - Classifier parameters (Sec. 3.1, 6-64-32-16-8-4 network): one FP64 block
 *    of 3228 values, row-major [out][in]:
 *      W1[64][6] b1[64] W2[32][64] b2[32] W3[16][32] b3[16] W4[8][16] b4[8]
 *      W5[4][8] b5[4]
 *    A candidate is discarded iff its output logit is > 0 (sigmoid > 1/2).
 */
#ifndef NENO6_H
#define NENO6_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define NENO6_OK 0
#define NENO6_BAD_ARG (-1)        /* null pointer, size or enum out of range */
#define NENO6_BAD_LAYOUT (-2)     /* precision / layout combination not valid */
#define NENO6_HIP_ERROR (-3)      /* a HIP launch or API call failed */
#define NENO6_NONPHYSICAL (-4)    /* (device status word) Euler: rho <= 0, p <= 0 or NaN;
                                   * Burgers: a non-finite value */
#define NENO6_UNSUPPORTED (-5)    /* feature not available for this equation */
#define NENO6_WORKSPACE_SMALL (-6)
#define NENO6_TOO_LARGE (-7)      /* beyond a fixed limit of the library (neno6_rhs_noalloc) */

/* ---- enums ---------------------------------------------------------------- */
/* Arithmetic of state, reconstruction and classifier.
 *  FP64: plain FP64 path in the canonical operation order of the reference
 *        implementation (fma chains in index order, IEEE division and sqrt);
 *        classification labels equal the FP64 oracle's exactly.
 *  FP32: FP32 state and reconstruction, FP32 classifier on the vector units.
 *  BF16 / FP16: FP32 state and reconstruction; classifier layers on MFMA in
 *        BF16 / FP16 with FP32 accumulation; evaluations whose smallest
 *        |logit| falls below the re-check margin are re-evaluated in FP32. */
#define NENO6_FP64 0
#define NENO6_FP32 1
#define NENO6_BF16 2
#define NENO6_FP16 3

#define NENO6_ADVECTION 0 /* u_t + u_x = 0 (Sec. 4.2) */
#define NENO6_BURGERS 1   /* u_t + (u^2/2)_x = 0 (Sec. 4.3), Rusanov split with the
                           * largest |u| over the six stencil cells */
#define NENO6_EULER1D 2   /* 1D Euler, gamma-law gas (Sec. 4.4) */
#define NENO6_EULER2D 3   /* 2D Euler, dimension by dimension (Sec. 4.4) */

#define NENO6_PERIODIC 0
#define NENO6_TRANSMISSIVE 1 /* zero-gradient ghost cells */

#define NENO6_SEL_MLP 0          /* the classifier decides (Alg. 2) */
#define NENO6_SEL_ALL_SMOOTH 1   /* every candidate kept: optimal linear scheme */
#define NENO6_SEL_ALL_DISCARD 2  /* every candidate discarded: upwind fallback */
#define NENO6_SEL_MASKS_IN 3     /* masks supplied by the caller */
#define NENO6_SEL_TENO 4         /* TENO6-opt smoothness indicators and cut-off
                                  * (Sec. 2.2-2.3), decided in FP64 in every mode */

#define NENO6_NPARAM 3228

/* Re-check arithmetic (neno6_mlp.recheck_mode). */
#define NENO6_RECHECK_FP32 0   /* evaluations within the margin again in FP32 (default) */
#define NENO6_RECHECK_FP16X2 1 /* FP16 operands only: again on FP16 MFMA with every weight and
                                  activation as two FP16 parts (value + rounding remainder), FP32
                                  sums; logit error about 2.5x the FP32 re-check's.  BF16 operands
                                  are re-checked in FP32 whatever the mode. */

/* Classifier handle.  `params` is the FP64 master block [dev]; `prepared` is a
 * device buffer of neno6_mlp_prepared_bytes() bytes that neno6_mlp_prepare()
 * fills with the reduced-precision copies the kernels read.  recheck_margin is
 * in logit units (BF16/FP16 modes); 0 disables the re-check.  recheck_mode:
 * NENO6_RECHECK_FP32 or NENO6_RECHECK_FP16X2 (other values: NENO6_BAD_ARG). */
typedef struct neno6_mlp {
  const double *params;
  void *prepared;
  float recheck_margin;
  int32_t recheck_mode;
} neno6_mlp;

/* Problem description (host struct; the pointers in it are [dev]).
 *  1D (ADVECTION, EULER1D): n_problems independent lines concatenated;
 *    offsets[n_problems+1] cell offsets (device and host copies, every line
 *    at least one cell), dx[n_problems] spacings; total_cells =
 *    offsets[n_problems].
 *    State layout SoA [var][total_cells]; faces of line p are numbered
 *    offsets[p] + p + k, k = 0..N_p (face k between cells k-1 and k);
 *    mask arrays are [field][total_cells + n_problems].
 *    total_cells + n_problems < 2^29.
 *    ADVECTION uses var = field = 1 and only the '+' nibble (the '-' split
 *    flux is identically zero, so its nibble is reported as 0).  BURGERS
 *    uses var = field = 1 with both nibbles.
 *  2D (EULER2D): one nx x ny grid (nx, ny <= 2^20, nx * ny <= 2^28), SoA
 *    [4][ny][nx] (x fastest), spacings dx2d, dy2d; x-face masks
 *    [4][ny][nx+1], y-face masks [4][ny+1][nx].
 *  A batch of 2D grids (EULER2D with grids_host != NULL): n_problems grids
 *    (1..65536) of their own sizes and spacings, each within the limits
 *    above; nx, ny, dx2d, dy2d and total_cells are then ignored.  Grid p's
 *    state is its own [4][ny_p][nx_p] block, following grid p-1's (it starts
 *    at element 4 sum_{r<p} nx_r ny_r), and so are its masks and face
 *    fluxes (x then y faces of grid p after those of grid p-1); time and
 *    status arrays hold one entry per grid.  The grids run one after another
 *    on the stream, each with the launches of a single grid (so a batch is
 *    captured into a HIP graph like a single grid; for many small grids the
 *    launch count, not the GPU, sets the pace).  neno6_recheck_count and
 *    neno6_rhs_noalloc do not take batches (NENO6_UNSUPPORTED); the autotuner
 *    tunes on the grid with the most faces. */
typedef struct neno6_grid2d {
  int64_t nx, ny;
  double dx, dy;
} neno6_grid2d;
/* Launch shapes of the BF16/FP16 kernels (from neno6_autotune, or chosen by
 * hand).  Any field left 0 takes the built-in default.
 *  face_waves:     64-lane waves per workgroup of the fused face kernel
 *                  (2, 4 or 8); each wave handles 64 consecutive faces per
 *                  iteration.
 *  face_blocks:    workgroups of the fused face kernel, which loop over the
 *                  64-face tiles (grid-stride); at most 65536.
 *  recheck_blocks: reserved, 0..65536 and otherwise ignored: the re-check
 *                  runs inside the face kernels.
 *  xcd_order:      1 = number the workgroups so that each of the eight XCDs
 *                  (each with its own L2) walks a contiguous run of tiles;
 *                  needs face_blocks to be a multiple of 8 (else ignored). */
typedef struct neno6_tuning {
  int32_t face_waves;
  int32_t face_blocks;
  int32_t recheck_blocks;
  int32_t xcd_order;
} neno6_tuning;

/* neno6_problem.flags */
#define NENO6_KEEP_MAP 1 /* 1D: the workspace already holds this problem's face -> line
                          * map, built by an earlier call with the same workspace and
                          * offsets on the same stream; the call skips rebuilding it */

typedef struct neno6_problem {
  int32_t equation;
  int32_t bc;
  int32_t precision;
  int32_t selector;
  int32_t n_problems;
  int32_t flags;               /* NENO6_KEEP_MAP or 0 */
  int64_t total_cells;
  int64_t nx, ny;
  const int64_t *offsets;      /* [dev]  cell offsets, 1D */
  const int64_t *offsets_host; /* [host] the same offsets, for argument checks */
  const double *dx;            /* [dev]  spacing per line, 1D */
  double dx2d, dy2d;
  double gamma;
  const neno6_tuning *tuning;  /* [host, may be NULL] launch shapes; NULL = defaults */
  const neno6_grid2d *grids_host; /* [host] EULER2D batch: grids[n_problems]; NULL = one grid */
} neno6_problem;

/* ---- library ------------------------------------------------------------- */
const char *neno6_status_string(int32_t status);
int32_t neno6_version(void);

/* ---- classifier preparation ---------------------------------------------- */
/* Bytes of the prepared-parameter buffer. */
size_t neno6_mlp_prepared_bytes(void);

/* Converts the FP64 master block into the FP32 copy and the BF16/FP16 MFMA
 * operand tiles (round to nearest even) the kernels read.  Call again after
 * every change of params.  Sec. 3.4: the trained parameters are loaded into
 * the solver. */
int32_t neno6_mlp_prepare(const neno6_mlp *mlp, hipStream_t stream);

/* Classifier on its own (Sec. 3.1; Alg. 2 steps 1-2): for n raw six-point
 * stencils s[n][6] [dev] (FP64 when precision = FP64, else FP32), scales each
 * by eq. normalizainput and writes the four output logits z[n][4] [dev]
 * (same float type) and the kept-candidate masks[n] [dev] (may be NULL).
 * In BF16/FP16 modes z holds the reduced-precision logits, except for the
 * evaluations within the re-check margin, which hold the re-check's (FP32, or
 * two-part FP16 by recheck_mode); masks are the signs of z. */
int32_t neno6_mlp_logits(const neno6_mlp *mlp, int32_t precision, const void *s, int64_t n,
                         void *z, uint8_t *masks, hipStream_t stream);

/* ---- reconstruction ------------------------------------------------------ */
/* Scalar NENO6 reconstruction at n_faces faces (Alg. 2; eq. convex,
 * eq. TENOweight_renormalize).  f [dev] holds n_faces + 5 point values; face k
 * uses f[k..k+5] (sign = +1) or f[k+5..k] (sign = -1).  fhat[n_faces] [dev]
 * receives the face values, masks_out[n_faces] [dev, may be NULL] the kept
 * masks; masks_in is read when selector = NENO6_SEL_MASKS_IN.
 * Element type: double for FP64, float otherwise. */
int32_t neno6_reconstruct(const neno6_mlp *mlp, const void *f, int64_t n_faces, int32_t sign,
                          int32_t precision, int32_t selector, const uint8_t *masks_in,
                          void *fhat, uint8_t *masks_out, hipStream_t stream);

/* ---- right-hand side ----------------------------------------------------- */
/* Workspace bytes for neno6_rhs / neno6_step / neno6_rhs_adjoint. */
size_t neno6_workspace_size(const neno6_problem *prob);

/* Semi-discrete right-hand side du/dt = -(F_{i+1/2} - F_{i-1/2})/dx
 * (eq. approximateEq) with NENO6 face fluxes: characteristic projection with
 * Roe-averaged eigenvectors, Rusanov splitting with the largest |lambda_m|
 * over the six stencil cells, classifier per field and sign, re-normalised
 * combine, back-projection (Sec. 4.4).  q, rhs [dev] in the problem's layout
 * (double for FP64, float otherwise).  masks_in / masks_out [dev, may be
 * NULL]: for 2D pass x masks then y masks back to back in one buffer
 * ([4][ny][nx+1] followed by [4][ny+1][nx]).  status[n_problems] [dev] is
 * set to NENO6_NONPHYSICAL for a problem with a cell that is not physical
 * (it is never cleared here).
 * 1D Euler in BF16/FP16: one fused kernel computes the face fluxes, the
 * re-check of near-cutoff evaluations and the flux difference.  A face whose
 * six stencil cells are equal has a constant split stencil, whose
 * re-normalised combination is that constant for every selection; the pass
 * takes it exactly, and re-checks such a face's near-cutoff labels only when
 * masks_out is given (they cannot change any value). */
int32_t neno6_rhs(const neno6_problem *prob, const neno6_mlp *mlp, const void *q, void *rhs,
                  const uint8_t *masks_in, uint8_t *masks_out, int32_t *status, void *ws,
                  size_t ws_bytes, hipStream_t stream);

/* neno6_rhs without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): it calls no allocating routine.  1D Euler in BF16/FP16
 * only (else NENO6_UNSUPPORTED); arguments, outputs and the kernels run are
 * those of neno6_rhs.  Its scratch (the face -> line map, 4 bytes per face) is
 * a fixed array in device memory that the library owns, one per GPU, held
 * from module load until the process ends: a batch with more than
 * NENO6_NOALLOC_MAX_FACES faces (cells + problems) is refused with
 * NENO6_TOO_LARGE before anything is enqueued.  The face map is rebuilt on
 * every call (NENO6_KEEP_MAP is ignored) and no re-check counters are kept
 * (neno6_recheck_count does not see these calls).  All calls on one GPU
 * share the array: calls that can overlap on one GPU (different streams or
 * host threads without ordering) race and must be serialised by the caller.
 * The current device must be the one that q, rhs and stream belong to. */
#define NENO6_NOALLOC_MAX_FACES ((int64_t)16 * 1024 * 1024)
int32_t neno6_rhs_noalloc(const neno6_problem *prob, const neno6_mlp *mlp, const void *q,
                          void *rhs, const uint8_t *masks_in, uint8_t *masks_out, int32_t *status,
                          hipStream_t stream);

/* Face fluxes only (the reconstruction of Alg. 2 at every face of the
 * problem, without the flux difference): F [dev] receives the face fluxes
 * ([var][faces] for 1D; x faces then y faces for 2D) and masks_out [dev, may
 * be NULL] the kept masks.  In BF16/FP16 modes this launches exactly the fused
 * classifier kernel (1D: the same kernel as neno6_rhs and neno6_step, writing
 * face fluxes instead of cells; the re-check is skipped when the margin
 * is 0); it exists so that kernel can be timed on its own. */
int32_t neno6_face_fluxes(const neno6_problem *prob, const neno6_mlp *mlp, const void *q, void *F,
                          uint8_t *masks_out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Diagnostic (synchronous: waits for `stream`): after neno6_face_fluxes or
 * neno6_rhs in BF16/FP16 mode with `mlp`, the number of classifier
 * evaluations of each sweep direction (count[0]: 1D or x, count[1]: y) that
 * were re-checked (0 when mlp's margin is 0: the re-check does not
 * run and its counters are not maintained).  1D: the pass works in tiles of
 * 64 faces that overlap by one face, so an overlap face's evaluations are
 * counted by both tiles; without masks_out the near-cutoff evaluations of
 * faces with six equal cells are not re-checked (see neno6_rhs).
 * count [host, 2 values]. */
int32_t neno6_recheck_count(const neno6_problem *prob, const neno6_mlp *mlp, const void *ws,
                            size_t ws_bytes, uint32_t *count, hipStream_t stream);

/* Autotuner (host-synchronous, not for graph capture): times the fused
 * face pass of `prob` (1D: the fused kernel with its in-pass re-check; 2D:
 * both sweeps of the sweep kernel with its in-tile re-check) on state q [dev]
 * for every launch shape of a candidate set -- waves per workgroup W in
 * {2, 4, 8} (2D: {4, 8}) x workgroup caps {16384, 65536, and k rounds of
 * resident workgroups for k = 1, 2, 3, 4, 6 (on the current device: 12 / W
 * workgroups per CU in 1D, one of eight waves; 8 / W in 2D)} x XCD ordering
 * {0, 1} -- with HIP events on `stream`, after about
 * 0.1 s of warm-up passes in the default shape, `reps` (1..1000) timed
 * passes each after one warm-up, and writes the fastest to *best [host] (its mean pass
 * time in ms to *best_ms [host], may be NULL).  Outputs of the passes land in
 * the workspace only; prob->tuning is ignored.  Euler problems in BF16 /
 * FP16 with SEL_MLP; NENO6_UNSUPPORTED otherwise. */
int32_t neno6_autotune(const neno6_problem *prob, const neno6_mlp *mlp, const void *q, void *ws,
                       size_t ws_bytes, int32_t reps, neno6_tuning *best, float *best_ms,
                       hipStream_t stream);

/* ---- time stepping -------------------------------------------------------- */
/* n_steps SSP-RK3 steps (Sec. 4.4), in place on q [dev].  Each step first
 * takes every problem's time step from its current state --
 * 1D: dt = cfl dx / max(|u| + c); 2D: dt = cfl / (max(|u|+c)/dx + max(|v|+c)/dy);
 * advection: dt = cfl dx (unit speed); Burgers: dt = cfl dx / max|u| (cfl dx
 * when u is identically 0) -- and advances only problems whose
 * status word is 0; a problem whose state is not physical at that point gets
 * NENO6_NONPHYSICAL and stays frozen.  t[n_problems] [dev, FP64] advances by
 * the dt taken.  status [dev]: one int32 per problem (one 2D grid: one; a
 * batch of 2D grids: one per grid). */
int32_t neno6_step(const neno6_problem *prob, const neno6_mlp *mlp, void *q, double cfl,
                   int32_t n_steps, double *t, int32_t *status, void *ws, size_t ws_bytes,
                   hipStream_t stream);

/* ---- differentiation ------------------------------------------------------ */
/* Adjoint of the advection right-hand side (eq. approximateEq with the
 * reconstruction of eq. convex / eq. TENOweight_renormalize, Sec. 4.2) with
 * respect to u at fixed masks: once the selection is fixed the map u -> rhs
 * is linear, rhs = A u, and this returns ubar = A^T rbar.
 * masks [dev] as returned by neno6_rhs; rbar, ubar [dev] [total_cells].
 * Only NENO6_ADVECTION, one line. */
int32_t neno6_rhs_adjoint(const neno6_problem *prob, const uint8_t *masks, const void *rbar,
                          void *ubar, hipStream_t stream);

/* Vector-Jacobian product of the BURGERS, EULER1D or EULER2D right-hand side
 * at state q with the labels held fixed: qbar = (d rhs / d q)^T rbar,
 * differentiating the physical flux, the Roe average and eigenvectors (2D: in
 * each sweep's normal/shear frame), the Rusanov speed (the max over the six
 * stencil cells, into the cell that attains it) and the split; the labels
 * masks [dev] (as returned by neno6_rhs; 2D: the x-face masks followed by the
 * y-face masks) select the fixed combination weights (eq.
 * TENOweight_renormalize).  q, rbar, qbar [dev] in the state layout, FP64 or
 * FP32 (the problem's precision must be FP64 or FP32).  ws [dev] of
 * neno6_vjp_workspace_size(prob) bytes.  Deterministic: each cell sums its
 * face contributions in a fixed order.  The map is not differentiable where
 * two cells tie for the Rusanov speed; there the first cell in stencil order
 * takes the derivative.  NENO6_UNSUPPORTED for ADVECTION (neno6_rhs_adjoint). */
size_t neno6_vjp_workspace_size(const neno6_problem *prob);
int32_t neno6_rhs_vjp(const neno6_problem *prob, const void *q, const uint8_t *masks,
                      const void *rbar, void *qbar, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* ---- classifier training (Sec. 3.3) ---------------------------------------- */
/* Workspace bytes for training with mini-batches of `batch` samples. */
/* Seeded synthetic training samples, generated on the device: the
 * six-point stencils f(x_c + (j - 2) dx), j = 0..5, of smooth functions
 * (polynomials of degree <= 5, sines with amplitude 1e-2..1e2) and of
 * functions with a step or a kink (jump ratio 1e-3..1e3), with the label of
 * each candidate sub-stencil (bit k set: candidate k crosses the jump) --
 * the kind of data the classifier of Sec. 3.2 is trained on, N in
 * {50, 100, 200} at 40/40/20 % as in Alg. 1.  Sample i depends only on
 * (seed, i) (Philox4x32-10 counters), so any range can be generated in
 * pieces.  s [dev, n x 6 FP32], y [dev, n bytes]; first >= 0, n >= 0.
 * Returns NENO6_BAD_ARG for null buffers with n > 0 or negative sizes. */
int32_t neno6_classifier_samples(uint64_t seed, int64_t first, int64_t n, float *s, uint8_t *y,
                                 hipStream_t stream);

size_t neno6_train_workspace_size(int32_t batch);

/* Adam on the binary cross entropy averaged over the four outputs and the
 * mini-batch (eq. Crossentropy).  Trains over samples idx[0..n_idx) [dev,
 * int64] in that order, in mini-batches of `batch` (the last may be shorter),
 * one Adam step each.  s[n][6] [dev, FP32] raw stencils (scaled inside by
 * eq. normalizainput), y[n] [dev] labels (bit k = 1: candidate k crossed by a
 * discontinuity).  params[3228], adam_m, adam_v [dev, FP64] are updated in
 * place; step [host] is the Adam step count (incremented per mini-batch).
 * precision: FP32 (vector units) or BF16 (MFMA, FP32 accumulation).
 * Forward activations are recomputed in the backward pass, not stored.
 * loss_out [dev, FP64, may be NULL] receives the mean loss over the samples,
 * each evaluated before its mini-batch's update. */
int32_t neno6_classifier_train(double *params, double *adam_m, double *adam_v, int64_t *step,
                               const float *s, const uint8_t *y, const int64_t *idx, int64_t n_idx,
                               int32_t batch, double lr, double beta1, double beta2, double eps,
                               int32_t precision, double *loss_out, void *ws, size_t ws_bytes,
                               hipStream_t stream);

/* Gradient of the mean loss over samples s[n][6], y[n] [dev] into grad[3228]
 * [dev, FP64] and the mean loss into *loss [dev, FP64] (the backward pass on
 * its own, for the autograd binding and for checking against the oracle). */
int32_t neno6_classifier_grad(const double *params, const float *s, const uint8_t *y, int64_t n,
                              int32_t precision, double *grad, double *loss, void *ws,
                              size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* NENO6_H */
