// Internal interface of the reduced-precision (BF16 / FP16 MFMA) path and of
// the classifier trainer.  Host-side declarations only.
#pragma once

#include "neno6_internal.h"

namespace n6 {

// Scratch of the fast path, carved from the caller's workspace.
struct FastScratch {
  uint8_t *masks;       // 2D: x|y masks when the caller passes none
  uint32_t *qcount;     // [QCOUNTERS] re-checked evaluations (diagnostic): 1D
                        // spread over all slots, 2D sweep d over slots 8 d .. 8 d + 7
};

// What the fused 1D Euler pass writes (one mode per launch).
constexpr int OUT_RHS = 0;    // dst[3][cells] = -(F_{i+1/2} - F_{i-1/2}) / dx
constexpr int OUT_STAGE = 1;  // dst[3][cells] = RK3 stage `stage` from q (= u_s) and u0
constexpr int OUT_FACES = 2;  // dst[3][faces] = face fluxes
struct Out1D {
  int mode = OUT_RHS;
  int stage = 1;
  float *dst = nullptr;
  const float *u0 = nullptr;        // OUT_STAGE: state at the start of the step
  const double *dt = nullptr;       // OUT_STAGE: [lines] time step
  const int32_t *frozen = nullptr;  // OUT_STAGE: [lines] nonzero = not advanced (dst = u0)
  int32_t *status = nullptr;        // OUT_RHS: [lines] NONPHYSICAL marks, may be null
  uint8_t *masks = nullptr;         // [3][faces] final labels, may be null
  uint32_t *nrecheck = nullptr;     // re-checked evaluations (diagnostic), may be null
};

struct FastArgs {
  int equation = 0, precision = 2, selector = 0;
  const void *prepared = nullptr;
  float margin = 0.f;
  bool split = false;  // FP16 operands: two-part FP16 re-check instead of FP32
  FastScratch scr{};
  // launch shapes (0 = default): waves per workgroup of the fused kernel,
  // its workgroup cap, recheck_blocks (reserved, unused), XCD-contiguous order
  int face_waves = 0, face_blocks = 0, recheck_blocks = 0, xcd_order = 0;
  int n_cu = 256;  // compute units of the device (default grid of the 1D pass)
};

size_t fast_prepared_bytes();
const void *fast_prepared_f32(const void *prepared);
hipError_t launch_fast_prepare(const double *P, void *prepared, hipStream_t s);

// split: FP16 operands re-checked in two-part FP16 instead of FP32.
hipError_t launch_fast_logits(const void *prepared, int precision, bool split, float margin,
                              const float *sten, int64_t n, float *z, uint8_t *masks,
                              hipStream_t s);
hipError_t launch_fast_reconstruct(const void *prepared, int precision, bool split, float margin,
                                   const float *f, int64_t n_faces, int sign, int selector,
                                   const uint8_t *masks_in, float *fhat, uint8_t *masks_out,
                                   hipStream_t s);
// Clears the re-check counters at the start of an API call (afterwards each
// stage's flux-difference kernel clears them for the next stage).
hipError_t launch_fast_reset(const FastArgs &fa, hipStream_t s);
// 1D Euler: one fused pass per right-hand side -- set-up, MFMA classifier,
// in-kernel re-check of near-cutoff evaluations, combine,
// back-projection and the output of `out` (face fluxes, right-hand side or
// RK3 stage).  Advection and Burgers: face fluxes only (out.mode ==
// OUT_FACES; their flux difference is a separate kernel).
hipError_t launch_fast_pass1d(const Line1D &ln, const FastArgs &fa, const float *q,
                              const uint8_t *masks_in, const Out1D &out, hipStream_t s);
hipError_t launch_fast_faces2d(const Grid2D &g, const FastArgs &fa, const float *q,
                               const uint8_t *masks_in, uint8_t *masks_out, float *Fx, float *Gy,
                               hipStream_t s);
hipError_t launch_fast_rhs2d(const Grid2D &g, const FastArgs &fa, const float *q, float *rhs,
                             const uint8_t *masks_in, uint8_t *masks_out, int32_t *status,
                             float *Fx, float *Gy, const Stage *st, hipStream_t s);

// ---- training ----------------------------------------------------------------
// Seeded classifier-training samples first .. first+n-1 (s [n][6], y [n]).
hipError_t launch_classifier_samples(uint64_t seed, int64_t first, int64_t n, float *s, uint8_t *y,
                                     hipStream_t st);
size_t train_workspace_bytes(int32_t batch);
bool train_precision_supported(int precision);
// BF16 MFMA gradient: per-wave partials part[train_mfma_waves(m)][3228] and
// lpart; tabs: train_mfma_tab_bytes() of scratch for the operand tables.
int train_mfma_waves(int64_t m);
size_t train_mfma_tab_bytes();
hipError_t launch_grad_mfma(const double *P, void *tabs, const float *s, const uint8_t *y,
                            const int64_t *idx, int64_t m, float *part, double *lpart,
                            hipStream_t st);
hipError_t launch_train_batch(double *P, double *m, double *v, int64_t step, const float *s,
                              const uint8_t *y, const int64_t *idx, int64_t mb, double lr,
                              double b1, double b2, double eps, int precision, double *loss_out,
                              double loss_scale, bool first, void *ws, hipStream_t st);
hipError_t launch_grad(const double *P, const float *s, const uint8_t *y, int64_t n,
                       int precision, double *grad, double *loss, void *ws, hipStream_t st);

}  // namespace n6
