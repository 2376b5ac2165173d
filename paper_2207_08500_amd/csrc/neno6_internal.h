// Internal launch interface between the C-ABI layer and the kernel files.
// Host-side declarations only; each launcher enqueues on `stream` and returns
// the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace n6 {

// Re-check counters in the workspace: 2D uses one per evaluation kind
// (field * 2 + sign), eight per sweep direction (sweep d at 8 * d); 1D spreads
// its diagnostic count of re-checked evaluations over all of them.  All are
// cleared together.
constexpr int QCOUNTERS = 64;

struct Line1D {            // a batch of independent 1D lines
  const int64_t *offsets;  // [dev] cell offsets [np+1]
  const double *dx;        // [dev] spacing per line
  int32_t np;              // number of lines
  int64_t total;           // cells in all lines
  __host__ __device__ int64_t faces() const { return total + np; }
  int32_t bc;
  double gamma;
  const int32_t *fmap = nullptr;  // [dev] line of every face, or null (binary search)
};

// Fills fmap[g] = line of face g for every face of the batch.
hipError_t launch_build_fmap(const Line1D &ln, int32_t *fmap, hipStream_t s);

struct Grid2D {
  int64_t nx, ny;
  double dx, dy, gamma;
  int32_t bc;
};

// Per-step RK3 stage descriptor: which stage (1, 2, 3), the stage state u_s
// (input of the rhs), u0 (start of step), and the output buffer.
struct Stage {
  int stage;
  const void *us;
  const void *u0;
  void *out;
  const double *dt;        // [dev] per problem
  const int32_t *status;   // [dev] per problem; nonzero = frozen
};

// ---- FP64 plain path (canonical order) and FP32 vector path ---------------
// T = double or float (float: classifier on the vector units).
template <typename T>
hipError_t launch_reconstruct(const T *P, const T *f, int64_t n_faces, int sign, int selector,
                              const uint8_t *masks_in, T *fhat, uint8_t *masks_out,
                              hipStream_t s);
template <typename T>
hipError_t launch_mlp_logits(const T *P, const T *sten, int64_t n, T *z, uint8_t *masks,
                             hipStream_t s);

// Face fluxes of 1D lines: Fhat [nvar][faces], masks [nvar][faces].
template <typename T>
hipError_t launch_faces_advection(const Line1D &ln, const T *P, int selector, const T *u,
                                  const uint8_t *masks_in, T *Fhat, uint8_t *masks_out,
                                  hipStream_t s);
template <typename T>
hipError_t launch_faces_burgers(const Line1D &ln, const T *P, int selector, const T *u,
                                const uint8_t *masks_in, T *Fhat, uint8_t *masks_out,
                                hipStream_t s);
// evals: scratch of plain_eval_bytes(6, faces, sizeof(T)) bytes.
template <typename T>
hipError_t launch_faces_euler1d(const Line1D &ln, const T *P, int selector, const T *q,
                                const uint8_t *masks_in, T *Fhat, uint8_t *masks_out, void *evals,
                                hipStream_t s);
// Scratch of the plain Euler face kernels: one value and one mask per
// evaluation.
size_t plain_eval_bytes(int nevals, int64_t faces, size_t elem);
// Flux difference (and, with st != nullptr, the RK3 stage update) of 1D lines;
// writes rhs (st == nullptr) or the stage output; sets status for cells that
// are not physical when status_out != nullptr.
// zero_after (may be null): two counters the kernel clears once it has run.
template <typename T>
hipError_t launch_diff1d(const Line1D &ln, int equation, const T *Fhat, const T *q, T *rhs,
                         const Stage *st, int32_t *status_out, hipStream_t s,
                         uint32_t *zero_after = nullptr);
// Per-line time step and status check at the start of a step; t += dt.
template <typename T>
hipError_t launch_cfl1d(const Line1D &ln, int equation, const T *q, double cfl, double *dt,
                        int32_t *status, double *t, hipStream_t s,
                        uint32_t *zero_after = nullptr);

// 2D: x faces [4][ny][nx+1], y faces [4][ny+1][nx].
// evals: scratch of plain_eval_bytes(8, max(x faces, y faces), sizeof(T)).
template <typename T>
hipError_t launch_faces_euler2d(const Grid2D &g, const T *P, int selector, const T *q,
                                const uint8_t *mx_in, const uint8_t *my_in, T *Fx, T *Gy,
                                uint8_t *mx_out, uint8_t *my_out, void *evals, hipStream_t s);
template <typename T>
hipError_t launch_diff2d(const Grid2D &g, const T *Fx, const T *Gy, const T *q, T *rhs,
                         const Stage *st, int32_t *status_out, hipStream_t s,
                         uint32_t *zero_after = nullptr);
// Grid-wide time step: partial maxima in `part` (>= cfl2d_parts() doubles x 2).
int cfl2d_parts();
template <typename T>
hipError_t launch_cfl2d(const Grid2D &g, const T *q, double cfl, double *part, double *dt,
                        int32_t *status, double *t, hipStream_t s);

// Vector-Jacobian product of the 1D right-hand side (Burgers or Euler) at
// fixed labels: qbar = (d rhs / d q)^T rbar; scratch holds 6 * nvar * faces
// values.
template <typename T>
hipError_t launch_vjp1d(const Line1D &ln, int equation, const T *q, const uint8_t *masks,
                        const T *rbar, T *qbar, T *scratch, hipStream_t s);
// 2D Euler: both sweeps; scratch of 24 x (x faces + y faces) values; masks
// are the x masks [4][x faces] followed by the y masks [4][y faces].
template <typename T>
hipError_t launch_vjp2d(const Grid2D &g, const T *q, const uint8_t *masks, const T *rbar, T *qbar,
                        T *scratch, hipStream_t s);
// Fixed-mask adjoint of the advection rhs (one line).
hipError_t launch_adjoint_advection(const Line1D &ln, const uint8_t *masks, const void *rbar,
                                    void *ubar, int is_fp64, hipStream_t s);

// Mirror of the MLP parameters into FP32 (prepared block).
hipError_t launch_params_to_f32(const double *P, float *P32, hipStream_t s);

}  // namespace n6
