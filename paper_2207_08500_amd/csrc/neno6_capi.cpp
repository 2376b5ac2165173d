// C-ABI entry points of libneno6.so: argument checks, workspace carving and
// the launch sequence of each call.  All numerical work is in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/neno6.h"
#include "neno6_fast.h"
#include "neno6_internal.h"

using namespace n6;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// Bump allocator over the caller's workspace.
struct Carve {
  char *base;
  size_t used = 0;
  template <typename T> T *take(size_t n) {
    T *p = base ? (T *)(base + used) : nullptr;
    used = align_up(used + n * sizeof(T));
    return p;
  }
};

inline int32_t hip_status(hipError_t e) { return e == hipSuccess ? NENO6_OK : NENO6_HIP_ERROR; }

bool valid_precision(int32_t p) { return p >= NENO6_FP64 && p <= NENO6_FP16; }
bool valid_selector(int32_t s) { return s >= NENO6_SEL_MLP && s <= NENO6_SEL_TENO; }

int32_t check_mlp(const neno6_mlp *mlp, int32_t selector, int32_t precision) {
  if (selector != NENO6_SEL_MLP) return NENO6_OK;
  if (!mlp || !mlp->params) return NENO6_BAD_ARG;
  if (precision != NENO6_FP64 && !mlp->prepared) return NENO6_BAD_ARG;
  if (mlp->recheck_mode != NENO6_RECHECK_FP32 && mlp->recheck_mode != NENO6_RECHECK_FP16X2)
    return NENO6_BAD_ARG;
  return NENO6_OK;
}

// The two-part FP16 re-check applies to FP16 operands only.
bool split_recheck(const neno6_mlp *mlp, int32_t precision) {
  return mlp && precision == NENO6_FP16 && mlp->recheck_mode == NENO6_RECHECK_FP16X2;
}

int nvar_of(int32_t eq) { return eq <= NENO6_BURGERS ? 1 : (eq == NENO6_EULER1D ? 3 : 4); }

int32_t check_tuning(const neno6_tuning *t) {
  if (!t) return NENO6_OK;
  if (t->face_waves != 0 && t->face_waves != 2 && t->face_waves != 4 && t->face_waves != 8)
    return NENO6_BAD_ARG;
  if (t->face_blocks < 0 || t->face_blocks > 65536) return NENO6_BAD_ARG;
  if (t->recheck_blocks < 0 || t->recheck_blocks > 65536) return NENO6_BAD_ARG;
  if (t->xcd_order != 0 && t->xcd_order != 1) return NENO6_BAD_ARG;
  return NENO6_OK;
}

int32_t check_problem(const neno6_problem *pb) {
  if (!pb) return NENO6_BAD_ARG;
  if (pb->flags & ~NENO6_KEEP_MAP) return NENO6_BAD_ARG;
  if (int32_t c = check_tuning(pb->tuning)) return c;
  if (pb->equation != NENO6_ADVECTION && pb->equation != NENO6_BURGERS &&
      pb->equation != NENO6_EULER1D && pb->equation != NENO6_EULER2D)
    return NENO6_BAD_ARG;
  if (pb->bc != NENO6_PERIODIC && pb->bc != NENO6_TRANSMISSIVE) return NENO6_BAD_ARG;
  if (!valid_precision(pb->precision) || !valid_selector(pb->selector)) return NENO6_BAD_ARG;
  if (pb->equation == NENO6_EULER2D) {
    if (pb->nx < 1 || pb->ny < 1 || !(pb->dx2d > 0) || !(pb->dy2d > 0) || !(pb->gamma > 1))
      return NENO6_BAD_ARG;
    if (pb->nx > (1 << 20) || pb->ny > (1 << 20) || pb->nx * pb->ny > (int64_t(1) << 28))
      return NENO6_BAD_ARG;  // in-grid indices are 32-bit
    return NENO6_OK;
  }
  if (pb->n_problems < 1 || !pb->offsets || !pb->offsets_host || !pb->dx) return NENO6_BAD_ARG;
  // face indices packed with an evaluation index stay within 32 bits
  if (pb->total_cells < 1 || pb->total_cells + pb->n_problems >= (int64_t(1) << 29))
    return NENO6_BAD_ARG;
  if (pb->offsets_host[0] != 0 || pb->offsets_host[pb->n_problems] != pb->total_cells)
    return NENO6_BAD_ARG;
  for (int32_t p = 0; p < pb->n_problems; ++p)
    if (pb->offsets_host[p + 1] <= pb->offsets_host[p]) return NENO6_BAD_ARG;
  if (pb->equation == NENO6_EULER1D && !(pb->gamma > 1)) return NENO6_BAD_ARG;
  return NENO6_OK;
}

Line1D line_of(const neno6_problem *pb, const int32_t *fmap = nullptr) {
  Line1D ln;
  ln.fmap = fmap;
  ln.offsets = pb->offsets;
  ln.dx = pb->dx;
  ln.np = pb->n_problems;
  ln.total = pb->total_cells;
  ln.bc = pb->bc;
  ln.gamma = pb->gamma;
  return ln;
}

Grid2D grid_of(const neno6_problem *pb) {
  Grid2D g;
  g.nx = pb->nx;
  g.ny = pb->ny;
  g.dx = pb->dx2d;
  g.dy = pb->dy2d;
  g.gamma = pb->gamma;
  g.bc = pb->bc;
  return g;
}

size_t elem_size(int32_t prec) { return prec == NENO6_FP64 ? sizeof(double) : sizeof(float); }

// Workspace layout (same carving for size query and use).
struct Work {
  void *F = nullptr, *G = nullptr;  // face fluxes (1D: F only)
  void *u1 = nullptr, *u2 = nullptr;
  double *dt = nullptr, *part = nullptr;
  int32_t *dummy_status = nullptr;
  int32_t *fmap = nullptr;          // 1D: line of every face
  void *evals = nullptr;            // FP64/FP32 Euler: value and mask per evaluation
  FastScratch scr{};                // reduced-precision path only
  size_t bytes = 0;
};

Work carve_work(const neno6_problem *pb, void *ws) {
  Carve c{(char *)ws};
  Work w;
  const size_t es = elem_size(pb->precision);
  const int nv = nvar_of(pb->equation);
  if (pb->equation == NENO6_EULER2D) {
    const size_t cells = (size_t)pb->nx * pb->ny;
    w.F = c.take<char>(es * 4 * (size_t)(pb->nx + 1) * pb->ny);
    w.G = c.take<char>(es * 4 * (size_t)pb->nx * (pb->ny + 1));
    w.u1 = c.take<char>(es * 4 * cells);
    w.u2 = c.take<char>(es * 4 * cells);
    w.dt = c.take<double>(1);
    w.part = c.take<double>(3 * (size_t)cfl2d_parts());
    w.dummy_status = c.take<int32_t>(1);
  } else {
    const size_t faces = (size_t)pb->total_cells + pb->n_problems;
    w.F = c.take<char>(es * nv * faces);
    w.u1 = c.take<char>(es * nv * (size_t)pb->total_cells);
    w.u2 = c.take<char>(es * nv * (size_t)pb->total_cells);
    w.dt = c.take<double>(pb->n_problems);
    w.dummy_status = c.take<int32_t>(pb->n_problems);
    w.fmap = c.take<int32_t>(faces);
  }
  if (pb->precision <= NENO6_FP32 && pb->equation >= NENO6_EULER1D) {
    const int64_t nf = pb->equation == NENO6_EULER2D
                           ? std::max((pb->nx + 1) * pb->ny, pb->nx * (pb->ny + 1))
                           : pb->total_cells + pb->n_problems;
    w.evals = c.take<char>(plain_eval_bytes(pb->equation == NENO6_EULER2D ? 8 : 6, nf, es));
  }
  if (pb->precision >= NENO6_BF16 && pb->equation == NENO6_EULER2D) {
    // masks of the x and y faces and the re-check counters
    const size_t faces = (size_t)(pb->nx + 1) * pb->ny + (size_t)pb->nx * (pb->ny + 1);
    w.scr.masks = c.take<uint8_t>(4 * faces);
    w.scr.qcount = c.take<uint32_t>(QCOUNTERS);
  } else if (pb->precision >= NENO6_BF16) {
    // 1D: the re-check runs inside the face pass; only its diagnostic counter
    w.scr.qcount = c.take<uint32_t>(QCOUNTERS);
  }
  w.bytes = c.used;
  return w;
}

// Face fluxes + flux difference (+ optional RK3 stage) for one state.
template <typename T>
int32_t rhs_impl(const neno6_problem *pb, const T *P, const void *q, void *rhs,
                 const uint8_t *masks_in, uint8_t *masks_out, int32_t *status, const Work &w,
                 const Stage *st, hipStream_t s) {
  hipError_t e;
  if (pb->equation == NENO6_EULER2D) {
    const Grid2D g = grid_of(pb);
    const size_t nfx = 4 * (size_t)(g.nx + 1) * g.ny;
    e = launch_faces_euler2d<T>(g, P, pb->selector, (const T *)q, masks_in,
                                masks_in ? masks_in + nfx : nullptr, (T *)w.F, (T *)w.G, masks_out,
                                masks_out ? masks_out + nfx : nullptr, w.evals, s);
    if (e != hipSuccess) return NENO6_HIP_ERROR;
    e = launch_diff2d<T>(g, (const T *)w.F, (const T *)w.G, (const T *)q, (T *)rhs, st, status, s);
    return hip_status(e);
  }
  const Line1D ln = line_of(pb, w.fmap);
  if (pb->equation == NENO6_ADVECTION)
    e = launch_faces_advection<T>(ln, P, pb->selector, (const T *)q, masks_in, (T *)w.F,
                                  masks_out, s);
  else if (pb->equation == NENO6_BURGERS)
    e = launch_faces_burgers<T>(ln, P, pb->selector, (const T *)q, masks_in, (T *)w.F, masks_out,
                                s);
  else
    e = launch_faces_euler1d<T>(ln, P, pb->selector, (const T *)q, masks_in, (T *)w.F, masks_out,
                                w.evals, s);
  if (e != hipSuccess) return NENO6_HIP_ERROR;
  e = launch_diff1d<T>(ln, pb->equation, (const T *)w.F, (const T *)q, (T *)rhs, st,
                       status, s);
  return hip_status(e);
}

// Compute units of the current device (queried once per device; 256 if the
// query fails).
int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int n = 0;
    cus[dev] = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0
                   ? n
                   : 256;
  }
  return cus[dev];
}

FastArgs fast_args(const neno6_problem *pb, const neno6_mlp *mlp, const Work &w) {
  FastArgs fa;
  fa.n_cu = device_cus();
  fa.equation = pb->equation;
  fa.precision = pb->precision;
  fa.selector = pb->selector;
  fa.prepared = mlp ? mlp->prepared : nullptr;
  fa.margin = mlp ? mlp->recheck_margin : 0.f;
  fa.split = split_recheck(mlp, pb->precision);
  fa.scr = w.scr;
  if (const neno6_tuning *t = pb->tuning) {
    fa.face_waves = t->face_waves;
    fa.face_blocks = t->face_blocks;
    fa.recheck_blocks = t->recheck_blocks;
    fa.xcd_order = t->xcd_order;
  }
  return fa;
}

// Per-call setup enqueued before the first kernel of an entry point: the
// face -> line map of a 1D batch and the re-check counters.
// (reset_counters = false: the call's first kernel clears the counters itself.)
int32_t begin_call(const neno6_problem *pb, const neno6_mlp *mlp, const Work &w, hipStream_t s,
                   bool reset_counters = true) {
  if (pb->equation != NENO6_EULER2D && !(pb->flags & NENO6_KEEP_MAP) &&
      launch_build_fmap(line_of(pb), w.fmap, s) != hipSuccess)
    return NENO6_HIP_ERROR;
  if (reset_counters && pb->precision >= NENO6_BF16 &&
      launch_fast_reset(fast_args(pb, mlp, w), s) != hipSuccess)
    return NENO6_HIP_ERROR;
  return NENO6_OK;
}

const float *prepared_f32(const neno6_mlp *mlp) {
  return mlp ? (const float *)fast_prepared_f32(mlp->prepared) : nullptr;
}

// Dispatch one right-hand side evaluation in the problem's precision.
int32_t rhs_dispatch(const neno6_problem *pb, const neno6_mlp *mlp, const void *q, void *rhs,
                     const uint8_t *masks_in, uint8_t *masks_out, int32_t *status, const Work &w,
                     const Stage *st, hipStream_t s) {
  switch (pb->precision) {
  case NENO6_FP64:
    return rhs_impl<double>(pb, mlp ? mlp->params : nullptr, q, rhs, masks_in, masks_out, status,
                            w, st, s);
  case NENO6_FP32:
    return rhs_impl<float>(pb, prepared_f32(mlp), q, rhs, masks_in, masks_out, status, w, st, s);
  default: {
    const FastArgs fa = fast_args(pb, mlp, w);
    if (pb->equation == NENO6_EULER2D) {
      const Grid2D g = grid_of(pb);
      return hip_status(launch_fast_rhs2d(g, fa, (const float *)q, (float *)rhs, masks_in,
                                          masks_out, status, (float *)w.F, (float *)w.G, st, s));
    }
    const Line1D ln = line_of(pb, w.fmap);
    Out1D out;
    out.masks = masks_out;
    if (pb->equation != NENO6_EULER1D) {  // scalar laws: face fluxes, then their difference
      out.mode = OUT_FACES;
      out.dst = (float *)w.F;
      hipError_t e = launch_fast_pass1d(ln, fa, (const float *)q, masks_in, out, s);
      if (e != hipSuccess) return NENO6_HIP_ERROR;
      return hip_status(launch_diff1d<float>(ln, pb->equation, (const float *)w.F, (const float *)q,
                                             (float *)rhs, st, status, s));
    }
    if (st) {
      out.mode = OUT_STAGE;
      out.stage = st->stage;
      out.dst = (float *)st->out;
      out.u0 = (const float *)st->u0;
      out.dt = st->dt;
      out.frozen = st->status;
    } else {
      out.mode = OUT_RHS;
      out.dst = (float *)rhs;
      out.status = status;
      out.nrecheck = w.scr.qcount;
    }
    return hip_status(launch_fast_pass1d(ln, fa, (const float *)q, masks_in, out, s));
  }
  }
}

// Scratch of neno6_rhs_noalloc: library-owned device memory for the face ->
// line map of a 1D batch (4 bytes per face), so that entry point allocates
// nothing.  Each GPU holds its own copy from module load until the process
// ends; calls on one GPU share it.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)NENO6_NOALLOC_MAX_FACES * sizeof(int32_t);
static_assert(NENO6_NOALLOC_MAX_FACES == 16777216, "status string states the limit");
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on the current device: looked up with
// hipGetSymbolAddress once per device (with that device current) and kept.
// The array's name is only a host-side handle; kernels and copies get this
// address.
int32_t noalloc_scratch(void **out) {
  constexpr int MAX_DEVICES = 64;
  static std::mutex mu;
  static void *addr[MAX_DEVICES] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return NENO6_HIP_ERROR;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NENO6_HIP_ERROR;
    addr[dev] = p;
  }
  *out = addr[dev];
  return NENO6_OK;
}

// ---- batches of 2D grids ------------------------------------------------------
// A 2D problem with grids_host runs its grids one after another on the
// stream, each as a one-grid problem; grid p's state, masks and face fluxes
// follow grid p-1's.
bool is_batch2d(const neno6_problem *pb) {
  return pb && pb->equation == NENO6_EULER2D && pb->grids_host;
}

neno6_problem grid_problem(const neno6_problem *pb, int32_t p) {
  neno6_problem s = *pb;
  const neno6_grid2d &g = pb->grids_host[p];
  s.n_problems = 1;
  s.nx = g.nx;
  s.ny = g.ny;
  s.dx2d = g.dx;
  s.dy2d = g.dy;
  s.total_cells = g.nx * g.ny;
  s.grids_host = nullptr;
  return s;
}

int32_t check_batch2d(const neno6_problem *pb) {
  if (pb->n_problems < 1 || pb->n_problems > 65536) return NENO6_BAD_ARG;
  for (int32_t p = 0; p < pb->n_problems; ++p) {
    const neno6_problem s = grid_problem(pb, p);
    if (int32_t c = check_problem(&s)) return c;
  }
  return NENO6_OK;
}

// Walks the grids of a batch: for each, f(sub-problem, p, cells before it,
// faces (x + y) before it); stops at the first error.
template <typename Fn>
int32_t for_each_grid(const neno6_problem *pb, Fn f) {
  if (int32_t c = check_batch2d(pb)) return c;
  int64_t cells = 0, faces = 0;
  for (int32_t p = 0; p < pb->n_problems; ++p) {
    const neno6_problem s = grid_problem(pb, p);
    if (int32_t c = f(s, p, cells, faces)) return c;
    cells += s.nx * s.ny;
    faces += (s.nx + 1) * s.ny + s.nx * (s.ny + 1);
  }
  return NENO6_OK;
}

template <typename T> T *at(T *base, int64_t offset) { return base ? base + offset : nullptr; }
inline const char *at_elems(const void *b, int64_t n, size_t es) {
  return b ? (const char *)b + n * (int64_t)es : nullptr;
}
inline char *at_elems(void *b, int64_t n, size_t es) { return b ? (char *)b + n * (int64_t)es : nullptr; }

}  // namespace

extern "C" {

const char *neno6_status_string(int32_t st) {
  switch (st) {
  case NENO6_OK: return "ok";
  case NENO6_BAD_ARG: return "bad argument";
  case NENO6_BAD_LAYOUT: return "precision/layout combination not valid";
  case NENO6_HIP_ERROR: return "HIP error";
  case NENO6_NONPHYSICAL: return "state not physical (rho <= 0, p <= 0 or not finite)";
  case NENO6_UNSUPPORTED: return "unsupported for this equation or precision";
  case NENO6_WORKSPACE_SMALL: return "workspace too small";
  case NENO6_TOO_LARGE:
    return "problem too large for the library's static scratch (neno6_rhs_noalloc: at most "
           "16777216 faces)";
  default: return "unknown status";
  }
}

int32_t neno6_version(void) { return 10000; }

size_t neno6_mlp_prepared_bytes(void) { return fast_prepared_bytes(); }

int32_t neno6_mlp_prepare(const neno6_mlp *mlp, hipStream_t stream) {
  if (!mlp || !mlp->params || !mlp->prepared) return NENO6_BAD_ARG;
  return hip_status(launch_fast_prepare(mlp->params, mlp->prepared, stream));
}

int32_t neno6_mlp_logits(const neno6_mlp *mlp, int32_t precision, const void *s, int64_t n,
                         void *z, uint8_t *masks, hipStream_t stream) {
  if (!valid_precision(precision) || n < 0 || (n > 0 && (!s || !z))) return NENO6_BAD_ARG;
  if (int32_t c = check_mlp(mlp, NENO6_SEL_MLP, precision)) return c;
  switch (precision) {
  case NENO6_FP64:
    return hip_status(launch_mlp_logits<double>(mlp->params, (const double *)s, n, (double *)z,
                                                masks, stream));
  case NENO6_FP32:
    return hip_status(launch_mlp_logits<float>(prepared_f32(mlp), (const float *)s, n, (float *)z,
                                               masks, stream));
  default:
    return hip_status(launch_fast_logits(mlp->prepared, precision, split_recheck(mlp, precision),
                                         mlp->recheck_margin,
                                         (const float *)s, n, (float *)z, masks, stream));
  }
}

int32_t neno6_reconstruct(const neno6_mlp *mlp, const void *f, int64_t n_faces, int32_t sign,
                          int32_t precision, int32_t selector, const uint8_t *masks_in,
                          void *fhat, uint8_t *masks_out, hipStream_t stream) {
  if (!valid_precision(precision) || !valid_selector(selector) || n_faces < 0 ||
      (sign != 1 && sign != -1))
    return NENO6_BAD_ARG;
  if (n_faces > 0 && (!f || !fhat)) return NENO6_BAD_ARG;
  if (selector == NENO6_SEL_MASKS_IN && !masks_in) return NENO6_BAD_ARG;
  if (int32_t c = check_mlp(mlp, selector, precision)) return c;
  switch (precision) {
  case NENO6_FP64:
    return hip_status(launch_reconstruct<double>(mlp ? mlp->params : nullptr, (const double *)f,
                                                 n_faces, sign, selector, masks_in,
                                                 (double *)fhat, masks_out, stream));
  case NENO6_FP32:
    return hip_status(launch_reconstruct<float>(prepared_f32(mlp), (const float *)f, n_faces, sign,
                                                selector, masks_in, (float *)fhat, masks_out,
                                                stream));
  default:
    return hip_status(launch_fast_reconstruct(mlp ? mlp->prepared : nullptr, precision,
                                              split_recheck(mlp, precision),
                                              mlp ? mlp->recheck_margin : 0.f, (const float *)f,
                                              n_faces, sign, selector, masks_in, (float *)fhat,
                                              masks_out, stream));
  }
}

size_t neno6_workspace_size(const neno6_problem *prob) {
  if (is_batch2d(prob)) {  // the largest grid's: the grids run one after another
    size_t most = 0;
    const int32_t c = for_each_grid(prob, [&](const neno6_problem &s, int32_t, int64_t, int64_t) {
      most = std::max(most, neno6_workspace_size(&s));
      return NENO6_OK;
    });
    return c == NENO6_OK ? most : 0;
  }
  if (check_problem(prob) != NENO6_OK) return 0;
  return carve_work(prob, nullptr).bytes;
}

int32_t neno6_rhs(const neno6_problem *prob, const neno6_mlp *mlp, const void *q, void *rhs,
                  const uint8_t *masks_in, uint8_t *masks_out, int32_t *status, void *ws,
                  size_t ws_bytes, hipStream_t stream) {
  if (is_batch2d(prob)) {
    if (!q || !rhs) return NENO6_BAD_ARG;
    const size_t es = elem_size(prob->precision);
    return for_each_grid(prob, [&](const neno6_problem &s, int32_t p, int64_t cells, int64_t faces) {
      return neno6_rhs(&s, mlp, at_elems(q, 4 * cells, es), at_elems(rhs, 4 * cells, es),
                       at(masks_in, 4 * faces), at(masks_out, 4 * faces), at(status, p), ws, ws_bytes,
                       stream);
    });
  }
  if (int32_t c = check_problem(prob)) return c;
  if (int32_t c = check_mlp(mlp, prob->selector, prob->precision)) return c;
  if (!q || !rhs || !ws) return NENO6_BAD_ARG;
  if (prob->selector == NENO6_SEL_MASKS_IN && !masks_in) return NENO6_BAD_ARG;
  const Work w = carve_work(prob, ws);
  if (ws_bytes < w.bytes) return NENO6_WORKSPACE_SMALL;
  if (int32_t c = begin_call(prob, mlp, w, stream)) return c;
  return rhs_dispatch(prob, mlp, q, rhs, masks_in, masks_out, status, w, nullptr, stream);
}

int32_t neno6_rhs_noalloc(const neno6_problem *prob, const neno6_mlp *mlp, const void *q,
                          void *rhs, const uint8_t *masks_in, uint8_t *masks_out, int32_t *status,
                          hipStream_t stream) {
  if (is_batch2d(prob)) return NENO6_UNSUPPORTED;
  if (int32_t c = check_problem(prob)) return c;
  if (int32_t c = check_mlp(mlp, prob->selector, prob->precision)) return c;
  if (prob->equation != NENO6_EULER1D || prob->precision < NENO6_BF16) return NENO6_UNSUPPORTED;
  if (!q || !rhs) return NENO6_BAD_ARG;
  if (prob->selector == NENO6_SEL_MASKS_IN && !masks_in) return NENO6_BAD_ARG;
  if (prob->total_cells + prob->n_problems > NENO6_NOALLOC_MAX_FACES) return NENO6_TOO_LARGE;
  void *base = nullptr;
  if (int32_t c = noalloc_scratch(&base)) return c;
  // the face map is the only scratch; no re-check counters are kept
  Work w;
  w.fmap = (int32_t *)base;
  // another call may have left another batch's map: always rebuild it
  neno6_problem pb = *prob;
  pb.flags &= ~NENO6_KEEP_MAP;
  if (int32_t c = begin_call(&pb, mlp, w, stream)) return c;
  return rhs_dispatch(&pb, mlp, q, rhs, masks_in, masks_out, status, w, nullptr, stream);
}

int32_t neno6_face_fluxes(const neno6_problem *prob, const neno6_mlp *mlp, const void *q, void *F,
                          uint8_t *masks_out, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (is_batch2d(prob)) {
    if (!q || !F) return NENO6_BAD_ARG;
    const size_t es = elem_size(prob->precision);
    return for_each_grid(prob, [&](const neno6_problem &s, int32_t, int64_t cells, int64_t faces) {
      return neno6_face_fluxes(&s, mlp, at_elems(q, 4 * cells, es), at_elems(F, 4 * faces, es),
                               at(masks_out, 4 * faces), ws, ws_bytes, stream);
    });
  }
  if (int32_t c = check_problem(prob)) return c;
  if (int32_t c = check_mlp(mlp, prob->selector, prob->precision)) return c;
  if (prob->selector == NENO6_SEL_MASKS_IN) return NENO6_UNSUPPORTED;
  if (!q || !F || !ws) return NENO6_BAD_ARG;
  const Work w = carve_work(prob, ws);
  if (ws_bytes < w.bytes) return NENO6_WORKSPACE_SMALL;
  if (int32_t c = begin_call(prob, mlp, w, stream)) return c;
  const bool is2d = prob->equation == NENO6_EULER2D;
  const size_t nfx = is2d ? 4 * (size_t)(prob->nx + 1) * prob->ny : 0;
  hipError_t e;
  if (prob->precision >= NENO6_BF16) {
    const FastArgs fa = fast_args(prob, mlp, w);
    if (is2d) {
      e = launch_fast_faces2d(grid_of(prob), fa, (const float *)q, nullptr, masks_out, (float *)F,
                              (float *)F + nfx, stream);
    } else {
      Out1D out;
      out.mode = OUT_FACES;
      out.dst = (float *)F;
      out.masks = masks_out;
      out.nrecheck = w.scr.qcount;
      e = launch_fast_pass1d(line_of(prob, w.fmap), fa, (const float *)q, nullptr, out, stream);
    }
    return hip_status(e);
  }
  const int nv = nvar_of(prob->equation);
  const uint8_t *mx = nullptr;
  if (prob->precision == NENO6_FP64) {
    const double *P = mlp ? mlp->params : nullptr;
    if (is2d)
      e = launch_faces_euler2d<double>(grid_of(prob), P, prob->selector, (const double *)q, mx, mx,
                                       (double *)F, (double *)F + nfx, masks_out,
                                       masks_out ? masks_out + nfx : nullptr, w.evals, stream);
    else if (prob->equation == NENO6_BURGERS)
      e = launch_faces_burgers<double>(line_of(prob, w.fmap), P, prob->selector, (const double *)q, mx,
                                    (double *)F, masks_out, stream);
    else if (nv == 1)
      e = launch_faces_advection<double>(line_of(prob, w.fmap), P, prob->selector, (const double *)q, mx,
                                         (double *)F, masks_out, stream);
    else
      e = launch_faces_euler1d<double>(line_of(prob, w.fmap), P, prob->selector, (const double *)q, mx,
                                       (double *)F, masks_out, w.evals, stream);
  } else {
    const float *P = prepared_f32(mlp);
    if (is2d)
      e = launch_faces_euler2d<float>(grid_of(prob), P, prob->selector, (const float *)q, mx, mx,
                                      (float *)F, (float *)F + nfx, masks_out,
                                      masks_out ? masks_out + nfx : nullptr, w.evals, stream);
    else if (prob->equation == NENO6_BURGERS)
      e = launch_faces_burgers<float>(line_of(prob, w.fmap), P, prob->selector, (const float *)q, mx,
                                    (float *)F, masks_out, stream);
    else if (nv == 1)
      e = launch_faces_advection<float>(line_of(prob, w.fmap), P, prob->selector, (const float *)q, mx,
                                        (float *)F, masks_out, stream);
    else
      e = launch_faces_euler1d<float>(line_of(prob, w.fmap), P, prob->selector, (const float *)q, mx,
                                      (float *)F, masks_out, w.evals, stream);
  }
  return hip_status(e);
}

int32_t neno6_recheck_count(const neno6_problem *prob, const neno6_mlp *mlp, const void *ws,
                            size_t ws_bytes, uint32_t *count, hipStream_t stream) {
  if (is_batch2d(prob)) return NENO6_UNSUPPORTED;
  if (int32_t c = check_problem(prob)) return c;
  if (!mlp || !ws || !count) return NENO6_BAD_ARG;
  if (prob->precision < NENO6_BF16) return NENO6_BAD_LAYOUT;
  const Work w = carve_work(prob, (void *)ws);
  if (ws_bytes < w.bytes) return NENO6_WORKSPACE_SMALL;
  if (hipStreamSynchronize(stream) != hipSuccess) return NENO6_HIP_ERROR;
  count[0] = count[1] = 0;
  // no re-check ran (its counters are then not maintained)
  if (!(mlp->recheck_margin > 0.f) || prob->selector != NENO6_SEL_MLP) return NENO6_OK;
  uint32_t qc[QCOUNTERS];
  if (hipMemcpy(qc, w.scr.qcount, sizeof(qc), hipMemcpyDeviceToHost) != hipSuccess)
    return NENO6_HIP_ERROR;
  if (prob->equation == NENO6_EULER2D) {  // one counter per evaluation kind and sweep
    for (int k = 0; k < 8; ++k) {
      count[0] += qc[k];
      count[1] += qc[8 + k];
    }
  } else {  // 1D: the count spread over all slots
    for (int k = 0; k < QCOUNTERS; ++k) count[0] += qc[k];
  }
  return NENO6_OK;
}

int32_t neno6_autotune(const neno6_problem *prob, const neno6_mlp *mlp, const void *q, void *ws,
                       size_t ws_bytes, int32_t reps, neno6_tuning *best, float *best_ms,
                       hipStream_t stream) {
  if (is_batch2d(prob)) {  // tuned on the grid with the most faces
    if (!q) return NENO6_BAD_ARG;
    neno6_problem big{};
    int64_t most = -1, at_cells = 0;
    if (int32_t c = for_each_grid(prob, [&](const neno6_problem &s, int32_t, int64_t cells, int64_t) {
          const int64_t nf = (s.nx + 1) * s.ny + s.nx * (s.ny + 1);
          if (nf > most) most = nf, big = s, at_cells = cells;
          return NENO6_OK;
        }))
      return c;
    return neno6_autotune(&big, mlp, at_elems(q, 4 * at_cells, elem_size(prob->precision)), ws,
                          ws_bytes, reps, best, best_ms, stream);
  }
  if (int32_t c = check_problem(prob)) return c;
  if (prob->precision < NENO6_BF16 || prob->selector != NENO6_SEL_MLP ||
      prob->equation <= NENO6_BURGERS)
    return NENO6_UNSUPPORTED;
  if (int32_t c = check_mlp(mlp, prob->selector, prob->precision)) return c;
  if (!q || !ws || !best || reps < 1 || reps > 1000) return NENO6_BAD_ARG;
  const Work w = carve_work(prob, ws);
  if (ws_bytes < w.bytes) return NENO6_WORKSPACE_SMALL;
  if (int32_t c = begin_call(prob, mlp, w, stream)) return c;
  static const int waves[] = {2, 4, 8};
  // workgroup caps: one to four and six full rounds of resident workgroups
  // (the fused kernel holds three waves per SIMD in 1D, twelve per compute
  // unit, and two in 2D), which split the tiles evenly over the SIMDs, and
  // two caps of many rounds.  A cap between whole rounds leaves part of the
  // chip idle in its last round: 2048 workgroups of four waves took 6 %
  // longer RK3 steps than 2304 on the 4096-problem batch.
  static const int fixed_blocks[] = {16384, 65536};
  static const int rounds[] = {1, 2, 3, 4, 6};
  const bool is2d = prob->equation == NENO6_EULER2D;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return NENO6_HIP_ERROR;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return NENO6_HIP_ERROR;
  }
  FastArgs fa = fast_args(prob, mlp, w);
  auto pass = [&]() -> hipError_t {
    hipError_t e = launch_fast_reset(fa, stream);
    if (e != hipSuccess) return e;
    if (is2d)
      return launch_fast_faces2d(grid_of(prob), fa, (const float *)q, nullptr, nullptr, (float *)w.F,
                                 (float *)w.G, stream);
    Out1D out;
    out.mode = OUT_FACES;
    out.dst = (float *)w.F;
    return launch_fast_pass1d(line_of(prob, w.fmap), fa, (const float *)q, nullptr, out, stream);
  };
  // about 0.1 s of passes in the default shape first, so that every candidate
  // is timed at steady clocks
  {
    float ms = 0.f;
    hipError_t e = pass();
    if (e == hipSuccess) e = hipEventRecord(e0, stream);
    if (e == hipSuccess) e = pass();
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const int n_warm = ms > 0.f ? (int)std::min(2000.f, 100.f / ms) : 100;
    for (int r = 0; r < n_warm && e == hipSuccess; ++r) e = pass();
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return NENO6_HIP_ERROR;
    }
  }
  float best_t = -1.f;
  neno6_tuning bt{};
  int32_t rc = NENO6_OK;
  for (int wv : waves) {
    if (is2d && wv == 2) continue;  // 2D sweeps run with 4 or 8 waves
    int blocks[8];
    int nbl = 0;
    for (int nb : fixed_blocks) blocks[nbl++] = nb;
    // resident workgroups per compute unit: 1D twelve waves (eight-wave
    // workgroups: one, by their LDS), 2D eight
    const int per_cu = is2d ? 8 / wv : (wv == 8 ? 1 : 12 / wv);
    for (int k : rounds) {
      const int nb = n_cu * per_cu * k;
      bool dup = nb < 1 || nb > 65536;
      for (int i = 0; i < nbl; ++i) dup = dup || blocks[i] == nb;
      if (!dup) blocks[nbl++] = nb;
    }
    for (int ib = 0; ib < nbl; ++ib)
      for (int xcd = 0; xcd < 2 && rc == NENO6_OK; ++xcd) {
          const int nb = blocks[ib];
          fa.face_waves = wv;
          fa.face_blocks = nb;
          fa.xcd_order = xcd;
          float ms = 0.f;
          hipError_t e = pass();
          if (e == hipSuccess) e = hipEventRecord(e0, stream);
          for (int r = 0; r < reps && e == hipSuccess; ++r) e = pass();
          if (e == hipSuccess) e = hipEventRecord(e1, stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess) {
            rc = NENO6_HIP_ERROR;
            break;
          }
          ms /= (float)reps;
          if (best_t < 0.f || ms < best_t) {
            best_t = ms;
            bt.face_waves = wv;
            bt.face_blocks = nb;
            bt.xcd_order = xcd;
          }
        }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != NENO6_OK) return rc;
  *best = bt;
  if (best_ms) *best_ms = best_t;
  return NENO6_OK;
}

int32_t neno6_step(const neno6_problem *prob, const neno6_mlp *mlp, void *q, double cfl,
                   int32_t n_steps, double *t, int32_t *status, void *ws, size_t ws_bytes,
                   hipStream_t stream) {
  if (is_batch2d(prob)) {
    if (!q || !t || !status) return NENO6_BAD_ARG;
    const size_t es = elem_size(prob->precision);
    return for_each_grid(prob, [&](const neno6_problem &s, int32_t p, int64_t cells, int64_t) {
      return neno6_step(&s, mlp, at_elems(q, 4 * cells, es), cfl, n_steps, t + p, status + p, ws,
                        ws_bytes, stream);
    });
  }
  if (int32_t c = check_problem(prob)) return c;
  if (int32_t c = check_mlp(mlp, prob->selector, prob->precision)) return c;
  if (prob->selector == NENO6_SEL_MASKS_IN) return NENO6_UNSUPPORTED;
  if (!q || !t || !status || !ws || n_steps < 0 || !(cfl > 0)) return NENO6_BAD_ARG;
  const Work w = carve_work(prob, ws);
  if (ws_bytes < w.bytes) return NENO6_WORKSPACE_SMALL;
  // steps maintain no re-check counters (the 2D time step clears them)
  if (int32_t c = begin_call(prob, mlp, w, stream, prob->equation == NENO6_EULER2D)) return c;
  const bool f64 = prob->precision == NENO6_FP64;
  for (int32_t it = 0; it < n_steps; ++it) {
    hipError_t e;
    if (prob->equation == NENO6_EULER2D) {
      const Grid2D g = grid_of(prob);
      e = f64 ? launch_cfl2d<double>(g, (const double *)q, cfl, w.part, w.dt, status, t, stream)
              : launch_cfl2d<float>(g, (const float *)q, cfl, w.part, w.dt, status, t, stream);
    } else {
      const Line1D ln = line_of(prob, w.fmap);
      e = f64 ? launch_cfl1d<double>(ln, prob->equation, (const double *)q, cfl, w.dt, status, t,
                                     stream)
              : launch_cfl1d<float>(ln, prob->equation, (const float *)q, cfl, w.dt, status, t,
                                    stream);
    }
    if (e != hipSuccess) return NENO6_HIP_ERROR;
    // u1 = stage 1 of q; u2 = stage 2 of u1; q = stage 3 of u2
    const void *ins[3] = {q, w.u1, w.u2};
    void *outs[3] = {w.u1, w.u2, q};
    for (int k = 0; k < 3; ++k) {
      Stage st;
      st.stage = k + 1;
      st.us = ins[k];
      st.u0 = q;
      st.out = outs[k];
      st.dt = w.dt;
      st.status = status;
      int32_t r = rhs_dispatch(prob, mlp, ins[k], nullptr, nullptr, nullptr, nullptr, w, &st,
                               stream);
      if (r != NENO6_OK) return r;
    }
  }
  return NENO6_OK;
}

int32_t neno6_classifier_samples(uint64_t seed, int64_t first, int64_t n, float *s, uint8_t *y,
                                 hipStream_t stream) {
  if (first < 0 || n < 0 || first > INT64_MAX - n) return NENO6_BAD_ARG;
  if (n > 0 && (!s || !y)) return NENO6_BAD_ARG;
  return hip_status(launch_classifier_samples(seed, first, n, s, y, stream));
}

int32_t neno6_rhs_adjoint(const neno6_problem *prob, const uint8_t *masks, const void *rbar,
                          void *ubar, hipStream_t stream) {
  if (int32_t c = check_problem(prob)) return c;
  if (prob->equation != NENO6_ADVECTION || prob->n_problems != 1) return NENO6_UNSUPPORTED;
  if (prob->precision != NENO6_FP64 && prob->precision != NENO6_FP32) return NENO6_BAD_LAYOUT;
  if (!masks || !rbar || !ubar) return NENO6_BAD_ARG;
  return hip_status(launch_adjoint_advection(line_of(prob), masks, rbar, ubar,
                                             prob->precision == NENO6_FP64, stream));
}

size_t neno6_vjp_workspace_size(const neno6_problem *prob) {
  if (is_batch2d(prob)) {
    size_t most = 0;
    const int32_t c = for_each_grid(prob, [&](const neno6_problem &s, int32_t, int64_t, int64_t) {
      most = std::max(most, neno6_vjp_workspace_size(&s));
      return NENO6_OK;
    });
    return c == NENO6_OK ? most : 0;
  }
  if (check_problem(prob) != NENO6_OK) return 0;
  if (prob->equation == NENO6_EULER2D) {
    const size_t nfx = (size_t)(prob->nx + 1) * prob->ny, nfy = (size_t)prob->nx * (prob->ny + 1);
    return align_up(24 * (nfx + nfy) * elem_size(prob->precision));
  }
  if (prob->equation != NENO6_BURGERS && prob->equation != NENO6_EULER1D) return 0;
  const size_t faces = (size_t)prob->total_cells + prob->n_problems;
  return align_up(faces * sizeof(int32_t)) +
         align_up(6 * (size_t)nvar_of(prob->equation) * faces * elem_size(prob->precision));
}

int32_t neno6_rhs_vjp(const neno6_problem *prob, const void *q, const uint8_t *masks,
                      const void *rbar, void *qbar, void *ws, size_t ws_bytes,
                      hipStream_t stream) {
  if (is_batch2d(prob)) {
    if (!q || !masks || !rbar || !qbar) return NENO6_BAD_ARG;
    const size_t es = elem_size(prob->precision);
    return for_each_grid(prob, [&](const neno6_problem &s, int32_t, int64_t cells, int64_t faces) {
      return neno6_rhs_vjp(&s, at_elems(q, 4 * cells, es), masks + 4 * faces,
                           at_elems(rbar, 4 * cells, es), at_elems(qbar, 4 * cells, es), ws,
                           ws_bytes, stream);
    });
  }
  if (int32_t c = check_problem(prob)) return c;
  if (prob->equation == NENO6_ADVECTION) return NENO6_UNSUPPORTED;
  if (prob->precision != NENO6_FP64 && prob->precision != NENO6_FP32) return NENO6_BAD_LAYOUT;
  if (!q || !masks || !rbar || !qbar || !ws) return NENO6_BAD_ARG;
  const size_t need = neno6_vjp_workspace_size(prob);
  if (ws_bytes < need) return NENO6_WORKSPACE_SMALL;
  if (prob->equation == NENO6_EULER2D) {
    const Grid2D g = grid_of(prob);
    hipError_t e = prob->precision == NENO6_FP64
                       ? launch_vjp2d<double>(g, (const double *)q, masks, (const double *)rbar,
                                              (double *)qbar, (double *)ws, stream)
                       : launch_vjp2d<float>(g, (const float *)q, masks, (const float *)rbar,
                                             (float *)qbar, (float *)ws, stream);
    return hip_status(e);
  }
  const size_t faces = (size_t)prob->total_cells + prob->n_problems;
  int32_t *fmap = (int32_t *)ws;
  void *scratch = (char *)ws + align_up(faces * sizeof(int32_t));
  const Line1D ln = line_of(prob, fmap);
  if (launch_build_fmap(line_of(prob), fmap, stream) != hipSuccess) return NENO6_HIP_ERROR;
  hipError_t e =
      prob->precision == NENO6_FP64
          ? launch_vjp1d<double>(ln, prob->equation, (const double *)q, masks,
                                 (const double *)rbar, (double *)qbar, (double *)scratch, stream)
          : launch_vjp1d<float>(ln, prob->equation, (const float *)q, masks, (const float *)rbar,
                                (float *)qbar, (float *)scratch, stream);
  return hip_status(e);
}

size_t neno6_train_workspace_size(int32_t batch) { return train_workspace_bytes(batch); }

int32_t neno6_classifier_train(double *params, double *adam_m, double *adam_v, int64_t *step,
                               const float *s, const uint8_t *y, const int64_t *idx, int64_t n_idx,
                               int32_t batch, double lr, double beta1, double beta2, double eps,
                               int32_t precision, double *loss_out, void *ws, size_t ws_bytes,
                               hipStream_t stream) {
  if (!params || !adam_m || !adam_v || !step || !s || !y || !idx || n_idx < 1 || batch < 1 ||
      batch > (1 << 20) || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) ||
      !(eps > 0) || !ws)
    return NENO6_BAD_ARG;
  if (precision != NENO6_FP32 && precision != NENO6_BF16) return NENO6_BAD_LAYOUT;
  if (!train_precision_supported(precision)) return NENO6_UNSUPPORTED;
  if (ws_bytes < train_workspace_bytes(batch)) return NENO6_WORKSPACE_SMALL;
  for (int64_t s0 = 0; s0 < n_idx; s0 += batch) {
    const int64_t mb = n_idx - s0 < batch ? n_idx - s0 : batch;
    *step += 1;
    hipError_t e = launch_train_batch(params, adam_m, adam_v, *step, s, y, idx + s0, mb, lr, beta1,
                                      beta2, eps, precision, loss_out, 1.0 / (double)n_idx,
                                      s0 == 0, ws, stream);
    if (e != hipSuccess) return NENO6_HIP_ERROR;
  }
  return NENO6_OK;
}

int32_t neno6_classifier_grad(const double *params, const float *s, const uint8_t *y, int64_t n,
                              int32_t precision, double *grad, double *loss, void *ws,
                              size_t ws_bytes, hipStream_t stream) {
  if (!params || !s || !y || n < 1 || n > (1 << 20) || !grad || !loss || !ws) return NENO6_BAD_ARG;
  if (precision != NENO6_FP32 && precision != NENO6_BF16) return NENO6_BAD_LAYOUT;
  if (!train_precision_supported(precision)) return NENO6_UNSUPPORTED;
  if (ws_bytes < train_workspace_bytes((int32_t)n)) return NENO6_WORKSPACE_SMALL;
  return hip_status(launch_grad(params, s, y, n, precision, grad, loss, ws, stream));
}

}  // extern "C"
