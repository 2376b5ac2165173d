"""ctypes binding of libneno6.so (the C ABI in include/neno6.h).

Argument marshalling only: every function takes torch tensors (device memory
and streams come from PyTorch), checks dtypes/shapes, and passes raw pointers
to the entry point of the same name.  All arithmetic happens in the HIP
kernels; if the library is missing this module raises instead of falling back
to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libneno6.so")

OK, BAD_ARG, BAD_LAYOUT, HIP_ERROR, NONPHYSICAL, UNSUPPORTED, WORKSPACE_SMALL = 0, -1, -2, -3, -4, -5, -6
TOO_LARGE = -7
NOALLOC_MAX_FACES = 16 * 1024 * 1024
FP64, FP32, BF16, FP16 = 0, 1, 2, 3
ADVECTION, BURGERS, EULER1D, EULER2D = 0, 1, 2, 3
PERIODIC, TRANSMISSIVE = 0, 1
SEL_MLP, SEL_ALL_SMOOTH, SEL_ALL_DISCARD, SEL_MASKS_IN, SEL_TENO = 0, 1, 2, 3, 4
RECHECK_FP32, RECHECK_FP16X2 = 0, 1
KEEP_MAP = 1
NPARAM = 3228

EXPORTS = (
    "neno6_status_string", "neno6_version", "neno6_mlp_prepared_bytes", "neno6_mlp_prepare",
    "neno6_mlp_logits", "neno6_reconstruct", "neno6_workspace_size", "neno6_rhs",
    "neno6_rhs_noalloc", "neno6_face_fluxes", "neno6_recheck_count", "neno6_autotune", "neno6_step",
    "neno6_rhs_adjoint", "neno6_vjp_workspace_size", "neno6_rhs_vjp",
    "neno6_train_workspace_size", "neno6_classifier_train",
    "neno6_classifier_grad", "neno6_classifier_samples",
)


class Neno6Error(RuntimeError):
    pass


class MlpStruct(C.Structure):
    _fields_ = [("params", C.c_void_p), ("prepared", C.c_void_p), ("recheck_margin", C.c_float),
                ("recheck_mode", C.c_int32)]


class TuningStruct(C.Structure):
    _fields_ = [("face_waves", C.c_int32), ("face_blocks", C.c_int32),
                ("recheck_blocks", C.c_int32), ("xcd_order", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class ProblemStruct(C.Structure):
    _fields_ = [("equation", C.c_int32), ("bc", C.c_int32), ("precision", C.c_int32),
                ("selector", C.c_int32), ("n_problems", C.c_int32), ("flags", C.c_int32),
                ("total_cells", C.c_int64), ("nx", C.c_int64), ("ny", C.c_int64),
                ("offsets", C.c_void_p), ("offsets_host", C.c_void_p), ("dx", C.c_void_p),
                ("dx2d", C.c_double), ("dy2d", C.c_double), ("gamma", C.c_double),
                ("tuning", C.POINTER(TuningStruct)), ("grids_host", C.c_void_p)]


class Grid2DStruct(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("dx", C.c_double), ("dy", C.c_double)]


_lock = threading.Lock()
_lib = None


def load(path: str = LIB_PATH):
    """Loads libneno6.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise Neno6Error("libneno6.so not built (run __graft_entry__.build() or "
                             "python -m paper_2207_08500_amd.build)")
        lib = C.CDLL(path)
        vp, i32, i64, f64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float, C.c_size_t
        P = C.POINTER
        lib.neno6_status_string.argtypes = [i32]
        lib.neno6_status_string.restype = C.c_char_p
        lib.neno6_version.restype = i32
        lib.neno6_mlp_prepared_bytes.restype = sz
        lib.neno6_mlp_prepare.argtypes = [P(MlpStruct), vp]
        lib.neno6_mlp_logits.argtypes = [P(MlpStruct), i32, vp, i64, vp, vp, vp]
        lib.neno6_reconstruct.argtypes = [P(MlpStruct), vp, i64, i32, i32, i32, vp, vp, vp, vp]
        lib.neno6_workspace_size.argtypes = [P(ProblemStruct)]
        lib.neno6_workspace_size.restype = sz
        lib.neno6_rhs.argtypes = [P(ProblemStruct), P(MlpStruct), vp, vp, vp, vp, vp, vp, sz, vp]
        lib.neno6_rhs_noalloc.argtypes = [P(ProblemStruct), P(MlpStruct), vp, vp, vp, vp, vp, vp]
        lib.neno6_face_fluxes.argtypes = [P(ProblemStruct), P(MlpStruct), vp, vp, vp, vp, sz, vp]
        lib.neno6_recheck_count.argtypes = [P(ProblemStruct), P(MlpStruct), vp, sz, P(C.c_uint32), vp]
        lib.neno6_autotune.argtypes = [P(ProblemStruct), P(MlpStruct), vp, vp, sz, i32,
                                       P(TuningStruct), P(C.c_float), vp]
        lib.neno6_step.argtypes = [P(ProblemStruct), P(MlpStruct), vp, f64, i32, vp, vp, vp, sz, vp]
        lib.neno6_rhs_adjoint.argtypes = [P(ProblemStruct), vp, vp, vp, vp]
        lib.neno6_vjp_workspace_size.argtypes = [P(ProblemStruct)]
        lib.neno6_vjp_workspace_size.restype = sz
        lib.neno6_rhs_vjp.argtypes = [P(ProblemStruct), vp, vp, vp, vp, vp, sz, vp]
        lib.neno6_train_workspace_size.argtypes = [i32]
        lib.neno6_train_workspace_size.restype = sz
        lib.neno6_classifier_train.argtypes = [vp, vp, vp, P(C.c_int64), vp, vp, vp, i64, i32, f64,
                                               f64, f64, f64, i32, vp, vp, sz, vp]
        lib.neno6_classifier_grad.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp, sz, vp]
        lib.neno6_classifier_samples.argtypes = [C.c_uint64, i64, i64, vp, vp, vp]
        for name in EXPORTS:
            fn = getattr(lib, name)
            if fn.restype is C.c_int:  # default
                fn.restype = i32
        _lib = lib
        return lib


def _check(rc: int, name: str):
    if rc != OK:
        msg = load().neno6_status_string(rc).decode()
        raise Neno6Error("%s failed: %s (%d)" % (name, msg, rc))


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _dev(t, dtype=None, name="tensor"):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def fdtype(precision: int):
    return torch.float64 if precision == FP64 else torch.float32


# ---------------------------------------------------------------------------
class Mlp:
    """Classifier handle: FP64 master parameters and the prepared block on device."""

    def __init__(self, params: torch.Tensor, recheck_margin: float = 0.0, prepare: bool = True,
                 recheck_mode: int = 0):
        """recheck_mode: RECHECK_FP32 (default) or RECHECK_FP16X2 (FP16 operands
        re-checked in two-part FP16 on MFMA)."""
        _dev(params, torch.float64, "params")
        if params.numel() != NPARAM:
            raise ValueError("params must hold %d values" % NPARAM)
        self.params = params.contiguous()
        nb = int(load().neno6_mlp_prepared_bytes())
        self.prepared = torch.empty(nb, dtype=torch.uint8, device=params.device)
        self.recheck_margin = float(recheck_margin)
        self.recheck_mode = int(recheck_mode)
        if prepare:
            neno6_mlp_prepare(self)

    def struct(self) -> MlpStruct:
        return MlpStruct(self.params.data_ptr(), self.prepared.data_ptr(), self.recheck_margin,
                         self.recheck_mode)


def _mlp(mlp):
    return None if mlp is None else C.byref(mlp.struct())


def neno6_mlp_prepare(mlp: Mlp, stream=None):
    _check(load().neno6_mlp_prepare(C.byref(mlp.struct()), _stream(stream)), "neno6_mlp_prepare")


def neno6_mlp_logits(mlp: Mlp, precision: int, s: torch.Tensor, z: torch.Tensor,
                     masks: torch.Tensor | None = None, stream=None):
    _dev(s, fdtype(precision), "s")
    _dev(z, fdtype(precision), "z")
    n = s.numel() // 6
    if s.numel() != 6 * n or z.numel() != 4 * n or (masks is not None and masks.numel() != n):
        raise ValueError("shape mismatch")
    _check(load().neno6_mlp_logits(_mlp(mlp), precision, _ptr(s), n, _ptr(z), _ptr(masks),
                                   _stream(stream)), "neno6_mlp_logits")


def neno6_reconstruct(mlp: Mlp | None, f: torch.Tensor, sign: int, precision: int, selector: int,
                      fhat: torch.Tensor, masks_in: torch.Tensor | None = None,
                      masks_out: torch.Tensor | None = None, stream=None):
    _dev(f, fdtype(precision), "f")
    _dev(fhat, fdtype(precision), "fhat")
    n = f.numel() - 5
    if n < 0 or fhat.numel() != n:
        raise ValueError("fhat must hold f.numel() - 5 values")
    for m in (masks_in, masks_out):
        if m is not None and (m.numel() != n or m.dtype != torch.uint8):
            raise ValueError("masks must be uint8 [n_faces]")
    _check(load().neno6_reconstruct(_mlp(mlp), _ptr(f), n, sign, precision, selector,
                                    _ptr(masks_in), _ptr(fhat), _ptr(masks_out), _stream(stream)),
           "neno6_reconstruct")


class Problem:
    """Holds a problem description and the device/host arrays it points to."""

    def __init__(self, equation: int, precision: int, selector: int = SEL_MLP, bc: int = TRANSMISSIVE,
                 offsets=None, dx=None, nx: int = 0, ny: int = 0, dx2d: float = 0.0,
                 dy2d: float = 0.0, gamma: float = 1.4, device="cuda", tuning=None, grids=None):
        """1D: offsets[n+1] and dx[n] of the lines.  2D: one grid (nx, ny, dx2d,
        dy2d), or a batch `grids` = [(nx, ny, dx, dy), ...] whose states,
        masks and face fluxes follow one another grid by grid."""
        self.equation, self.precision, self.selector, self.bc = equation, precision, selector, bc
        self.gamma = float(gamma)
        self.flags = 0  # KEEP_MAP once the caller's workspace holds the face map
        self.tuning = None
        self.set_tuning(tuning)
        self.grids = None
        if equation == EULER2D and grids is not None:
            g = [(int(a), int(b), float(c), float(d)) for a, b, c, d in grids]
            self.grids = (Grid2DStruct * len(g))(*[Grid2DStruct(*x) for x in g])
            self.grid_list = g
            self.n_problems = len(g)
            self.total_cells = sum(a * b for a, b, _, _ in g)
            self.nx = self.ny = 0
            self.dx2d = self.dy2d = 0.0
            self.offsets_host = self.offsets = self.dx = None
        elif equation == EULER2D:
            self.nx, self.ny, self.dx2d, self.dy2d = int(nx), int(ny), float(dx2d), float(dy2d)
            self.n_problems = 1
            self.total_cells = self.nx * self.ny
            self.offsets_host = self.offsets = self.dx = None
        else:
            oh = torch.as_tensor(offsets, dtype=torch.int64).contiguous().cpu()
            self.offsets_host = oh
            self.offsets = oh.to(device)
            self.n_problems = oh.numel() - 1
            self.total_cells = int(oh[-1])
            self.dx = torch.as_tensor(dx, dtype=torch.float64).expand(self.n_problems).contiguous().to(device)
            self.nx = self.ny = 0
            self.dx2d = self.dy2d = 0.0

    def set_tuning(self, tuning):
        """Launch shapes (dict with the neno6_tuning fields, a TuningStruct,
        or None for the library defaults)."""
        if tuning is None or isinstance(tuning, TuningStruct):
            self.tuning = tuning
        else:
            self.tuning = TuningStruct(*(int(tuning.get(k, 0)) for k, _ in TuningStruct._fields_))

    @property
    def nvar(self) -> int:
        return {ADVECTION: 1, BURGERS: 1, EULER1D: 3, EULER2D: 4}[self.equation]

    @property
    def n_faces(self) -> int:
        if self.equation == EULER2D and self.grids is not None:
            return sum((a + 1) * b + a * (b + 1) for a, b, _, _ in self.grid_list)
        if self.equation == EULER2D:
            return (self.nx + 1) * self.ny + self.nx * (self.ny + 1)
        return self.total_cells + self.n_problems

    def mask_count(self) -> int:
        return self.nvar * self.n_faces

    def struct(self) -> ProblemStruct:
        return ProblemStruct(self.equation, self.bc, self.precision, self.selector, self.n_problems,
                             self.flags,
                             self.total_cells, self.nx, self.ny,
                             None if self.offsets is None else self.offsets.data_ptr(),
                             None if self.offsets_host is None else self.offsets_host.data_ptr(),
                             None if self.dx is None else self.dx.data_ptr(),
                             self.dx2d, self.dy2d, self.gamma,
                             None if self.tuning is None else C.pointer(self.tuning),
                             None if self.grids is None else C.addressof(self.grids))

    def workspace(self, device="cuda") -> torch.Tensor:
        nb = int(load().neno6_workspace_size(C.byref(self.struct())))
        if nb == 0:
            raise Neno6Error("invalid problem description")
        return torch.empty(nb, dtype=torch.uint8, device=device)


def neno6_rhs(prob: Problem, mlp: Mlp | None, q: torch.Tensor, rhs: torch.Tensor,
              ws: torch.Tensor, masks_in=None, masks_out=None, status=None, stream=None):
    dt = fdtype(prob.precision)
    _dev(q, dt, "q")
    _dev(rhs, dt, "rhs")
    if q.numel() != prob.nvar * prob.total_cells or rhs.numel() != q.numel():
        raise ValueError("state size mismatch")
    for m in (masks_in, masks_out):
        if m is not None and (m.numel() != prob.mask_count() or m.dtype != torch.uint8):
            raise ValueError("masks must be uint8 with %d entries" % prob.mask_count())
    if status is not None:
        _dev(status, torch.int32, "status")
    ps = prob.struct()
    _check(load().neno6_rhs(C.byref(ps), _mlp(mlp), _ptr(q), _ptr(rhs), _ptr(masks_in),
                            _ptr(masks_out), _ptr(status), _ptr(ws), ws.numel(), _stream(stream)),
           "neno6_rhs")


def neno6_rhs_noalloc(prob: Problem, mlp: Mlp, q: torch.Tensor, rhs: torch.Tensor, masks_in=None,
                      masks_out=None, status=None, stream=None):
    """neno6_rhs without a workspace: the library's static device scratch
    holds the face map (1D Euler, BF16/FP16, at most NOALLOC_MAX_FACES faces;
    calls on one GPU share it and must not overlap)."""
    dt = fdtype(prob.precision)
    _dev(q, dt, "q")
    _dev(rhs, dt, "rhs")
    if q.numel() != prob.nvar * prob.total_cells or rhs.numel() != q.numel():
        raise ValueError("state size mismatch")
    for m in (masks_in, masks_out):
        if m is not None and (m.numel() != prob.mask_count() or m.dtype != torch.uint8):
            raise ValueError("masks must be uint8 with %d entries" % prob.mask_count())
    if status is not None:
        _dev(status, torch.int32, "status")
    ps = prob.struct()
    _check(load().neno6_rhs_noalloc(C.byref(ps), _mlp(mlp), _ptr(q), _ptr(rhs), _ptr(masks_in),
                                    _ptr(masks_out), _ptr(status), _stream(stream)),
           "neno6_rhs_noalloc")


def neno6_face_fluxes(prob: Problem, mlp: Mlp | None, q: torch.Tensor, F: torch.Tensor,
                      ws: torch.Tensor, masks_out=None, stream=None):
    dt = fdtype(prob.precision)
    _dev(q, dt, "q")
    _dev(F, dt, "F")
    if F.numel() != prob.nvar * prob.n_faces:
        raise ValueError("F must hold nvar * faces values")
    ps = prob.struct()
    _check(load().neno6_face_fluxes(C.byref(ps), _mlp(mlp), _ptr(q), _ptr(F), _ptr(masks_out),
                                    _ptr(ws), ws.numel(), _stream(stream)), "neno6_face_fluxes")


def neno6_recheck_count(prob: Problem, mlp: Mlp, ws: torch.Tensor, stream=None):
    """Evaluations re-checked by the last neno6_face_fluxes call with
    this mlp (x, y); (0, 0) when its margin is 0."""
    cnt = (C.c_uint32 * 2)()
    ps = prob.struct()
    _check(load().neno6_recheck_count(C.byref(ps), _mlp(mlp), _ptr(ws), ws.numel(), cnt,
                                      _stream(stream)), "neno6_recheck_count")
    return int(cnt[0]), int(cnt[1])


def neno6_autotune(prob: Problem, mlp: Mlp, q: torch.Tensor, ws: torch.Tensor, reps: int = 3,
                   stream=None):
    """Times the fused face pass for the library's candidate launch shapes;
    returns (TuningStruct of the fastest, its mean pass time in ms)."""
    _dev(q, fdtype(prob.precision), "q")
    if q.numel() != prob.nvar * prob.total_cells:
        raise ValueError("state size mismatch")
    best, ms = TuningStruct(), C.c_float(0.0)
    ps = prob.struct()
    _check(load().neno6_autotune(C.byref(ps), _mlp(mlp), _ptr(q), _ptr(ws), ws.numel(), int(reps),
                                 C.byref(best), C.byref(ms), _stream(stream)), "neno6_autotune")
    return best, float(ms.value)


def neno6_step(prob: Problem, mlp: Mlp | None, q: torch.Tensor, cfl: float, n_steps: int,
               t: torch.Tensor, status: torch.Tensor, ws: torch.Tensor, stream=None):
    _dev(q, fdtype(prob.precision), "q")
    _dev(t, torch.float64, "t")
    _dev(status, torch.int32, "status")
    if q.numel() != prob.nvar * prob.total_cells:
        raise ValueError("state size mismatch")
    if t.numel() != prob.n_problems or status.numel() != prob.n_problems:
        raise ValueError("t and status need one entry per problem")
    ps = prob.struct()
    _check(load().neno6_step(C.byref(ps), _mlp(mlp), _ptr(q), float(cfl), int(n_steps), _ptr(t),
                             _ptr(status), _ptr(ws), ws.numel(), _stream(stream)), "neno6_step")


def neno6_rhs_adjoint(prob: Problem, masks: torch.Tensor, rbar: torch.Tensor, ubar: torch.Tensor,
                      stream=None):
    dt = fdtype(prob.precision)
    _dev(rbar, dt, "rbar")
    _dev(ubar, dt, "ubar")
    ps = prob.struct()
    _check(load().neno6_rhs_adjoint(C.byref(ps), _ptr(masks), _ptr(rbar), _ptr(ubar),
                                    _stream(stream)), "neno6_rhs_adjoint")


def neno6_rhs_vjp(prob: Problem, q: torch.Tensor, masks: torch.Tensor, rbar: torch.Tensor,
                  qbar: torch.Tensor, ws: torch.Tensor | None = None, stream=None):
    """qbar = (d rhs / d q)^T rbar at q with fixed labels (BURGERS, EULER1D, EULER2D)."""
    dt = fdtype(prob.precision)
    for t, nm in ((q, "q"), (rbar, "rbar"), (qbar, "qbar")):
        _dev(t, dt, nm)
        if t.numel() != prob.nvar * prob.total_cells:
            raise ValueError("%s size mismatch" % nm)
    if masks.numel() != prob.mask_count() or masks.dtype != torch.uint8:
        raise ValueError("masks must be uint8 with %d entries" % prob.mask_count())
    ps = prob.struct()
    if ws is None:
        nb = int(load().neno6_vjp_workspace_size(C.byref(ps)))
        if nb == 0:
            raise Neno6Error("neno6_rhs_vjp: unsupported problem")
        ws = torch.empty(nb, dtype=torch.uint8, device=q.device)
    _check(load().neno6_rhs_vjp(C.byref(ps), _ptr(q), _ptr(masks), _ptr(rbar), _ptr(qbar), _ptr(ws),
                                ws.numel(), _stream(stream)), "neno6_rhs_vjp")


def neno6_train_workspace_size(batch: int) -> int:
    return int(load().neno6_train_workspace_size(int(batch)))


def neno6_classifier_train(params, adam_m, adam_v, step: int, s, y, idx, batch: int, lr: float,
                           beta1=0.9, beta2=0.999, eps=1e-8, precision=BF16, loss_out=None,
                           ws=None, stream=None) -> int:
    for t, d, nm in ((params, torch.float64, "params"), (adam_m, torch.float64, "adam_m"),
                     (adam_v, torch.float64, "adam_v"), (s, torch.float32, "s"),
                     (y, torch.uint8, "y"), (idx, torch.int64, "idx")):
        _dev(t, d, nm)
    if ws is None:
        ws = torch.empty(neno6_train_workspace_size(batch), dtype=torch.uint8, device=params.device)
    st = C.c_int64(int(step))
    _check(load().neno6_classifier_train(_ptr(params), _ptr(adam_m), _ptr(adam_v), C.byref(st),
                                         _ptr(s), _ptr(y), _ptr(idx), idx.numel(), int(batch),
                                         float(lr), float(beta1), float(beta2), float(eps),
                                         int(precision), _ptr(loss_out), _ptr(ws), ws.numel(),
                                         _stream(stream)), "neno6_classifier_train")
    return int(st.value)


def neno6_classifier_grad(params, s, y, precision, grad, loss, ws=None, stream=None):
    n = y.numel()
    if ws is None:
        ws = torch.empty(neno6_train_workspace_size(n), dtype=torch.uint8, device=params.device)
    _check(load().neno6_classifier_grad(_ptr(params), _ptr(s), _ptr(y), n, int(precision),
                                        _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(),
                                        _stream(stream)), "neno6_classifier_grad")


def neno6_classifier_samples(seed: int, first: int, n: int, s=None, y=None, device="cuda",
                             stream=None):
    """Seeded training samples first .. first+n-1 generated on the device:
    returns (s [n][6] float32, y [n] uint8) (given tensors are filled)."""
    if s is None:
        s = torch.empty((n, 6), dtype=torch.float32, device=device)
    if y is None:
        y = torch.empty(n, dtype=torch.uint8, device=device)
    _dev(s, torch.float32, "s")
    _dev(y, torch.uint8, "y")
    if s.numel() != 6 * n or y.numel() != n:
        raise ValueError("s needs 6 n floats and y n bytes")
    _check(load().neno6_classifier_samples(int(seed) & 0xFFFFFFFFFFFFFFFF, int(first), int(n),
                                           _ptr(s), _ptr(y), _stream(stream)),
           "neno6_classifier_samples")
    return s, y
