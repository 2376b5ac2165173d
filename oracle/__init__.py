"""NENO6 FP64 CPU oracle (Li, Fu & Adams, arXiv 2207.08500).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may use this package; the product library never does.  It shares
no code with the HIP library; both sides only take the same seeded inputs.

The arithmetic lives in ``neno6_oracle.c`` (plain C, FP64, no FP contraction),
compiled with gcc into ``_build/liboracle_neno6.so`` on first use.  This module
only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "neno6_oracle.c")
_SO = os.path.join(_HERE, "_build", "liboracle_neno6.so")
_lock = threading.Lock()
_lib = None

SEL_MLP, SEL_ALL_SMOOTH, SEL_ALL_DISCARD, SEL_MASKS_IN, SEL_TENO = 0, 1, 2, 3, 4
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
NPARAM = 3228


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64, -ffp-contract=off)."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    deps = [_SRC, os.path.join(_HERE, "teno_beta.h")]
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < max(map(os.path.getmtime, deps)):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = C.CDLL(_SO)
            d, i64, i32, u8 = (C.POINTER(C.c_double), C.POINTER(C.c_int64),
                               C.POINTER(C.c_int32), C.POINTER(C.c_uint8))
            sig = {
                "oracle_reconstruct": [d, C.c_int64, C.c_int32, d, C.c_int32, u8, d, u8],
                "oracle_mlp_logits": [d, d, C.c_int64, d, d],
                "oracle_mlp_logits_raw": [d, d, C.c_int64, d],
                "oracle_teno": [d, C.c_int64, d, d, d, u8],
                "oracle_burgers_rhs": [d, i64, C.c_int32, d, C.c_int32, d, C.c_int32, u8, d, u8,
                                       i32],
                "oracle_burgers_step": [d, i64, C.c_int32, d, C.c_int32, C.c_double, C.c_int32, d,
                                        C.c_int32, d, i32],
                "oracle_advection_rhs": [d, C.c_int64, C.c_double, C.c_int32, d, C.c_int32, u8, d, u8],
                "oracle_advection_step": [d, C.c_int64, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                          d, C.c_int32, u8],
                "oracle_advection_rhs_adjoint": [u8, C.c_int64, C.c_double, C.c_int32, d, d],
                "oracle_euler1d_rhs": [d, i64, C.c_int32, d, C.c_double, C.c_int32, d, C.c_int32,
                                       u8, d, u8, i32],
                "oracle_euler1d_step": [d, i64, C.c_int32, d, C.c_double, C.c_int32, C.c_double,
                                        C.c_int32, d, C.c_int32, d, i32],
                "oracle_euler1d_stencils": [d, i64, C.c_int32, C.c_double, C.c_int32, d],
                "oracle_euler2d_rhs": [d, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double,
                                       C.c_int32, d, C.c_int32, u8, u8, d, u8, u8, i32],
                "oracle_euler2d_step": [d, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double,
                                        C.c_int32, C.c_double, C.c_int32, d, C.c_int32, d, i32],
                "oracle_bce_grad": [d, d, u8, C.c_int64, d, d],
                "oracle_train": [d, d, d, i64, d, u8, i64, C.c_int64, C.c_int32, C.c_double,
                                 C.c_double, C.c_double, C.c_double, d],
            }
            for name, args in sig.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = C.c_int
            for name, args in {
                "oracle_linear_weights": [d], "oracle_candidate_coeffs": [d],
                "oracle_euler1d_eigen": [d, d, C.c_double, d, d],
                "oracle_euler2d_eigen": [d, d, C.c_double, C.c_int32, d, d],
                "oracle_euler1d_flux": [d, C.c_double, d],
                "oracle_euler2d_flux": [d, C.c_double, C.c_int32, d],
            }.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = None
            lib.oracle_num_threads.restype = C.c_int
            lib.oracle_set_num_threads.argtypes = [C.c_int]
            lib.oracle_set_num_threads.restype = None
            _lib = lib
    return _lib


def _p(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def _check(rc, name):
    if rc != 0:
        raise ValueError("%s returned status %d" % (name, rc))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the loops over independent problems (timing only)."""
    _load().oracle_set_num_threads(int(n))


def linear_weights() -> np.ndarray:
    out = np.zeros(4)
    _load().oracle_linear_weights(_p(out, C.c_double))
    return out


def candidate_coeffs() -> np.ndarray:
    """[4][6]: coefficient of stencil position j (cells i-2..i+3) in candidate k."""
    out = np.zeros(24)
    _load().oracle_candidate_coeffs(_p(out, C.c_double))
    return out.reshape(4, 6)


def reconstruct(f, sign=1, params=None, selector=SEL_MLP, masks_in=None):
    """Face values from f[n_faces+5]; returns (fhat[n_faces], masks[n_faces])."""
    f = _f64(f)
    n = f.size - 5
    P = None if params is None else _f64(params)
    fh = np.zeros(n)
    m = np.zeros(n, np.uint8)
    mi = _u8(masks_in)
    _check(_load().oracle_reconstruct(_p(f, C.c_double), n, sign, _p(P, C.c_double), selector,
                                      _p(mi, C.c_uint8), _p(fh, C.c_double), _p(m, C.c_uint8)),
           "oracle_reconstruct")
    return fh, m


def mlp_logits(params, stencils):
    """Scaled features and logits of stencils s[n][6]: returns (x[n][6], z[n][4])."""
    s = _f64(stencils).reshape(-1, 6)
    P = _f64(params)
    x = np.zeros_like(s)
    z = np.zeros((s.shape[0], 4))
    _check(_load().oracle_mlp_logits(_p(P, C.c_double), _p(s, C.c_double), s.shape[0],
                                     _p(x, C.c_double), _p(z, C.c_double)), "oracle_mlp_logits")
    return x, z


def mlp_logits_raw(params, x):
    x = _f64(x).reshape(-1, 6)
    P = _f64(params)
    z = np.zeros((x.shape[0], 4))
    _check(_load().oracle_mlp_logits_raw(_p(P, C.c_double), _p(x, C.c_double), x.shape[0],
                                         _p(z, C.c_double)), "oracle_mlp_logits_raw")
    return z


def teno(s):
    """TENO6-opt quantities of stencils s[n][6]: (beta[n][5] = beta_0..3 and
    beta_6, tau_6[n], chi[n][4], masks[n]) -- Sec. 2.2-2.3."""
    s = _f64(np.atleast_2d(s))
    n = s.shape[0]
    beta, tau, chi = np.zeros((n, 5)), np.zeros(n), np.zeros((n, 4))
    m = np.zeros(n, np.uint8)
    _check(_load().oracle_teno(_p(s, C.c_double), n, _p(beta, C.c_double), _p(tau, C.c_double),
                               _p(chi, C.c_double), _p(m, C.c_uint8)), "oracle_teno")
    return beta, tau, chi, m


def advection_rhs(u, dx, bc=BC_PERIODIC, params=None, selector=SEL_MLP, masks_in=None):
    u = _f64(u)
    n = u.size
    P = None if params is None else _f64(params)
    r = np.zeros(n)
    m = np.zeros(n + 1, np.uint8)
    mi = _u8(masks_in)
    _check(_load().oracle_advection_rhs(_p(u, C.c_double), n, dx, bc, _p(P, C.c_double), selector,
                                        _p(mi, C.c_uint8), _p(r, C.c_double), _p(m, C.c_uint8)),
           "oracle_advection_rhs")
    return r, m


def advection_step(u, dx, dt, n_steps, bc=BC_PERIODIC, params=None, selector=SEL_MLP,
                   masks_in=None):
    u = _f64(u).copy()
    P = None if params is None else _f64(params)
    mi = _u8(masks_in)
    _check(_load().oracle_advection_step(_p(u, C.c_double), u.size, dx, dt, n_steps, bc,
                                         _p(P, C.c_double), selector, _p(mi, C.c_uint8)),
           "oracle_advection_step")
    return u


def advection_rhs_adjoint(masks, dx, rbar, bc=BC_PERIODIC):
    rbar = _f64(rbar)
    m = _u8(masks)
    ub = np.zeros_like(rbar)
    _check(_load().oracle_advection_rhs_adjoint(_p(m, C.c_uint8), rbar.size, dx, bc,
                                                _p(rbar, C.c_double), _p(ub, C.c_double)),
           "oracle_advection_rhs_adjoint")
    return ub


def euler1d_rhs(q, offsets, dx, gamma=1.4, bc=BC_TRANSMISSIVE, params=None, selector=SEL_MLP,
                masks_in=None):
    """q: [3][total]; offsets: [n_problems+1]; dx: [n_problems].
    Returns (rhs[3][total], masks[3][total+n_problems], status[n_problems])."""
    q = _f64(q)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    npb = off.size - 1
    dxa = _f64(np.broadcast_to(np.asarray(dx, np.float64), (npb,)))
    P = None if params is None else _f64(params)
    total = int(off[-1])
    r = np.zeros((3, total))
    m = np.zeros((3, total + npb), np.uint8)
    st = np.zeros(npb, np.int32)
    mi = _u8(masks_in)
    _check(_load().oracle_euler1d_rhs(_p(q, C.c_double), _p(off, C.c_int64), npb,
                                      _p(dxa, C.c_double), gamma, bc, _p(P, C.c_double), selector,
                                      _p(mi, C.c_uint8), _p(r, C.c_double), _p(m, C.c_uint8),
                                      _p(st, C.c_int32)), "oracle_euler1d_rhs")
    return r, m, st


def euler1d_stencils(q, offsets, gamma=1.4, bc=BC_TRANSMISSIVE):
    """The classifier inputs of euler1d_rhs: the '+' and '-' characteristic
    split stencils of every field at every face, [faces][6][6] with
    evaluation e = 2 m + sign ('-' mirrored), faces numbered as the masks."""
    q = _f64(q)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    npb = off.size - 1
    out = np.zeros((int(off[-1]) + npb, 6, 6))
    _check(_load().oracle_euler1d_stencils(_p(q, C.c_double), _p(off, C.c_int64), npb, gamma, bc,
                                           _p(out, C.c_double)), "oracle_euler1d_stencils")
    return out


def euler1d_step(q, offsets, dx, cfl, n_steps, gamma=1.4, bc=BC_TRANSMISSIVE, params=None,
                 selector=SEL_MLP, t=None, status=None):
    q = _f64(q).copy()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    npb = off.size - 1
    dxa = _f64(np.broadcast_to(np.asarray(dx, np.float64), (npb,)))
    P = None if params is None else _f64(params)
    tt = np.zeros(npb) if t is None else _f64(t).copy()
    st = np.zeros(npb, np.int32) if status is None else np.ascontiguousarray(status, np.int32).copy()
    _check(_load().oracle_euler1d_step(_p(q, C.c_double), _p(off, C.c_int64), npb,
                                       _p(dxa, C.c_double), gamma, bc, cfl, n_steps,
                                       _p(P, C.c_double), selector, _p(tt, C.c_double),
                                       _p(st, C.c_int32)), "oracle_euler1d_step")
    return q, tt, st


def burgers_rhs(u, offsets, dx, bc=BC_TRANSMISSIVE, params=None, selector=SEL_TENO, masks_in=None):
    """Inviscid Burgers (Sec. 4.3) on a batch of lines u[total].
    Returns (rhs[total], masks[total + n_problems], status[n_problems])."""
    u = _f64(u)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    npb = off.size - 1
    dxa = _f64(np.broadcast_to(np.asarray(dx, np.float64), (npb,)))
    P = None if params is None else _f64(params)
    total = int(off[-1])
    r = np.zeros(total)
    m = np.zeros(total + npb, np.uint8)
    st = np.zeros(npb, np.int32)
    mi = _u8(masks_in)
    _check(_load().oracle_burgers_rhs(_p(u, C.c_double), _p(off, C.c_int64), npb, _p(dxa, C.c_double),
                                      bc, _p(P, C.c_double), selector, _p(mi, C.c_uint8),
                                      _p(r, C.c_double), _p(m, C.c_uint8), _p(st, C.c_int32)),
           "oracle_burgers_rhs")
    return r, m, st


def burgers_step(u, offsets, dx, cfl, n_steps, bc=BC_TRANSMISSIVE, params=None, selector=SEL_TENO,
                 t=None, status=None):
    u = _f64(u).copy()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    npb = off.size - 1
    dxa = _f64(np.broadcast_to(np.asarray(dx, np.float64), (npb,)))
    P = None if params is None else _f64(params)
    tt = np.zeros(npb) if t is None else _f64(t).copy()
    st = np.zeros(npb, np.int32) if status is None else np.ascontiguousarray(status, np.int32).copy()
    _check(_load().oracle_burgers_step(_p(u, C.c_double), _p(off, C.c_int64), npb, _p(dxa, C.c_double),
                                       bc, cfl, n_steps, _p(P, C.c_double), selector,
                                       _p(tt, C.c_double), _p(st, C.c_int32)), "oracle_burgers_step")
    return u, tt, st


def euler2d_rhs(q, dx, dy, gamma=1.4, bc=BC_TRANSMISSIVE, params=None, selector=SEL_MLP,
                masks_in=None):
    """q: [4][ny][nx].  Returns (rhs, masks_x[4][ny][nx+1], masks_y[4][ny+1][nx], status)."""
    q = _f64(q)
    _, ny, nx = q.shape
    P = None if params is None else _f64(params)
    r = np.zeros_like(q)
    mx = np.zeros((4, ny, nx + 1), np.uint8)
    my = np.zeros((4, ny + 1, nx), np.uint8)
    st = np.zeros(1, np.int32)
    mxi = myi = None
    if masks_in is not None:
        mxi, myi = _u8(masks_in[0]), _u8(masks_in[1])
    _check(_load().oracle_euler2d_rhs(_p(q, C.c_double), nx, ny, dx, dy, gamma, bc,
                                      _p(P, C.c_double), selector, _p(mxi, C.c_uint8),
                                      _p(myi, C.c_uint8), _p(r, C.c_double), _p(mx, C.c_uint8),
                                      _p(my, C.c_uint8), _p(st, C.c_int32)), "oracle_euler2d_rhs")
    return r, mx, my, st


def euler2d_step(q, dx, dy, cfl, n_steps, gamma=1.4, bc=BC_TRANSMISSIVE, params=None,
                 selector=SEL_MLP, t=0.0):
    q = _f64(q).copy()
    _, ny, nx = q.shape
    P = None if params is None else _f64(params)
    tt = np.array([t], np.float64)
    st = np.zeros(1, np.int32)
    _check(_load().oracle_euler2d_step(_p(q, C.c_double), nx, ny, dx, dy, gamma, bc, cfl, n_steps,
                                       _p(P, C.c_double), selector, _p(tt, C.c_double),
                                       _p(st, C.c_int32)), "oracle_euler2d_step")
    return q, float(tt[0]), int(st[0])


def euler1d_eigen(qL, qR, gamma=1.4):
    L = np.zeros(9)
    R = np.zeros(9)
    _load().oracle_euler1d_eigen(_p(_f64(qL), C.c_double), _p(_f64(qR), C.c_double), gamma,
                                 _p(L, C.c_double), _p(R, C.c_double))
    return L.reshape(3, 3), R.reshape(3, 3)


def euler2d_eigen(qL, qR, gamma=1.4, direction=0):
    L = np.zeros(16)
    R = np.zeros(16)
    _load().oracle_euler2d_eigen(_p(_f64(qL), C.c_double), _p(_f64(qR), C.c_double), gamma,
                                 direction, _p(L, C.c_double), _p(R, C.c_double))
    return L.reshape(4, 4), R.reshape(4, 4)


def euler1d_flux(q, gamma=1.4):
    F = np.zeros(3)
    _load().oracle_euler1d_flux(_p(_f64(q), C.c_double), gamma, _p(F, C.c_double))
    return F


def euler2d_flux(q, gamma=1.4, direction=0):
    F = np.zeros(4)
    _load().oracle_euler2d_flux(_p(_f64(q), C.c_double), gamma, direction, _p(F, C.c_double))
    return F


def bce_grad(params, x, y):
    """Mean BCE loss and its gradient over raw stencils x[n][6] (scaled inside), labels y[n]."""
    P = _f64(params)
    x = _f64(x).reshape(-1, 6)
    y = _u8(y)
    g = np.zeros(NPARAM)
    loss = np.zeros(1)
    _check(_load().oracle_bce_grad(_p(P, C.c_double), _p(x, C.c_double), _p(y, C.c_uint8),
                                   x.shape[0], _p(loss, C.c_double), _p(g, C.c_double)),
           "oracle_bce_grad")
    return float(loss[0]), g


def train(params, adam_m, adam_v, adam_t, x, y, idx, batch, lr, beta1=0.9, beta2=0.999,
          eps=1e-8):
    """Adam over the samples idx in order; updates params/adam_m/adam_v in place.
    Returns (mean loss, new step count)."""
    for a in (params, adam_m, adam_v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    x = _f64(x).reshape(-1, 6)
    y = _u8(y)
    idx = np.ascontiguousarray(idx, np.int64)
    t = np.array([adam_t], np.int64)
    loss = np.zeros(1)
    _check(_load().oracle_train(_p(params, C.c_double), _p(adam_m, C.c_double),
                                _p(adam_v, C.c_double), _p(t, C.c_int64), _p(x, C.c_double),
                                _p(y, C.c_uint8), _p(idx, C.c_int64), idx.size, batch, lr, beta1,
                                beta2, eps, _p(loss, C.c_double)), "oracle_train")
    return float(loss[0]), int(t[0])
