"""TENO6-opt selector (NENO6_SEL_TENO) on the GPU against the FP64 oracle.

The selection is decided in FP64 in every mode from the stencil values as
the kernel holds them, with the operation order the oracle uses, so:
* FP64 mode: labels, face values and right-hand sides bit for bit;
* FP32 / BF16 / FP16 modes on scalar stencils (no projection): labels bit for
  bit against the oracle on the same FP32-rounded values, face values to
  FP32 round-off;
* Euler in the fast modes: right-hand side against the FP64 path on the
  same state (TENO labels near smooth extrema follow the FP32 round-off of
  the projected stencils; the flip rate is printed).
"""
import numpy as np
import pytest

import oracle
from paper_2207_08500_amd import inputs
from tests._helpers import dev, host, label_flip_rate, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    return native, torch


def _same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape
    bad = ~((a == b) | (np.isnan(a) & np.isnan(b)))
    assert not bad.any(), "first mismatch at %s: %r vs %r (%d of %d differ)" % (
        np.argwhere(bad)[0], a[bad][0], b[bad][0], bad.sum(), bad.size)


def _stencil_data(seed, n):
    """Smooth pieces, jumps of several sizes and exactly constant runs."""
    f = inputs.random_stencils(seed, (n + 10) // 6 + 1).ravel()[: n + 5].copy()
    f[n // 3: n // 3 + 40] = 2.5  # constant run: every indicator exactly 0
    return f


@pytest.mark.parametrize("n", [1, 64, 65, 3001])
@pytest.mark.parametrize("sign", [1, -1])
def test_teno_reconstruct_fp64_bitwise(ctx, n, sign):
    native, torch = ctx
    f = _stencil_data(300 + n, n)
    fh_o, m_o = oracle.reconstruct(f, sign, None, oracle.SEL_TENO)
    fh = torch.zeros(n, dtype=torch.float64, device="cuda")
    m = torch.zeros(n, dtype=torch.uint8, device="cuda")
    native.neno6_reconstruct(None, dev(f), sign, native.FP64, native.SEL_TENO, fh, masks_out=m)
    torch.cuda.synchronize()
    _same(host(m), m_o)
    _same(host(fh), fh_o)
    if n >= 64:
        assert 0 < (m_o == 15).mean() < 1  # both smooth and non-smooth stencils occur


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_teno_reconstruct_reduced_labels_bitwise(ctx, prec):
    native, torch = ctx
    n = 4097
    f32 = _stencil_data(31, n).astype(np.float32)
    fh_o, m_o = oracle.reconstruct(f32.astype(np.float64), 1, None, oracle.SEL_TENO)
    fh = torch.zeros(n, dtype=torch.float32, device="cuda")
    m = torch.zeros(n, dtype=torch.uint8, device="cuda")
    native.neno6_reconstruct(None, dev(f32), 1, prec, native.SEL_TENO, fh, masks_out=m)
    torch.cuda.synchronize()
    _same(host(m), m_o)
    assert np.allclose(host(fh), fh_o, rtol=2e-6, atol=2e-6 * np.abs(fh_o).max())


def test_teno_euler1d_rhs_fp64_bitwise(ctx):
    native, torch = ctx
    sizes = [1, 2, 7, 64, 65, 300, 1000]
    q, off, dx = inputs.riemann1d_batch(77, sizes, perturb=True)
    r_o, m_o, st_o = oracle.euler1d_rhs(q, off, dx, 1.4, oracle.BC_TRANSMISSIVE, None,
                                        oracle.SEL_TENO)
    prob = native.Problem(native.EULER1D, native.FP64, native.SEL_TENO, native.TRANSMISSIVE, off, dx)
    qg = dev(q)
    r = torch.zeros_like(qg)
    m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
    st = torch.zeros(len(sizes), dtype=torch.int32, device="cuda")
    native.neno6_rhs(prob, None, qg, r, prob.workspace(), masks_out=m, status=st)
    torch.cuda.synchronize()
    _same(host(st), st_o)
    _same(host(m).reshape(m_o.shape), m_o)
    _same(host(r).reshape(r_o.shape), r_o)


def test_teno_euler2d_rhs_fp64_bitwise(ctx):
    native, torch = ctx
    nx, ny = 70, 45
    q = inputs.riemann2d(78, nx, ny)
    r_o, mx_o, my_o, st_o = oracle.euler2d_rhs(q, 1 / nx, 1 / ny, 1.4, oracle.BC_TRANSMISSIVE,
                                               None, oracle.SEL_TENO)
    prob = native.Problem(native.EULER2D, native.FP64, native.SEL_TENO, native.TRANSMISSIVE,
                          nx=nx, ny=ny, dx2d=1 / nx, dy2d=1 / ny)
    qg = dev(q)
    r = torch.zeros_like(qg)
    m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
    native.neno6_rhs(prob, None, qg, r, prob.workspace(), masks_out=m)
    torch.cuda.synchronize()
    mh = host(m)
    _same(mh[: mx_o.size].reshape(mx_o.shape), mx_o)
    _same(mh[mx_o.size:].reshape(my_o.shape), my_o)
    _same(host(r).reshape(r_o.shape), r_o)


def test_teno_advection_steps_fp64_bitwise(ctx):
    native, torch = ctx
    n, dx = 200, 2.0 / 200
    u0 = inputs.advection_c1(inputs.BASE_SEED, n)
    u_o = oracle.advection_step(u0, dx, 0.4 * dx, 25, oracle.BC_PERIODIC, None, oracle.SEL_TENO)
    prob = native.Problem(native.ADVECTION, native.FP64, native.SEL_TENO, native.PERIODIC, [0, n], [dx])
    u = dev(u0)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    native.neno6_step(prob, None, u, 0.4, 25, t, st, prob.workspace())
    torch.cuda.synchronize()
    _same(host(u), u_o)


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_teno_euler1d_fast_modes(ctx, prec):
    """Riemann batch in FP32 state against the FP64 path on the same
    (FP32-rounded) state.  tau_6 measures a sixth-order cancellation, so near
    smooth extrema the FP32 round-off of the projected stencils decides
    which smooth candidates TENO keeps: labels there differ from the FP64
    path (about 28 % of labels on this batch, in the nearly constant
    acoustic fields), and the right-hand side moves by a few 1e-4 (relative
    L1), since every candidate kept or dropped there is a smooth one.  On the
    unperturbed batch (piecewise constant states) labels agree exactly."""
    native, torch = ctx
    for perturb in (False, True):
        q, off, dx = inputs.riemann1d_batch(79, (4000,) * 16, perturb=perturb)
        q32 = dev(q, torch.float32)
        masks, rhs = {}, {}
        for pr, qq in ((native.FP64, q32.double().contiguous()), (prec, q32)):
            prob = native.Problem(native.EULER1D, pr, native.SEL_TENO, native.TRANSMISSIVE, off, dx)
            m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
            r = torch.zeros_like(qq)
            native.neno6_rhs(prob, None, qq, r, prob.workspace(), masks_out=m)
            torch.cuda.synchronize()
            masks[pr], rhs[pr] = host(m), host(r).astype(np.float64).reshape(3, -1)
        flip = label_flip_rate(masks[prec], masks[native.FP64])
        d = np.abs(rhs[prec] - rhs[native.FP64]).sum(axis=1) / np.abs(rhs[native.FP64]).sum(axis=1)
        print("TENO prec %d vs FP64, perturb=%s: label flip rate %.3g, rhs relative L1 %.3g"
              % (prec, perturb, flip, d.max()))
        if not perturb:
            assert flip < 1e-4 and d.max() < 1e-5
        else:
            assert d.max() < 1e-3
